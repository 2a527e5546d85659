"""Continuous-batching server for shot simulations and FWI gradients.

Requests -- forward modelling, or misfit and gradient, of one shot on its own
2-D or 3-D grid -- arrive as a Poisson stream.  A request is admitted when a
slot is free and its HBM footprint (the job memory of fwi_job_bytes plus its
inputs and outputs) fits the free budget; its velocity model and wavefield
state then stay resident on the device until it finishes.  Every chunk of K
time steps, the scheduled jobs advance together through fwi_jobs_advance,
whose launches each cover the tiles of every job; requests that arrived in
the meantime join at the next chunk boundary and finished ones leave.  By
default each chunk runs the resident jobs with the least remaining work that
fit the fill limit (preemptive shortest-remaining-work first); long jobs
pause, resident, while short ones pass.

The plain baseline is the same loop with one slot: one request at a time,
each with launches of its own.

    python -m paper_1912_08063_amd.serve --requests 200 --rate 0.8
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time
from typing import List, Optional

import numpy as np

from . import workloads as wl


@dataclasses.dataclass
class Request:
    rid: int
    kind: str                      # "forward" or "gradient"
    arrival: float                 # seconds after the stream starts
    problem: wl.Problem            # one shot
    obs: Optional[np.ndarray] = None   # gradient: observed traces [1][nt][R]
    ckpt: Optional[str] = None     # gradient: checkpoint spec (None: the server's)


@dataclasses.dataclass
class Result:
    rid: int
    kind: str
    arrival: float
    admitted: float
    done: float
    traces: Optional[np.ndarray] = None
    dv: Optional[np.ndarray] = None
    misfit: Optional[float] = None
    seq: int = -1                  # completion index within the run
    work: int = 0                  # padded cells x time steps, at admission
    error: Optional[str] = None    # set when the request was refused or failed

    @property
    def latency(self):
        return self.done - self.arrival


def _round16(x):
    return max(16, int(round(x / 16.0)) * 16)


def make_request_problem(rid, seed=4, scale=1.0, force=None):
    """One request of the mixed stream: 2-D N^2 with N ~ U[256, 2048] or 3-D N^3
    with N ~ U[128, 384] (50/50, rounded to 16), 1000-4000 steps, layered
    model (8-12 layers, 1500-4500 m/s, 5 % noise), 10 Hz Ricker at the surface,
    dt from CFL 0.4, 20 (2-D) / 24 (3-D) sponge cells.  `scale` shrinks the
    grid edge and the step count (tests)."""
    rng = np.random.default_rng(seed + rid)
    kind = "gradient" if rng.random() < 0.3 else "forward"
    dim = 2 if rng.random() < 0.5 else 3
    if force:
        kind = force.get("kind", kind)
        dim = force.get("dim", dim)
    if dim == 2:
        n = _round16(rng.uniform(256, 2048) * scale)
        shape = (n, n)
        nb = 20
    else:
        n = _round16(rng.uniform(128, 384) * scale)
        shape = (n, n, n)
        nb = 24
    nt = max(8, int(rng.integers(1000, 4001) * scale))
    v = wl.layered(shape, rng)
    dx = 10.0
    dt = wl.dt_from_cfl(float(v.max()), dx, 0.4)
    src = [[4] + [s // 2 for s in shape[1:]]]
    rec = wl.surface_receivers(shape, 4, stride=1 if dim == 2 else 4)
    P = wl._pack("req%d-%s-%dd-%d-nt%d" % (rid, kind, dim, n, nt), v, dx, dt, nt, 8, nb, 10.0,
                 src, rec)
    return kind, P


def make_stream(n, rate, seed=4, scale=1.0, force=None) -> List[Request]:
    """n requests with exponential inter-arrival times of mean 1/rate seconds."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n)) if rate > 0 else np.zeros(n)
    out = []
    for i in range(n):
        kind, P = make_request_problem(i, seed, scale, force)
        out.append(Request(i, kind, float(t[i]), P))
    return out


def attach_observed(requests, device="cuda", perturb=1.02):
    """Observed data of gradient requests: the library's forward on perturb * v
    (computed before the stream starts, not timed)."""
    import torch
    from . import api
    for r in requests:
        if r.kind != "gradient" or r.obs is not None:
            continue
        P = r.problem
        t = lambda a, d: torch.as_tensor(np.ascontiguousarray(a), device=device).to(d)
        cfg = api.Config(dt=P.dt, dx=P.dx, order=P.order, nsponge=P.nb, eta_max=P.eta_max)
        tr = api.forward(t(P.v * perturb, torch.float32), t(P.wavelet, torch.float32),
                         t(P.src_pos, torch.int32), t(P.rec_pos, torch.int32), cfg)
        r.obs = tr.cpu().numpy()
    return requests


class _Active:
    pass


POLICIES = ("srpt", "srpt_oldest", "fifo")


class Server:
    """Admission by HBM footprint, resident job state, continuous batching.

    policy "srpt": every arrived request that fits the memory budget is
    admitted and stays resident; each chunk advances the resident jobs with
    the least remaining work (padded cells x time steps left) while
    their cells stay within fill_cells, so a long job yields the GPU to short
    ones that arrive during it and resumes afterwards.
    policy "srpt_oldest": as srpt, and the job that arrived first among the
    resident ones also advances every chunk (its cells outside the fill
    limit), which bounds how long any job can be paused.
    policy "fifo": requests are admitted in arrival order while their cells
    fit fill_cells, and every admitted job advances each chunk.
    grad_ckpt: the checkpoint policy of gradient requests that name none, a
    spec as for api.gradient ("all", "every:K", "revolve:SLOTS|BUDGET";
    None: every chunk steps); a revolve job keeps SLOTS snapshots in place
    of nt/K and recomputes more.
    At 0.8x the saturated rate, srpt cuts the median latency 4x to 8x
    against one-at-a-time serving.  On the stream at x0.25 size its p99 is
    also 27 % lower; at full size p99 is the largest 3-D gradient jobs,
    which yield to every shorter job and finish 15-45 % later than
    one-at-a-time, while fifo keeps one-at-a-time's p99 within 2 %.
    fill_cells 8 M: at x0.25 size p50 0.035 s and p99 0.32 s, against
    0.042 s and 0.53 s with 24 M (more co-scheduled cells make every step of
    the jobs that share a launch longer) and 0.011 s and 0.76 s with 1 M."""

    def __init__(self, device="cuda", hbm_budget=None, max_active=64, chunk=50,
                 keep_outputs=False, fill_cells=8_000_000, policy="srpt", grad_ckpt=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        if hbm_budget is None:
            # blocks that torch's caching allocator holds from earlier work
            # are free for jobs: hand them back before measuring
            torch.cuda.empty_cache()
            free, _ = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(0.8 * free)
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.chunk = int(chunk)
        self.keep = keep_outputs
        # co-schedule jobs only while their padded cells per step stay below
        # what saturates the GPU: small jobs batch, a big job runs (nearly)
        # alone instead of slowing every other job down
        self.fill_cells = fill_cells
        if policy not in POLICIES:
            raise ValueError("policy must be one of %s" % (POLICIES,))
        self.policy = policy
        self.grad_ckpt = grad_ckpt
        self.ws = None

    # ---------------------------------------------------------------- sizes
    def _problem(self, P):
        from . import _lib
        p = _lib.FwiProblem()
        p.ndim = P.v.ndim
        for i, n in enumerate(P.v.shape):
            p.shape[i] = int(n)
        p.dx, p.dt, p.nt = P.dx, P.dt, P.nt
        p.order, p.nsponge, p.eta_max = P.order, P.nb, P.eta_max
        p.nshots, p.nrec = 1, P.nrec
        return p

    def _ckpt(self, req: Request):
        """The checkpoint policy of a gradient request (None: every chunk)."""
        spec = req.ckpt or self.grad_ckpt
        if req.kind != "gradient" or spec is None:
            return None
        from . import api
        return api.parse_ckpt(spec)

    def footprint(self, req: Request) -> int:
        from . import _lib
        P = req.problem
        kind = _lib.JOB_GRADIENT if req.kind == "gradient" else _lib.JOB_FORWARD
        job = _lib.fwi_job_bytes(self._problem(P), kind, self.chunk, self._ckpt(req))
        io = 4 * (P.v.size + P.nt + P.nt * P.nrec * (2 if req.kind == "gradient" else 1))
        io += 4 * P.v.size if req.kind == "gradient" else 0
        return job + io + 4 * P.src_pos.size + 4 * P.rec_pos.size

    # -------------------------------------------------------------- admission
    @staticmethod
    def check_request(req: Request):
        """The arrays of a one-shot request against its problem (the job API
        reads them by the problem's sizes)."""
        P = req.problem
        D, nt = P.v.ndim, P.nt
        if req.kind not in ("forward", "gradient"):
            raise ValueError("request %d: kind must be forward or gradient" % req.rid)
        if D not in (2, 3):
            raise ValueError("request %d: the model must be 2-D or 3-D" % req.rid)
        if np.shape(P.src_pos) != (1, D):
            raise ValueError("request %d: src_pos must be [1][%d]" % (req.rid, D))
        if np.ndim(P.rec_pos) != 3 or np.shape(P.rec_pos)[0] != 1 or np.shape(P.rec_pos)[2] != D:
            raise ValueError("request %d: rec_pos must be [1][R][%d]" % (req.rid, D))
        if np.shape(P.wavelet) != (1, nt):
            raise ValueError("request %d: wavelet must be [1][%d]" % (req.rid, nt))
        if req.kind == "gradient" and np.shape(req.obs) != (1, nt, P.nrec):
            raise ValueError("request %d: obs must be [1][%d][%d]" % (req.rid, nt, P.nrec))
        if req.ckpt is not None:
            from . import api
            try:
                api.parse_ckpt(req.ckpt)
            except (ValueError, IndexError):
                raise ValueError("request %d: bad checkpoint spec %r" % (req.rid, req.ckpt))

    def _admit(self, req: Request, now):
        from . import _lib
        torch = self.torch
        P = req.problem
        dev = self.device
        t = lambda a, d: torch.as_tensor(np.ascontiguousarray(a), device=dev).to(d)
        a = _Active()
        a.req = req
        a.admitted = now
        a.v = t(P.v, torch.float32)
        a.w = t(P.wavelet, torch.float32)
        a.s = t(P.src_pos, torch.int32)
        a.r = t(P.rec_pos, torch.int32)
        grad = req.kind == "gradient"
        a.obs = t(req.obs, torch.float32) if grad else None
        a.traces = torch.empty((1, P.nt, P.nrec), dtype=torch.float32, device=dev)
        a.dv = torch.empty_like(a.v) if grad else None
        kind = _lib.JOB_GRADIENT if grad else _lib.JOB_FORWARD
        prob = self._problem(P)
        ckpt = self._ckpt(req)
        nbytes = _lib.fwi_job_bytes(prob, kind, self.chunk, ckpt)
        a.mem = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
        a.footprint = self.footprint(req)
        stream = torch.cuda.current_stream(dev).cuda_stream
        a.handle = _lib.fwi_job_create(
            prob, kind, self.chunk, ckpt, a.v.data_ptr(), a.w.data_ptr(), a.s.data_ptr(),
            a.r.data_ptr() if P.nrec else None, a.obs.data_ptr() if grad and P.nrec else None,
            a.traces.data_ptr() if P.nrec else None, a.dv.data_ptr() if grad else None,
            a.mem.data_ptr(), a.mem.numel(), stream)
        a.work = P.padded_cells * _lib.fwi_job_query(a.handle)[1]
        if grad:
            # the misfit is a double inside the job memory: a view of it can be
            # copied to the host without synchronising the stream
            a.mis_off = _lib.fwi_job_misfit_device(a.handle) - a.mem.data_ptr()
        return a

    def _collect(self, a):
        """Enqueues the copies of a finished job's outputs to pinned host memory
        (read once the stream has passed them)."""
        torch = self.torch
        pin = lambda t: torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
        a.host = {}
        if a.req.kind == "gradient":
            m = a.mem[a.mis_off:a.mis_off + 8].view(torch.float64)
            a.host["misfit"] = pin(m)
            a.host["misfit"].copy_(m, non_blocking=True)
        if self.keep:
            for name in ("traces", "dv"):
                t = getattr(a, name)
                if t is not None:
                    a.host[name] = pin(t)
                    a.host[name].copy_(t, non_blocking=True)

    def _finish(self, a, now):
        """Result of a job whose work (and output copies) the stream has passed."""
        from . import _lib
        res = Result(a.req.rid, a.req.kind, a.req.arrival, a.admitted, now, work=a.work)
        if "misfit" in a.host:
            res.misfit = float(a.host["misfit"][0])
        if "traces" in a.host:
            res.traces = a.host["traces"].numpy()
        if "dv" in a.host:
            res.dv = a.host["dv"].numpy()
        _lib.fwi_job_destroy(a.handle)
        a.handle = None
        return res

    def _select(self, active):
        """The jobs that advance this chunk (see the class docstring)."""
        from . import _lib
        if self.policy == "fifo" or not self.fill_cells:
            return active

        def work(a):
            _, left = _lib.fwi_job_query(a.handle)
            return (a.req.problem.padded_cells * left, a.req.arrival, a.req.rid)
        chosen, cells = [], 0
        rest = active
        if self.policy == "srpt_oldest":
            # the longest-waiting job always advances, outside the fill limit:
            # a long job is never starved by a stream of short ones
            oldest = min(active, key=lambda a: (a.req.arrival, a.req.rid))
            chosen.append(oldest)
            rest = [a for a in active if a is not oldest]
        for a in sorted(rest, key=work):
            c = a.req.problem.padded_cells
            if chosen and cells + c > self.fill_cells:
                continue
            chosen.append(a)
            cells += c
        return chosen

    # ------------------------------------------------------------------- loop
    def _reject(self, req: Request, now, err):
        """A request that is refused or fails: retired with its error."""
        return Result(req.rid, req.kind, req.arrival, now, now, error=str(err))

    def run(self, requests: List[Request], realtime=True, log=None):
        """Serves the stream; returns (results, report dict).  A request that
        the library refuses (shapes, stability limit, positions, memory) or
        whose work fails is retired with Result.error set; the others are
        served as if it had not been there."""
        active = []
        try:
            return self._run(requests, realtime, log, active)
        finally:
            # every job handle still held (an exception left the loop) is freed
            from . import _lib
            for a in active:
                if getattr(a, "handle", None):
                    _lib.fwi_job_destroy(a.handle)
                    a.handle = None

    def _run(self, requests, realtime, log, active):
        """The serving loop.  Chunks are pipelined: the next chunk is enqueued
        before the previous one has finished, and a job's completion time is
        taken when the stream has passed the chunk that finished it (one HIP
        event per chunk), so the GPU never waits for the host between
        chunks."""
        import collections
        from . import _lib
        torch = self.torch
        results = []
        pending = []
        for r in sorted(requests, key=lambda r: (r.arrival, r.rid)):
            try:
                if r.kind == "gradient" and r.obs is None:
                    raise ValueError("gradient request %d has no observed data" % r.rid)
                self.check_request(r)
                pending.append(r)
            except ValueError as e:
                results.append(self._reject(r, r.arrival, e))
        used = 0
        cells = 0
        st = torch.cuda.current_stream(self.device)
        stream = st.cuda_stream
        ws_bytes = _lib.fwi_jobs_ws_bytes(self.max_active, self.chunk)
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else None
        virtual = 0.0
        chunks = 0
        inflight = collections.deque()   # (event, jobs finished by that chunk)
        closing = []                     # finished jobs whose chunk is still in flight

        def retire(wait_all):
            nonlocal used
            while inflight and (wait_all or len(inflight) > 1):
                ev, done = inflight.popleft()
                ev.synchronize()
                now = clock() if realtime else virtual
                for a in done:
                    results.append(self._finish(a, now))
                    results[-1].seq = len(results) - 1
                    used -= a.footprint
                    closing.remove(a)
                    if log and len(results) % 10 == 0:
                        log("%d requests done (last: %d, %s, latency %.3f s)" % (
                            len(results), a.req.rid, a.req.kind, results[-1].latency))

        try:
            while pending or active or inflight:
                now = clock() if realtime else virtual
                # admit arrived requests while slots and memory allow
                while pending and len(active) + len(closing) < self.max_active:
                    r = pending[0]
                    if realtime and r.arrival > now:
                        break
                    try:
                        need = self.footprint(r)
                    except _lib.FwiError as e:
                        pending.pop(0)
                        results.append(self._reject(r, now, e))
                        continue
                    if used + need > self.budget and (active or closing):
                        break
                    if (self.policy == "fifo" and self.fill_cells and active
                            and cells + r.problem.padded_cells > self.fill_cells):
                        break
                    pending.pop(0)
                    if need > self.budget:
                        results.append(self._reject(
                            r, now, "needs %d bytes, more than the budget %d" % (need, self.budget)))
                        continue
                    try:
                        a = self._admit(r, now)
                    except _lib.FwiError as e:
                        results.append(self._reject(r, now, e))
                        continue
                    used += a.footprint
                    cells += r.problem.padded_cells
                    active.append(a)
                if not active:
                    if inflight:
                        retire(True)
                    elif realtime and pending:
                        time.sleep(max(0.0, min(0.01, pending[0].arrival - clock())))
                    elif pending:
                        virtual = max(virtual, pending[0].arrival)
                    continue
                chosen = self._select(active)
                failed = {}
                try:
                    _lib.fwi_jobs_advance([a.handle for a in chosen], self.chunk,
                                          self.ws.data_ptr(), ws_bytes, stream)
                except _lib.FwiError:
                    # isolate the failing job(s): the others advance one by one
                    for a in chosen:
                        try:
                            _lib.fwi_jobs_advance([a.handle], self.chunk, self.ws.data_ptr(),
                                                  ws_bytes, stream)
                        except _lib.FwiError as e:
                            failed[id(a)] = e
                chunks += 1
                done, still = [], []
                for a in active:
                    if id(a) in failed:
                        torch.cuda.synchronize(self.device)   # its memory may still be read
                        now = clock() if realtime else virtual
                        results.append(self._reject(a.req, now, failed[id(a)]))
                        results[-1].admitted = a.admitted
                        _lib.fwi_job_destroy(a.handle)
                        a.handle = None
                        used -= a.footprint
                        cells -= a.req.problem.padded_cells
                    elif _lib.fwi_job_query(a.handle)[0]:
                        self._collect(a)
                        done.append(a)
                        cells -= a.req.problem.padded_cells
                    else:
                        still.append(a)
                active[:] = still
                closing.extend(done)
                ev = torch.cuda.Event()
                ev.record(st)
                inflight.append((ev, done))
                retire(False)
            retire(True)
        finally:
            for a in closing:
                active.append(a)
        makespan = (clock() if realtime else virtual)
        ok = [r for r in results if r.error is None]
        lat = np.array([r.latency for r in ok])
        report = {
            "requests": len(ok), "failed": len(results) - len(ok),
            "chunks": chunks, "chunk_steps": self.chunk,
            "max_active": self.max_active, "fill_cells": self.fill_cells, "policy": self.policy,
            "makespan_s": makespan,
            "shots_per_s": len(ok) / makespan if makespan > 0 else None,
            "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_latency_s": float(lat.mean()) if len(lat) else None,
        }
        return sorted(results, key=lambda r: r.rid), report


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--rate", type=float, default=None,
                    help="arrivals per second (default: 0.8 x the measured saturated rate)")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--chunk", type=int, default=50)
    ap.add_argument("--max-active", type=int, default=64)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--policy", choices=list(POLICIES), default="srpt",
                    help="batched server's scheduling (the plain server runs one job at a time)")
    ap.add_argument("--compare", default="",
                    help="comma list of other batched policies to serve the same stream with")
    args = ap.parse_args(argv)
    log = lambda m: print("[serve] " + m, file=sys.stderr, flush=True)
    reqs = []
    for i in range(args.requests):   # generated one by one, with progress
        kind, P = make_request_problem(i, args.seed, args.scale)
        reqs.append(Request(i, kind, 0.0, P))
        if (i + 1) % 20 == 0:
            log("generated %d requests" % (i + 1))
    log("observed data for %d gradient requests" % sum(r.kind == "gradient" for r in reqs))
    for i in range(0, len(reqs), 20):
        attach_observed(reqs[i:i + 20])
        log("observed data up to request %d" % min(i + 20, len(reqs)))
    rate = args.rate
    out = {}
    if rate is None:
        # saturated throughput: everything arrives at t = 0
        for r in reqs:
            r.arrival = 0.0
        _, sat = Server(max_active=args.max_active, chunk=args.chunk,
                        policy=args.policy).run(reqs, realtime=True, log=log)
        out["saturated"] = sat
        rate = 0.8 * sat["shots_per_s"]
        log("saturated: %.2f shots/s" % sat["shots_per_s"])
    arr = np.cumsum(np.random.default_rng(args.seed).exponential(1.0 / rate, len(reqs)))
    for r, t in zip(reqs, arr):
        r.arrival = float(t)
    _, rep = Server(max_active=args.max_active, chunk=args.chunk,
                    policy=args.policy).run(reqs, realtime=True, log=log)
    out["batched"] = dict(rep, rate=rate)
    log("batched: p50 %.3f s p99 %.3f s" % (rep["p50_latency_s"], rep["p99_latency_s"]))
    for pol in [p for p in args.compare.split(",") if p and p != args.policy]:
        _, repo = Server(max_active=args.max_active, chunk=args.chunk,
                         policy=pol).run(reqs, realtime=True, log=log)
        out["batched_" + pol] = dict(repo, rate=rate)
        log("batched %s: p50 %.3f s p99 %.3f s" % (pol, repo["p50_latency_s"],
                                                    repo["p99_latency_s"]))
    if not args.skip_plain:
        _, rep1 = Server(max_active=1, chunk=args.chunk).run(reqs, realtime=True, log=log)
        out["plain"] = dict(rep1, rate=rate)
        log("plain: p50 %.3f s p99 %.3f s" % (rep1["p50_latency_s"], rep1["p99_latency_s"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
