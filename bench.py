#!/usr/bin/env python3
"""Benchmark of the FWI hot path on one MI355X.

A step is one complete forward modelling run of the 3-D workload (256^3 model
grid, 24-cell sponge, 8th-order stencil, 2000 time steps, 256x256 receivers,
seeded layered velocity), with every input already resident in HBM.  The
line printed on stdout is JSON:

    value      Gcell-updates/s over padded cells (cells x time steps / s)
    roofline   the stencil step kernel against the HBM peak (16 algorithmic
               bytes per cell-update: read p, p_prev, kappa; write p_next)
    cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload

Only one GPU is used: --gpus above 1 exits with a message.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gcell-updates/s + %HBM roofline; gradient shots/s vs plain; p99 latency"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = 16


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def recorded_traffic():
    """HBM bytes per step launch from the rocprofv3 counter runs recorded in
    profiles/, or None if the kernel or runtime source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_k_step3d_fwd_layered304.json")
    try:
        rec = json.load(open(path))
        for src, digest in rec["sources_sha1"].items():
            if hashlib.sha1(open(os.path.join(ROOT, src), "rb").read()).hexdigest() != digest:
                return None
        return rec["traffic_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        return None


def cpu_model():
    """The host CPU's model name (Linux), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(P, nt_sample):
    """The oracle as it stands, on the same model for nt_sample steps."""
    import oracle
    t0 = time.perf_counter()
    oracle.forward(P.v, P.wavelet[:, :nt_sample], P.src_pos, P.rec_pos, P.dx, P.dt, P.order,
                   P.nb, P.eta_max)
    secs = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": P.padded_cells * nt_sample / secs / 1e9, "unit": "Gcell-updates/s",
            "cores": cores, "cpu": cpu_model(), "host_cpus": os.cpu_count(), "kind": "oracle",
            "sample": "fp64 oracle forward on the same 304^3 padded grid, %d of %d time steps "
                      "(%.1f s, set-up included)" % (nt_sample, P.nt, secs)}


def fstride_of(P):
    """Floats per field allocation of a 3-D problem (the library's layout: the
    padded grid plus an M-cell zero frame, rows padded to 64 floats)."""
    M = P.order // 2
    nz, ny, nx = (n + 2 * P.nb for n in P.v.shape)
    pitch = -(-(nx + 2 * M) // 64) * 64
    return (nz + 2 * M) * (ny + 2 * M) * pitch


def median_time(fn, reps, sync):
    """Median wall-clock seconds of `reps` calls of fn, each synchronised."""
    times = []
    for _ in range(reps):
        sync()
        t0 = time.perf_counter()
        fn()
        sync()
        times.append(time.perf_counter() - t0)
    return sorted(times)[len(times) // 2]


def tile_march(dev, P, step_us, reps=50):
    """The forward step's memory pattern without its stencil (fwi_tile_probe):
    the same 64 x 16 tiles, z-chunks (the step's own choice for this grid),
    block order and buffer loads, writing 2 cur + kappa prv.  Timed with HIP
    events bare, with the halo loads, with the LDS staging and barrier, and
    with the z-chunk warm-up planes as well (the step's whole access pattern),
    and the bare march and its halo loads with 64-bit loads per lane;
    `step_frac_of_pattern` is the whole pattern's time over the step's."""
    import torch
    from paper_1912_08063_amd import _lib
    st = torch.cuda.current_stream(dev)
    nz, ny, nx = (n + 2 * P.nb for n in P.v.shape)
    fs = fstride_of(P)
    bufs = [torch.zeros(fs, dtype=torch.float32, device=dev) for _ in range(4)]
    res = {}
    for name, mode in (("bare_us", 0), ("halos_us", 1), ("halos_lds_us", 3), ("pattern_us", 7),
                       ("bare_64bit_us", 8), ("halos_64bit_us", 9)):
        k = [0]

        def launch():
            i = k[0]
            k[0] += 1
            cur, prv, out = bufs[i % 3], bufs[(i + 1) % 3], bufs[(i + 2) % 3]
            return _lib.fwi_tile_probe(cur.data_ptr(), prv.data_ptr(), bufs[3].data_ptr(),
                                       out.data_ptr(), nz, ny, nx, 0, mode, st.cuda_stream)
        for _ in range(3):
            zc = launch()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            launch()
        e1.record(st)
        torch.cuda.synchronize()
        res[name] = round(e0.elapsed_time(e1) * 1e3 / reps, 2)
        res["zc"] = zc
    del bufs
    torch.cuda.empty_cache()
    res["pattern_GBps"] = round(BYTES_PER_UPDATE * P.padded_cells / (res["pattern_us"] * 1e-6) / 1e9, 1)
    res["step_frac_of_pattern"] = round(res["pattern_us"] / step_us, 4)
    return res


def stream_ceiling(dev, fstride, reps=50):
    """The hand-written 3-read/1-write stream (fwi_stream_probe) over four
    fields of the headline grid's size, rotated like the step's ring: the rate
    any kernel that reads p, p_prev and kappa' and writes p_next can reach on
    this GPU.  Every variant (load width, cache policy, grid) is timed with
    HIP events; the best is reported."""
    import torch
    from paper_1912_08063_amd import _lib
    st = torch.cuda.current_stream(dev)
    bufs = [torch.zeros(fstride, dtype=torch.float32, device=dev) for _ in range(4)]
    best = None
    names = {0: "32-bit", 1: "64-bit", 2: "128-bit"}
    for var in (0, 1, 2, 4, 5, 6, 8, 9, 10, 12, 13, 14):
        k = [0]

        def launch():
            i = k[0]
            k[0] += 1
            a, b, c, o = bufs[i % 3], bufs[(i + 1) % 3], bufs[3], bufs[(i + 2) % 3]
            _lib.fwi_stream_probe(a.data_ptr(), b.data_ptr(), c.data_ptr(), o.data_ptr(),
                                  fstride, var, st.cuda_stream)
        for _ in range(3):
            launch()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            launch()
        e1.record(st)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        gbs = 16.0 * fstride / (us * 1e-6) / 1e9
        if best is None or gbs > best["GBps"]:
            best = {"GBps": round(gbs, 1), "us_per_launch": round(us, 2),
                    "variant": "%s loads%s%s" % (names[var & 3], ", non-temporal" if var & 4 else "",
                                                 ", 2048-block grid" if var & 8 else "")}
    del bufs
    torch.cuda.empty_cache()
    best["frac_of_peak"] = round(best["GBps"] / HBM_PEAK_GBS, 4)
    return best


def c1_section(dev, calls=11):
    """The 2-D one-shot forward (128^2 Gaussian anomaly + 20-cell sponge,
    168^2 padded, 500 steps, 128 receivers): latency of one fwi_forward call
    (median of `calls`) and its Gcell-updates/s.  The grid is far too small to
    fill the GPU, so this measures the launch-bound path, not HBM."""
    import numpy as np
    import torch

    from paper_1912_08063_amd import api, workloads as wl
    P = wl.anomaly_2d()
    t = lambda a, d: torch.as_tensor(np.ascontiguousarray(a), device=dev).to(d)
    v, w = t(P.v, torch.float32), t(P.wavelet, torch.float32)
    s, r = t(P.src_pos, torch.int32), t(P.rec_pos, torch.int32)
    cfg = api.Config(dt=P.dt, dx=P.dx, order=P.order, nsponge=P.nb, eta_max=P.eta_max)
    ws = api.Workspace()
    tr = api.forward(v, w, s, r, cfg, workspace=ws)
    secs = median_time(lambda: api.forward(v, w, s, r, cfg, workspace=ws, out=tr), calls,
                       torch.cuda.synchronize)
    log("2-D one-shot forward: %.3f ms per call" % (secs * 1e3))
    return {"workload": "2-D acoustic forward, 128^2 Gaussian anomaly + 20-cell sponge "
                        "(168^2 padded), 8th order, 500 steps, 128 receivers",
            "latency_ms": round(secs * 1e3, 3), "us_per_step": round(secs * 1e6 / P.nt, 2),
            "Gcell_updates_per_s": round(P.padded_cells * P.nt / secs / 1e9, 3),
            "calls": calls}


def cpu_c1():
    """The oracle on the whole 2-D one-shot forward (all 500 steps)."""
    import oracle
    from paper_1912_08063_amd import workloads as wl
    P = wl.anomaly_2d()
    t0 = time.perf_counter()
    oracle.forward(P.v, P.wavelet, P.src_pos, P.rec_pos, P.dx, P.dt, P.order, P.nb, P.eta_max)
    secs = time.perf_counter() - t0
    return {"value": round(secs * 1e3, 2), "unit": "ms per 500-step forward", "kind": "oracle",
            "Gcell_updates_per_s": round(P.padded_cells * P.nt / secs / 1e9, 4),
            "sample": "fp64 oracle forward of the whole 2-D one-shot workload"}


def forward16_section(dev, nt):
    """The headline geometry at 16th order (M = 8, a 49-point star): the
    stencil step's rate and its HIP-event launch time."""
    import numpy as np
    import torch

    from paper_1912_08063_amd import api, workloads as wl
    P = wl.layered_3d(nt=nt, order=16)
    t = lambda a, d: torch.as_tensor(np.ascontiguousarray(a), device=dev).to(d)
    v, w = t(P.v, torch.float32), t(P.wavelet, torch.float32)
    s, r = t(P.src_pos, torch.int32), t(P.rec_pos, torch.int32)
    cfg = api.Config(dt=P.dt, dx=P.dx, order=P.order, nsponge=P.nb, eta_max=P.eta_max)
    ws = api.Workspace()
    api.forward(v, w, s, r, cfg, workspace=ws)                      # warm-up
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    api.forward(v, w, s, r, cfg, workspace=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    log("16th-order forward: %d steps in %.1f ms" % (nt, ms))
    us = ms * 1e3 / nt
    return {"workload": "3-D acoustic forward, 256^3 model + 24-cell sponge (304^3 padded), "
                        "16th order, %d steps" % nt,
            "Gcell_updates_per_s": round(P.padded_cells * nt / (ms * 1e-3) / 1e9, 3),
            "avg_launch_us": round(us, 2),
            "hbm_frac": round(BYTES_PER_UPDATE * P.padded_cells / (us * 1e-6) / 1e9
                              / HBM_PEAK_GBS, 4)}


def slab_section(dev, nt, reps=3):
    """The forward step on one GPU's share of a domain-decomposed model: a
    128 x 1024 x 1024 slab of a 1024^3 model split along z over 8 GPUs, at its
    real shape (halo exchange not included; the zero frame stands in for the
    received ghost planes).  Median of `reps` runs."""
    import numpy as np
    import torch

    from paper_1912_08063_amd import api, workloads as wl
    P = wl.slab_3d(nt=nt)
    t = lambda a, d: torch.as_tensor(np.ascontiguousarray(a), device=dev).to(d)
    v, w = t(P.v, torch.float32), t(P.wavelet, torch.float32)
    s, r = t(P.src_pos, torch.int32), t(P.rec_pos, torch.int32)
    cfg = api.Config(dt=P.dt, dx=P.dx, order=P.order, nsponge=P.nb, eta_max=P.eta_max)
    ws = api.Workspace()
    tr = api.forward(v, w, s, r, cfg, workspace=ws)                 # warm-up
    secs = median_time(lambda: api.forward(v, w, s, r, cfg, workspace=ws, out=tr), reps,
                       torch.cuda.synchronize)
    log("slab forward: %d steps in %.1f ms (median of %d)" % (nt, secs * 1e3, reps))
    us = secs * 1e6 / nt
    return {"workload": "3-D acoustic forward on one of 8 z-slabs of a 1024^3 layered model "
                        "(128 x 1024 x 1024 cells, no sponge), 8th order, %d steps, "
                        "256x256 receivers" % nt,
            "Gcell_updates_per_s": round(P.padded_cells * nt / secs / 1e9, 3),
            "us_per_step": round(us, 2),
            "hbm_frac": round(BYTES_PER_UPDATE * P.padded_cells / (us * 1e-6) / 1e9
                              / HBM_PEAK_GBS, 4),
            "runs": reps}


def cpu_gradient_2d(nt):
    """The oracle's misfit + gradient for one shot of the 2-D gradient workload,
    full length, beside the GPU's batched shots/s."""
    import numpy as np

    import oracle
    from paper_1912_08063_amd import workloads as wl
    P = wl.shots_2d(nt=nt, nshots=32)
    obs = np.zeros((1, P.nt, P.nrec))
    t0 = time.perf_counter()
    oracle.gradient(P.v_start, P.wavelet[:1], P.src_pos[:1], P.rec_pos[:1], obs, P.dx, P.dt,
                    P.order, P.nb, P.eta_max)
    secs = time.perf_counter() - t0
    return {"value": round(1.0 / secs, 4), "unit": "shots/s", "kind": "oracle",
            "sample": "fp64 oracle gradient (forward with stored states, adjoint, imaging "
                      "condition) of one of the 32 shots, all %d steps (%.1f s)" % (nt, secs)}


def cpu_gradient_3d(nt_sample, nt):
    """The oracle's gradient on the 3-D headline grid over two bounded step
    counts (its stored states grow with nt): set-up plus a per-step cost from
    their difference, extrapolated to the GPU section's nt."""
    import numpy as np

    import oracle
    from paper_1912_08063_amd import workloads as wl
    secs = []
    for n in (nt_sample // 2, nt_sample):
        P = wl.layered_3d(nt=n)
        obs = np.zeros((1, P.nt, P.nrec))
        t0 = time.perf_counter()
        oracle.gradient(0.98 * P.v, P.wavelet, P.src_pos, P.rec_pos, obs, P.dx, P.dt,
                        P.order, P.nb, P.eta_max)
        secs.append(time.perf_counter() - t0)
    per_step = (secs[1] - secs[0]) / (nt_sample - nt_sample // 2)
    total = secs[1] + (nt - nt_sample) * per_step
    return {"value": round(total, 1), "unit": "s per %d-step gradient" % nt, "kind": "oracle",
            "sample": "fp64 oracle gradient on the 304^3 padded grid at %d and %d steps "
                      "(%.1f s, %.1f s), extrapolated with the per-step difference to %d steps"
                      % (nt_sample // 2, nt_sample, secs[0], secs[1], nt)}


def _lib_workspace_bytes(prob, spec):
    from paper_1912_08063_amd import _lib, api
    return _lib.fwi_workspace_bytes(prob, _lib.MODE_GRADIENT, api.parse_ckpt(spec))


def gradient_section(dev, nt, shots, every, plain=True, reps=5):
    """2-D FWI gradient, 1024x320 model, 32 shots (median of `reps` runs each).
    Batched: one fwi_gradient call for all shots (each launch covers every
    shot's tiles); also with every forward level kept instead of every-50
    checkpoints, where the workspace fits.  Autograd: the same shots through FWIForward (forward with
    checkpoints, then backward of the least-squares loss).  Plain: one
    fwi_gradient call per shot."""
    import numpy as np
    import torch

    from paper_1912_08063_amd import api, workloads as wl
    from paper_1912_08063_amd.autograd import FWIForward
    P = wl.shots_2d(nt=nt, nshots=shots)
    t = lambda a, d: torch.as_tensor(np.ascontiguousarray(a), device=dev).to(d)
    w, s, r = t(P.wavelet, torch.float32), t(P.src_pos, torch.int32), t(P.rec_pos, torch.int32)
    cfg = api.Config(dt=P.dt, dx=P.dx, order=P.order, nsponge=P.nb, eta_max=P.eta_max,
                     ckpt="every:%d" % every)
    obs = api.forward(t(P.v, torch.float32), w, s, r, cfg)          # untimed
    v0 = t(P.v_start, torch.float32)
    ws = api.Workspace()
    sync = torch.cuda.synchronize
    out_mis = []
    api.gradient(v0, obs, w, s, r, cfg, workspace=ws)               # warm-up
    tb = median_time(lambda: out_mis.append(api.gradient(v0, obs, w, s, r, cfg, workspace=ws)[0]),
                     reps, sync)
    log("gradient batched: %d shots in %.3f s (median of %d)" % (shots, tb, reps))

    def autograd_step():
        vt = v0.clone().requires_grad_(True)
        tr = FWIForward.apply(vt, w, s, r, cfg)
        ((tr - obs) ** 2).sum().backward()
    autograd_step()                                                 # warm-up
    ta = median_time(autograd_step, reps, sync)
    log("gradient autograd: %d shots in %.3f s (median of %d)" % (shots, ta, reps))
    out = {"workload": "2-D FWI gradient, 1024x320 model + 20-cell sponge, %d shots, %d steps, "
                       "1024 receivers, every-%d checkpoints" % (shots, nt, every),
           "batched_shots_per_s": round(shots / tb, 3),
           "autograd_shots_per_s": round(shots / ta, 3),
           "misfit": out_mis[-1], "runs": reps}
    # the same batched call keeping every forward level in HBM (no recompute):
    # 3001 levels of 32 shots take 147 GB, which one MI355X holds
    import dataclasses
    cfg_all = dataclasses.replace(cfg, ckpt="all")
    prob = api.make_problem(v0, nt, cfg_all, shots, P.nrec)
    need = _lib_workspace_bytes(prob, "all")
    free, _ = torch.cuda.mem_get_info(dev)
    if need < 0.9 * free:
        ws_all = api.Workspace()
        mis_all = []
        api.gradient(v0, obs, w, s, r, cfg_all, workspace=ws_all)   # warm-up
        tl = median_time(lambda: mis_all.append(api.gradient(v0, obs, w, s, r, cfg_all,
                                                             workspace=ws_all)[0]), 3, sync)
        log("gradient batched, all levels kept: %d shots in %.3f s" % (shots, tl))
        out.update(all_levels_shots_per_s=round(shots / tl, 3),
                   all_levels_workspace_GB=round(need / 1e9, 1),
                   all_levels_misfit_equal=bool(mis_all[-1] == out_mis[-1]))
        del ws_all
        torch.cuda.empty_cache()
    if not plain:
        return out
    ws1 = api.Workspace()
    api.gradient(v0, obs[:1], w[:1], s[:1], r[:1], cfg, workspace=ws1)

    def plain_run():
        for i in range(shots):
            api.gradient(v0, obs[i:i + 1], w[i:i + 1], s[i:i + 1], r[i:i + 1], cfg,
                         workspace=ws1)
    tp = median_time(plain_run, max(1, reps // 2 + 1), sync)
    log("gradient plain: %d shots in %.3f s" % (shots, tp))
    out.update(plain_shots_per_s=round(shots / tp, 3), speedup=round(tp / tb, 3))
    return out


def gradient3d_section(dev, nt, every, order=8, reps=5):
    """3-D gradient on the headline geometry (304^3 padded, 8th order) over nt
    steps with every-k checkpoints: forward, recompute of each segment,
    adjoint and imaging condition.  Reported against the forward alone, and
    with every level kept instead where the workspace fits."""
    import numpy as np
    import torch

    from paper_1912_08063_amd import api, workloads as wl
    P = wl.layered_3d(nt=nt, order=order)
    t = lambda a, d: torch.as_tensor(np.ascontiguousarray(a), device=dev).to(d)
    v, w = t(P.v, torch.float32), t(P.wavelet, torch.float32)
    s, r = t(P.src_pos, torch.int32), t(P.rec_pos, torch.int32)
    cfg = api.Config(dt=P.dt, dx=P.dx, order=P.order, nsponge=P.nb, eta_max=P.eta_max,
                     ckpt="every:%d" % every)
    obs = api.forward(v, w, s, r, cfg)                              # untimed
    v0 = 0.98 * v
    ws, wf = api.Workspace(), api.Workspace()
    api.gradient(v0, obs, w, s, r, cfg, workspace=ws)               # warm-up
    api.forward(v0, w, s, r, cfg, workspace=wf)
    mis = []
    sync = torch.cuda.synchronize
    tg = median_time(lambda: mis.append(api.gradient(v0, obs, w, s, r, cfg, workspace=ws)[0]),
                     reps, sync)
    tf = median_time(lambda: api.forward(v0, w, s, r, cfg, workspace=wf), reps, sync)
    log("3-D gradient: %.3f s (forward %.3f s), medians of %d" % (tg, tf, reps))
    out = {"workload": "3-D FWI gradient, 256^3 model + 24-cell sponge (304^3 padded), "
                       "order %d, %d steps, every-%d checkpoints" % (order, nt, every),
           "gradient_s": round(tg, 4), "forward_s": round(tf, 4),
           "gradient_over_forward": round(tg / tf, 3), "misfit": mis[-1], "runs": reps}
    # every forward level kept in HBM (no recompute), where it fits: 601
    # levels of the 304^3 grid take 75 GB
    import dataclasses
    del ws
    torch.cuda.empty_cache()
    cfg_all = dataclasses.replace(cfg, ckpt="all")
    need = _lib_workspace_bytes(api.make_problem(v0, nt, cfg_all, 1, P.nrec), "all")
    free, _ = torch.cuda.mem_get_info(dev)
    if need < 0.9 * free:
        wa, mis_all = api.Workspace(), []
        api.gradient(v0, obs, w, s, r, cfg_all, workspace=wa)           # warm-up
        ta = median_time(lambda: mis_all.append(api.gradient(v0, obs, w, s, r, cfg_all,
                                                             workspace=wa)[0]), 3, sync)
        log("3-D gradient, all levels kept: %.3f s" % ta)
        out.update(all_levels_gradient_s=round(ta, 4), all_levels_workspace_GB=round(need / 1e9, 1),
                   all_levels_misfit_equal=bool(mis_all[-1] == mis[-1]))
        del wa
        torch.cuda.empty_cache()
    return out


def salt3d_section(dev, nt, crop_nt=600, budget="40e9", reps=5):
    """3-D salt workload (512x512x256 model + 24-cell sponge, 560x560x304
    padded, 8th order, 512x512 receivers): the forward's rate, and the
    gradient with binomial (revolve) checkpointing under a snapshot budget,
    against every-50 snapshots."""
    import dataclasses

    import numpy as np
    import torch

    from paper_1912_08063_amd import _lib, api, workloads as wl
    P = wl.salt_3d(nt=nt)
    t = lambda a, d: torch.as_tensor(np.ascontiguousarray(a), device=dev).to(d)
    v, w = t(P.v, torch.float32), t(P.wavelet, torch.float32)
    s, r = t(P.src_pos, torch.int32), t(P.rec_pos, torch.int32)
    cfg = api.Config(dt=P.dt, dx=P.dx, order=P.order, nsponge=P.nb, eta_max=P.eta_max,
                     ckpt="revolve:%s" % budget)
    obs = torch.empty((1, nt, P.nrec), dtype=torch.float32, device=dev)
    ws = api.Workspace()
    sync = torch.cuda.synchronize
    api.forward(v, w, s, r, cfg, workspace=ws, out=obs)            # warm-up
    tf = median_time(lambda: api.forward(v, w, s, r, cfg, workspace=ws, out=obs), reps, sync)
    log("salt forward: %d steps in %.3f s (median of %d)" % (nt, tf, reps))
    v0 = t(P.v_start, torch.float32)
    del ws
    out = {"workload": "3-D FWI, salt model 512x512x256 + 24-cell sponge (560x560x304 padded), "
                       "8th order, %d steps, 512x512 receivers" % nt,
           "forward_s": round(tf, 4),
           "forward_Gcell_updates_per_s": round(P.padded_cells * nt / tf / 1e9, 3),
           "forward_hbm_frac": round(BYTES_PER_UPDATE * P.padded_cells * nt / tf / 1e9
                                     / HBM_PEAK_GBS, 4)}
    # bytes per snapshot slot (two levels of the padded, framed field), from
    # the gradient's workspace size at one and at two slots
    prob = api.make_problem(v0, nt, cfg, 1, P.nrec)
    wsb = [_lib.fwi_workspace_bytes(prob, _lib.MODE_GRADIENT, api.parse_ckpt("revolve:%d" % k))
           for k in (1, 2)]
    slot_bytes = wsb[1] - wsb[0]
    slots = int(float(budget)) // slot_bytes
    fwd_steps = _lib.fwi_revolve_schedule(nt, slots, with_actions=False)[1]
    for spec in ("revolve:%s" % budget, "every:50"):
        cg = dataclasses.replace(cfg, ckpt=spec)
        wg = api.Workspace()
        api.gradient(v0, obs, w, s, r, cg, workspace=wg)           # warm-up (and sizing)
        mis = []
        tg = median_time(lambda: mis.append(api.gradient(v0, obs, w, s, r, cg, workspace=wg)[0]),
                         reps, sync)
        log("salt gradient %s: %.3f s (median of %d)" % (spec, tg, reps))
        key = spec.split(":")[0]
        out[key] = {"gradient_s": round(tg, 4), "gradient_over_forward": round(tg / tf, 3),
                    "misfit": mis[-1], "runs": reps}
        del wg
        torch.cuda.empty_cache()
    out["revolve"].update(slots=slots, snapshot_bytes=slots * slot_bytes,
                          forward_steps=fwd_steps, adjoint_steps=nt)
    del v, v0, obs
    torch.cuda.empty_cache()
    # the 64^3 crop the oracle can run, timed beside the oracle's gradient
    C = salt_crop(crop_nt)
    vc, wc = t(C.v, torch.float32), t(C.wavelet, torch.float32)
    sc, rc = t(C.src_pos, torch.int32), t(C.rec_pos, torch.int32)
    cc = api.Config(dt=C.dt, dx=C.dx, order=C.order, nsponge=C.nb, eta_max=C.eta_max,
                    ckpt="all")
    oc = api.forward(vc, wc, sc, rc, cc)
    vc0 = t(C.v_start, torch.float32)
    api.gradient(vc0, oc, wc, sc, rc, cc)                           # warm-up
    tcrop = median_time(lambda: api.gradient(vc0, oc, wc, sc, rc, cc), reps, sync)
    out["crop"] = {"workload": "64^3 crop of the salt model + 24-cell sponge (112^3 padded), "
                               "%d steps, 64x64 receivers, all levels kept" % crop_nt,
                   "gradient_s": round(tcrop, 4), "runs": reps}
    return out


_crop_cache = {}


def salt_crop(nt):
    """The 64^3 salt crop workload (built once per process: it cuts the full model)."""
    from paper_1912_08063_amd import workloads as wl
    if nt not in _crop_cache:
        _crop_cache[nt] = wl.salt_3d_crop(nt=nt)
    return _crop_cache[nt]


def cpu_salt_crop(nt):
    """The oracle's gradient on the 64^3 salt crop (its sponge included)."""
    import numpy as np

    import oracle
    C = salt_crop(nt)
    obs = np.zeros((1, C.nt, C.nrec))
    t0 = time.perf_counter()
    oracle.gradient(C.v_start, C.wavelet, C.src_pos, C.rec_pos, obs, C.dx, C.dt, C.order,
                    C.nb, C.eta_max)
    secs = time.perf_counter() - t0
    return {"value": round(secs, 2), "unit": "s per %d-step gradient" % nt, "kind": "oracle",
            "sample": "fp64 oracle gradient on the 64^3 salt crop (112^3 padded), all %d steps"
                      % nt}


def serve_section(nreq, scale, chunk):
    """Serving: a Poisson stream of mixed 2-D/3-D forward and gradient
    requests (grid edges and step counts times `scale` of the configured
    stream) at 0.8x the saturated rate; continuous batching against one
    request at a time on the same stream."""
    import numpy as np

    from paper_1912_08063_amd import serve
    t0 = time.perf_counter()
    reqs = serve.make_stream(nreq, 1.0, seed=4, scale=scale)
    serve.attach_observed(reqs)
    log("serving x%.2f: %d requests generated in %.1f s" % (scale, nreq, time.perf_counter() - t0))
    for r in reqs:
        r.arrival = 0.0
    _, sat = serve.Server(max_active=64, chunk=chunk).run(reqs, realtime=True)
    rate = 0.8 * sat["shots_per_s"]
    arr = np.cumsum(np.random.default_rng(4).exponential(1.0 / rate, nreq))
    for r, a in zip(reqs, arr):
        r.arrival = float(a)
    _, b = serve.Server(max_active=64, chunk=chunk).run(reqs, realtime=True)
    log("serving x%.2f batched: p50 %.3f p99 %.3f s" % (scale, b["p50_latency_s"],
                                                       b["p99_latency_s"]))
    _, bf = serve.Server(max_active=64, chunk=chunk, policy="fifo").run(reqs, realtime=True)
    log("serving x%.2f batched fifo: p50 %.3f p99 %.3f s" % (scale, bf["p50_latency_s"],
                                                            bf["p99_latency_s"]))
    _, p = serve.Server(max_active=1, chunk=chunk).run(reqs, realtime=True)
    log("serving x%.2f plain: p50 %.3f p99 %.3f s" % (scale, p["p50_latency_s"],
                                                     p["p99_latency_s"]))
    keep = ("shots_per_s", "p50_latency_s", "p99_latency_s", "mean_latency_s", "makespan_s",
            "failed")
    n3 = sum(r.problem.v.ndim == 3 for r in reqs)
    ng = sum(r.kind == "gradient" for r in reqs)
    return {"workload": "Poisson stream of %d requests (%d gradient, %d forward; %d 3-D, %d 2-D; "
                        "layered models), grid edges and step counts x%.2f of the configured "
                        "stream (2-D 256^2-2048^2, 3-D 128^3-384^3, 1000-4000 steps), arrival "
                        "rate 0.8x saturated" % (nreq, ng, nreq - ng, n3, nreq - n3, scale),
            "requests": nreq,
            "p99_tail_samples": max(1, int(round(0.01 * nreq))),
            "rate_per_s": round(rate, 3),
            "saturated_shots_per_s": round(sat["shots_per_s"], 3),
            "batched": dict({k: round(b[k], 4) for k in keep}, policy=b["policy"]),
            "batched_fifo": dict({k: round(bf[k], 4) for k in keep}, policy=bf["policy"]),
            "plain": {k: round(p[k], 4) for k in keep}}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nt", type=int, default=2000)
    ap.add_argument("--cpu-steps", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sections",
                    default="forward,ceiling,c1,forward16,slab,gradient,gradient3d,salt3d,serve",
                    help="comma list of: forward (headline), ceiling (3-read/1-write stream "
                         "probe and the step's tile-march pattern), c1 (2-D one-shot latency), forward16 (16th order), slab (one "
                         "GPU's z-slab of a 1024^3 model), gradient (2-D, 32 shots), "
                         "gradient3d (headline geometry), salt3d (salt model, revolve), serve "
                         "(request streams)")
    ap.add_argument("--salt-nt", type=int, default=3000)
    ap.add_argument("--slab-nt", type=int, default=200)
    ap.add_argument("--grad-nt", type=int, default=3000)
    ap.add_argument("--grad-shots", type=int, default=32)
    ap.add_argument("--grad3d-nt", type=int, default=600)
    ap.add_argument("--grad3d-order", type=int, default=8)
    ap.add_argument("--no-grad-plain", action="store_true",
                    help="gradient section: time only the batched call")
    ap.add_argument("--fwd16-nt", type=int, default=500)
    ap.add_argument("--cpu-grad3d-steps", type=int, default=20)
    ap.add_argument("--serve-requests", type=int, default=80,
                    help="requests of the full-size serving stream")
    ap.add_argument("--serve-small-requests", type=int, default=400,
                    help="requests of the serving stream at --serve-small-scale (0: skip)")
    ap.add_argument("--serve-small-scale", type=float, default=0.25)
    ap.add_argument("--calibrate-copy", type=float, default=0.0, metavar="GIB",
                    help="only time a plain device copy of GIB GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (got --gpus %d); the multi-GPU "
              "sharding is a design note, not an implementation" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1912_08063_amd import api, workloads as wl

    dev = torch.device("cuda:0")
    if args.calibrate_copy > 0:
        n = int(args.calibrate_copy * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                          "ms_per_copy": ms, "GBps_read_plus_write": 8 * n / ms / 1e6}),
              flush=True)
        return
    log("generating workload")
    P = wl.layered_3d(nt=args.nt)
    t = lambda a, d: torch.as_tensor(np.ascontiguousarray(a), device=dev).to(d)
    v, w = t(P.v, torch.float32), t(P.wavelet, torch.float32)
    s, r = t(P.src_pos, torch.int32), t(P.rec_pos, torch.int32)
    cfg = api.Config(dt=P.dt, dx=P.dx, order=P.order, nsponge=P.nb, eta_max=P.eta_max)
    traces = torch.empty((P.nshots, P.nt, P.nrec), dtype=torch.float32, device=dev)
    ws = api.Workspace()

    def run():
        api.forward(v, w, s, r, cfg, workspace=ws, out=traces)

    for i in range(args.warmup):
        run()
        torch.cuda.synchronize()
        log("warmup %d done" % i)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(args.steps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    log("timed %d steps: %.1f ms" % (args.steps, ms))
    assert bool(torch.isfinite(traces).all()), "non-finite traces"

    updates = P.padded_cells * P.nt * args.steps
    value = updates / (ms * 1e-3) / 1e9
    launches = P.nt * args.steps
    avg_launch_s = ms * 1e-3 / launches
    bytes_per_launch = BYTES_PER_UPDATE * P.padded_cells
    achieved = bytes_per_launch / avg_launch_s / 1e9
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded layered velocity model, Ricker source",
        "config": {
            "workload": "3-D acoustic forward, 256^3 model + 24-cell sponge (304^3 padded), "
                        "8th order, %d steps, 256x256 receivers" % P.nt,
            "padded_cells": P.padded_cells, "model_cells": P.model_cells, "nt": P.nt,
            "order": P.order, "parallelism": "single GPU",
            "model_cell_updates_per_s": round(P.model_cells * P.nt * args.steps
                                              / (ms * 1e-3) / 1e9, 3),
        },
        "roofline": {
            "bound": "hbm", "kernel": "k_step3d<4,0,4,4> (forward stencil step, one launch per time step)",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(),
            "bytes_per_launch": bytes_per_launch,
            "avg_launch_us": round(avg_launch_s * 1e6, 2),
        },
    }
    sections = set(args.sections.split(","))
    if "ceiling" in sections:
        ceil = stream_ceiling(dev, fstride_of(P))
        ceil["step_frac_of_ceiling"] = round(achieved / ceil["GBps"], 4)
        out["roofline"]["stream_ceiling"] = ceil
        log("stream ceiling: %.1f GB/s (%s)" % (ceil["GBps"], ceil["variant"]))
        tm = tile_march(dev, P, avg_launch_s * 1e6)
        out["roofline"]["tile_march"] = tm
        log("tile march: bare %.1f, halos %.1f, + LDS %.1f, + warm-up %.1f us per launch"
            % (tm["bare_us"], tm["halos_us"], tm["halos_lds_us"], tm["pattern_us"]))
    if "c1" in sections:
        out["c1"] = c1_section(dev)
    if "gradient" in sections:
        out["gradient"] = gradient_section(dev, args.grad_nt, args.grad_shots, 50,
                                           plain=not args.no_grad_plain)
    if "forward16" in sections:
        out["forward16"] = forward16_section(dev, args.fwd16_nt)
    if "slab" in sections:
        out["slab"] = slab_section(dev, args.slab_nt)
    if "gradient3d" in sections:
        out["gradient3d"] = gradient3d_section(dev, args.grad3d_nt, 50, args.grad3d_order)
    if "salt3d" in sections:
        out["salt3d"] = salt3d_section(dev, args.salt_nt)
    if "serve" in sections:
        out["serving"] = serve_section(args.serve_requests, 1.0, 50)
        if args.serve_small_requests > 0:
            out["serving_small"] = serve_section(args.serve_small_requests,
                                                 args.serve_small_scale, 50)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, %d steps)" % args.cpu_steps)
        out["cpu_baseline"] = cpu_baseline(P, args.cpu_steps)
        if "c1" in sections:
            log("cpu baseline: oracle 2-D one-shot forward")
            out["cpu_baseline"]["c1"] = cpu_c1()
        if "gradient" in sections:
            log("cpu baseline: oracle 2-D gradient, one shot")
            out["cpu_baseline"]["gradient"] = cpu_gradient_2d(args.grad_nt)
        if "salt3d" in sections:
            log("cpu baseline: oracle gradient on the salt crop")
            out["cpu_baseline"]["salt_crop"] = cpu_salt_crop(600)
        if "gradient3d" in sections:
            log("cpu baseline: oracle 3-D gradient sample")
            out["cpu_baseline"]["gradient3d"] = cpu_gradient_3d(args.cpu_grad3d_steps,
                                                                 args.grad3d_nt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
