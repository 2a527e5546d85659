"""Serving: jobs of different grids batched into shared launches.

Each job's results must be bitwise those of the stand-alone entry points
(fwi_forward / fwi_gradient with the same checkpoint interval) and the same
alone and in a mix; a job served in a mix also matches the FP64 oracle.
"""
import numpy as np
import pytest

from gpu_common import f32, oracle_forward, oracle_gradient, rel_l2
from paper_1912_08063_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _stream(n, scale, seed=21, force=None):
    from paper_1912_08063_amd import serve
    reqs = serve.make_stream(n, 0.0, seed=seed, scale=scale, force=force)
    for r in reqs:
        r.problem = f32(r.problem)
    serve.attach_observed(reqs)
    return reqs


def _standalone(req, chunk, ckpt=None):
    import torch
    from gpu_common import cfg, dev, inputs
    from paper_1912_08063_amd import api
    P = req.problem
    v, w, s, r = inputs(P)
    if req.kind == "forward":
        tr = api.forward(v, w, s, r, cfg(P))
        torch.cuda.synchronize()
        return tr.cpu().numpy(), None, None
    mis, dv, tr = api.gradient(v, dev(req.obs, torch.float32), w, s, r,
                               cfg(P, ckpt or "every:%d" % chunk), return_traces=True)
    torch.cuda.synchronize()
    return tr.cpu().numpy(), dv.cpu().numpy(), mis


def test_mixed_jobs_bitwise_equal_standalone_calls():
    from paper_1912_08063_amd import serve
    reqs = _stream(10, 0.08)
    kinds = {(r.kind, r.problem.ndim) for r in reqs}
    assert len(kinds) >= 3, kinds
    chunk = 16
    results, rep = serve.Server(max_active=10, chunk=chunk, keep_outputs=True).run(
        reqs, realtime=False)
    assert rep["requests"] == 10
    for req, res in zip(reqs, results):
        tr, dv, mis = _standalone(req, chunk)
        assert np.array_equal(res.traces, tr), req.problem.name
        if req.kind == "gradient":
            assert np.array_equal(res.dv, dv), req.problem.name
            assert res.misfit == mis


def test_alone_and_in_a_mix_are_identical():
    from paper_1912_08063_amd import serve
    reqs = _stream(8, 0.06, seed=33)
    alone, _ = serve.Server(max_active=1, chunk=20, keep_outputs=True).run(reqs, realtime=False)
    mixed, rep = serve.Server(max_active=8, chunk=20, keep_outputs=True).run(reqs,
                                                                             realtime=False)
    assert rep["requests"] == 8
    for a, b in zip(alone, mixed):
        assert np.array_equal(a.traces, b.traces)
        if a.kind == "gradient":
            assert np.array_equal(a.dv, b.dv) and a.misfit == b.misfit


def test_served_job_matches_oracle():
    from paper_1912_08063_amd import serve
    reqs = _stream(4, 0.05, seed=5, force={"dim": 2})
    reqs[0].kind = "gradient"
    serve.attach_observed(reqs)
    results, _ = serve.Server(max_active=4, chunk=12, keep_outputs=True).run(reqs,
                                                                            realtime=False)
    for req, res in zip(reqs, results):
        P = req.problem
        if req.kind == "forward":
            assert rel_l2(res.traces.astype(np.float64), oracle_forward(P)) <= 1e-4
        else:
            obs = req.obs.astype(np.float64)
            mis_o, dv_o = oracle_gradient(P, P.v, obs)
            assert rel_l2(res.dv.astype(np.float64), dv_o) <= 1e-3
            assert abs(res.misfit - mis_o) <= 1e-3 * mis_o


def test_admission_respects_budget():
    from paper_1912_08063_amd import serve
    reqs = _stream(6, 0.05, seed=8)
    srv = serve.Server(max_active=6, chunk=10)
    biggest = max(srv.footprint(r) for r in reqs)
    srv.budget = biggest + 1   # at most one large job at a time
    results, rep = srv.run(reqs, realtime=False)
    assert rep["requests"] == 6


def test_srpt_pauses_long_jobs_without_changing_results():
    """A fill limit of one cell lets one job advance per chunk: the one with the
    least remaining work.  Jobs then finish in order of their work, and every
    result is bitwise that of the FIFO server, which advances all jobs at once."""
    from paper_1912_08063_amd import serve
    reqs = _stream(6, 0.06, seed=41)
    srpt, rep = serve.Server(max_active=6, chunk=10, keep_outputs=True, fill_cells=1).run(
        reqs, realtime=False)
    fifo, _ = serve.Server(max_active=6, chunk=10, keep_outputs=True, policy="fifo",
                           fill_cells=10 ** 12).run(reqs, realtime=False)
    assert rep["requests"] == 6 and rep["policy"] == "srpt"
    order = [r.rid for r in sorted(srpt, key=lambda r: r.seq)]
    by_work = [r.rid for r in sorted(srpt, key=lambda r: (r.work, r.arrival, r.rid))]
    assert order == by_work
    for a, b in zip(srpt, fifo):
        assert np.array_equal(a.traces, b.traces)
        if a.kind == "gradient":
            assert np.array_equal(a.dv, b.dv) and a.misfit == b.misfit


def test_every_policy_gives_the_same_results():
    """The scheduling policy decides only which jobs advance in which chunk:
    under a fill limit that forces pauses, every policy's results are bitwise
    those of the FIFO server."""
    from paper_1912_08063_amd import serve
    reqs = _stream(7, 0.06, seed=43)
    ref, _ = serve.Server(max_active=7, chunk=12, keep_outputs=True, policy="fifo",
                          fill_cells=10 ** 12).run(reqs, realtime=False)
    for policy in serve.POLICIES:
        got, rep = serve.Server(max_active=7, chunk=12, keep_outputs=True, policy=policy,
                                fill_cells=150_000).run(reqs, realtime=False)
        assert rep["requests"] == 7 and rep["policy"] == policy
        for a, b in zip(ref, got):
            assert np.array_equal(a.traces, b.traces), policy
            if a.kind == "gradient":
                assert np.array_equal(a.dv, b.dv) and a.misfit == b.misfit, policy


def test_mixed_orders_in_one_advance():
    """8th- and 16th-order jobs, 2-D and 3-D, forward and gradient, advanced
    together: each (dimension, order, phase) forms its own launch group, and
    every result is bitwise that of the stand-alone call."""
    from paper_1912_08063_amd import serve
    probs = [("forward", wl.small_2d(nz=30, nx=90, nt=60, order=16, nrec=9, seed=3)),
             ("gradient", wl.small_2d(nz=28, nx=75, nt=55, order=8, nrec=7, seed=4)),
             ("gradient", wl.small_3d(shape=(14, 12, 70), nt=40, order=16, nrec=6, seed=5)),
             ("forward", wl.small_3d(shape=(12, 15, 66), nt=45, order=8, nrec=8, seed=6))]
    reqs = [serve.Request(i, kind, 0.0, f32(P)) for i, (kind, P) in enumerate(probs)]
    serve.attach_observed(reqs)
    chunk = 16
    results, rep = serve.Server(max_active=4, chunk=chunk, keep_outputs=True,
                                policy="fifo").run(reqs, realtime=False)
    assert rep["requests"] == 4
    for req, res in zip(reqs, results):
        tr, dv, mis = _standalone(req, chunk)
        assert np.array_equal(res.traces, tr), req.problem.name
        if req.kind == "gradient":
            assert np.array_equal(res.dv, dv) and res.misfit == mis


def _sized_request(rid, kind, shape, nt, seed):
    """A request of the configured stream's structure at a chosen size:
    layered model, 10 Hz Ricker at the surface centre, dt from CFL 0.4, surface
    receivers (every cell in 2-D, every 4th in 3-D)."""
    from paper_1912_08063_amd import serve
    rng = np.random.default_rng(seed)
    v = wl.layered(shape, rng)
    dx = 10.0
    dt = wl.dt_from_cfl(float(v.max()), dx, 0.4)
    src = [[4] + [s // 2 for s in shape[1:]]]
    rec = wl.surface_receivers(shape, 4, stride=1 if len(shape) == 2 else 4)
    P = wl._pack("sized%d" % rid, v, dx, dt, nt, 8, 20 if len(shape) == 2 else 24, 10.0, src,
                 rec)
    return serve.Request(rid, kind, 0.0, f32(P))


def test_full_size_jobs_in_a_mix_equal_standalone_calls():
    """A 1024^2 2-D gradient and a 256^3 3-D forward (the configured stream's
    sizes, 1200 steps) served together with two small jobs: each result is
    bitwise that of its stand-alone fwi_gradient / fwi_forward call, the calls
    the full-size parity tests check against the oracle."""
    from paper_1912_08063_amd import serve
    reqs = [_sized_request(0, "gradient", (1024, 1024), 1200, 61),
            _sized_request(1, "forward", (256, 256, 256), 1200, 62),
            _sized_request(2, "forward", (300, 300), 900, 63),
            _sized_request(3, "gradient", (64, 80, 72), 700, 64)]
    serve.attach_observed(reqs)
    chunk = 50
    results, rep = serve.Server(max_active=4, chunk=chunk, keep_outputs=True,
                                policy="fifo", fill_cells=10 ** 12).run(reqs, realtime=False)
    assert rep["requests"] == 4 and rep["failed"] == 0
    for req, res in zip(reqs, results):
        tr, dv, mis = _standalone(req, chunk)
        assert np.array_equal(res.traces, tr), req.problem.name
        if req.kind == "gradient":
            assert np.array_equal(res.dv, dv), req.problem.name
            assert res.misfit == mis


def test_a_failing_request_is_retired_and_the_others_are_unchanged():
    """One request violates the stability limit (dt 1.5x its CFL bound) and one
    has a receiver outside its model: both are retired with an error, and every
    other result is bitwise that of a run of the stream without them."""
    import dataclasses
    from paper_1912_08063_amd import serve
    good = _stream(6, 0.06, seed=71)
    bad_cfl = _stream(1, 0.06, seed=72)[0]
    P = bad_cfl.problem
    bad_cfl.problem = dataclasses.replace(P, dt=float(np.float32(1.5 * P.dt / 0.4 * 0.5546)))
    bad_cfl.rid = 100
    bad_pos = _stream(1, 0.06, seed=73)[0]
    bad_pos.problem.rec_pos[0, 0, 0] = bad_pos.problem.v.shape[0] + 5
    bad_pos.rid = 101
    clean, rep0 = serve.Server(max_active=8, chunk=16, keep_outputs=True).run(good,
                                                                            realtime=False)
    mixed, rep1 = serve.Server(max_active=8, chunk=16, keep_outputs=True).run(
        good[:3] + [bad_cfl] + good[3:] + [bad_pos], realtime=False)
    assert rep0["failed"] == 0 and rep1["failed"] == 2 and rep1["requests"] == 6
    errs = {r.rid: r.error for r in mixed if r.error}
    assert set(errs) == {100, 101}
    assert "stability" in errs[100] and "outside" in errs[101]
    ok = [r for r in mixed if r.error is None]
    for a, b in zip(clean, ok):
        assert a.rid == b.rid
        assert np.array_equal(a.traces, b.traces)
        if a.kind == "gradient":
            assert np.array_equal(a.dv, b.dv) and a.misfit == b.misfit


@pytest.mark.parametrize("chunk", [7, 16])
def test_revolve_jobs_equal_standalone_revolve_calls(chunk):
    """Gradient jobs with binomial checkpointing turn between recomputation
    and adjoint steps inside a chunk (per-step level lists).  Served with
    every-K gradients and forward jobs, 2-D and 3-D, 8th and 16th order, each
    is bitwise the stand-alone fwi_gradient with the same revolve:S policy
    (which keeps its snapshots in place instead of copying them)."""
    from paper_1912_08063_amd import serve
    probs = [("gradient", "revolve:3", wl.small_2d(nz=28, nx=75, nt=61, order=8, nrec=7, seed=4)),
             ("gradient", "revolve:5", wl.small_3d(shape=(14, 12, 70), nt=47, order=16, nrec=6,
                                                   seed=5)),
             ("gradient", "revolve:1", wl.small_2d(nz=30, nx=40, nt=23, order=16, nrec=5, seed=7)),
             ("gradient", "revolve:2", wl.small_3d(shape=(12, 15, 66), nt=39, order=8, nrec=8,
                                                   seed=6)),
             ("gradient", None, wl.small_2d(nz=26, nx=50, nt=44, order=8, nrec=6, seed=8)),
             ("forward", None, wl.small_3d(shape=(13, 14, 60), nt=35, order=8, nrec=5, seed=9))]
    reqs = [serve.Request(i, kind, 0.0, f32(P), ckpt=ck) for i, (kind, ck, P) in enumerate(probs)]
    serve.attach_observed(reqs)
    results, rep = serve.Server(max_active=6, chunk=chunk, keep_outputs=True,
                                policy="fifo").run(reqs, realtime=False)
    assert rep["requests"] == 6 and rep["failed"] == 0
    for req, res in zip(reqs, results):
        tr, dv, mis = _standalone(req, chunk, req.ckpt)
        assert np.array_equal(res.traces, tr), req.problem.name
        if req.kind == "gradient":
            assert np.array_equal(res.dv, dv), req.problem.name
            assert res.misfit == mis


def test_revolve_job_alone_matches_oracle():
    """A served revolve job alone (fill limit 1: nothing shares its launches
    after the first chunk) against the FP64 oracle's misfit and gradient."""
    from paper_1912_08063_amd import serve
    P = f32(wl.small_2d(nz=36, nx=64, nt=80, order=8, nrec=9, seed=12))
    req = serve.Request(0, "gradient", 0.0, P, ckpt="revolve:4")
    serve.attach_observed([req])
    (res,), rep = serve.Server(max_active=1, chunk=9, keep_outputs=True).run([req],
                                                                             realtime=False)
    assert rep["failed"] == 0
    obs = req.obs.astype(np.float64)
    mis_o, dv_o = oracle_gradient(P, P.v, obs)
    assert rel_l2(res.dv.astype(np.float64), dv_o) <= 1e-3
    assert abs(res.misfit - mis_o) <= 1e-3 * mis_o
