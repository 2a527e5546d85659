"""Misfit and gradient: HIP library vs the FP64 oracle; checkpoint invariance;
the autograd.Function against fwi_gradient.

Tolerances: relative L2 <= 1e-3 on dv, relative 1e-4 on traces and 1e-3 on
the misfit.  Every checkpoint policy must give bitwise the same dv, since all
of them recompute exactly the same forward levels with the same kernels.
"""
import numpy as np
import pytest

from gpu_common import (cfg, dev, f32, gpu_gradient, inputs, oracle_forward, oracle_gradient,
                        rel_l2)
from paper_1912_08063_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _setup(P, smooth=3.0):
    P = f32(P)
    obs = np.asarray(oracle_forward(P), dtype=np.float32).astype(np.float64)
    v0 = np.asarray(wl.smooth(P.v, smooth), dtype=np.float32).astype(np.float64)
    return P, obs, v0


def _check(P, obs, v0, ckpt="all"):
    mis_o, dv_o = oracle_gradient(P, v0, obs)
    mis_g, dv_g, tr_g = gpu_gradient(P, v0, obs, ckpt)
    assert rel_l2(tr_g, oracle_forward(P, v0)) <= 1e-4
    assert abs(mis_g - mis_o) <= 1e-3 * abs(mis_o), (mis_g, mis_o)
    assert rel_l2(dv_g, dv_o) <= 1e-3, rel_l2(dv_g, dv_o)
    return dv_g


@pytest.mark.parametrize("order", [8, 16])
def test_gradient_2d(order):
    P, obs, v0 = _setup(wl.small_2d(nz=48, nx=131, nt=220, order=order, nshots=2, nrec=40))
    _check(P, obs, v0, "every:25")


@pytest.mark.parametrize("direct", ["0", "1"])
def test_gradient_2d_receivers_on_tile_and_chunk_edges(direct, monkeypatch):
    """2-D adjoint steps add the adjoint source themselves, per tile and row:
    a full receiver row (64 cells per tile), cells on both sides of tile and
    row-chunk edges, and a duplicated cell, for two shots.  With nb = 6 and
    an M = 4 frame, model column c is memory column c + 10 (tiles start at
    multiples of 64) and model row r is padded row r + 6 (chunks of 10 rows).
    Both 2-D kernels: the marching one and the one-cell-per-lane one."""
    monkeypatch.setenv("FWI_ZCHUNK", "10")
    monkeypatch.setenv("FWI_DIRECT2D", direct)
    P = wl.small_2d(nz=40, nx=150, nt=120, nb=6, nshots=2, nrec=156)
    rec = [[4, x] for x in range(150)] + [[3, 53], [3, 54], [13, 117], [14, 118], [39, 149],
                                          [3, 53]]
    P.rec_pos[:] = np.array(rec, dtype=np.int32)
    P.src_pos[:] = [[20, 75], [5, 10]]
    P, obs, v0 = _setup(P)
    _check(P, obs, v0, "every:10")


@pytest.mark.parametrize("order", [8, 16])
def test_gradient_3d(order):
    P, obs, v0 = _setup(wl.small_3d(shape=(26, 22, 75), nt=90, order=order, nshots=2, nrec=30),
                        1.5)
    _check(P, obs, v0, "revolve:4")


def test_gradient_duplicate_receivers_and_sponge_edges():
    P = wl.small_2d(nz=30, nx=70, nt=120, nrec=8, nb=9)
    P.rec_pos[0, 4:] = P.rec_pos[0, 0]
    P.src_pos[0] = [0, 69]
    P, obs, v0 = _setup(P)
    _check(P, obs, v0, "all")


def test_checkpoint_policies_bitwise_identical():
    P, obs, v0 = _setup(wl.small_2d(nz=40, nx=100, nt=97, nshots=3, nrec=20))
    ref_mis, ref_dv, ref_tr = gpu_gradient(P, v0, obs, "all")
    for ck in ["every:1", "every:7", "every:50", "every:97", "every:500", "revolve:0",
               "revolve:1", "revolve:3", "revolve:10", "revolve:200"]:
        mis, dv, tr = gpu_gradient(P, v0, obs, ck)
        assert mis == ref_mis, ck
        assert np.array_equal(tr, ref_tr), ck
        assert np.array_equal(dv, ref_dv), ck


@pytest.mark.parametrize("order", [8, 16])
def test_3d_checkpoint_policies_bitwise_identical(order):
    P, obs, v0 = _setup(wl.small_3d(shape=(20, 18, 66), nt=41, nrec=12, order=order), 1.5)
    ref_mis, ref, ref_tr = gpu_gradient(P, v0, obs, "all")
    for ck in ["every:6", "revolve:1", "revolve:2", "revolve:5", "revolve:40"]:
        mis, dv, tr = gpu_gradient(P, v0, obs, ck)
        assert mis == ref_mis, ck
        assert np.array_equal(tr, ref_tr), ck
        assert np.array_equal(dv, ref), ck


@pytest.mark.parametrize("order", [8, 16])
def test_3d_block_shapes_bitwise_identical(order, monkeypatch):
    """Every 3-D block shape (waves x rows per thread: 4x4, 8x4, 4x2, 8x2) for
    the forward and the adjoint launches gives the same traces, misfit and
    gradient bit for bit: a cell's arithmetic does not depend on its tile.
    The grid's y extent (37) leaves a ragged last tile row for each shape."""
    P, obs, v0 = _setup(wl.small_3d(shape=(22, 37, 100), nt=45, nshots=2, nrec=15, order=order))
    ref = gpu_gradient(P, v0, obs, "every:8")
    for fwd, adj in [("4", "4"), ("8", "8"), ("42", "42"), ("82", "82"), ("4", "82")]:
        monkeypatch.setenv("FWI_WAVES", fwd)
        monkeypatch.setenv("FWI_WAVES_ADJ", adj)
        got = gpu_gradient(P, v0, obs, "every:8")
        assert got[0] == ref[0], (fwd, adj)
        assert np.array_equal(got[1], ref[1]), (fwd, adj)
        assert np.array_equal(got[2], ref[2]), (fwd, adj)


@pytest.mark.parametrize("shape", ["82", "42", "4", "8"])
def test_split_adjoint_equals_fused(shape, monkeypatch):
    """At 8th order FWI_SPLIT_ADJ=1 runs the adjoint as a psi pass and an
    imaging pass instead of the fused kernel: the same values bit for bit, for
    every block shape of the adjoint launches."""
    P, obs, v0 = _setup(wl.small_3d(shape=(30, 37, 100), nt=57, nshots=2, nrec=15))
    monkeypatch.setenv("FWI_WAVES_ADJ", shape)
    ref = gpu_gradient(P, v0, obs, "every:8")
    monkeypatch.setenv("FWI_SPLIT_ADJ", "1")
    got = gpu_gradient(P, v0, obs, "every:8")
    assert got[0] == ref[0]
    assert np.array_equal(got[1], ref[1])


def test_revolve_without_copies_equals_copies(monkeypatch):
    """Binomial checkpointing reads restored states from their slots and
    writes snapshot states straight into them; FWI_REVOLVE_COPY=1 copies
    instead.  Both give the same gradient and traces, bit for bit."""
    P, obs, v0 = _setup(wl.small_3d(shape=(25, 30, 90), nt=75, nshots=2, nrec=15))
    got = gpu_gradient(P, v0, obs, "revolve:4")
    monkeypatch.setenv("FWI_REVOLVE_COPY", "1")
    ref = gpu_gradient(P, v0, obs, "revolve:4")
    assert got[0] == ref[0]
    assert np.array_equal(got[2], ref[2])
    assert np.array_equal(got[1], ref[1])


def test_zero_residual_gives_zero_gradient():
    import torch
    from paper_1912_08063_amd import api
    P = f32(wl.small_2d(nz=30, nx=80, nt=60, nrec=10))
    v, w, s, r = inputs(P)
    obs = api.forward(v, w, s, r, cfg(P))
    mis, dv = api.gradient(v, obs, w, s, r, cfg(P, "every:9"))
    torch.cuda.synchronize()
    assert mis == 0.0 and float(dv.abs().max()) == 0.0


@pytest.mark.parametrize("ckpt", ["every:11", "revolve:3"])
def test_autograd_function_matches_fwi_gradient(ckpt):
    import torch
    from paper_1912_08063_amd.autograd import FWIForward
    P, obs, v0 = _setup(wl.small_2d(nz=40, nx=90, nt=130, nshots=2, nrec=21))
    mis_g, dv_g, _ = gpu_gradient(P, v0, obs, ckpt)
    vt, w, s, r = inputs(P, v0)
    vt.requires_grad_(True)
    tr = FWIForward.apply(vt, w, s, r, cfg(P, ckpt))
    loss = ((tr - dev(obs, torch.float32)) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    g = vt.grad.cpu().numpy().astype(np.float64)
    assert rel_l2(g, dv_g) <= 1e-6
    assert abs(float(loss.detach()) - mis_g) <= 1e-5 * mis_g
    # a second backward through consumed checkpoints must fail loudly
    tr2 = FWIForward.apply(vt, w, s, r, cfg(P, ckpt))
    l2 = tr2.sum()
    l2.backward(retain_graph=True)
    with pytest.raises(RuntimeError):
        l2.backward()


def test_autograd_matches_central_differences():
    """<dv, dir> from the autograd backward against central differences of the
    GPU forward misfit in fp64 sums (h chosen for fp32 traces)."""
    import torch
    from paper_1912_08063_amd import api
    from paper_1912_08063_amd.autograd import FWIForward
    P, obs, v0 = _setup(wl.small_2d(nz=40, nx=90, nt=160, nrec=30), 4.0)
    rng = np.random.default_rng(0)
    direction = wl.smooth(rng.standard_normal(v0.shape), 2.0)
    direction /= np.abs(direction).max()
    vt, w, s, r = inputs(P, v0)
    vt.requires_grad_(True)
    tr = FWIForward.apply(vt, w, s, r, cfg(P, "every:20"))
    ((tr - dev(obs, torch.float32)) ** 2).sum().backward()
    an = float(np.sum(vt.grad.cpu().numpy().astype(np.float64) * direction))

    def phi(v):
        vv, _, _, _ = inputs(P, v)
        d = api.forward(vv, w, s, r, cfg(P)).cpu().numpy().astype(np.float64)
        return float(np.sum((d - obs) ** 2))

    h = 2.0   # m/s
    fd = (phi(v0 + h * direction) - phi(v0 - h * direction)) / (2 * h)
    assert abs(fd - an) <= 1e-2 * abs(an), (fd, an)


def test_lbfgs_reduces_the_misfit():
    """A few L-BFGS iterations driven by fwi_gradient lower the misfit and move
    the model towards the truth (a smooth start, sponge held fixed)."""
    import torch
    from paper_1912_08063_amd import api, inversion
    P = f32(wl.small_2d(nz=40, nx=96, nt=260, nshots=4, nrec=48))
    vt, w, s, r = inputs(P)
    c = cfg(P, "every:20")
    obs = api.forward(vt, w, s, r, c)
    v0 = dev(wl.smooth(P.v, 4.0), torch.float32)
    v, hist = inversion.lbfgs(v0, obs, w, s, r, c, iters=4, vmin=float(P.v.min()) - 100,
                              vmax=float(P.v.max()) + 100)
    assert len(hist) >= 3
    assert all(b < a for a, b in zip(hist, hist[1:]))
    assert hist[-1] < 0.5 * hist[0]
    assert float((v - vt).norm()) < float((v0 - vt).norm())


def test_lbfgs_matches_the_oracle_reference():
    """Three iterations of the GPU inversion loop (misfit and gradient from the
    HIP library, fp32 models) against the same iterations of the FP64
    reference over the oracle (oracle/lbfgs.py, written separately from the
    textbook algorithm): the misfit history to 1e-3 relative, the accepted
    steps to 1e-3, and the model update to 1e-2 of its size."""
    import torch
    from oracle import lbfgs as ref
    from paper_1912_08063_amd import api, inversion
    P = f32(wl.small_2d(nz=40, nx=96, nt=260, nshots=4, nrec=48))
    vt, w, s, r = inputs(P)
    c = cfg(P, "every:20")
    obs_t = api.forward(vt, w, s, r, c)
    obs = obs_t.cpu().numpy().astype(np.float64)      # the same data on both sides
    v0 = np.asarray(wl.smooth(P.v, 4.0), np.float32).astype(np.float64)
    lo, hi = float(P.v.min()) - 100.0, float(P.v.max()) + 100.0
    steps_g = []
    v, hist = inversion.lbfgs(dev(v0, torch.float32), obs_t, w, s, r, c, iters=3, vmin=lo,
                              vmax=hi, steps=steps_g)
    torch.cuda.synchronize()
    vr, hr, steps_r = ref.fwi(v0, P.wavelet, P.src_pos, P.rec_pos, obs, P.dx, P.dt, P.order,
                              P.nb, P.eta_max, iters=3, vmin=lo, vmax=hi)
    assert len(hist) == len(hr) == 4
    for a, b in zip(hist, hr):
        assert abs(a - b) <= 1e-3 * b, (hist, hr)
    # the same backtracking decisions: accepted steps agree to rounding (the
    # first is first_step / max|g|, the others 1 / 2^k)
    np.testing.assert_allclose(steps_g, steps_r, rtol=1e-3)
    up_g = v.cpu().numpy().astype(np.float64) - v0
    up_r = vr - v0
    assert rel_l2(up_g, up_r) <= 1e-2, rel_l2(up_g, up_r)


@pytest.mark.parametrize("order", [8, 16, 2])
def test_2d_direct_and_marching_kernels_bitwise_equal(order, monkeypatch):
    """The one-cell-per-lane 2-D kernels (small grids) and the marching ones
    evaluate the same terms in the same order: traces, misfit and dv of a
    three-shot gradient (every-13 snapshots, sponge, receivers on tile edges)
    are bitwise equal."""
    P, obs, v0 = _setup(wl.small_2d(nz=45, nx=140, nt=150, order=order, nshots=3, nrec=33))
    P.rec_pos[1, :4] = [[0, 0], [0, 63 - 6], [44, 139], [20, 64 - 6]]
    out = {}
    for d in ("0", "1"):
        monkeypatch.setenv("FWI_DIRECT2D", d)
        out[d] = gpu_gradient(P, v0, obs, "every:13")
    (m0, g0, t0), (m1, g1, t1) = out["0"], out["1"]
    assert np.array_equal(t0, t1) and np.array_equal(g0, g1) and m0 == m1


def test_automatic_checkpoint_policy_bitwise_equal():
    """ckpt="auto" (every level kept here) and "auto:BUDGET" with a budget that
    forces binomial checkpointing give the gradient of every-K bit for bit,
    through fwi_gradient and through the autograd Function."""
    import torch

    from paper_1912_08063_amd import _lib, api
    from paper_1912_08063_amd.autograd import FWIForward
    P, obs, v0 = _setup(wl.small_2d(nz=30, nx=80, nt=70, nrec=9, seed=17))
    ref = gpu_gradient(P, v0, obs, "every:8")
    assert gpu_gradient(P, v0, obs, "auto")[0] == ref[0]
    vt, w, s, r = inputs(P, v0)
    prob = api.make_problem(vt, P.nt, cfg(P), 1, P.nrec)
    small = _lib.fwi_workspace_bytes(prob, _lib.MODE_GRADIENT, api.parse_ckpt("revolve:3"))
    assert api.resolve_ckpt("auto:%d" % small, prob, vt.device).startswith("revolve:")
    for spec in ("auto", "auto:%d" % small):
        mis, dv, tr = gpu_gradient(P, v0, obs, spec)
        assert mis == ref[0] and np.array_equal(dv, ref[1]) and np.array_equal(tr, ref[2]), spec
    vt.requires_grad_(True)
    tr = FWIForward.apply(vt, w, s, r, cfg(P, "auto"))
    ((tr - dev(obs, torch.float32)) ** 2).sum().backward()
    torch.cuda.synchronize()
    assert rel_l2(vt.grad.cpu().numpy().astype(np.float64), ref[1]) <= 1e-6


def _run_on(ws_fill, P, v0, obs, ckpt, ws):
    """Forward traces and gradient through one workspace whose bytes are all
    set to ws_fill before each call."""
    import torch
    from paper_1912_08063_amd import api
    vt, w, s, r = inputs(P)
    v0t = dev(v0, torch.float32)
    obs_t = dev(obs, torch.float32)
    outs = []
    for call in ("forward", "gradient"):
        if ws.buf is not None:
            ws.buf.fill_(ws_fill)
        if call == "forward":
            tr = api.forward(vt, w, s, r, cfg(P), workspace=ws)
            outs.append(tr.cpu().numpy())
        else:
            mis, dv, tr = api.gradient(v0t, obs_t, w, s, r, cfg(P, ckpt), return_traces=True,
                                       workspace=ws)
            outs += [np.float64(mis), dv.cpu().numpy(), tr.cpu().numpy()]
    torch.cuda.synchronize()
    return outs


@pytest.mark.parametrize("case", ["3d", "2d_direct", "2d_marching"])
@pytest.mark.parametrize("ckpt", ["all", "every:7", "revolve:3"])
def test_results_do_not_depend_on_workspace_contents(case, ckpt, monkeypatch):
    """Level stores are cleared only where the steps never write (the frame
    and row padding) plus the zero initial levels: every other cell of a
    level is written before it is read.  A workspace whose bytes are all 0xFF
    (NaN as floats) must therefore give bitwise the results of a zeroed one,
    for the forward and under every checkpoint policy."""
    from paper_1912_08063_amd import api
    if case == "3d":
        P = f32(wl.small_3d(shape=(37, 29, 70), nt=48, order=8, nshots=2, nrec=23))
    else:
        monkeypatch.setenv("FWI_DIRECT2D", "1" if case == "2d_direct" else "0")
        P = f32(wl.small_2d(nz=48, nx=131, nt=90, order=8, nshots=2, nrec=40))
    obs = np.asarray(oracle_forward(P), dtype=np.float32).astype(np.float64)
    v0 = np.asarray(wl.smooth(P.v, 3.0), dtype=np.float32).astype(np.float64)
    ws = api.Workspace()
    _run_on(0, P, v0, obs, ckpt, ws)          # sizes the workspace
    clean = _run_on(0, P, v0, obs, ckpt, ws)
    dirty = _run_on(255, P, v0, obs, ckpt, ws)
    for a, b in zip(clean, dirty):
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b)
