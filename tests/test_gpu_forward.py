"""Forward modelling: HIP library vs the FP64 oracle, element by element.

Tolerance: relative L2 <= 1e-4 on traces (fp32 kernels against an fp64
reference), per shot and overall.  Sizes span several tiles in every axis and
ragged tails; edge cases cover empty receiver lists, no sponge, duplicated
receivers, sources and receivers on the model corners, one time step, and
every supported stencil order, and models smaller than the stencil radius.
"""
import numpy as np
import pytest

from gpu_common import f32, gpu_forward, oracle_forward, rel_l2
from paper_1912_08063_amd import workloads as wl

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _check(P, tol=TOL):
    P = f32(P)
    g = gpu_forward(P)
    o = oracle_forward(P)
    assert g.shape == o.shape
    assert np.all(np.isfinite(g))
    for s in range(P.nshots):
        assert rel_l2(g[s], o[s]) <= tol, (P.name, s, rel_l2(g[s], o[s]))
    return g, o


@pytest.mark.parametrize("order", [8, 16, 4, 2])
def test_small_2d_ragged(order):
    _check(wl.small_2d(nz=150, nx=203, nt=160, order=order, nshots=2, nrec=31))


@pytest.mark.parametrize("order", [8, 16, 4, 2])
def test_small_3d_ragged(order):
    _check(wl.small_3d(shape=(45, 37, 150), nt=80, order=order, nshots=2, nrec=29))


def test_3d_many_tiles_thin_z():
    # many xy tiles, few z planes: z chunks shorter than the register queue
    _check(wl.small_3d(shape=(6, 70, 200), nt=40, nb=3, nrec=40))


def test_anomaly_2d_full():
    g, o = _check(wl.anomaly_2d())
    assert np.abs(g).max() > 0


def test_no_sponge_and_corners():
    P = wl.small_2d(nz=40, nx=77, nt=90, nb=0, nrec=4)
    P.src_pos[0] = [0, 0]
    P.rec_pos[0] = [[0, 76], [39, 0], [39, 76], [0, 0]]
    _check(P)
    P3 = wl.small_3d(shape=(12, 13, 70), nt=40, nb=0, nrec=2)
    P3.src_pos[0] = [11, 12, 69]
    P3.rec_pos[0] = [[0, 0, 0], [11, 0, 69]]
    _check(P3)


def test_degenerate_grids():
    """Models smaller than the stencil radius, one cell thick, with and without
    a sponge: the frames and the clamped loads carry the whole computation."""
    P = wl.small_2d(nz=1, nx=1, nt=30, nb=0, nrec=1)
    P.src_pos[0] = [0, 0]
    P.rec_pos[0] = [[0, 0]]
    _check(P)
    P = wl.small_2d(nz=2, nx=3, nt=30, nb=4, nrec=2)
    P.src_pos[0] = [1, 2]
    P.rec_pos[0] = [[0, 0], [1, 1]]
    _check(P)
    for nb in (0, 3):
        P3 = wl.small_3d(shape=(1, 2, 3), nt=25, nb=nb, nrec=2)
        P3.src_pos[0] = [0, 1, 2]
        P3.rec_pos[0] = [[0, 0, 0], [0, 1, 1]]
        _check(P3)


def test_duplicate_receivers_and_single_step():
    P = wl.small_2d(nz=30, nx=70, nt=1, nrec=6)
    P.rec_pos[0] = [P.src_pos[0]] * 3 + [[1, 1]] * 3
    _check(P)
    P = wl.small_2d(nz=30, nx=70, nt=50, nrec=6)
    P.rec_pos[0, 3:] = P.rec_pos[0, 0]
    g, _ = _check(P)
    assert np.array_equal(g[0, :, 3], g[0, :, 0])


def test_no_receivers():
    import torch
    from gpu_common import cfg, inputs
    from paper_1912_08063_amd import api
    P = f32(wl.small_2d(nz=30, nx=70, nt=20, nrec=1))
    v, w, s, r = inputs(P)
    tr = api.forward(v, w, s, r[:, :0], cfg(P))
    torch.cuda.synchronize()
    assert tr.shape == (1, 20, 0)


def test_batched_shots_equal_single_shot_runs_bitwise():
    P = f32(wl.small_2d(nz=60, nx=130, nt=100, nshots=5, nrec=20))
    g = gpu_forward(P)
    for s in range(P.nshots):
        Q = wl.Problem(P.name, P.v, P.dx, P.dt, P.nt, P.order, P.nb, P.eta_max,
                       P.wavelet[s:s + 1], P.src_pos[s:s + 1], P.rec_pos[s:s + 1])
        assert np.array_equal(gpu_forward(Q)[0], g[s])


def test_run_twice_bitwise():
    P = f32(wl.small_3d(shape=(30, 33, 90), nt=50, nrec=20))
    assert np.array_equal(gpu_forward(P), gpu_forward(P))


def _tile_edge_problem(order, nt, nshots=1, seed=31):
    """A 2-D problem whose receivers cover one whole row and one whole column of
    the padded grid's model part (crossing every tile edge of the multi-step
    launches: output tiles of 56, 48 or 32 columns and 16 rows) and whose
    source sits on a tile corner."""
    nb = 6
    P = wl.small_2d(nz=45, nx=97, nt=nt, order=order, nb=nb, seed=seed, nshots=nshots, nrec=1)
    nz, nx = P.v.shape
    row = [(16 - nb, x) for x in range(nx)]
    col = [(z, 32 - nb) for z in range(nz)]
    rec = np.array([row + col] * nshots, dtype=np.int64)
    src = np.array([[16 - nb, 32 - nb]] * nshots, dtype=np.int64)
    return wl._pack(P.name + "-edges", P.v, P.dx, P.dt, nt, order, nb, 25.0, src, rec,
                    eta_max=P.eta_max)


@pytest.mark.parametrize("order", [8, 4, 2])
def test_2d_multi_step_launches_bitwise_equal_single_steps(order, monkeypatch):
    """Small forward-only 2-D calls advance up to 4 steps per launch in LDS
    (FWI_MULTI2D=0 keeps one step per launch): traces bitwise equal for step
    counts that leave every remainder (1 .. 14 steps, a single last step
    included), for receivers on every tile edge and a source on a tile corner,
    and for several shots in one call."""
    for nt, nshots in [(1, 1), (2, 1), (3, 1), (4, 2), (5, 1), (6, 1), (7, 3), (14, 1)]:
        P = f32(_tile_edge_problem(order, nt, nshots))
        monkeypatch.setenv("FWI_MULTI2D", "0")
        ref = gpu_forward(P)
        monkeypatch.setenv("FWI_MULTI2D", "1")
        got = gpu_forward(P)
        assert np.array_equal(got, ref), (order, nt, nshots)


def test_2d_multi_step_launches_match_the_oracle():
    P = _tile_edge_problem(8, 61)
    _check(P)
