"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: each checks a property that a
dropped term, a wrong sign, a wrong index or a transposed operand would break
(exactness on polynomials, energy conservation, reciprocity, the adjoint
dot-product identity, central finite differences of the misfit, analytic
Green's functions, symmetry, linearity, time invariance, stability limit).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1912_08063_amd import workloads as wl


# ------------------------------------------------------------------ weights
@pytest.mark.parametrize("order", [2, 4, 8, 16])
def test_weights_exact_on_polynomials(order):
    """Second-derivative weights are exact on x^k for k <= 2M+1 and first fail at 2M+2."""
    c = oracle.fd_weights(order)
    M = order // 2
    for k in range(0, 2 * M + 2):
        # FD second derivative of x^k at x = 0 with dx = 1
        s = c[0] * (1 if k == 0 else 0) + sum(c[m] * (Fraction(m) ** k + Fraction(-m) ** k)
                                              for m in range(1, M + 1))
        exact = 2 if k == 2 else 0
        assert s == exact, (order, k, s)
    k = 2 * M + 2
    s = sum(c[m] * (Fraction(m) ** k + Fraction(-m) ** k) for m in range(1, M + 1))
    assert s != 0


def test_weights_textbook_8th_order():
    """8th-order central weights (Fornberg's table)."""
    assert oracle.fd_weights(8) == [Fraction(-205, 72), Fraction(8, 5), Fraction(-1, 5),
                                    Fraction(8, 315), Fraction(-1, 560)]


def test_weights_16th_order_leading_terms():
    c = oracle.fd_weights(16)
    assert c[1] == Fraction(16, 9) and c[2] == Fraction(-14, 45) and c[8] == Fraction(-1, 411840)


@pytest.mark.parametrize("order", [8, 16])
@pytest.mark.parametrize("ndim", [2, 3])
def test_c_laplacian_exact_on_polynomials(order, ndim):
    """The C stencil reproduces lap(x^a y^b z^c) exactly away from the ghost cells,
    with the 1/dx^2 factor (dx != 1), on every axis."""
    M = order // 2
    dx = 0.37
    n = 2 * M + 9
    rng = np.random.default_rng(0)
    coords = [(np.arange(n) - n / 2 + rng.uniform(-.3, .3)) * dx for _ in range(ndim)]
    grids = np.meshgrid(*coords, indexing="ij")
    for trial in range(6):
        exps = rng.integers(0, 2 * M + 2, size=ndim)
        p = np.ones_like(grids[0])
        for g, e in zip(grids, exps):
            p = p * g ** int(e)
        ana = np.zeros_like(p)
        for a in range(ndim):
            e = int(exps[a])
            if e < 2:
                continue
            term = e * (e - 1) * np.ones_like(p)
            for b in range(ndim):
                eb = int(exps[b]) - (2 if b == a else 0)
                term = term * grids[b] ** eb
            ana = ana + term
        num = oracle.laplacian(p, dx, order)
        sl = tuple(slice(M, n - M) for _ in range(ndim))
        scale = np.abs(p[sl]).max() / dx ** 2 + 1.0
        assert np.abs(num[sl] - ana[sl]).max() <= 1e-9 * scale, (exps, order, ndim)


@pytest.mark.parametrize("order", [8, 16])
def test_laplacian_symmetric_with_zero_ghosts(order):
    """<q, L p> == <L q, p> on a grid with zero ghost cells (the adjoint relies on it)."""
    rng = np.random.default_rng(1)
    for shape in [(13, 17), (9, 11, 14)]:
        p, q = rng.standard_normal(shape), rng.standard_normal(shape)
        a = np.sum(q * oracle.laplacian(p, 1.3, order))
        b = np.sum(oracle.laplacian(q, 1.3, order) * p)
        assert abs(a - b) <= 1e-12 * abs(a)


def test_paper_stencil_is_8th_order_star():
    """Fig. 3 right: the 8th-order 3-D star has 25 points (24 neighbours + centre)."""
    p = np.zeros((11, 11, 11))
    p[5, 5, 5] = 1.0
    lp = oracle.laplacian(p, 1.0, 8)
    assert np.count_nonzero(lp) == 25


# ------------------------------------------------------------ stability (CFL)
def test_cfl_limits_values():
    assert abs(oracle.max_symbol(8) - 6.501587) < 1e-6
    assert abs(oracle.cfl_limit(2, 8) - 0.5546) < 1e-4
    assert abs(oracle.cfl_limit(3, 8) - 0.4529) < 1e-4
    assert abs(oracle.cfl_limit(3, 16) - 0.4237) < 1e-4


@pytest.mark.parametrize("factor,grows", [(0.99, False), (1.01, True)])
def test_cfl_limit_is_the_stability_edge(factor, grows):
    nz = nx = 40
    v = np.full((nz, nx), 2000.0)
    dx = 10.0
    dt = factor * oracle.cfl_limit(2, 8) * dx / 2000.0
    nt = 3000
    rng = np.random.default_rng(3)
    w = np.zeros(nt)
    w[:20] = rng.standard_normal(20)
    tr = oracle.forward(v, w, [[20, 20]], [[20, 21]], dx, dt, 8, nb=0)[0, :, 0]
    early = np.abs(tr[20:200]).max()
    late = np.abs(tr[-200:]).max()
    if grows:
        assert not np.isfinite(late) or late > 1e6 * early
    else:
        assert late < 10 * early


# ------------------------------------------------------------------ energy
@pytest.mark.parametrize("shape,order", [((40, 45), 8), ((18, 20, 22), 8), ((40, 45), 16)])
def test_energy_conserved_without_sponge(shape, order):
    """Sponge off, source switched off: the leapfrog energy is constant (FP64)."""
    rng = np.random.default_rng(4)
    v = 1500.0 + 1500.0 * wl.smooth(rng.random(shape), 2.0)
    dx = 10.0
    dt = 0.3 * dx / v.max()
    nt = 200
    w = np.zeros(nt)
    w[:15] = rng.standard_normal(15)
    src = [n // 2 for n in shape]
    _, st = oracle.forward(v, w, [src], [src], dx, dt, order, nb=0, return_states=True)
    e = oracle.energy(st[0][16:], v, dx, dt, order, 0)
    assert e.min() > 0
    assert np.abs(e - e[0]).max() <= 1e-11 * e[0]


def test_energy_non_increasing_with_sponge():
    shape = (40, 45)
    v = np.full(shape, 2000.0)
    dx, nb = 10.0, 10
    dt = 0.3 * dx / 2000.0
    nt = 400
    w = wl.ricker(25.0, nt, dt)
    w[100:] = 0.0
    eta = wl.default_eta_max(2000.0, nb, dx)
    _, st = oracle.forward(v, w, [[20, 22]], [[20, 22]], dx, dt, 8, nb=nb, eta_max=eta,
                           return_states=True)
    # energy of the padded grid (the sponge cells carry the same kappa)
    vpad = oracle.pad_model(v, nb)
    e = oracle.energy(st[0][101:], vpad, dx, dt, 8, 0)
    assert np.all(np.diff(e) <= 1e-12 * e[0])
    assert e[-1] < 0.05 * e[0]   # the sponge removes most of it


# ------------------------------------------------------------- reciprocity
def test_reciprocity_heterogeneous_with_sponge():
    """v_s^2 d(s -> r) == v_r^2 d(r -> s) for the discrete operator."""
    rng = np.random.default_rng(5)
    shape = (30, 41)
    v = 1500.0 + 2000.0 * wl.smooth(rng.random(shape), 1.5)
    dx, nb = 10.0, 8
    dt = 0.3 * dx / v.max()
    nt = 300
    w = wl.ricker(20.0, nt, dt)
    eta = wl.default_eta_max(v.max(), nb, dx)
    s, r = (3, 5), (21, 33)
    d_sr = oracle.forward(v, w, [s], [r], dx, dt, 8, nb, eta)[0, :, 0]
    d_rs = oracle.forward(v, w, [r], [s], dx, dt, 8, nb, eta)[0, :, 0]
    a = v[s] ** 2 * d_sr
    b = v[r] ** 2 * d_rs
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_reciprocity_3d():
    rng = np.random.default_rng(6)
    shape = (14, 15, 16)
    v = 1500.0 + 2000.0 * wl.smooth(rng.random(shape), 1.0)
    dx, nb = 10.0, 4
    dt = 0.3 * dx / v.max()
    w = wl.ricker(30.0, 120, dt)
    eta = wl.default_eta_max(v.max(), nb, dx)
    s, r = (2, 3, 4), (10, 11, 9)
    a = v[s] ** 2 * oracle.forward(v, w, [s], [r], dx, dt, 8, nb, eta)[0, :, 0]
    b = v[r] ** 2 * oracle.forward(v, w, [r], [s], dx, dt, 8, nb, eta)[0, :, 0]
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


# ------------------------------------------------------------- dot product
@pytest.mark.parametrize("shape", [(25, 31), (11, 12, 13)])
def test_adjoint_dot_product(shape):
    """<F w, y> == <w, F^T y> where F maps the wavelet to the traces."""
    rng = np.random.default_rng(7)
    v = 1500.0 + 2000.0 * wl.smooth(rng.random(shape), 1.5)
    dx, nb = 10.0, 5
    dt = 0.3 * dx / v.max()
    nt = 90
    eta = wl.default_eta_max(v.max(), nb, dx)
    src = tuple(int(rng.integers(0, n)) for n in shape)
    rec = np.stack([rng.integers(0, n, 9) for n in shape], axis=1)
    w = rng.standard_normal(nt)
    y = rng.standard_normal((nt, 9))
    Fw = oracle.forward(v, w, [src], rec, dx, dt, 8, nb, eta)[0]
    FTy = oracle.adjoint_source_probe(v, src, rec, y, dx, dt, 8, nb, eta)
    a, b = np.sum(Fw * y), np.sum(w * FTy)
    assert abs(a - b) <= 1e-11 * max(abs(a), abs(b))


def test_fold_is_transpose_of_pad():
    rng = np.random.default_rng(8)
    for shape in [(7, 9), (5, 6, 7)]:
        v = rng.standard_normal(shape)
        g = rng.standard_normal(tuple(n + 6 for n in shape))
        a = np.sum(oracle.pad_model(v, 3) * g)
        b = np.sum(v * oracle.fold_model(g, 3))
        assert abs(a - b) <= 1e-12 * abs(a)


# -------------------------------------------------------- gradient vs FD
@pytest.mark.parametrize("ndim", [2, 3])
def test_gradient_matches_central_differences(ndim):
    """dv from the adjoint equals central differences of the misfit, O(h^2)."""
    rng = np.random.default_rng(9)
    shape = (16, 23) if ndim == 2 else (9, 10, 11)
    v_true = 1800.0 + 900.0 * wl.smooth(rng.random(shape), 1.5)
    v0 = wl.smooth(v_true, 3.0)
    dx, nb = 10.0, 4
    dt = 0.3 * dx / 2700.0
    nt = 110 if ndim == 2 else 70
    eta = wl.default_eta_max(2700.0, nb, dx)
    src = [[1] * ndim, [shape[0] - 2] + [n // 2 for n in shape[1:]]]
    rec = np.stack([rng.integers(0, n, 12) for n in shape], axis=1)
    w = wl.ricker(30.0, nt, dt)
    obs = oracle.forward(v_true, w, src, rec, dx, dt, 8, nb, eta)
    phi, dv = oracle.gradient(v0, w, src, rec, obs, dx, dt, 8, nb, eta)
    direction = rng.standard_normal(shape)   # touches edge cells too (fold)
    errs = []
    for h in [0.1, 0.01]:
        pp = oracle.misfit_residual(oracle.forward(v0 + h * direction, w, src, rec, dx, dt, 8, nb, eta), obs)[0]
        pm = oracle.misfit_residual(oracle.forward(v0 - h * direction, w, src, rec, dx, dt, 8, nb, eta), obs)[0]
        fd = (pp - pm) / (2 * h)
        an = np.sum(dv * direction)
        errs.append(abs(fd - an) / abs(an))
    assert errs[1] < 1e-6
    assert errs[1] < errs[0] / 20      # second-order convergence in h


def test_zero_residual_gives_zero_gradient():
    v = wl.gaussian_anomaly_2d(30, 30, centre=(15, 15), sigma=3)
    w = wl.ricker(25.0, 80, 1e-3)
    obs = oracle.forward(v, w, [[4, 15]], [[4, 3], [4, 27]], 10.0, 1e-3, 8, 5, 100.0)
    phi, dv = oracle.gradient(v, w, [[4, 15]], [[4, 3], [4, 27]], obs, 10.0, 1e-3, 8, 5, 100.0)
    assert phi == 0.0 and np.all(dv == 0.0)


# ----------------------------------------- linearity, shift, mirror symmetry
def test_linearity_and_time_invariance():
    v = wl.gaussian_anomaly_2d(30, 34, centre=(15, 17), sigma=4)
    dt = 1e-3
    w = wl.ricker(25.0, 150, dt)
    rec = [[4, 3], [20, 30], [29, 0]]
    d1 = oracle.forward(v, w, [[4, 17]], rec, 10.0, dt, 8, 6, 120.0)
    d2 = oracle.forward(v, 2.0 * w, [[4, 17]], rec, 10.0, dt, 8, 6, 120.0)
    assert np.array_equal(2.0 * d1, d2)          # scaling by 2 is exact in binary
    k = 17
    ws = np.concatenate([np.zeros(k), w[:-k]])
    d3 = oracle.forward(v, ws, [[4, 17]], rec, 10.0, dt, 8, 6, 120.0)
    assert np.array_equal(d3[0, k:], d1[0, :-k]) and np.all(d3[0, :k] == 0.0)


def test_mirror_symmetry_homogeneous():
    nx = 41
    v = np.full((30, nx), 2500.0)
    dt = 1e-3
    w = wl.ricker(20.0, 200, dt)
    rec = [[10, 20 - j] for j in range(1, 15)] + [[10, 20 + j] for j in range(1, 15)]
    d = oracle.forward(v, w, [[5, 20]], rec, 10.0, dt, 8, 7, 150.0)[0]
    assert np.abs(d[:, :14] - d[:, 14:]).max() <= 1e-13 * np.abs(d).max()


# -------------------------------------------------- analytic Green's functions
def _ricker_t(f, t, t0):
    a = (np.pi * f * (t - t0)) ** 2
    return (1 - 2 * a) * np.exp(-a)


@pytest.mark.slow
def test_green_3d_homogeneous():
    """3-D point source: p(r, t) = w(t - r/v) / (4 pi v^2 r)."""
    v0, dx, f = 2000.0, 10.0, 8.0
    dt = 0.2 * dx / v0
    n = 64
    v = np.full((n, n, n), v0)
    t0 = 1.5 / f
    nt = 330
    w = wl.ricker(f, nt, dt, t0)
    src = (20, 32, 32)
    rec = (20, 32, 57)   # r = 250 m along x
    r = 25 * dx
    nb = 20
    d = oracle.forward(v, w, [src], [rec], dx, dt, 8, nb, wl.default_eta_max(v0, nb, dx))[0, :, 0]
    t = (np.arange(nt) + 1) * dt
    ana = _ricker_t(f, t - r / v0, t0) / (4 * np.pi * v0 ** 2 * r)
    err = np.linalg.norm(d - ana) / np.linalg.norm(ana)
    assert err < 3e-3, err


@pytest.mark.slow
def test_green_2d_homogeneous():
    """2-D line source: P = irfft(W(w) * (-i / (4 v^2)) H0^(2)(w r / v)), exp(-iwt) FFT."""
    from scipy.special import hankel2
    v0, dx, f = 2000.0, 5.0, 10.0
    dt = 0.2 * dx / v0
    t0 = 1.5 / f
    nt = 700
    r_cells = 60
    n_z, n_x = 200, 200
    v = np.full((n_z, n_x), v0)
    src = (100, 70)
    rec = (100, 70 + r_cells)
    nb = 30
    w = wl.ricker(f, nt, dt, t0)
    d = oracle.forward(v, w, [src], [rec], dx, dt, 8, nb, wl.default_eta_max(v0, nb, dx))[0, :, 0]
    N = 16 * nt
    wpad = np.zeros(N)
    wpad[:nt] = w
    W = np.fft.rfft(wpad)
    om = 2 * np.pi * np.fft.rfftfreq(N, dt)
    G = np.zeros_like(W)
    r = r_cells * dx
    G[1:] = -1j / (4 * v0 ** 2) * hankel2(0, om[1:] * r / v0)
    P = np.fft.irfft(W * G, N)   # sum_n G(t - t_n) w_n dt == irfft(rfft(w) * G_hat)
    ana = P[1:nt + 1]
    err = np.linalg.norm(d - ana) / np.linalg.norm(ana)
    assert err < 3e-3, err


# ------------------------------------------------- the paper's own arithmetic
def test_table1_gcells_per_second(tmp_path):
    """Table 1: Gcells/s = N^3 * steps / time, the metric used throughout."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table1.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for n, steps, secs, gcells in rows:
        rate = int(n) ** 3 * int(steps) / float(secs) / 1e9
        assert abs(rate - float(gcells)) < 0.006, (n, rate, gcells)
