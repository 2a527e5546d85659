"""FP64 CPU oracle for the acoustic FWI hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (the HIP library under
``paper_1912_08063_amd/`` and its binding) never imports, links or calls it,
and the two share no code: only the seeded input generators
(``paper_1912_08063_amd.workloads``, which holds none of the method's
arithmetic) feed both.

What is computed, and where it comes from (Huot et al., "High-resolution
imaging on TPUs"):

* Eq. 1 -- least-squares misfit  phi = ||d_mod - d_obs||_2^2  (no 1/2, no dt),
  summed over shots.
* Eq. 2 -- constant-density acoustic wave equation  P_tt = v^2 lap P + s.
* Eq. 3 -- leapfrog update  P^{n+1} = -P^{n-1} + 2P^n + v^2 dt^2 lap P^n + dt^2 s^n,
  extended by a sponge (damping 2*eta*P_t, centred), which reduces to Eq. 3
  exactly where eta = 0 (the whole model grid).
* Fig. 3 / Section 3 (stencils of order 8 and above) -- central 2M-th order
  star Laplacian; Section 4 -- 8th and 16th order.
* Section 1 (the misfit and its gradient, the costly part of each FWI
  iteration) -- the gradient here is the exact gradient of the discrete
  misfit (discretise, then differentiate), computed with the adjoint
  recurrence in the scaled variable psi = kappa*alpha*lambda.

Readings of points the paper leaves open (source scaling dt^2 w / dx^D,
trace n = field at time (n+1) dt, zero initial state, sponge outside the
model grid with edge-replicated velocity, zero ghost cells beyond the sponge,
positions as integer cells in array-axis order) follow the project's design
notes; every pin that fixes them lives in ``tests/test_oracle_*.py``.

Layout: 2-D arrays are [nz][nx], 3-D arrays [nz][ny][nx] (x fastest).
Positions are model-grid integer indices in the same axis order.
"""
from __future__ import annotations

import ctypes
import math
import os
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    lp = ctypes.POINTER(ctypes.c_long)
    L, I, D = ctypes.c_long, ctypes.c_int, ctypes.c_double
    lib.orc_laplacian.argtypes = [I, L, L, L, I, dp, D, dp, dp]
    lib.orc_laplacian.restype = None
    lib.orc_forward.argtypes = [I, L, L, L, I, dp, D, D, dp, dp, dp, L, L, dp,
                                L, lp, dp, dp]
    lib.orc_forward.restype = I
    lib.orc_adjoint.argtypes = [I, L, L, L, I, dp, D, D, dp, dp, dp, L, L, lp,
                                dp, dp, dp, L, dp]
    lib.orc_adjoint.restype = I
    _lib = lib
    return lib


def _dp(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _lp(a):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_long))


# --------------------------------------------------------------------------
# Stencil weights (Fig. 3; order 8 or more, Section 3; 8th and 16th, Section 4)
# --------------------------------------------------------------------------
def fd_weights(order: int) -> list:
    """Exact central second-derivative weights c_0..c_M for spatial order 2M.

    Closed form of the maximal-order central formula:
        c_m = 2 (-1)^{m+1} (M!)^2 / (m^2 (M-m)! (M+m)!),  m = 1..M,
        c_0 = -2 sum_m c_m.
    Returned as Fractions so that tests can check them exactly.
    """
    if order < 2 or order % 2:
        raise ValueError("order must be a positive even integer")
    M = order // 2
    fM = math.factorial(M)
    c = [Fraction(0)] * (M + 1)
    for m in range(1, M + 1):
        c[m] = Fraction(2 * (-1) ** (m + 1) * fM * fM,
                        m * m * math.factorial(M - m) * math.factorial(M + m))
    c[0] = -2 * sum(c[1:])
    return c


def fd_weights_f64(order: int) -> np.ndarray:
    return np.array([float(x) for x in fd_weights(order)], dtype=np.float64)


def max_symbol(order: int) -> float:
    """max_k of -(c0 + 2 sum_m c_m cos(m k)) over k in [0, pi] (per axis, dx=1)."""
    c = fd_weights_f64(order)
    k = np.linspace(0.0, np.pi, 20001)
    m = np.arange(1, len(c))
    s = -(c[0] + 2.0 * (c[1:, None] * np.cos(np.outer(m, k))).sum(axis=0))
    return float(s.max())


def cfl_limit(ndim: int, order: int) -> float:
    """Largest v dt / dx for which the undamped leapfrog stays bounded:
    dt^2 v^2 / dx^2 * D * S <= 4, with S the largest symbol of one axis."""
    return math.sqrt(4.0 / (ndim * max_symbol(order)))


# --------------------------------------------------------------------------
# Model padding (sponge outside the model, edge-replicated velocity)
# --------------------------------------------------------------------------
def pad_model(v: np.ndarray, nb: int) -> np.ndarray:
    """E v: extend the model by nb cells on every face, copying edge cells."""
    return np.pad(np.asarray(v, dtype=np.float64), nb, mode="edge")


def fold_model(g_pad: np.ndarray, nb: int) -> np.ndarray:
    """E^T g: add every padded cell's value onto the model cell it copies."""
    g_pad = np.asarray(g_pad, dtype=np.float64)
    shape = tuple(n - 2 * nb for n in g_pad.shape)
    out = np.zeros(shape)
    # map each padded index to the model index it replicates, per axis
    maps = [np.clip(np.arange(n) - nb, 0, m - 1) for n, m in zip(g_pad.shape, shape)]
    grids = np.meshgrid(*maps, indexing="ij")
    np.add.at(out, tuple(grids), g_pad)
    return out


def sponge_coefficients(shape_pad, nb: int, eta_max: float, dt: float):
    """alpha, beta over the padded grid.

    eta = eta_max * sum_axes (d_a / nb)^2 with d_a the distance (in cells)
    into the sponge along axis a:  d_a = max(nb - i, i - (n_a - 1 - nb), 0).
    The damped equation P_tt + 2 eta P_t = v^2 lap P + s, with P_t centred,
    gives alpha = 1 / (1 + eta dt), beta = (1 - eta dt) / (1 + eta dt).
    """
    eta = np.zeros(shape_pad)
    if nb > 0 and eta_max != 0.0:
        for a, n in enumerate(shape_pad):
            i = np.arange(n)
            d = np.maximum(np.maximum(nb - i, i - (n - 1 - nb)), 0).astype(np.float64)
            prof = eta_max * (d / nb) ** 2
            sh = [1] * len(shape_pad)
            sh[a] = n
            eta = eta + prof.reshape(sh)
    alpha = 1.0 / (1.0 + eta * dt)
    beta = (1.0 - eta * dt) / (1.0 + eta * dt)
    return alpha, beta


# --------------------------------------------------------------------------
# Problem set-up shared by the oracle entry points
# --------------------------------------------------------------------------
class _Setup:
    def __init__(self, v, dx, dt, order, nb, eta_max):
        v = np.asarray(v, dtype=np.float64)
        if v.ndim not in (2, 3):
            raise ValueError("v must be 2-D [nz][nx] or 3-D [nz][ny][nx]")
        self.ndim = v.ndim
        self.nb = int(nb)
        self.dx = float(dx)
        self.dt = float(dt)
        self.order = int(order)
        self.M = self.order // 2
        self.c = fd_weights_f64(self.order)
        self.model_shape = v.shape
        self.v_pad = pad_model(v, self.nb)
        self.shape_pad = self.v_pad.shape
        self.kappa = np.ascontiguousarray(self.v_pad ** 2 * self.dt ** 2)
        a, b = sponge_coefficients(self.shape_pad, self.nb, float(eta_max), self.dt)
        self.alpha = np.ascontiguousarray(a)
        self.beta = np.ascontiguousarray(b)
        if self.ndim == 2:
            self.nz, self.ny, self.nx = self.shape_pad[0], 1, self.shape_pad[1]
        else:
            self.nz, self.ny, self.nx = self.shape_pad
        self.ncell = self.nz * self.ny * self.nx

    def cell(self, pos):
        """Linear padded-grid index of a model-grid position (array-axis order)."""
        pos = [int(q) for q in pos]
        if len(pos) != self.ndim:
            raise ValueError("position has wrong dimension")
        for q, n in zip(pos, self.model_shape):
            if not 0 <= q < n:
                raise ValueError("position outside the model grid")
        pp = [q + self.nb for q in pos]
        if self.ndim == 2:
            z, x = pp
            y = 0
        else:
            z, y, x = pp
        return (z * self.ny + y) * self.nx + x

    def args(self):
        return (self.ndim, self.nz, self.ny, self.nx, self.M, _dp(self.c), self.dx)


def _shots(src_pos, rec_pos, ndim):
    src_pos = np.asarray(src_pos, dtype=np.int64).reshape(-1, ndim)
    S = src_pos.shape[0]
    rec_pos = np.asarray(rec_pos, dtype=np.int64)
    if rec_pos.ndim == 2:
        rec_pos = np.broadcast_to(rec_pos, (S,) + rec_pos.shape)
    return src_pos, rec_pos.reshape(S, -1, ndim)


def laplacian(p: np.ndarray, dx: float, order: int) -> np.ndarray:
    """Star Laplacian with zero ghost cells, on a 2-D or 3-D array."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    c = fd_weights_f64(order)
    if p.ndim == 2:
        nz, ny, nx = p.shape[0], 1, p.shape[1]
    else:
        nz, ny, nx = p.shape
    out = np.empty_like(p)
    _load().orc_laplacian(p.ndim, nz, ny, nx, order // 2, _dp(c), float(dx), _dp(p), _dp(out))
    return out


def forward(v, w, src_pos, rec_pos, dx, dt, order=8, nb=20, eta_max=0.0,
            return_states=False):
    """Forward modelling (Eq. 3 with sponge), one point source per shot.

    v        model velocity, [nz][nx] or [nz][ny][nx]
    w        source wavelet samples, [nt] (all shots) or [S][nt]; w[n] = w(n dt)
    src_pos  [S][D] model-grid cells
    rec_pos  [R][D] (shared) or [S][R][D]
    returns  traces [S][nt][R] with traces[s][n][r] = p^{n+1}(rec_r),
             plus, if return_states, a list over shots of [nt+1][padded] states.
    """
    st = _Setup(v, dx, dt, order, nb, eta_max)
    src_pos, rec_pos = _shots(src_pos, rec_pos, st.ndim)
    S, R = src_pos.shape[0], rec_pos.shape[1]
    w = np.asarray(w, dtype=np.float64)
    if w.ndim == 1:
        w = np.broadcast_to(w, (S, w.shape[0]))
    nt = w.shape[1]
    traces = np.zeros((S, nt, R))
    states_all = []
    for s in range(S):
        src = st.cell(src_pos[s])
        rec = np.array([st.cell(r) for r in rec_pos[s]], dtype=np.int64)
        ws = np.ascontiguousarray(w[s])
        tr = np.zeros((nt, R))
        states = np.zeros((nt + 1,) + st.shape_pad) if return_states else None
        rc = _load().orc_forward(*st.args(), st.dt, _dp(st.kappa), _dp(st.alpha),
                                 _dp(st.beta), nt, src, _dp(ws), R, _lp(rec),
                                 _dp(tr), _dp(states))
        if rc != 0:
            raise MemoryError("oracle forward: allocation failed")
        traces[s] = tr
        if return_states:
            states_all.append(states)
    if return_states:
        return traces, states_all
    return traces


def adjoint_source_probe(v, src_pos, rec_pos, y, dx, dt, order=8, nb=20, eta_max=0.0):
    """Transpose of the map (wavelet -> traces) of one shot applied to y [nt][R].

    (F^T y)^n = (dt^2 / dx^D) psi^{n+1}(src) / kappa(src), n = 0..nt-1.
    """
    st = _Setup(v, dx, dt, order, nb, eta_max)
    src = st.cell(src_pos)
    rec = np.array([st.cell(r) for r in np.asarray(rec_pos).reshape(-1, st.ndim)],
                   dtype=np.int64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    nt = y.shape[0]
    probe = np.zeros(nt + 2)
    rc = _load().orc_adjoint(*st.args(), st.dt, _dp(st.kappa), _dp(st.alpha),
                             _dp(st.beta), nt, len(rec), _lp(rec), _dp(y), None,
                             None, src, _dp(probe))
    if rc != 0:
        raise MemoryError("oracle adjoint: allocation failed")
    return (st.dt ** 2 / st.dx ** st.ndim) * probe[1:nt + 1] / st.kappa.reshape(-1)[src]


def misfit_residual(traces, obs):
    """Eq. 1: phi = sum (d - d_obs)^2 and its derivative res = 2 (d - d_obs)."""
    d = np.asarray(traces, dtype=np.float64) - np.asarray(obs, dtype=np.float64)
    return float(np.sum(d * d)), 2.0 * d


def backward(v, w, src_pos, rec_pos, grad_traces, dx, dt, order=8, nb=20, eta_max=0.0):
    """Vector-Jacobian product of forward() w.r.t. v for cotangent grad_traces [S][nt][R].

    dv = E^T [ (2 / v_pad) * sum_shots sum_{n=1}^{nt-1} psi^{n+1} * lap(p^n) ].
    """
    st = _Setup(v, dx, dt, order, nb, eta_max)
    src_pos, rec_pos = _shots(src_pos, rec_pos, st.ndim)
    S = src_pos.shape[0]
    w = np.asarray(w, dtype=np.float64)
    if w.ndim == 1:
        w = np.broadcast_to(w, (S, w.shape[0]))
    grad_traces = np.asarray(grad_traces, dtype=np.float64)
    g = np.zeros(st.shape_pad)
    for s in range(S):
        _, states = forward(v, w[s], src_pos[s:s + 1], rec_pos[s], dx, dt, order, nb,
                            eta_max, return_states=True)
        states = states[0]
        rec = np.array([st.cell(r) for r in rec_pos[s]], dtype=np.int64)
        res = np.ascontiguousarray(grad_traces[s])
        nt = res.shape[0]
        gs = np.zeros(st.shape_pad)
        rc = _load().orc_adjoint(*st.args(), st.dt, _dp(st.kappa), _dp(st.alpha),
                                 _dp(st.beta), nt, len(rec), _lp(rec), _dp(res),
                                 _dp(states), _dp(gs), 0, None)
        if rc != 0:
            raise MemoryError("oracle adjoint: allocation failed")
        del states
        g += gs
    dv_pad = (2.0 / st.v_pad) * g
    return fold_model(dv_pad, st.nb)


def gradient(v, w, src_pos, rec_pos, obs, dx, dt, order=8, nb=20, eta_max=0.0):
    """Misfit (Eq. 1) and its exact gradient with respect to the model velocity."""
    traces = forward(v, w, src_pos, rec_pos, dx, dt, order, nb, eta_max)
    phi, res = misfit_residual(traces, obs)
    dv = backward(v, w, src_pos, rec_pos, res, dx, dt, order, nb, eta_max)
    return phi, dv


def energy(states, v, dx, dt, order, nb):
    """Discrete energy E^{n+1/2} = <(p^{n+1}-p^n)^2 / kappa> - <p^{n+1}, lap p^n>,
    which the undamped, source-free leapfrog conserves exactly."""
    v_pad = pad_model(v, nb)
    kappa = v_pad ** 2 * dt ** 2
    out = []
    for n in range(len(states) - 1):
        a = states[n + 1] - states[n]
        out.append(float(np.sum(a * a / kappa) - np.sum(states[n + 1] * laplacian(states[n], dx, order))))
    return np.array(out)
