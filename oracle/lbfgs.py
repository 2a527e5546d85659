"""L-BFGS outer iteration in FP64 NumPy -- TEST INFRASTRUCTURE ONLY.

The reference the GPU inversion loop is checked against.  Only ``tests/``
imports it; the product never does, and it imports nothing from the product.

What it computes.  Full-waveform inversion minimises the least-squares misfit
of Eq. 1 over the velocity model; Section 1 of the paper names the misfit and
its gradient as the costly part of every iteration.  The paper prescribes no
optimiser, so this is the standard limited-memory BFGS method written from
its textbook definition (Nocedal & Wright, *Numerical Optimization*, 2nd ed.:
the two-loop recursion of Algorithm 7.4 with the initial scaling
gamma_k = s'y / y'y of Eq. 7.20, and backtracking under the Armijo condition of
Algorithm 3.1), with each trial model projected onto the box [lo, hi]:

* direction  d = -H g, H the inverse-Hessian approximation of the last
  `memory` pairs (s_i, y_i) = (x_{i+1} - x_i, g_{i+1} - g_i);
* first trial step 1 once pairs exist, otherwise the step whose largest
  component change is `first_step`;
* trial x_t = clip(x + step d, lo, hi), accepted when
  f(x_t) <= f(x) + c1 step g'd, otherwise step /= 2 (at most `max_backtracks`
  trials; if none is accepted the iteration stops);
* a pair is stored only if s'y > 1e-30 max(y'y, 1e-300) (curvature), and a
  direction that is not a descent direction discards the memory and falls
  back to -g.

``fwi`` runs it on the oracle's misfit and gradient.
"""
from __future__ import annotations

import numpy as np


def two_loop(g, S, Y):
    """H g for the L-BFGS matrix of the pairs S, Y (oldest first), H_0 = gamma I."""
    q = np.array(g, dtype=np.float64, copy=True)
    m = len(S)
    rho = [1.0 / float(np.vdot(Y[i], S[i])) for i in range(m)]
    alpha = [0.0] * m
    for i in range(m - 1, -1, -1):          # newest to oldest
        alpha[i] = rho[i] * float(np.vdot(S[i], q))
        q = q - alpha[i] * Y[i]
    gamma = float(np.vdot(S[-1], Y[-1])) / float(np.vdot(Y[-1], Y[-1])) if m else 1.0
    r = gamma * q
    for i in range(m):                      # oldest to newest
        beta = rho[i] * float(np.vdot(Y[i], r))
        r = r + (alpha[i] - beta) * S[i]
    return r


def minimise(f, fg, x0, iters, lo, hi, memory=5, first_step=20.0, c1=1e-4, max_backtracks=8):
    """Projected L-BFGS.  f(x) -> value, fg(x) -> (value, gradient).
    Returns (x, history of values, accepted steps)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    phi, g = fg(x)
    hist, steps = [float(phi)], []
    S, Y = [], []
    for _ in range(iters):
        d = -two_loop(g, S, Y)
        gd = float(np.vdot(g, d))
        if gd >= 0.0:
            S, Y = [], []
            d = -np.asarray(g, dtype=np.float64)
            gd = float(np.vdot(g, d))
        step = 1.0 if S else first_step / max(float(np.abs(d).max()), 1e-30)
        xt = None
        for _ in range(max_backtracks):
            trial = np.clip(x + step * d, lo, hi)
            if f(trial) <= phi + c1 * step * gd:
                xt = trial
                break
            step *= 0.5
        if xt is None:
            break
        phi_t, g_t = fg(xt)
        s, y = xt - x, np.asarray(g_t, dtype=np.float64) - g
        if float(np.vdot(s, y)) > 1e-30 * max(float(np.vdot(y, y)), 1e-300):
            S.append(s)
            Y.append(y)
            if len(S) > memory:
                S.pop(0)
                Y.pop(0)
        x, g, phi = xt, np.asarray(g_t, dtype=np.float64), float(phi_t)
        hist.append(phi)
        steps.append(step)
    return x, hist, steps


def fwi(v0, w, src_pos, rec_pos, obs, dx, dt, order, nb, eta_max, iters, vmin, vmax,
        **kw):
    """L-BFGS on the oracle's Eq. 1 misfit and its exact gradient."""
    import oracle

    def f(v):
        d = oracle.forward(v, w, src_pos, rec_pos, dx, dt, order, nb, eta_max)
        return oracle.misfit_residual(d, obs)[0]

    def fg(v):
        return oracle.gradient(v, w, src_pos, rec_pos, obs, dx, dt, order, nb, eta_max)

    return minimise(f, fg, v0, iters, vmin, vmax, **kw)
