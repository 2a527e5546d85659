"""Pins of the FP64 L-BFGS reference (oracle/lbfgs.py) that checks the GPU
inversion loop: each against a definition computed another way.

* The two-loop recursion equals the dense BFGS inverse-Hessian update
  H_{k+1} = V_k' H_k V_k + rho_k s_k s_k', V_k = I - rho_k y_k s_k',
  from H_0 = gamma I (Nocedal & Wright, Eqs. 7.16-7.20): a dropped term, a
  swapped loop order or a wrong rho fails it.
* The secant condition H y_newest = s_newest.
* Unconstrained convex quadratic: converges to A^-1 b, the value never rises.
* Box constraints: the first iterate is the projected steepest-descent step
  of the stated length, and every iterate stays inside the box.
"""
import numpy as np

from oracle import lbfgs


def _pairs(n, m, seed):
    rng = np.random.default_rng(seed)
    S, Y = [], []
    for _ in range(m):
        s = rng.standard_normal(n)
        y = s + 0.3 * rng.standard_normal(n)      # s'y > 0 with high probability
        assert s @ y > 0
        S.append(s)
        Y.append(y)
    return S, Y


def test_two_loop_equals_dense_bfgs_update():
    n = 7
    for m in (1, 2, 4):
        S, Y = _pairs(n, m, seed=m)
        gamma = (S[-1] @ Y[-1]) / (Y[-1] @ Y[-1])
        H = gamma * np.eye(n)
        for s, y in zip(S, Y):
            rho = 1.0 / (y @ s)
            V = np.eye(n) - rho * np.outer(y, s)
            H = V.T @ H @ V + rho * np.outer(s, s)
        g = np.random.default_rng(99).standard_normal(n)
        np.testing.assert_allclose(lbfgs.two_loop(g, S, Y), H @ g, rtol=1e-12, atol=1e-12)


def test_secant_condition_on_the_newest_pair():
    S, Y = _pairs(9, 3, seed=5)
    np.testing.assert_allclose(lbfgs.two_loop(Y[-1], S, Y), S[-1], rtol=1e-11, atol=1e-12)


def test_no_pairs_is_the_gradient():
    g = np.arange(5.0)
    np.testing.assert_array_equal(lbfgs.two_loop(g, [], []), g)


def test_quadratic_converges_to_the_solution():
    rng = np.random.default_rng(3)
    n = 12
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    b = rng.standard_normal(n)
    f = lambda x: 0.5 * x @ A @ x - b @ x
    fg = lambda x: (f(x), A @ x - b)
    x, hist, steps = lbfgs.minimise(f, fg, np.zeros(n), 60, -1e9, 1e9, memory=5,
                                    first_step=0.1)
    assert all(b2 <= a2 + 1e-12 for a2, b2 in zip(hist, hist[1:]))
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-6, atol=1e-8)
    assert steps[1:] and max(steps[1:]) == 1.0      # unit quasi-Newton steps accepted


def test_box_constraints_first_step_and_feasibility():
    """The first iteration is a projected steepest-descent step whose largest
    component change is first_step; every iterate stays in the box and the
    value never rises (projected L-BFGS need not reach the box optimum)."""
    a = np.array([1.0, 2.0, 4.0, 0.5, 3.0])
    b = np.array([3.0, -4.0, 1.0, 2.0, -0.3])
    lo, hi = -1.0, 1.0
    f = lambda x: float(np.sum(0.5 * a * x * x - b * x))
    fg = lambda x: (f(x), a * x - b)
    x0 = np.zeros(5)
    x1, h1, s1 = lbfgs.minimise(f, fg, x0, 1, lo, hi, memory=3, first_step=0.5)
    g0 = a * x0 - b
    step = 0.5 / np.abs(g0).max()
    assert s1 == [step]                           # accepted at the first trial
    np.testing.assert_allclose(x1, np.clip(x0 - step * g0, lo, hi), rtol=0, atol=1e-15)
    x, hist, _ = lbfgs.minimise(f, fg, x0, 40, lo, hi, memory=3, first_step=0.5)
    assert np.all(x >= lo) and np.all(x <= hi)
    assert all(b2 <= a2 + 1e-12 for a2, b2 in zip(hist, hist[1:]))
    assert hist[-1] < f(np.clip(x0 - step * g0, lo, hi))
