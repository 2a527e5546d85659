"""Phase error of the star stencil's second derivative, and the grid spacing it
allows (the trade-off of Section 4, Fig. 6: a higher order samples the same
wavefield with fewer cells per axis).

For a plane wave cos(k x) sampled at spacing dx, the order-2M central second
derivative returns -k_eff^2 cos(k x) with

    k_eff^2 dx^2 = sum_m 2 c_m (1 - cos(m k dx)),   c_m the stencil weights,

so the relative phase (wavenumber) error is |k_eff / k - 1|, a function of
theta = k dx alone.  It grows with theta; for a tolerance tau, theta_max(tau)
is the coarsest sampling that stays within it, i.e. 2 pi / theta_max points
per wavelength.  At equal tolerance, going from order a to order b shrinks
every axis by 1 - theta_max,a / theta_max,b.

This is host-side planning arithmetic (no GPU work).

    python -m paper_1912_08063_amd.dispersion --tol 1e-3
"""
from __future__ import annotations

import argparse
import math

import numpy as np


def weights(order: int) -> np.ndarray:
    """c_1..c_M of the maximal-order central second derivative (M = order / 2):
    c_m = 2 (-1)^{m+1} (M!)^2 / (m^2 (M-m)! (M+m)!)."""
    if order < 2 or order % 2:
        raise ValueError("order must be an even integer >= 2")
    M = order // 2
    f = math.factorial
    return np.array([2.0 * (-1) ** (m + 1) * f(M) ** 2 / (m * m * f(M - m) * f(M + m))
                     for m in range(1, M + 1)])


def phase_error(order: int, theta) -> np.ndarray:
    """|k_eff / k - 1| at theta = k dx (0 < theta <= pi)."""
    th = np.asarray(theta, dtype=np.float64)
    c = weights(order)
    s = np.zeros_like(th)
    for m, cm in enumerate(c, start=1):
        # 1 - cos(m th) = 2 sin^2(m th / 2): no cancellation at small theta
        s = s + 4.0 * cm * np.sin(0.5 * m * th) ** 2
    return np.abs(np.sqrt(s) / th - 1.0)


def max_theta(order: int, tol: float, samples: int = 4096) -> float:
    """Largest theta in (0, pi] with phase_error <= tol on all of (0, theta]."""
    if tol <= 0:
        raise ValueError("tol must be positive")
    grid = np.linspace(math.pi / samples, math.pi, samples)
    bad = np.nonzero(phase_error(order, grid) > tol)[0]
    if bad.size == 0:
        return math.pi
    hi = grid[bad[0]]
    lo = grid[bad[0] - 1] if bad[0] > 0 else 0.0
    for _ in range(80):   # the error is increasing between two samples
        mid = 0.5 * (lo + hi)
        if phase_error(order, mid) <= tol:
            lo = mid
        else:
            hi = mid
    return lo


def points_per_wavelength(order: int, tol: float) -> float:
    return 2.0 * math.pi / max_theta(order, tol)


def domain_reduction(order_from: int, order_to: int, tol: float) -> float:
    """Fraction of cells saved on each axis at equal phase-error tolerance."""
    return 1.0 - max_theta(order_from, tol) / max_theta(order_to, tol)


def max_dx(order: int, tol: float, vmin: float, fmax: float) -> float:
    """Coarsest spacing for which the shortest wavelength vmin / fmax keeps
    the phase error within tol."""
    return vmin / (fmax * points_per_wavelength(order, tol))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--tol", type=float, nargs="+", default=[0.05, 1e-2, 1e-3, 1e-4])
    ap.add_argument("--orders", type=int, nargs="+", default=[4, 8, 16])
    args = ap.parse_args(argv)
    print("tolerance  " + "  ".join("ppw(order %d)" % o for o in args.orders)
          + "  8->16 saving per axis")
    for tol in args.tol:
        ppw = ["%13.2f" % points_per_wavelength(o, tol) for o in args.orders]
        print("%9.0e  %s  %6.1f %%" % (tol, "  ".join(ppw), 100 * domain_reduction(8, 16, tol)))


if __name__ == "__main__":
    main()
