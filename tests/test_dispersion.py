"""Phase-error tool (Section 4, Fig. 6) against closed forms.

* Order 2: k_eff dx = 2 sin(theta / 2) exactly.
* Any order 2M: k_eff^2 dx^2 = theta^2 - eps theta^(2M+2) + O(theta^(2M+4)) with
  eps = 2 (M!)^2 / (2M+2)!, so the phase error tends to eps theta^(2M) / 2.
* The weights equal the oracle's exact rational weights.
* The Fig. 6 saving: 8th -> 16th order saves about 12 % per axis only at a
  5 % phase-error tolerance; at 1e-3 it is about 30 % (the paper's Table 1
  moves from 1024 to 768 cells per axis, 25 %).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1912_08063_amd import dispersion


def test_second_order_closed_form():
    th = np.linspace(1e-3, math.pi, 500)
    ref = np.abs(np.sin(th / 2) / (th / 2) - 1.0)
    assert np.allclose(dispersion.phase_error(2, th), ref, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("order", [2, 4, 6, 8, 12, 16])
def test_leading_error_term(order):
    M = order // 2
    eps = 2.0 * math.factorial(M) ** 2 / math.factorial(2 * M + 2)
    th = 0.02 if order <= 8 else 0.15
    got = dispersion.phase_error(order, th)
    assert got == pytest.approx(0.5 * eps * th ** (2 * M), rel=2e-2)


@pytest.mark.parametrize("order", [2, 8, 16])
def test_weights_match_oracle(order):
    ref = [float(c) for c in oracle.fd_weights(order)[1:]]
    assert np.allclose(dispersion.weights(order), ref, rtol=1e-14, atol=0)


@pytest.mark.parametrize("order", [2, 4, 8, 16])
def test_error_increases_with_sampling(order):
    # above rounding level (the error is ~1e-7 or more from theta = 1 on)
    th = np.linspace(1.0, math.pi, 2000)
    e = dispersion.phase_error(order, th)
    assert np.all(np.diff(e) > 0)


def test_fig6_saving_depends_on_tolerance():
    assert 0.11 <= dispersion.domain_reduction(8, 16, 0.05) <= 0.14
    assert 0.28 <= dispersion.domain_reduction(8, 16, 1e-3) <= 0.32
    # a higher order never needs more points per wavelength
    for tol in (0.05, 1e-2, 1e-3):
        assert (dispersion.points_per_wavelength(16, tol)
                < dispersion.points_per_wavelength(8, tol)
                < dispersion.points_per_wavelength(4, tol))


def test_max_theta_meets_tolerance_and_max_dx():
    for order in (8, 16):
        th = dispersion.max_theta(order, 1e-3)
        assert dispersion.phase_error(order, th) <= 1e-3
        assert dispersion.phase_error(order, th * 1.001) > 1e-3
    dx = dispersion.max_dx(8, 1e-3, vmin=1500.0, fmax=25.0)
    assert dx == pytest.approx(1500.0 / 25.0 / dispersion.points_per_wavelength(8, 1e-3))
