"""Pins of the oracle's Hankel functions (scipy) against mpmath and the Wronskian."""
import mpmath as mp
import numpy as np
import pytest

from oracle.special import h0, h1

mp.mp.dps = 40
ZS = [1e-3, 0.1, 0.5, 1.0, 3.7, 7.9, 12.0, 19.5, 24.9, 25.1, 40.0, 97.3, 411.0, 1234.5, 6624.0, 25000.0]


@pytest.mark.parametrize("z", ZS)
def test_hankel_vs_mpmath(z):
    ref0 = complex(mp.hankel1(0, mp.mpf(z)))
    ref1 = complex(mp.hankel1(1, mp.mpf(z)))
    # absolute error relative to |H|; large z is limited by rounding z itself
    tol = max(2e-14, 4 * z * 1.1e-16)
    assert abs(h0(z) - ref0) / abs(ref0) < tol
    assert abs(h1(z) - ref1) / abs(ref1) < tol


def test_wronskian():
    z = np.geomspace(1e-2, 1e4, 200)
    H0, H1 = h0(z), h1(z)
    lhs = H1.real * H0.imag - H0.real * H1.imag      # J1 Y0 - J0 Y1
    assert np.max(np.abs(lhs * np.pi * z / 2 - 1)) < 1e-11
