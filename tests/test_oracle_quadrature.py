"""Pins of the Kress weights and the spectral derivative (closed forms)."""
import numpy as np
import pytest

from oracle import nystrom as ny


@pytest.mark.parametrize("n", [16, 64, 256])
def test_kress_weights_exact_on_log_cos(n):
    # int_0^{2pi} log(4 sin^2((t-tau)/2)) cos(m tau) dtau = -2pi/m cos(m t) (m >= 1), 0 (m = 0)
    R = ny.kress_R(n)
    t = 2 * np.pi * np.arange(n) / n
    N = n // 2
    for m in range(0, N):
        for i in (0, 3, n - 1):
            approx = sum(R[abs(i - j)] * np.cos(m * t[j]) for j in range(n))
            exact = 0.0 if m == 0 else -2 * np.pi / m * np.cos(m * t[i])
            assert abs(approx - exact) < 1e-12


@pytest.mark.parametrize("n", [16, 64, 300])
def test_spectral_derivative(n):
    d = ny.spectral_derivative_row(n)
    k = np.arange(1, n)
    # closed form for even n: d_k = (1/2) (-1)^k cot(pi k / n), d_0 = 0
    ref = 0.5 * (-1.0) ** k / np.tan(np.pi * k / n)
    assert abs(d[0]) < 1e-14
    assert np.max(np.abs(d[1:] - ref)) < 1e-11 * n
    t = 2 * np.pi * np.arange(n) / n
    D = ny.circulant(d)
    for m in range(1, n // 2):
        assert np.max(np.abs(D @ np.sin(m * t) - m * np.cos(m * t))) < 1e-10 * n
