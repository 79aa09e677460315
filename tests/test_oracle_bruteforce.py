"""Pin of the oracle's layer matrices on a non-circular curve against adaptive
quadrature of the singular integrals (independent of the Kress rule)."""
import numpy as np
import pytest
from scipy import integrate, special as sp

from oracle import nystrom as ny
from synth import sample_boundary
from synth.geometry import curve_by_name


def _arclength_curve(b, curve_name, m=4096):
    """Exact curve points at arclength parameter sigma via dense root finding."""
    from synth.geometry import sample_boundary as sb
    fine = sb(curve_name, m)
    return fine


@pytest.mark.parametrize("name", ["S", "D", "Dp"])
def test_layer_rows_vs_adaptive_quadrature(name):
    # kite at low frequency; density = low-order trig polynomial in sigma
    n, om = 512, 3.0
    b = sample_boundary("kite", n)
    fine = _arclength_curve(b, "kite", 512 * 16)
    lay = ny.layer_rows(b, om, np.array([0, 17, 50]))
    sig_b = 2 * np.pi * np.arange(n) / n
    dens = lambda s: np.cos(2 * s) + 0.5j * np.sin(3 * s) + 0.25

    # continuous integral in arclength: int k(x_i, y(rho)) phi(rho) drho, via a
    # piecewise-cubic-free approach: high-order trapezoid is not allowed near the
    # singularity, so integrate with scipy quad over the fine arclength nodes'
    # trigonometric interpolant of position and normal.
    X = np.fft.fft(fine.x, axis=0) / fine.n
    NU = np.fft.fft(fine.nu, axis=0) / fine.n
    mm = np.fft.fftfreq(fine.n, 1.0 / fine.n)
    keep = np.abs(mm) < fine.n // 2

    def geom(s):
        e = np.exp(1j * mm[keep] * s)
        x = (e @ X[keep]).real
        nu = (e @ NU[keep]).real
        return x, nu / np.linalg.norm(nu)

    sp_len = b.L / (2 * np.pi)
    for r, i in enumerate([0, 17, 50]):
        xi, ni = geom(sig_b[i])

        def integrand(s, part):
            y, ny_ = geom(s)
            d = xi - y
            rr = np.linalg.norm(d)
            if name == "S":
                k = 1j / 4 * sp.hankel1(0, om * rr)
            elif name == "D":
                k = 1j * om / 4 * sp.hankel1(1, om * rr) * (ny_ @ d) / rr
            else:
                k = -1j * om / 4 * sp.hankel1(1, om * rr) * (ni @ d) / rr
            v = k * dens(s) * sp_len
            return v.real if part == 0 else v.imag

        s0 = sig_b[i]
        exact = 0
        for part, fac in ((0, 1.0), (1, 1j)):
            exact += fac * integrate.quad(integrand, s0 + 1e-15, s0 + 2 * np.pi - 1e-15,
                                          args=(part,), limit=400, epsabs=1e-14, epsrel=1e-13)[0]
        approx = lay[name][r] @ dens(sig_b)
        assert abs(approx - exact) < 1e-9 * max(1.0, abs(exact)), (name, i, approx, exact)
