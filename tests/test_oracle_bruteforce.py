"""Pin of the oracle's layer matrices on a non-circular curve against adaptive
quadrature of the singular integrals (independent of the Kress rule)."""
import warnings

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

    # continuous integral in arclength, int k(x_i, y(rho)) phi(rho) drho, by
    # adaptive quadrature (no quadrature rule of the oracle involved) over the
    # trigonometric interpolant of a 16x finer arclength sampling of the curve
    X = np.fft.fft(fine.x, axis=0) / fine.n
    mm = np.fft.fftfreq(fine.n, 1.0 / fine.n)
    keep = np.abs(mm) < fine.n // 2
    Xk, mk = X[keep], mm[keep]

    def geom(s):
        # position and outward normal of the trigonometric interpolant
        e = np.exp(1j * mk * s)
        x = (e @ Xk).real
        t = ((1j * mk * e) @ Xk).real
        return x, np.array([t[1], -t[0]]) / np.linalg.norm(t)

    def chord(s0, u):
        # x(s0) - x(s0 + u) without cancellation for small |u|:
        # e^{i m s0} - e^{i m (s0 + u)} = -2i sin(m u/2) e^{i m (s0 + u/2)}
        e = -2j * np.sin(mk * u / 2) * np.exp(1j * mk * (s0 + u / 2))
        return (e @ Xk).real

    sp_len = b.L / (2 * np.pi)
    for r, i in enumerate([0, 17, 50]):
        _, ni = geom(sig_b[i])

        def integrand(u, part):
            s = s0 + u
            _, ny_ = geom(s)
            d = chord(s0, u)
            rr = np.linalg.norm(d)
            if name == "S":
                k = 1j / 4 * sp.hankel1(0, om * rr)
            elif name == "D":
                k = 1j * om / 4 * sp.hankel1(1, om * rr) * (ny_ @ d) / rr
            else:
                k = -1j * om / 4 * sp.hankel1(1, om * rr) * (ni @ d) / rr
            v = k * dens(s) * sp_len
            return v.real if part == 0 else v.imag

        # one period u in [-pi, pi] around the target, s = s0 + u; the log
        # singularity at u = 0 is approached by pieces graded geometrically,
        # every piece converged (warnings are errors)
        s0 = sig_b[i]
        g = np.array([1e-8, 1e-6, 1e-4, 1e-2, 0.1, 0.5, np.pi])
        edges = np.concatenate([-g[::-1], [0.0], g])
        exact = 0
        with warnings.catch_warnings():
            warnings.simplefilter("error", integrate.IntegrationWarning)
            for part, fac in ((0, 1.0), (1, 1j)):
                for lo, hi in zip(edges[:-1], edges[1:]):
                    exact += fac * integrate.quad(integrand, lo, hi, args=(part,), limit=400,
                                                  epsabs=1e-13, epsrel=1e-12)[0]
        approx = lay[name][r] @ dens(sig_b)
        assert abs(approx - exact) < 1e-9 * max(1.0, abs(exact)), (name, i, approx, exact)
