"""Closed forms on the unit disk (oracle pins; test infrastructure).

With G(x, y) = sum_m (i/4) J_m(omega r_<) H_m(omega r_>) e^{i m (theta - phi)}
(Graf's addition theorem), every layer operator on the unit circle is
diagonal in e^{i m theta}:
    S_m  = (i pi/2) J_m H_m
    D_m  = D'_m = (i pi omega/4)(J_m' H_m + J_m H_m')
    N_m  = (i pi omega^2/2) J_m' H_m'
(arguments omega, H = H^(1)).  The CFIE symbols of Sec. 1 follow:
    soft  (1/2 + D - i eta S)_m      = (i pi/2) H_m (omega J_m' - i eta J_m)
    hard  (1/2 - D' + N/(i eta))_m   = -(i pi omega/2) H_m' (J_m + i (omega/eta) J_m')
For the plane wave u_I = e^{i omega x_1} = sum_m i^m J_m(omega r) e^{i m theta}
(Jacobi-Anger) the exact densities and scattered fields are
    soft  q_m = -i^m J_m / soft_m,     u = -sum i^m J_m H_m(omega r)/H_m e^{i m theta}
    hard  q_m = -i^m omega J_m' / hard_m, u = -sum i^m J_m' H_m(omega r)/H_m' e^{i m theta}
"""
import numpy as np
from scipy import special as sp


def _bessels(m, omega):
    J = sp.jv(m, omega)
    Jp = sp.jvp(m, omega)
    H = sp.hankel1(m, omega)
    Hp = sp.h1vp(m, omega)
    return J, Jp, H, Hp


def layer_eigs(m, omega):
    J, Jp, H, Hp = _bessels(m, omega)
    S = 1j * np.pi / 2 * J * H
    D = 1j * np.pi * omega / 4 * (Jp * H + J * Hp)
    N = 1j * np.pi * omega ** 2 / 2 * Jp * Hp
    return S, D, N


def cfie_eigs(m, omega, eta, kind):
    J, Jp, H, Hp = _bessels(m, omega)
    if kind == 0:
        return 1j * np.pi / 2 * H * (omega * Jp - 1j * eta * J)
    return -1j * np.pi * omega / 2 * Hp * (J + 1j * (omega / eta) * Jp)


def _modes(omega, extra=100):
    M = int(np.ceil(omega + extra))
    return np.arange(-M, M + 1)


def density(theta, omega, eta, kind):
    """Exact CFIE density q(theta) for the plane wave along +x."""
    m = _modes(omega)
    J, Jp, _, _ = _bessels(m, omega)
    lam = cfie_eigs(m, omega, eta, kind)
    coef = -(1j ** m) * (J if kind == 0 else omega * Jp) / lam
    return np.exp(1j * np.outer(theta, m)) @ coef


def scattered_field(r, theta, omega, kind):
    m = _modes(omega)
    J, Jp, H, Hp = _bessels(m, omega)
    ratio = J / H if kind == 0 else Jp / Hp
    coef = -(1j ** m) * ratio
    Hr = sp.hankel1(m[None, :], omega * np.asarray(r)[:, None])
    return (Hr * np.exp(1j * np.outer(theta, m))) @ coef
