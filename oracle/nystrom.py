"""Nystrom discretisation of the CFIEs of Sec. 1 (oracle; test infrastructure).

Sound-soft, eq. (3) / eq. (1):   (1/2 I + D - i eta S) q = -u_I
Sound-hard, eq. (2):             (1/2 I - D' + (1/(i eta)) N) q = -du_I/dn
(The hard operator follows the integral equation eq. (2), which is what the
exterior Neumann problem with ansatz u = -S q + (1/(i eta)) D q gives under
outward normals; the displayed operator form eq. (4) flips the signs of D'
and N.  That reading is pinned by the disk eigenvalues in tests.)

Operators (Sec. 1): S, D, D', N with G(x, y) = (i/4) H_0^(1)(omega |x - y|).
The paper leaves the quadrature open ("the Nystrom method", Sec. 1); this
oracle uses Kress's product rule for logarithmic kernels on a 2*pi-periodic
parametrisation (nodes t_j = 2*pi*j/n, n = 2N):

    int_0^{2pi} K(t_i, tau) phi(tau) dtau
        ~ sum_j [ R_{|i-j|} K1(t_i, t_j) + (pi/N) K2(t_i, t_j) ] phi_j,
    K = K1 log(4 sin^2((t - tau)/2)) + K2,
    R_k = -(2pi/N) sum_{m=1}^{N-1} cos(m k pi/N)/m - (pi/N^2) cos(k pi),

and Maue's identity for the hypersingular operator,
    N = D_s S D_s + omega^2 (nu_1 S nu_1 + nu_2 S nu_2),
with D_s the trigonometric-interpolation derivative in arclength (Nyquist
mode dropped).  Every function here is plain and dense.
"""
from __future__ import annotations

import numpy as np

from .special import EULER_GAMMA, h0, h1


# ------------------------------------------------------------ quadrature
def _cos_table(n):
    return np.cos(2 * np.pi * np.arange(n) / n), np.sin(2 * np.pi * np.arange(n) / n)


def kress_R(n: int) -> np.ndarray:
    """R_k for k = 0..n-1 (Kress weights for the log(4 sin^2) factor)."""
    if n % 2:
        raise ValueError("n must be even")
    N = n // 2
    c, _ = _cos_table(n)
    m = np.arange(1, N)
    out = np.empty(n)
    for k0 in range(0, n, 2048):
        k = np.arange(k0, min(n, k0 + 2048))
        idx = np.outer(k, m) % n          # cos(m k pi / N) = cos(2 pi (m k mod n) / n)
        out[k] = -(2 * np.pi / N) * (c[idx] @ (1.0 / m))
    out -= (np.pi / N ** 2) * np.cos(np.arange(n) * np.pi)
    return out


def log4sin2(n: int) -> np.ndarray:
    """log(4 sin^2(pi k / n)) for k = 0..n-1 (k = 0 entry is -inf, unused)."""
    k = np.arange(n)
    with np.errstate(divide="ignore"):
        return np.log(4 * np.sin(np.pi * k / n) ** 2)


def spectral_derivative_row(n: int) -> np.ndarray:
    """d_k, k = 0..n-1, with (d phi/dt)_i = sum_j d_{(i-j) mod n} phi_j.

    Derivative of the trigonometric interpolant with modes |m| <= N-1:
    d_k = -(2/n) sum_{m=1}^{N-1} m sin(2 pi m k / n).
    """
    N = n // 2
    _, s = _cos_table(n)
    m = np.arange(1, N)
    out = np.empty(n)
    for k0 in range(0, n, 2048):
        k = np.arange(k0, min(n, k0 + 2048))
        out[k] = -(2.0 / n) * (s[np.outer(k, m) % n] @ m)
    return out


def circulant(row: np.ndarray) -> np.ndarray:
    n = row.size
    i = np.arange(n)
    return row[(i[:, None] - i[None, :]) % n]


def arclength_derivative_matrix(b) -> np.ndarray:
    """Dense D_s: d/ds = (1/|x'(t)|) d/dt on the periodic node sequence."""
    return circulant(spectral_derivative_row(b.n)) / b.speed[:, None]


# ------------------------------------------------------------ layer operators
def layer_rows(b, omega: float, rows=None):
    """Rows of the discrete S, D, D' (Kress-corrected), as a dict of arrays.

    Kernels (r = |x_i - x_j|, rhat = (x_i - x_j)/r, all times |x'(t_j)|):
      S : K  = (i/4) H0(omega r),                 K1 = -J0(omega r)/(4 pi)
      D : K  = (i omega/4) H1(omega r) nu_j.rhat, K1 = -(omega/(4 pi)) J1 nu_j.rhat
      D': K  = -(i omega/4) H1(omega r) nu_i.rhat, K1 = (omega/(4 pi)) J1 nu_i.rhat
    Diagonal limits: K1_S = -1/(4 pi), K2_S = i/4 - gamma/(2 pi)
    - log(omega |x'|/2)/(2 pi); K1_D = K1_D' = 0, K2_D = K2_D' = -kappa/(4 pi).
    """
    n = b.n
    N = n // 2
    rows = np.arange(n) if rows is None else np.asarray(rows)
    R = kress_R(n)
    lg = log4sin2(n)
    out = {k: np.empty((rows.size, n), np.complex128) for k in ("S", "D", "Dp")}
    j = np.arange(n)
    for c0 in range(0, rows.size, 512):
        ii = rows[c0:c0 + 512]
        d = b.x[ii, None, :] - b.x[None, :, :]
        r = np.linalg.norm(d, axis=-1)
        diag = ii[:, None] == j[None, :]
        r_safe = np.where(diag, 1.0, r)
        H0, H1 = h0(omega * r_safe), h1(omega * r_safe)
        J0, J1 = H0.real, H1.real
        nj_r = np.einsum("jk,ijk->ij", b.nu, d) / r_safe
        ni_r = np.einsum("ik,ijk->ij", b.nu[ii], d) / r_safe
        sp = b.speed[None, :]
        kd = (ii[:, None] - j[None, :]) % n
        Rk = R[kd]
        L = np.where(diag, 0.0, lg[kd])
        kernels = {
            "S": ((1j / 4) * H0 * sp, -J0 / (4 * np.pi) * sp),
            "D": ((1j * omega / 4) * H1 * nj_r * sp, -(omega / (4 * np.pi)) * J1 * nj_r * sp),
            "Dp": (-(1j * omega / 4) * H1 * ni_r * sp, (omega / (4 * np.pi)) * J1 * ni_r * sp),
        }
        spi = b.speed[ii]
        kap = b.kappa[ii]
        diag_k1 = {"S": -spi / (4 * np.pi), "D": 0 * spi, "Dp": 0 * spi}
        diag_k2 = {"S": (1j / 4 - EULER_GAMMA / (2 * np.pi)
                         - np.log(omega * spi / 2) / (2 * np.pi)) * spi,
                   "D": -kap * spi / (4 * np.pi), "Dp": -kap * spi / (4 * np.pi)}
        for name, (K, K1) in kernels.items():
            K2 = K - K1 * L
            K1 = np.where(diag, 0, K1)
            K2 = np.where(diag, 0, K2)
            loc = np.nonzero(diag)
            K1[loc] = diag_k1[name][loc[0]]
            K2[loc] = diag_k2[name][loc[0]]
            out[name][c0:c0 + 512] = Rk * K1 + (np.pi / N) * K2
    return out


def soft_matrix(b, omega, eta, rows=None):
    """Rows of A = 1/2 I + D - i eta S (eq. (3))."""
    rows = np.arange(b.n) if rows is None else np.asarray(rows)
    lay = layer_rows(b, omega, rows)
    A = lay["D"] - 1j * eta * lay["S"]
    A[np.arange(rows.size), rows] += 0.5
    return A


def hard_matrix(b, omega, eta):
    """Full A = 1/2 I - D' + (1/(i eta)) N, N by Maue's identity (eq. (2))."""
    lay = layer_rows(b, omega)
    S = lay["S"]
    Ds = arclength_derivative_matrix(b)
    n1, n2 = b.nu[:, 0], b.nu[:, 1]
    N = Ds @ S @ Ds + omega ** 2 * (n1[:, None] * S * n1[None, :]
                                    + n2[:, None] * S * n2[None, :])
    A = -lay["Dp"] + N / (1j * eta)
    A[np.diag_indices(b.n)] += 0.5
    return A


def cfie_matrix(b, omega, eta, kind):
    return soft_matrix(b, omega, eta) if kind == 0 else hard_matrix(b, omega, eta)


# ------------------------------------------------------------ data and field
def plane_wave_rhs(b, omega, angles, kind):
    """f = -u_I (soft) or -du_I/dnu (hard), u_I = exp(i omega d.x); (n, nrhs)."""
    angles = np.atleast_1d(angles)
    d = np.stack([np.cos(angles), np.sin(angles)], 0)          # (2, nrhs)
    ui = np.exp(1j * omega * (b.x @ d))
    if kind == 0:
        return -ui
    return -1j * omega * (b.nu @ d) * ui


def point_source_data(b, omega, z0, kind):
    """Boundary data of the radiating field G(., z0), z0 inside the obstacle.

    soft: f = G(x_i, z0); hard: f = dG(x_i, z0)/dnu(x_i).
    """
    d = b.x - np.asarray(z0)[None, :]
    r = np.linalg.norm(d, axis=1)
    if kind == 0:
        return (1j / 4) * h0(omega * r)
    return -(1j * omega / 4) * h1(omega * r) * np.einsum("ij,ij->i", b.nu, d) / r


def green(omega, x, z0):
    r = np.linalg.norm(np.asarray(x) - np.asarray(z0)[None, :], axis=1)
    return (1j / 4) * h0(omega * r)


def field(b, omega, eta, kind, q, pts):
    """Scattered field at exterior points by the trapezoid rule.

    soft: u = D q - i eta S q;  hard: u = -S q + (1/(i eta)) D q.
    Accurate for points a few node spacings away from the boundary.
    """
    pts = np.atleast_2d(pts)
    d = pts[:, None, :] - b.x[None, :, :]
    r = np.linalg.norm(d, axis=-1)
    G = (1j / 4) * h0(omega * r)
    dG = (1j * omega / 4) * h1(omega * r) * np.einsum("jk,ijk->ij", b.nu, d) / r
    w = b.w[None, :]
    if kind == 0:
        return (dG * w - 1j * eta * G * w) @ q
    return (-G * w + dG * w / (1j * eta)) @ q
