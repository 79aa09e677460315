"""Directional preconditioner of Sec. 2 (dense reference; test infrastructure).

Steps, in the paper's order and notation:
  Sec. 2.1  segments P_1..P_m (hierarchical bisection, almost-planar test);
            flat diagonal blocks B_j; direction grids K_i; rounding [k]_i;
            partial Fourier factors U_i (eq. (12)); non-oscillatory part
            M~_ij (eq. (13)) sampled on Chebyshev grids R_i x R_j; rank-1
            entries e_ij (eq. (14)); M ~ B + U E U^t (eq. (15)).
  Sec. 2.2  augmented system eq. (16), factorisation eq. (17) with
            S = U^t B^{-1} U, T = S^{-1}, W = E + T, exact inverse eq. (18),
            and the approximate apply eq. (19) with floor(T) (thresholded)
            and floor(W) = E + antidiag(T).

Readings where the paper is silent or loose (each also listed in the design
notes of the repository):
  * initial segment count 2^round(log2 sqrt(L/lambda)) (the paper's 2^q with
    L = 4^q lambda); almost-planar when length <= sqrt(L lambda / c_max);
    non-planar leaf when length <= m_ell lambda (m_ell = 4) or s <= 8;
  * K_i has 2J+1 points, J = ceil(s/p), p = lambda/ds, spacing 2 pi/(s ds)
    (= omega/2^l when s = 2^l p); the same rule for K_j;
  * [k]_i rounds half away from zero and clamps to [-J, J];
  * U^t is the plain transpose; rho(x_a) - rho(c_i) = (a - (s-1)/2) ds, the
    centre c_i is the curve point at the arclength midpoint, t_i the unit
    tangent there;
  * R_i: m_c first-kind Chebyshev points on the segment's arclength interval
    (centre +- s ds/2); positions and normals there by trigonometric
    interpolation of the node sequence; w^dagger = w^t/s so e_ij is the
    interpolated block mean of M~;
  * M(x, y) = kernel(x, y) * ds; M~ = M / (U_i(x, k^i) U_j(y, k^j));
  * B_j: the Kress-discretised operator on a straight segment of s points
    (soft: 1/2 - i eta S_flat; hard: 1/2 + N_flat/(i eta) with the Laplace
    hypersingular part by the finite-part trapezoid correction);
  * floor(B^{-1}) = exact dense inverse (no H-matrix compression);
  * floor(T_i) keeps the antidiagonal and every entry whose modulus is within
    a 1e-8 relative margin of the (t_keep |K_i|)-th largest (t_keep = 0: dense).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .nystrom import kress_R, log4sin2
from .special import EULER_GAMMA, h0, h1


# ---------------------------------------------------------------- options
@dataclass
class Options:
    m_ell: float = 4.0      # non-planar leaf length in wavelengths
    min_pts: int = 8        # never split below this many points
    m_c: int = 10           # Chebyshev grid size (Sec. 3)
    t_keep: float = 3.0     # nnz(floor(T_i)) ~ t_keep * |K_i|; 0 = keep all


# ---------------------------------------------------------------- geometry
def round_half_away(x):
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def trig_interp(b, sig):
    """Trigonometric interpolant of the node positions at parameters sig.

    Returns (x(sig), dx/dsig), sig = 2 pi rho / L; modes |m| < n/2 plus the
    Nyquist mode as a cosine.
    """
    n = b.n
    N = n // 2
    X = np.fft.fft(b.x, axis=0) / n
    m = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    sig = np.atleast_1d(sig)
    keep = np.abs(m) < N
    E = np.exp(1j * np.outer(sig, m[keep]))
    pos = (E @ X[keep]).real
    der = ((E * (1j * m[keep])) @ X[keep]).real
    if n % 2 == 0:
        XN = X[m == -N][0]
        pos += np.outer(np.cos(N * sig), XN.real)
        der += np.outer(-N * np.sin(N * sig), XN.real)
    return pos, der


def segment(b, omega, opt: Options):
    """List of (offset, s) for the segments P_1..P_m, ordered along the curve."""
    lam = 2 * np.pi / omega
    n, L, ds = b.n, b.L, b.ds
    m0 = 2 ** int(round(np.log2(np.sqrt(L / lam))))
    m0 = max(1, min(m0, n))
    while n % m0:
        m0 //= 2
    out = []

    def rec(off, s):
        length = s * ds
        cmax = np.max(np.abs(b.kappa[off:off + s]))
        if cmax == 0 or length <= np.sqrt(L * lam / cmax):
            out.append((off, s))
            return
        if length <= opt.m_ell * lam or s <= opt.min_pts or s % 2:
            out.append((off, s))
            return
        rec(off, s // 2)
        rec(off + s // 2, s // 2)

    s0 = n // m0
    for t in range(m0):
        rec(t * s0, s0)
    return out


def cheb_nodes(m_c):
    b = np.arange(m_c)
    return np.cos((2 * b + 1) * np.pi / (2 * m_c))


def lagrange_mean(s, m_c):
    """alpha_s(b) = (1/s) sum_a l_b(xi_a), xi_a = (a - (s-1)/2)/(s/2)."""
    xc = cheb_nodes(m_c)
    xa = (np.arange(s) - (s - 1) / 2) / (s / 2)
    I = np.ones((s, m_c))
    for bb in range(m_c):
        for c in range(m_c):
            if c != bb:
                I[:, bb] *= (xa - xc[c]) / (xc[bb] - xc[c])
    return I.mean(axis=0)


def n_dirs(s, omega, ds):
    """J for a segment of s points: ceil(s/p), p = (2 pi/omega)/ds."""
    return int(np.ceil(s * omega * ds / (2 * np.pi) - 1e-9))


def partial_fourier(s, J):
    """U(a, j) = exp(2 pi i j (a - (s-1)/2)/s), j = -J..J (eq. (12))."""
    a = np.arange(s) - (s - 1) / 2
    j = np.arange(-J, J + 1)
    return np.exp(2j * np.pi * np.outer(a, j) / s)


# ---------------------------------------------------------------- kernels
def kernel(kind, omega, eta, x, nx, y, ny):
    """CFIE kernel without the identity part, broadcast over (x, y) pairs.

    soft:  dG/dn_y - i eta G
    hard: -dG/dn_x + (1/(i eta)) d2G/dn_x dn_y
    """
    d = x - y
    r = np.linalg.norm(d, axis=-1)
    rh = d / r[..., None]
    H0, H1 = h0(omega * r), h1(omega * r)
    if kind == 0:
        return (1j * omega / 4) * H1 * np.sum(ny * rh, -1) + (eta / 4) * H0
    nxr = np.sum(nx * rh, -1)
    nyr = np.sum(ny * rh, -1)
    hyp = (1j * omega / 4) * ((omega * H0 - 2 * H1 / r) * nxr * nyr
                              + H1 * np.sum(nx * ny, -1) / r)
    return (1j * omega / 4) * H1 * nxr + hyp / (1j * eta)


def flat_block(s, n, L, omega, eta, kind):
    """B_s: the Kress-discretised operator on a straight segment of s points.

    Spacing ds = L/n, parameter speed L/(2 pi), correction table
    C_k = R_k - (2 pi/n) log(4 sin^2(pi k/n)) of the global rule.
    soft: 1/2 - i eta S_flat.
    hard: 1/2 + N_flat/(i eta), N_flat = f.p. (i omega/4) H1(omega r)/r split
          as 1/(2 pi r^2) (finite-part trapezoid: sum_{d!=0} ds/(2 pi (d ds)^2)
          - pi/(6 ds) at d = 0, plus (q_{+1} - 2 q_0 + q_{-1})/(4 pi ds)) and a
          log-singular remainder under the Kress rule.
    """
    ds = L / n
    sp = L / (2 * np.pi)
    R = kress_R(n)
    lg = log4sin2(n)
    C = R - (2 * np.pi / n) * lg
    d = np.arange(s)
    r = d * ds
    row = np.zeros(s, np.complex128)
    if kind == 0:
        z = omega * r[1:]
        H0 = h0(z)
        row[1:] = ds * (1j / 4) * H0 + C[1:s] * (-H0.real / (4 * np.pi)) * sp
        row[0] = R[0] * (-sp / (4 * np.pi)) + (2 * np.pi / n) * (
            1j / 4 - EULER_GAMMA / (2 * np.pi) - np.log(omega * sp / 2) / (2 * np.pi)) * sp
        row = -1j * eta * row
    else:
        z = omega * r[1:]
        H1 = h1(z)
        nrem = (1j * omega / 4) * H1 / r[1:] - 1 / (2 * np.pi * r[1:] ** 2)
        k1 = -(omega / (4 * np.pi)) * H1.real / r[1:] * sp
        row[1:] = ds * nrem + C[1:s] * k1 + 1 / (2 * np.pi * r[1:] ** 2) * ds
        k1_0 = -(omega ** 2 / (8 * np.pi)) * sp
        k2_0 = sp * (1j * omega ** 2 / 8
                     - (omega ** 2 / (4 * np.pi)) * (np.log(omega * sp / 2) + EULER_GAMMA - 0.5))
        row[0] = R[0] * k1_0 + (2 * np.pi / n) * k2_0 - np.pi / (6 * ds)
        row[0] += -2 / (4 * np.pi * ds)
        if s > 1:
            row[1] += 1 / (4 * np.pi * ds)
        row = row / (1j * eta)
    row[0] += 0.5
    return sla.toeplitz(row, row)


def threshold_T(T, t_keep):
    """floor(T_i): antidiagonal plus entries within 1e-8 of the k-th largest."""
    K = T.shape[0]
    if t_keep <= 0:
        return T.copy()
    k = int(min(K * K, round(t_keep * K)))
    mag = np.abs(T)
    tau = np.sort(mag.ravel())[::-1][k - 1]
    keep = mag >= tau * (1 - 1e-8)
    keep |= np.fliplr(np.eye(K, dtype=bool))
    return np.where(keep, T, 0)


# ---------------------------------------------------------------- builder
@dataclass
class Preconditioner:
    segs: list
    J: np.ndarray
    offK: np.ndarray
    NW: int
    classes: dict = field(default_factory=dict)   # s -> dict(B, Binv, U, S, T, Tt)
    E: list = field(default_factory=list)         # (i, j, ki, kj, e_ij)
    W: np.ndarray = None
    W_lu: tuple = None
    kind: int = 0


def build(b, omega, eta, kind, opt: Options = Options()):
    """Assemble every piece of Sec. 2.1-2.2 densely."""
    n, L, ds = b.n, b.L, b.ds
    segs = segment(b, omega, opt)
    m = len(segs)
    J = np.array([n_dirs(s, omega, ds) for _, s in segs])
    offK = np.concatenate([[0], np.cumsum(2 * J + 1)])
    P = Preconditioner(segs, J, offK, int(offK[-1]), kind=kind)

    # size classes (B_j, U_j, S_j, T_j depend only on s)
    for s in sorted({s for _, s in segs}):
        Js = n_dirs(s, omega, ds)
        B = flat_block(s, n, L, omega, eta, kind)
        Binv = np.linalg.inv(B)
        U = partial_fourier(s, Js)
        S = U.T @ Binv @ U
        T = np.linalg.inv(S)
        P.classes[s] = dict(B=B, Binv=Binv, U=U, S=S, T=T,
                            Tt=threshold_T(T, opt.t_keep), alpha=lagrange_mean(s, opt.m_c))

    # centres, tangents and Chebyshev grids by trigonometric interpolation
    xc = cheb_nodes(opt.m_c)
    cen, tan, gx, gn, goff = [], [], [], [], []
    for off, s in segs:
        rho_c = (off + (s - 1) / 2) * ds
        delta = xc * (s * ds / 2)
        sig = 2 * np.pi * (np.concatenate([[rho_c], rho_c + delta])) / L
        pos, der = trig_interp(b, sig)
        tvec = der / np.linalg.norm(der, axis=1)[:, None]
        nvec = np.stack([tvec[:, 1], -tvec[:, 0]], 1)
        cen.append(pos[0])
        tan.append(tvec[0])
        gx.append(pos[1:])
        gn.append(nvec[1:])
        goff.append(delta)

    # rank-1 entries e_ij (eq. (14)) for all ordered pairs i != j
    for i in range(m):
        si = segs[i][1]
        hi = 2 * np.pi / (si * ds)
        for j in range(m):
            if i == j:
                continue
            sj = segs[j][1]
            hj = 2 * np.pi / (sj * ds)
            a = cen[i] - cen[j]
            a = a / np.linalg.norm(a)
            ki = int(np.clip(round_half_away(omega * (a @ tan[i]) / hi), -J[i], J[i]))
            kj = int(np.clip(round_half_away(-omega * (a @ tan[j]) / hj), -J[j], J[j]))
            Mblk = ds * kernel(kind, omega, eta, gx[i][:, None, :], gn[i][:, None, :],
                               gx[j][None, :, :], gn[j][None, :, :])
            Mt = Mblk / np.outer(np.exp(1j * ki * hi * goff[i]), np.exp(1j * kj * hj * goff[j]))
            e = P.classes[si]["alpha"] @ Mt @ P.classes[sj]["alpha"]
            P.E.append((i, j, ki, kj, e))

    # floor(W) = E + antidiag(T)
    W = np.zeros((P.NW, P.NW), np.complex128)
    for i, (off, s) in enumerate(segs):
        T = P.classes[s]["T"]
        K = T.shape[0]
        o = offK[i]
        for r in range(K):
            W[o + r, o + K - 1 - r] += T[r, K - 1 - r]
    for (i, j, ki, kj, e) in P.E:
        W[offK[i] + ki + J[i], offK[j] + kj + J[j]] += e
    P.W = W
    P.W_lu = sla.lu_factor(W)
    return P


# ---------------------------------------------------------------- apply
def _per_seg(P, v, fn):
    out = []
    for i, (off, s) in enumerate(P.segs):
        out.append(fn(i, off, s, v))
    return out


def apply(P, f, exact=False):
    """Preconditioner: first block of eq. (19) applied to (f, 0, 0).

    y = floor(B^{-1}) f;  g = U^t y;  z = floor(T) g;  u = floor(W)^{-1} z;
    z' = floor(T) u;  h = z - z';  q = y - floor(B^{-1}) U h.
    exact=True uses T and W = E + T (eq. (18)) instead of their floors.
    """
    f = np.asarray(f, np.complex128)
    squeeze = f.ndim == 1
    F = f.reshape(f.shape[0], -1)
    Tkey = "T" if exact else "Tt"
    y = np.zeros_like(F)
    g = np.zeros((P.NW, F.shape[1]), np.complex128)
    for i, (off, s) in enumerate(P.segs):
        c = P.classes[s]
        y[off:off + s] = c["Binv"] @ F[off:off + s]
        g[P.offK[i]:P.offK[i + 1]] = c["U"].T @ y[off:off + s]
    z = np.zeros_like(g)
    for i, (off, s) in enumerate(P.segs):
        sl = slice(P.offK[i], P.offK[i + 1])
        z[sl] = P.classes[s][Tkey] @ g[sl]
    if exact:
        u = np.linalg.solve(exact_W(P), z)
    else:
        u = sla.lu_solve(P.W_lu, z)
    h = z.copy()
    q = y.copy()
    for i, (off, s) in enumerate(P.segs):
        sl = slice(P.offK[i], P.offK[i + 1])
        c = P.classes[s]
        h[sl] = z[sl] - c[Tkey] @ u[sl]
        q[off:off + s] = y[off:off + s] - c["Binv"] @ (c["U"] @ h[sl])
    return q[:, 0] if squeeze else q


def exact_W(P):
    """W = E + T with the full blocks T_i."""
    W = np.zeros((P.NW, P.NW), np.complex128)
    for i, (off, s) in enumerate(P.segs):
        sl = slice(P.offK[i], P.offK[i + 1])
        W[sl, sl] = P.classes[s]["T"]
    for (i, j, ki, kj, e) in P.E:
        W[P.offK[i] + ki + P.J[i], P.offK[j] + kj + P.J[j]] += e
    return W


def dense_pieces(P, n):
    """Dense B (block diagonal), U (block diagonal) and E of eq. (15)."""
    B = np.zeros((n, n), np.complex128)
    U = np.zeros((n, P.NW), np.complex128)
    for i, (off, s) in enumerate(P.segs):
        B[off:off + s, off:off + s] = P.classes[s]["B"]
        U[off:off + s, P.offK[i]:P.offK[i + 1]] = P.classes[s]["U"]
    E = np.zeros((P.NW, P.NW), np.complex128)
    for (i, j, ki, kj, e) in P.E:
        E[P.offK[i] + ki + P.J[i], P.offK[j] + kj + P.J[j]] += e
    return B, U, E
