"""Pins of the reference directional preconditioner (Sec. 2) by identities,
closed forms, independent quadrature, least squares and structural invariants."""
import warnings

import numpy as np
import pytest
from scipy import integrate, special as sp

from oracle import nystrom as ny, precond as pc
from oracle.gmres import gmres
from synth import config_boundary, sample_boundary, omega_for_ppw


@pytest.fixture(scope="module")
def star_small():
    b = sample_boundary("star", 512)
    om = omega_for_ppw(512, b.L, 10.0)
    return b, om, pc.build(b, om, om, 0)


def test_exact_inverse_formula(star_small):
    # eq. (18) with exact B^-1, T and W = E + T equals (B + U E U^t)^{-1} f
    b, om, P = star_small
    B, U, E = pc.dense_pieces(P, b.n)
    f = np.random.default_rng(0).standard_normal(b.n) + 0j
    q = pc.apply(P, f, exact=True)
    qe = np.linalg.solve(B + U @ E @ U.T, f)
    assert np.linalg.norm(q - qe) / np.linalg.norm(qe) < 1e-10


def test_factorisation_multiplies_back(star_small):
    # eq. (17) reproduces the augmented matrix eq. (16)
    b, om, P = star_small
    B, U, E = pc.dense_pieces(P, b.n)
    n, K = b.n, P.NW
    S = U.T @ np.linalg.inv(B) @ U
    T = np.linalg.inv(S)
    W = E + T
    I_n, I_k, Z = np.eye(n), np.eye(K), np.zeros
    aug = np.block([[B, U, Z((n, K))], [U.T, Z((K, K)), I_k], [Z((K, n)), I_k, E]])
    Binv = np.linalg.inv(B)
    F1 = np.block([[I_n, Z((n, K)), Z((n, K))], [U.T @ Binv, I_k, Z((K, K))], [Z((K, n)), Z((K, K)), I_k]])
    F2 = np.block([[I_n, Z((n, K)), Z((n, K))], [Z((K, n)), I_k, Z((K, K))], [Z((K, n)), -T, I_k]])
    F3 = np.block([[B, Z((n, K)), Z((n, K))], [Z((K, n)), -S, Z((K, K))], [Z((K, n)), Z((K, K)), W]])
    F4 = np.block([[I_n, Z((n, K)), Z((n, K))], [Z((K, n)), I_k, -T], [Z((K, n)), Z((K, K)), I_k]])
    F5 = np.block([[I_n, Binv @ U, Z((n, K))], [Z((K, n)), I_k, Z((K, K))], [Z((K, n)), Z((K, K)), I_k]])
    prod = F1 @ F2 @ F3 @ F4 @ F5
    assert np.max(np.abs(prod - aug)) < 1e-9 * np.max(np.abs(aug))


def test_identity_B_gives_exchange_T():
    for s, J in ((64, 7), (256, 32), (100, 11)):
        U = pc.partial_fourier(s, J)
        T = np.linalg.inv(U.T @ U)
        X = np.fliplr(np.eye(2 * J + 1))
        assert np.max(np.abs(T - X / s)) < 1e-15


@pytest.mark.parametrize("kind", [0, 1])
def test_flat_block_symbol_and_antidiagonal(kind):
    # Fig. 2 setting: l = 5, p = 8 -> s = 256, |K| = 65
    s, n, L = 256, 8192, 1.0
    ds = L / n
    om = 2 * np.pi / (8 * ds)
    B = pc.flat_block(s, n, L, om, om, kind)
    J = pc.n_dirs(s, om, ds)
    assert 2 * J + 1 == 65
    U = pc.partial_fourier(s, J)
    T = np.linalg.inv(U.T @ np.linalg.inv(B) @ U)
    K = 2 * J + 1
    ad = T[np.arange(K), K - 1 - np.arange(K)]
    assert np.sum(np.abs(ad) ** 2) / np.sum(np.abs(T) ** 2) > 0.95
    xi = np.arange(-J, J + 1) * 2 * np.pi / (s * ds)
    sel = np.abs(xi) < 0.8 * om
    root = np.sqrt(om ** 2 - xi[sel] ** 2)
    sig = 0.5 + om / (2 * root) if kind == 0 else 0.5 + root / (2 * om)
    assert np.median(np.abs(s * ad[sel] - sig) / np.abs(sig)) < 0.02


def test_flat_soft_block_vs_quadrature():
    s, n, L = 256, 4096, 1.0
    ds = L / n
    om = 2 * np.pi / (8 * ds)
    x = np.arange(s) * ds
    xi = 0.3 * om
    wfun = lambda y: np.exp(-((y - x.mean()) / (0.3 * np.ptp(x))) ** 8)
    u = np.exp(1j * xi * x) * wfun(x)
    B = pc.flat_block(s, n, L, om, om, 0)
    a = s // 2 + 3
    xa = x[a]

    def f(y, part):
        v = (1j / 4) * sp.hankel1(0, om * abs(xa - y)) * np.exp(1j * xi * y) * wfun(y) * (-1j * om)
        return v.real if part == 0 else v.imag
    val = 0.5 * u[a]
    for part, fac in ((0, 1), (1, 1j)):
        for lo, hi in ((x[0] - ds / 2, xa), (xa, x[-1] + ds / 2)):
            val += fac * integrate.quad(f, lo, hi, args=(part,), limit=4000,
                                        epsabs=1e-13, epsrel=1e-12)[0]
    assert abs((B @ u)[a] - val) < 1e-10


def test_structure(star_small):
    b, om, P = star_small
    m = len(P.segs)
    # segments tile the boundary in order
    offs = [o for o, _ in P.segs]
    assert offs[0] == 0 and sum(s for _, s in P.segs) == b.n
    assert all(o2 == o1 + s1 for (o1, s1), (o2, _) in zip(P.segs, P.segs[1:]))
    # one rank-1 entry per ordered pair, structurally symmetric pattern
    assert len(P.E) == m * (m - 1)
    idx = {(i, j): (ki, kj) for i, j, ki, kj, _ in P.E}
    for (i, j), (ki, kj) in idx.items():
        assert idx[(j, i)] == (kj, ki)
    # nnz(floor(W)) = N_W + m(m-1)
    assert np.count_nonzero(P.W) == P.NW + m * (m - 1)


def test_lagrange_mean_exact_on_polynomials():
    s, mc = 128, 10
    al = pc.lagrange_mean(s, mc)
    xc = pc.cheb_nodes(mc)
    xa = (np.arange(s) - (s - 1) / 2) / (s / 2)
    for d in range(mc):
        assert abs(al @ xc ** d - np.mean(xa ** d)) < 1e-13


def test_trig_interp_on_disk():
    b = sample_boundary("disk", 64)
    sig = np.array([0.1, 1.3, 2.9, 6.0])
    pos, der = pc.trig_interp(b, sig)
    assert np.max(np.abs(pos - np.stack([np.cos(sig), np.sin(sig)], 1))) < 1e-14
    assert np.max(np.abs(der - np.stack([-np.sin(sig), np.cos(sig)], 1))) < 1e-13


@pytest.mark.parametrize("kind", [0, 1])
def test_preconditioner_reduces_iterations(kind):
    b, om, eta, _ = config_boundary("disk")
    A = ny.cfie_matrix(b, om, eta, kind)
    f = ny.plane_wave_rhs(b, om, 0.0, kind)[:, 0]
    P = pc.build(b, om, eta, kind)
    _, nn, _ = gmres(A, f, tol=1e-8)
    x, npc, _ = gmres(A, f, tol=1e-8, M=lambda v: pc.apply(P, v))
    assert npc < nn
    assert np.linalg.norm(A @ x - f) / np.linalg.norm(f) < 1e-8


# ---------------------------------------------------------------- kernels and e_ij
@pytest.mark.parametrize("kind", [0, 1])
def test_kernel_vs_finite_differences(kind):
    # Sec. 1: G(x, y) = (i/4) H0(omega |x - y|); soft kernel dG/dn_y - i eta G,
    # hard kernel -dG/dn_x + (1/(i eta)) d2G/dn_x dn_y, here by central
    # differences of G itself (omega h = 1e-3: truncation ~ 2e-7 relative)
    rng = np.random.default_rng(3)
    om, eta = 40.0, 55.0
    G = lambda x, y: (1j / 4) * sp.hankel1(0, om * np.linalg.norm(x - y))
    h = 1e-3 / om
    for _ in range(6):
        x, y = rng.uniform(-1, 1, 2), rng.uniform(-1, 1, 2)
        if np.linalg.norm(x - y) < 0.2:
            continue
        ax, ay = rng.uniform(0, 2 * np.pi, 2)
        nx, ny_ = np.array([np.cos(ax), np.sin(ax)]), np.array([np.cos(ay), np.sin(ay)])
        dGy = (G(x, y + h * ny_) - G(x, y - h * ny_)) / (2 * h)
        dGx = (G(x + h * nx, y) - G(x - h * nx, y)) / (2 * h)
        d2 = (G(x + h * nx, y + h * ny_) - G(x + h * nx, y - h * ny_)
              - G(x - h * nx, y + h * ny_) + G(x - h * nx, y - h * ny_)) / (4 * h * h)
        want = dGy - 1j * eta * G(x, y) if kind == 0 else -dGx + d2 / (1j * eta)
        got = pc.kernel(kind, om, eta, x, nx, y, ny_)
        assert abs(got - want) < 1e-5 * abs(want), (got, want)


def _separated_pairs(b, P, factor=3.0):
    """Ordered segment pairs whose node sets are at least factor x (larger length) apart."""
    out = []
    for (i, j, ki, kj, e) in P.E:
        oi, si = P.segs[i]
        oj, sj = P.segs[j]
        xi, xj = b.x[oi:oi + si], b.x[oj:oj + sj]
        dmin = np.min(np.linalg.norm(xi[:, None] - xj[None], axis=-1))
        if dmin >= factor * max(si, sj) * b.ds:
            out.append((i, j, ki, kj, e))
    return out


@pytest.mark.parametrize("kind", [0, 1])
def test_eij_is_the_rank1_least_squares_coefficient(kind):
    # eq. (13)-(14): M_ij ~ U_i(:, k^i) e_ij U_j(:, k^j)^t with e_ij the
    # w^dagger-weighted (least-squares) constant of the non-oscillatory part,
    # interpolated from the Chebyshev grids R_i x R_j.  Independent of the
    # oracle's interpolation: the least-squares coefficient of the rank-1
    # pattern U_i(:, k^i) U_j(:, k^j)^t fitted to the kernel block at the
    # nodes themselves.  The Chebyshev value must agree to interpolation
    # accuracy (m_c = 10 points of a function with under a quarter turn of
    # residual phase per segment).
    b = sample_boundary("kite", 2048)
    om = omega_for_ppw(2048, b.L, 10.0)
    P = pc.build(b, om, om, kind)
    pairs = _separated_pairs(b, P)
    assert len(pairs) > 100
    rel, fit = [], []
    for (i, j, ki, kj, e) in pairs:
        oi, si = P.segs[i]
        oj, sj = P.segs[j]
        M = b.ds * pc.kernel(kind, om, om, b.x[oi:oi + si][:, None], b.nu[oi:oi + si][:, None],
                             b.x[oj:oj + sj][None], b.nu[oj:oj + sj][None])
        R1 = np.outer(P.classes[si]["U"][:, ki + P.J[i]], P.classes[sj]["U"][:, kj + P.J[j]])
        estar = np.linalg.lstsq(R1.reshape(-1, 1), M.ravel(), rcond=None)[0][0]
        rel.append(abs(e - estar) / abs(estar))
        fit.append(np.linalg.norm(M - e * R1) / np.linalg.norm(M))
    rel = np.array(rel)
    assert np.median(rel) < 1e-4 and rel.max() < 2e-2, (np.median(rel), rel.max())
    # the rank-1 term removes part of every separated block
    assert max(fit) < 1.0


@pytest.mark.parametrize("kind", [0, 1])
def test_direction_indices_pick_the_dominant_plane_wave(kind):
    # Sec. 2.1: k^i_ij is the grid direction of K_i nearest to the direction
    # a_ij between the segment centres.  Independent of that rounding: over all
    # grid pairs (k, k'), the projection |U_i(:, k)^H M_ij conj(U_j(:, k'))| of
    # the kernel block is largest at the chosen pair for most separated pairs
    # and within one grid step for nearly all of them (floor instead of
    # rounding drops the first fraction to about 0.2)
    b = sample_boundary("kite", 2048)
    om = omega_for_ppw(2048, b.L, 10.0)
    P = pc.build(b, om, om, kind)
    exact = near = 0
    pairs = _separated_pairs(b, P)
    for (i, j, ki, kj, e) in pairs:
        oi, si = P.segs[i]
        oj, sj = P.segs[j]
        M = b.ds * pc.kernel(kind, om, om, b.x[oi:oi + si][:, None], b.nu[oi:oi + si][:, None],
                             b.x[oj:oj + sj][None], b.nu[oj:oj + sj][None])
        proj = np.abs(P.classes[si]["U"].conj().T @ M @ P.classes[sj]["U"].conj())
        bi, bj = np.unravel_index(np.argmax(proj), proj.shape)
        di, dj = bi - P.J[i] - ki, bj - P.J[j] - kj
        exact += di == 0 and dj == 0
        near += abs(di) <= 1 and abs(dj) <= 1
    assert exact / len(pairs) > 0.5 and near / len(pairs) > 0.9, (exact, near, len(pairs))


def test_hard_flat_block_vs_quadrature():
    # B_s for the sound-hard CFIE on a straight segment: 1/2 + N_flat/(i eta).
    # On a line, Maue's identity gives N u(x) = int G(x - y) (u'' + omega^2 u)(y) dy
    # (u compactly supported), computed here by adaptive quadrature.  The
    # finite-part trapezoid with the second-difference term is exact up to the
    # remainder of that difference, h^3 u''''/(48 pi) per unit of 1/(i eta):
    # the raw error must be of that size and vanish to 1e-6 once it is removed.
    s, n, L = 256, 4096, 1.0
    ds = L / n
    om = 2 * np.pi / (8 * ds)
    x = np.arange(s) * ds
    c, sg, xi = x.mean(), 0.3 * np.ptp(x), 0.3 * om
    w = lambda y: np.exp(-((y - c) / sg) ** 8)
    w1 = lambda y: -8 * ((y - c) / sg) ** 7 / sg * w(y)
    w2 = lambda y: (64 * ((y - c) / sg) ** 14 - 56 * ((y - c) / sg) ** 6) / sg ** 2 * w(y)
    u = lambda y: np.exp(1j * xi * y) * w(y)
    upp = lambda y: np.exp(1j * xi * y) * (w2(y) + 2j * xi * w1(y) - xi ** 2 * w(y))
    B = pc.flat_block(s, n, L, om, om, 1)
    Bu = B @ u(x)
    for a in (s // 2 + 3, s // 2 - 17):
        xa = x[a]

        def f(y, part):
            v = (1j / 4) * sp.hankel1(0, om * abs(xa - y)) * (upp(y) + om ** 2 * u(y))
            return v.real if part == 0 else v.imag
        Nu = 0
        with warnings.catch_warnings():
            warnings.simplefilter("error", integrate.IntegrationWarning)
            for part, fac in ((0, 1), (1, 1j)):
                for lo, hi in ((x[0] - ds / 2, xa), (xa, x[-1] + ds / 2)):
                    Nu += fac * integrate.quad(f, lo, hi, args=(part,), limit=4000,
                                               epsabs=1e-13, epsrel=1e-12)[0]
        want = 0.5 * u(xa) + Nu / (1j * om)
        lead = ds ** 3 * xi ** 4 * u(xa) / (48 * np.pi * 1j * om)
        assert abs(Bu[a] - want) < 1e-4 * abs(want)
        assert abs(Bu[a] - want - lead) < 1e-6 * abs(want), (abs(Bu[a] - want), abs(lead))


# ---------------------------------------------------------------- floor(T_i)
def test_threshold_T_hand_counted():
    # Sec. 2.2: floor(T_i) keeps ~t_keep |K_i| largest entries (ties together)
    # and always the antidiagonal; masks below counted by hand
    T = np.array([[9, 1, 5], [2, 8, 3], [7, 4, 6]], dtype=np.complex128)
    keep1 = np.array([[1, 0, 1], [0, 1, 0], [1, 0, 0]], bool)      # 3 largest: 9 8 7
    keep2 = np.array([[1, 0, 1], [0, 1, 0], [1, 1, 1]], bool)      # 6 largest: 9 8 7 6 5 4
    assert np.array_equal(pc.threshold_T(T, 1.0) != 0, keep1)
    assert np.array_equal(pc.threshold_T(T, 2.0) != 0, keep2)
    assert np.array_equal(pc.threshold_T(T, 0.0), T)
    # equal moduli at the threshold stay together: 2 largest of {4, 4i, -4, 1}
    Tt = np.array([[4, 4j], [-4, 1]], dtype=np.complex128)
    assert np.array_equal(pc.threshold_T(Tt, 1.0) != 0, np.array([[1, 1], [1, 0]], bool))
    # kept values are the original entries
    assert np.array_equal(pc.threshold_T(T, 1.0)[keep1], T[keep1])


def test_threshold_T_keeps_the_largest(star_small):
    b, om, P = star_small
    for s, c in P.classes.items():
        T, Tt = c["T"], c["Tt"]
        K = T.shape[0]
        k = int(round(3.0 * K))
        anti = np.fliplr(np.eye(K, dtype=bool))
        kept = Tt != 0
        assert kept[anti].all()
        mag = np.abs(T)
        # the k largest moduli are all kept ...
        assert kept.ravel()[np.argsort(-mag.ravel(), kind="stable")[:k]].all()
        # ... and nothing dropped exceeds a kept entry off the antidiagonal
        if (~kept).any():
            assert mag[~kept].max() <= mag[kept & ~anti].min()


# ---------------------------------------------------------------- segmentation
def _stops(b, omega, off, s, opt=pc.Options()):
    """Which stop rules of Sec. 2.1 a segment meets (almost planar; short; tiny/odd)."""
    lam = 2 * np.pi / omega
    length = s * b.ds
    cmax = np.max(np.abs(b.kappa[off:off + s]))
    planar = cmax == 0 or length <= np.sqrt(b.L * lam / cmax)
    return planar or length <= opt.m_ell * lam or s <= opt.min_pts or s % 2 == 1


def test_segmentation_disk_by_hand():
    # unit disk, omega = 100 (lambda = 0.0628): 2^round(log2 sqrt(100)) = 8 initial
    # segments of 128 points (length 0.785 > sqrt(L lambda) = 0.628, > 4 lambda),
    # bisected once to 16 almost-planar segments of 64 points (length 0.393)
    b = sample_boundary("disk", 1024)
    segs = pc.segment(b, 100.0, pc.Options())
    assert segs == [(64 * k, 64) for k in range(16)]


@pytest.mark.parametrize("name,n", [("kite", 4096), ("star", 4096), ("randstar0", 8192)])
def test_segmentation_leaves_minimal(name, n):
    # every leaf meets a stop rule, and the segment it was bisected from met none
    b = sample_boundary(name, n)
    om = omega_for_ppw(n, b.L, 10.0)
    segs = pc.segment(b, om, pc.Options())
    lam = 2 * np.pi / om
    m0 = 2 ** int(round(np.log2(np.sqrt(b.L / lam))))
    s0 = n // m0
    assert sum(s for _, s in segs) == n
    for off, s in segs:
        assert _stops(b, om, off, s), (off, s)
        if s < s0:
            poff = off - off % (2 * s)
            assert not _stops(b, om, poff, 2 * s), (off, s)
