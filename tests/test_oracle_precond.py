"""Pins of the reference directional preconditioner (Sec. 2) by identities,
closed forms and structural invariants."""
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
