"""GPU parity of the HIP Nystrom matvec against the CPU oracle.

Tolerance: the kernels are FP64; each pair's value carries the rounding of
z = omega r (relative ~ z eps) on top of ~1e-15 from the Hankel evaluation,
so a matvec over n pairs per row is checked at 1e-11 relative (L2) for
z_max <= 1e4 (tight enough that any formula slip fails by orders of
magnitude)."""
import numpy as np
import pytest
from scipy import special as sps

import paper_1408_1578_amd as dp
from oracle import disk, nystrom as ny
from synth import config_boundary, random_density, sample_boundary, omega_for_ppw
from tests.gpu_util import ctx, empty, problem, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu
TOL = 1e-11


def test_hankel_device_vs_scipy():
    import torch
    from scipy import special as sp
    z = np.concatenate([np.geomspace(1e-3, 3e4, 4000), np.linspace(24.0, 26.0, 401)])
    zt = torch.from_numpy(z).to("cuda:0")
    out = torch.zeros(4 * z.size, dtype=torch.float64, device="cuda:0")
    dp.dp_hankel_dev(ctx(), zt, out)
    o = out.cpu().numpy().reshape(-1, 4)
    tol = np.maximum(3e-15, 4 * z * 1.1e-16) + 2e-15
    for nu, (re, im) in ((0, (0, 1)), (1, (2, 3))):
        ref = sp.hankel1(nu, z)
        err = np.abs(o[:, re] + 1j * o[:, im] - ref) / np.abs(ref)
        assert np.all(err < tol), (nu, err.max(), z[np.argmax(err / tol)])


@pytest.mark.parametrize("nrhs", [1, 3, 8, 70])
def test_soft_disk_matvec(nrhs):
    b, om, eta, kind = config_boundary("disk", 1024)
    A = ny.cfie_matrix(b, om, eta, kind)
    q = random_density(b.n, nrhs, seed=nrhs)
    p = problem(b, om, eta, kind)
    y = empty(b.n, nrhs)
    dp.dp_matvec(p, to_dev(q), y)
    assert relerr(to_host(y), A @ q) < TOL


@pytest.mark.parametrize("n", [1000, 1536])
def test_soft_star_ragged_matvec(n):
    # n not a multiple of the 256-row / 64-row tiles
    b = sample_boundary("star", n)
    om = omega_for_ppw(n, b.L, 10.0)
    A = ny.soft_matrix(b, om, om)
    q = random_density(n, 2, seed=5)
    p = problem(b, om, om, 0)
    y = empty(n, 2)
    dp.dp_matvec(p, to_dev(q), y)
    assert relerr(to_host(y), A @ q) < TOL


@pytest.mark.parametrize("n,nrhs", [(1024, 1), (1024, 16), (1000, 3), (1536, 64)])
def test_hard_kite_matvec(n, nrhs):
    # n = 1000, 1536: the spectral derivative of Maue's form by Bluestein's DFT
    b = sample_boundary("kite", n)
    om = omega_for_ppw(n, b.L, 10.0)
    A = ny.hard_matrix(b, om, om)
    q = random_density(b.n, nrhs, seed=7)
    p = problem(b, om, om, 1)
    y = empty(b.n, nrhs)
    dp.dp_matvec(p, to_dev(q), y)
    assert relerr(to_host(y), A @ q) < TOL


# Pairs with omega r < 25 take the small-argument Hankel branch in a separate
# near-field pass.  omega = 3 on the unit disk puts every pair there (a dense,
# unbanded near list); omega = 30 puts about a quarter of them there; the
# kite at 40 points per wavelength has long near bands in every row.
@pytest.mark.parametrize("kind,omega,nrhs", [(0, 3.0, 1), (1, 3.0, 70), (0, 30.0, 64), (1, 30.0, 5)])
def test_near_field_heavy_disk(kind, omega, nrhs):
    b = sample_boundary("disk", 512)
    A = ny.cfie_matrix(b, omega, omega, kind)
    q = random_density(b.n, nrhs, seed=13)
    p = problem(b, omega, omega, kind)
    y = empty(b.n, nrhs)
    dp.dp_matvec(p, to_dev(q), y)
    assert relerr(to_host(y), A @ q) < TOL


@pytest.mark.parametrize("nrhs", [2, 32, 64])
def test_near_field_dense_bands_kite(nrhs):
    b = sample_boundary("kite", 2048)
    om = omega_for_ppw(2048, b.L, 40.0)
    A = ny.hard_matrix(b, om, om)
    q = random_density(b.n, nrhs, seed=17)
    p = problem(b, om, om, 1)
    y = empty(b.n, nrhs)
    dp.dp_matvec(p, to_dev(q), y)
    assert relerr(to_host(y), A @ q) < TOL
    y32 = empty(b.n, nrhs)
    dp.dp_matvec_mixed(p, to_dev(q), y32)
    assert relerr(to_host(y32), A @ q) < 1e-5


# At 10 points per wavelength every near pair of an evenly sampled smooth
# curve lies within about 25/(omega h) = 40 rows of its target: the
# 64-column apply then stages each block's band of source densities in LDS
# (at 40 points per wavelength, above, the band is too wide and the entry
# list is used).  Soft and hard, FP64 and single-precision densities.
@pytest.mark.parametrize("kind", [0, 1])
def test_near_field_band_64_columns(kind):
    b = sample_boundary("kite", 4096)
    om = omega_for_ppw(4096, b.L, 10.0)
    A = ny.cfie_matrix(b, om, om, kind)
    q = random_density(b.n, 64, seed=19)
    p = problem(b, om, om, kind)
    y = empty(b.n, 64)
    dp.dp_matvec(p, to_dev(q), y)
    ref = A @ q
    assert relerr(to_host(y), ref) < TOL
    y32 = empty(b.n, 64)
    dp.dp_matvec_mixed(p, to_dev(q), y32)
    assert relerr(to_host(y32), ref) < 1e-5


@pytest.mark.parametrize("op,name", [(dp.DP_OP_S, "S"), (dp.DP_OP_D, "D"), (dp.DP_OP_DP, "Dp")])
def test_layers(op, name):
    b = sample_boundary("randstar2", 1000)
    om = omega_for_ppw(1000, b.L, 10.0)
    lay = ny.layer_rows(b, om)
    q = random_density(b.n, 3, seed=11)
    p = problem(b, om, om, 0)
    y = empty(b.n, 3)
    dp.dp_layer_apply(p, op, to_dev(q), y)
    assert relerr(to_host(y), lay[name] @ q) < TOL


# n > 4096 takes the four-step path with n = n1 n2: 8192 = 128 x 64,
# 32768 = 256 x 128, 65536 = 256 x 256.  Other even n go through Bluestein's
# chirp-z DFT with power-of-two FFTs of length M >= 2n - 1 (1000: 2048 in LDS,
# 3008: 8192, 64 * 1021 = 65344: 131072).  The Nyquist mode n/2 is dropped.
@pytest.mark.parametrize("n", [64, 4096, 8192, 32768, 65536, 1000, 3008, 64 * 1021])
def test_spectral_derivative(n):
    b = sample_boundary("disk", n)
    t = 2 * np.pi * np.arange(n) / n
    m = np.array([1, 7, -3, n // 2 - 1, n // 2])
    q = np.stack([np.exp(1j * mm * t) for mm in m], 1)
    om = max(10.0, n / 16)  # D_s does not depend on omega; this keeps the near list small
    p = problem(b, om, om, 1)
    y = empty(n, len(m))
    dp.dp_layer_apply(p, dp.DP_OP_DS, to_dev(q), y)
    mult = np.where(m == n // 2, 0, m)
    ref = q * (1j * mult)[None, :] / b.speed[:, None]
    # inputs at mode n/2 - 1 carry rounding ~ m t eps; allow eps * n * log2(n)
    assert relerr(to_host(y), ref) < max(1e-12, 1.1e-16 * n * np.log2(n))
    if n <= 4096:
        Ds = ny.arclength_derivative_matrix(b)
        q2 = random_density(n, 2, seed=3)
        y2 = empty(n, 2)
        dp.dp_layer_apply(p, dp.DP_OP_DS, to_dev(q2), y2)
        assert relerr(to_host(y2), Ds @ q2) < 1e-12


@pytest.mark.parametrize("kind", [0, 1])
def test_plane_wave_rhs(kind):
    b = sample_boundary("kite", 512)
    om = 77.0
    ang = np.array([0.0, 0.3, 2.0, 5.5])
    p = problem(b, om, om, kind)
    f = empty(b.n, 4)
    dp.dp_rhs_plane_wave(p, ang, f)
    assert relerr(to_host(f), ny.plane_wave_rhs(b, om, ang, kind)) < 1e-12


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("prec", [dp.DP_PREC_FP64, dp.DP_PREC_MIXED])
def test_disk_eigenfunctions_large_n(kind, prec):
    # property at the full size and column count of the bench: the equispaced
    # disk matrix is circulant with the closed-form symbols of Sec. 1 (Graf's
    # addition theorem), so A applied to 64 Fourier modes at n = 32768 runs the
    # 64-column matrix-core sweeps (FP64, and the single-precision one) with
    # their full source chunking.  The discrete symbols match the closed forms
    # to 3e-12 for |m| <= 4500 (omega = 3277)
    n = 32768
    b = sample_boundary("disk", n)
    om = omega_for_ppw(n, b.L, 10.0)
    t = 2 * np.pi * np.arange(n) / n
    rng = np.random.default_rng(kind)
    m = np.concatenate([[0, 1, -1, 5, 1000, -2000, 3000, -4500], rng.integers(-4500, 4501, 56)])
    q = np.stack([np.exp(1j * mm * t) for mm in m], 1)
    p = problem(b, om, om, kind)
    y = empty(n, len(m))
    (dp.dp_matvec if prec == dp.DP_PREC_FP64 else dp.dp_matvec_mixed)(p, to_dev(q), y)
    lam = disk.cfie_eigs(m, om, om, kind)
    err = np.abs(to_host(y) - q * lam[None, :]).max(0)
    if prec == dp.DP_PREC_FP64:
        assert np.all(err < 1e-10 * np.abs(lam)), (err / np.abs(lam)).max()
        return
    # single precision: the error of a row sum is relative to the sum of the
    # moduli of its terms, not to the result.  With c = sum_j |S_0j| those
    # are eta c (soft: S-part) and (m^2 + omega^2) c / eta (hard, Maue: the
    # S-sweeps of D_s q and omega^2 nu q), which near |m| = omega exceed
    # |lambda_m| 10-30x; measured errors stay below 1e-6 of that scale
    j = np.arange(1, n)
    c = np.sum(np.abs(sps.hankel1(0, om * 2 * np.sin(np.pi * j / n)))) / 4 * b.ds
    if kind == 0:
        scale = np.abs(lam) + om * c
    else:
        scale = np.abs(lam) + (m.astype(float) ** 2 + om ** 2) * c / om
    assert np.all(err < 2e-6 * scale), (err / scale).max()
    # typical mode: ~6e-7 |lambda_m| soft, ~5e-6 hard (D_s multiplies by |m|
    # twice around the S-sweep)
    assert np.median(err / np.abs(lam)) < (3e-6 if kind == 0 else 1e-5), np.median(err / np.abs(lam))
    assert (err / np.abs(lam)).max() > 1e-12      # it really is the single-precision operator


def test_soft_star_sampled_rows_16384():
    n = 16384
    b = sample_boundary("star", n)
    om = omega_for_ppw(n, b.L, 10.0)
    rows = np.sort(np.random.default_rng(0).choice(n, 48, replace=False))
    rows = np.concatenate([[0, 1, n - 1], rows])
    A = ny.soft_matrix(b, om, om, rows)
    q = random_density(n, 1, seed=1)
    p = problem(b, om, om, 0)
    y = empty(n, 1)
    dp.dp_matvec(p, to_dev(q), y)
    assert relerr(to_host(y)[rows], A @ q) < TOL


@pytest.mark.parametrize("nrhs", [2, 64])
def test_hard_layers_sampled_rows_32768(nrhs):
    # the full-size sound-hard workload: S and D' rows against the oracle, with
    # 2 columns (one row per lane) and the bench's 64 (matrix-core sweep)
    b, om, eta, kind = config_boundary("kite", 32768)
    rng = np.random.default_rng(1)
    rows = np.concatenate([[0, 5, 32767], rng.choice(32768, 13 if nrhs == 2 else 29, replace=False)])
    lay = ny.layer_rows(b, om, rows)
    q = random_density(b.n, nrhs, seed=2)
    p = problem(b, om, eta, kind)
    for op, name in ((dp.DP_OP_S, "S"), (dp.DP_OP_DP, "Dp")):
        y = empty(b.n, nrhs)
        dp.dp_layer_apply(p, op, to_dev(q), y)
        assert relerr(to_host(y)[rows], lay[name] @ q) < 5 * TOL


@pytest.mark.parametrize("kind,nrhs,prec", [(1, 16, 0), (1, 64, 1), (0, 3, 0), (0, 8, 0)])
def test_autotune_keeps_parity_and_determinism(kind, nrhs, prec):
    b = sample_boundary("kite", 2048)
    om = omega_for_ppw(2048, b.L, 10.0)
    A = ny.cfie_matrix(b, om, om, kind)
    q = random_density(b.n, nrhs, seed=21)
    p = problem(b, om, om, kind)
    info = dp.dp_autotune(p, nrhs, prec)
    assert info["candidates"] >= 4 and 0 < info["t_best_ms"] <= info["t_default_ms"]
    mv = dp.dp_matvec if prec == 0 else dp.dp_matvec_mixed
    y1, y2 = empty(b.n, nrhs), empty(b.n, nrhs)
    mv(p, to_dev(q), y1)
    mv(p, to_dev(q), y2)
    assert np.array_equal(to_host(y1), to_host(y2))
    assert relerr(to_host(y1), A @ q) < (1e-11 if prec == 0 else 1e-5)
