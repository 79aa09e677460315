"""Mixed-precision path: the single-precision operator against the oracle,
and iterative refinement to an FP64 residual of 1e-8 with q matching the
oracle's dense solve (small n) or an exterior point-source field (full n)."""
import numpy as np
import pytest

import paper_1408_1578_amd as dp
from oracle import nystrom as ny
from synth import config_boundary, plane_wave_angles, random_density, sample_boundary, omega_for_ppw
from tests.gpu_util import empty, problem, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

# FP32 kernel values (~2e-7 relative) and FP32 products accumulated over
# source chunks: the operator is checked at 1e-5 relative (L2).
TOL32 = 1e-5


@pytest.mark.parametrize("cfg,n,nrhs", [("disk", 1024, 1), ("disk", 1024, 3), ("disk", 1024, 70),
                                        ("kite", 1024, 16), ("kite", 2048, 64), ("disk", 1000, 64)])
def test_mixed_operator(cfg, n, nrhs):
    b = sample_boundary(cfg, n)
    om = 100.0 if cfg == "disk" else omega_for_ppw(n, b.L, 10.0)
    kind = 0 if cfg == "disk" else 1
    A = ny.cfie_matrix(b, om, om, kind)
    q = random_density(n, nrhs, seed=nrhs)
    p = problem(b, om, om, kind)
    y = empty(n, nrhs)
    dp.dp_matvec_mixed(p, to_dev(q), y)
    err = relerr(to_host(y), A @ q)
    assert err < TOL32
    assert err > 1e-12      # it really is the reduced-precision operator


@pytest.mark.parametrize("kind,n", [(0, 4096), (1, 2048)])
def test_mixed_solve_small(kind, n):
    b = sample_boundary("kite", n)
    om = omega_for_ppw(n, b.L, 10.0)
    A = ny.cfie_matrix(b, om, om, kind)
    F = ny.plane_wave_rhs(b, om, plane_wave_angles(5), kind)
    Q = np.linalg.solve(A, F)
    p = problem(b, om, om, kind)
    dp.dp_precond_build(p)
    q = empty(n, 5)
    info = dp.dp_solve(p, to_dev(F), q, tol=1e-8, use_precond=True, precision=dp.DP_PREC_MIXED)
    assert info["converged"] and info["relres_max"] <= 1e-8
    assert info["refinements"] >= 2
    Qg = to_host(q)
    assert relerr(Qg, Q) < 1e-6
    # the reported residual is the FP64 one: recompute it with the oracle
    res = np.linalg.norm(F - A @ Qg, axis=0) / np.linalg.norm(F, axis=0)
    assert np.all(res < 2e-8)


def test_mixed_solve_full_size_point_source():
    # the 32768-point sound-hard kite with 64 right-hand sides, checked by a
    # property that holds at any size: data from an interior point source
    # must reproduce its exterior field
    b, om, eta, kind = config_boundary("kite", 32768)
    z0 = np.array([0.1, 0.2])
    f = ny.point_source_data(b, om, z0, kind)
    F = np.repeat(f[:, None], 64, axis=1) * np.exp(1j * np.arange(64))[None, :]
    p = problem(b, om, eta, kind)
    dp.dp_precond_build(p)
    q = empty(b.n, 64)
    info = dp.dp_solve(p, to_dev(F), q, tol=1e-8, use_precond=True, precision=dp.DP_PREC_MIXED)
    assert info["converged"] and info["relres_max"] <= 1e-8
    Q = to_host(q)
    th = np.linspace(0, 2 * np.pi, 5, endpoint=False)
    pts = np.stack([2.6 * np.cos(th), 2.6 * np.sin(th)], 1)
    ue = ny.green(om, pts, z0)
    for c in (0, 17, 63):
        u = ny.field(b, om, eta, kind, Q[:, c] * np.exp(-1j * c), pts)
        assert np.max(np.abs(u - ue)) / np.max(np.abs(ue)) < 1e-6


def test_random_star_131072_mixed_single_rhs():
    # the 131072-point seeded random star (omega = 11889, sound-soft, one
    # right-hand side): FP32 sweep, FP64 near field and residuals.  Checked by
    # a property that holds at any size: data from an interior point source
    # reproduces its exterior field; plus oracle rows of A q at sampled targets
    # for the FP64 operator on the solution
    b, om, eta, kind = config_boundary("randstar", 131072)
    z0 = np.array([0.05, -0.1])
    f = ny.point_source_data(b, om, z0, kind)
    p = problem(b, om, eta, kind)
    dp.dp_precond_build(p)
    # 320 segments coupled all-to-all: floor(W) (N_W = 26922) is factored densely on the device
    assert dp.dp_precond_get_info(p)["dense_w"] == 1
    q = empty(b.n, 1)
    info = dp.dp_solve(p, to_dev(f[:, None]), q, tol=1e-8, use_precond=True, precision=dp.DP_PREC_MIXED)
    assert info["converged"] and info["relres_max"] <= 1e-8
    Q = to_host(q)[:, 0]
    th = np.linspace(0, 2 * np.pi, 6, endpoint=False)
    pts = np.stack([1.8 * np.cos(th), 1.8 * np.sin(th)], 1)
    ue = ny.green(om, pts, z0)
    u = ny.field(b, om, eta, kind, Q, pts)
    assert np.max(np.abs(u - ue)) / np.max(np.abs(ue)) < 1e-6
    rows = np.arange(0, b.n, b.n // 12)[:12]
    lay = ny.layer_rows(b, om, rows)
    Arow = 0.5 * np.eye(b.n)[rows] + lay["D"] - 1j * eta * lay["S"]
    res = np.abs(Arow @ Q - f[rows]) / np.linalg.norm(f) * np.sqrt(b.n)
    assert np.max(res) < 1e-6


def test_star_mixed_solve_4096_vs_dense_oracle():
    # the five-petal star at n = 4096 (10 points per wavelength, sound-soft),
    # one plane wave at a seeded angle: FP32 preconditioner and single-precision
    # corrections inside FP64 refinement, against the oracle's dense solve
    b, om, eta, kind = config_boundary("star", 4096)
    ang = plane_wave_angles(1, "random", seed=0)
    A = ny.soft_matrix(b, om, eta)
    F = ny.plane_wave_rhs(b, om, ang, kind)
    Q = np.linalg.solve(A, F)
    p = problem(b, om, eta, kind)
    dp.dp_precond_build(p)
    q = empty(b.n, 1)
    info = dp.dp_solve(p, to_dev(F), q, tol=1e-8, use_precond=True, precision=dp.DP_PREC_MIXED)
    assert info["converged"] and info["relres_max"] <= 1e-8 and info["refinements"] >= 2
    Qg = to_host(q)
    assert relerr(Qg, Q) < 1e-6
    res = np.linalg.norm(F - A @ Qg) / np.linalg.norm(F)
    assert res < 2e-8


def test_star_mixed_solve_16384_sampled_oracle_rows():
    # the star at n = 16384: no dense oracle solve, so the FP64 residual
    # f - A q of the mixed solve is recomputed by the oracle at 64 sampled rows
    # (root-mean-square residual <= 1e-8 ||f||/sqrt(n) allows rows a few times
    # that; 1e-7 leaves a margin of ten)
    b, om, eta, kind = config_boundary("star", 16384)
    ang = plane_wave_angles(1, "random", seed=0)
    F = ny.plane_wave_rhs(b, om, ang, kind)
    p = problem(b, om, eta, kind)
    dp.dp_precond_build(p)
    q = empty(b.n, 1)
    info = dp.dp_solve(p, to_dev(F), q, tol=1e-8, use_precond=True, precision=dp.DP_PREC_MIXED)
    assert info["converged"] and info["relres_max"] <= 1e-8
    Qg = to_host(q)[:, 0]
    rows = np.concatenate([[0, 1, b.n - 1], np.sort(np.random.default_rng(2).choice(b.n, 61, replace=False))])
    r = ny.soft_matrix(b, om, eta, rows) @ Qg - F[rows, 0]
    rms_f = np.linalg.norm(F) / np.sqrt(b.n)
    assert np.max(np.abs(r)) < 1e-7 * rms_f, np.max(np.abs(r)) / rms_f
    # and the FP64 solver reaches the same density
    q64 = empty(b.n, 1)
    dp.dp_solve(p, to_dev(F), q64, tol=1e-8, use_precond=True)
    assert relerr(Qg, to_host(q64)[:, 0]) < 1e-6
