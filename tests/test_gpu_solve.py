"""GPU GMRES solves against the oracle's dense direct solve.  q parity bar:
relative L2 1e-6 (FP64 path) with GMRES tolerance 1e-8 and cond(A) < 100."""
import numpy as np
import pytest

import paper_1408_1578_amd as dp
from oracle import disk, nystrom as ny
from oracle.gmres import gmres
from synth import config_boundary, plane_wave_angles, sample_boundary, omega_for_ppw
from tests.gpu_util import empty, problem, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", [0, 1])
def test_disk_solve_vs_series(kind):
    b, om, eta, _ = config_boundary("disk", 1024)
    p = problem(b, om, eta, kind)
    f = empty(b.n, 1)
    dp.dp_rhs_plane_wave(p, np.array([0.0]), f)
    q = empty(b.n, 1)
    info = dp.dp_solve(p, f, q, tol=1e-10)
    assert info["converged"]
    theta = 2 * np.pi * np.arange(b.n) / b.n
    qe = disk.density(theta, om, eta, kind)
    assert relerr(to_host(q)[:, 0], qe) < 1e-8


@pytest.mark.parametrize("kind,n", [(0, 2048), (1, 1024)])
def test_kite_solve_multi_rhs(kind, n):
    b = sample_boundary("kite", n)
    om = omega_for_ppw(n, b.L, 10.0)
    ang = plane_wave_angles(5)
    A = ny.cfie_matrix(b, om, om, kind)
    F = ny.plane_wave_rhs(b, om, ang, kind)
    Q = np.linalg.solve(A, F)
    p = problem(b, om, om, kind)
    f = to_dev(F)
    q = empty(n, 5)
    info = dp.dp_solve(p, f, q, tol=1e-8)
    assert info["converged"] and info["relres_max"] <= 1e-8
    assert relerr(to_host(q), Q) < 1e-6
    # iteration counts agree with the oracle's textbook GMRES
    _, its, _ = gmres(A, F[:, 0], tol=1e-8)
    assert abs(int(info["iters"][0]) - its) <= 2


def test_solve_restart_and_nonconvergence():
    b, om, eta, kind = config_boundary("disk", 1024)
    p = problem(b, om, eta, kind)
    f = empty(b.n, 1)
    dp.dp_rhs_plane_wave(p, np.array([0.0]), f)
    q = empty(b.n, 1)
    info = dp.dp_solve(p, f, q, tol=1e-10, restart=5)
    assert info["converged"]
    info = dp.dp_solve(p, f, q, tol=1e-10, max_iters=2)
    assert not info["converged"] and info["iters_max"] == 2


def test_zero_rhs_column():
    b, om, eta, kind = config_boundary("disk", 1024)
    p = problem(b, om, eta, kind)
    F = np.zeros((b.n, 2), complex)
    F[:, 1] = ny.plane_wave_rhs(b, om, 0.0, kind)[:, 0]
    q = empty(b.n, 2)
    info = dp.dp_solve(p, to_dev(F), q, tol=1e-8)
    assert info["converged"]
    assert np.all(to_host(q)[:, 0] == 0)


@pytest.mark.parametrize("precision", [dp.DP_PREC_FP64, dp.DP_PREC_MIXED])
def test_repeated_solves_reuse_workspaces(precision):
    # the GMRES and refinement workspaces stay with the problem between
    # solves: a solve after others with different column counts and restart
    # lengths reproduces a solve on a fresh problem bit for bit
    b = sample_boundary("kite", 1024)
    om = omega_for_ppw(b.n, b.L, 10.0)
    ang = plane_wave_angles(4)

    def solve(p, cols, restart):
        f, q = empty(b.n, len(cols)), empty(b.n, len(cols))
        dp.dp_rhs_plane_wave(p, ang[cols], f)
        info = dp.dp_solve(p, f, q, tol=1e-9, restart=restart, use_precond=True, precision=precision)
        assert info["converged"]
        return to_host(q)

    fresh = problem(b, om, om, 1)
    dp.dp_precond_build(fresh)
    ref = solve(fresh, [0, 1, 2, 3], 40)
    fresh.close()
    p = problem(b, om, om, 1)
    dp.dp_precond_build(p)
    solve(p, [3], 80)
    solve(p, [0, 2], 10)
    dp.dp_precond_build(p)  # the rebuild takes over the previous buffers
    assert np.array_equal(solve(p, [0, 1, 2, 3], 40), ref)
    p.close()
