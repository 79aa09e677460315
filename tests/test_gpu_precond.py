"""GPU parity of the directional preconditioner (Sec. 2) against the dense
oracle reference: integer structure bit-exact, e_ij and the apply in FP64."""
import numpy as np
import pytest

import paper_1408_1578_amd as dp
from oracle import nystrom as ny, precond as pc
from oracle.gmres import gmres
from synth import config_boundary, random_density, sample_boundary, omega_for_ppw
from tests.gpu_util import empty, problem, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [("disk", 1024, 0), ("disk", 1024, 1), ("star", 4096, 0), ("kite", 4096, 1), ("kite", 2048, 0),
         ("kite", 1000, 1)]


def _setup(cfg, n, kind):
    b, om, eta, _ = config_boundary(cfg, n)
    P = pc.build(b, om, eta, kind)
    p = problem(b, om, eta, kind)
    dp.dp_precond_build(p)
    return b, om, eta, P, p


@pytest.mark.parametrize("cfg,n,kind", CASES)
def test_structure_and_entries(cfg, n, kind):
    b, om, eta, P, p = _setup(cfg, n, kind)
    off, ln, eidx, ev = dp.dp_precond_export(p)
    assert [tuple(x) for x in zip(off, ln)] == [tuple(s) for s in P.segs]
    info = dp.dp_precond_get_info(p)
    m = len(P.segs)
    assert info["m"] == m and info["NW"] == P.NW and info["nnzE"] == m * (m - 1)
    ref = {(i, j): (ki, kj, e) for i, j, ki, kj, e in P.E}
    evals = np.array([ref[(int(i), int(j))][2] for i, j, _, _ in eidx])
    for (i, j, ki, kj) in eidx:
        assert (ki, kj) == ref[(int(i), int(j))][:2]          # rounded directions: bit-exact
    assert np.max(np.abs(ev - evals)) < 1e-11 * np.max(np.abs(evals))
    assert info["nnzW"] == np.count_nonzero(P.W)


@pytest.mark.parametrize("cfg,n,kind", CASES)
def test_apply_parity(cfg, n, kind):
    b, om, eta, P, p = _setup(cfg, n, kind)
    for nrhs in (1, 5, 20):
        v = random_density(b.n, nrhs, seed=nrhs)
        z = empty(b.n, nrhs)
        dp.dp_precond_apply(p, to_dev(v), z)
        assert relerr(to_host(z), pc.apply(P, v)) < 1e-10


@pytest.mark.parametrize("gj_steps", [0, 1, 2, 3, 4, 8])
def test_apply_parity_gauss_jordan_panels(gj_steps):
    # the size-class inverses with each panel width of the batched
    # Gauss-Jordan elimination (0: automatic; 1: one launch per step; 3: a
    # ragged last panel)
    b, om, eta, _ = config_boundary("kite", 4096)
    P = pc.build(b, om, eta, 1)
    p = problem(b, om, eta, 1)
    dp.dp_precond_build(p, gj_steps=gj_steps)
    v = random_density(b.n, 5, seed=4)
    z = empty(b.n, 5)
    dp.dp_precond_apply(p, to_dev(v), z)
    assert relerr(to_host(z), pc.apply(P, v)) < 1e-10


@pytest.mark.parametrize("cfg,n,kind", [("star", 4096, 0), ("kite", 4096, 1), ("kite", 1000, 1), ("kite", 3008, 1)])
def test_preconditioned_solve(cfg, n, kind):
    b, om, eta, P, p = _setup(cfg, n, kind)
    A = ny.cfie_matrix(b, om, eta, kind)
    F = ny.plane_wave_rhs(b, om, np.array([0.0, 1.0, 2.5]), kind)
    Q = np.linalg.solve(A, F)
    q = empty(b.n, 3)
    info_p = dp.dp_solve(p, to_dev(F), q, tol=1e-8, use_precond=True)
    assert info_p["converged"] and relerr(to_host(q), Q) < 1e-6
    q2 = empty(b.n, 3)
    info_n = dp.dp_solve(p, to_dev(F), q2, tol=1e-8, use_precond=False)
    assert info_p["iters_max"] < info_n["iters_max"]
    _, its_p, _ = gmres(A, F[:, 0], tol=1e-8, M=lambda v: pc.apply(P, v))
    assert abs(int(info_p["iters"][0]) - its_p) <= 2


def test_apply_before_build_is_an_error():
    b, om, eta, kind = config_boundary("disk", 1024)
    p = problem(b, om, eta, kind)
    with pytest.raises(dp.DpError) as e:
        dp.dp_precond_apply(p, empty(b.n, 1), empty(b.n, 1))
    assert e.value.code == dp.DP_ESTATE


def test_full_size_kite_hard_apply():
    # the 32768-point sound-hard kite: apply parity against the dense reference
    b, om, eta, kind = config_boundary("kite", 32768)
    P = pc.build(b, om, eta, kind)
    p = problem(b, om, eta, kind)
    dp.dp_precond_build(p)
    v = random_density(b.n, 2, seed=9)
    z = empty(b.n, 2)
    dp.dp_precond_apply(p, to_dev(v), z)
    assert relerr(to_host(z), pc.apply(P, v)) < 1e-10
    # the FP64 apply with the bench's 64 columns
    v64 = random_density(b.n, 64, seed=10)
    ref64 = pc.apply(P, v64)
    z64 = empty(b.n, 64)
    dp.dp_precond_apply(p, to_dev(v64), z64)
    assert relerr(to_host(z64), ref64) < 1e-10
    # the single-precision apply of the correction solves with the bench's
    # 64 columns (matrix-core segment products, one wave per column in the
    # triangular solves): FP32 tables and vectors, checked at 2e-5
    z64 = empty(b.n, 64)
    dp.dp_precond_apply_mixed(p, to_dev(v64), z64)
    err = relerr(to_host(z64), ref64)
    assert 1e-12 < err < 2e-5


@pytest.mark.parametrize("cfg,n,kind", [("disk", 1024, 1), ("star", 4096, 0), ("kite", 4096, 1)])
def test_dense_w_apply_parity(cfg, n, kind):
    # floor(W) factored densely on the device (forced): same apply as the
    # oracle's dense LU, for column counts below, at and above one 64-column tile
    b, om, eta, _ = config_boundary(cfg, n)
    P = pc.build(b, om, eta, kind)
    p = problem(b, om, eta, kind)
    dp.dp_precond_build(p, w_solver=dp.W_DENSE)
    info = dp.dp_precond_get_info(p)
    assert info["dense_w"] == 1 and info["nnzLU"] == P.NW ** 2
    for nrhs in (1, 64, 70):
        v = random_density(b.n, nrhs, seed=nrhs + 3)
        z = empty(b.n, nrhs)
        dp.dp_precond_apply(p, to_dev(v), z)
        assert relerr(to_host(z), pc.apply(P, v)) < 1e-10
    # and the same as the host sparse factors
    p2 = problem(b, om, eta, kind)
    dp.dp_precond_build(p2, w_solver=dp.W_SPARSE)
    assert dp.dp_precond_get_info(p2)["dense_w"] == 0
    v = random_density(b.n, 3, seed=1)
    z1, z2 = empty(b.n, 3), empty(b.n, 3)
    dp.dp_precond_apply(p, to_dev(v), z1)
    dp.dp_precond_apply(p2, to_dev(v), z2)
    assert relerr(to_host(z1), to_host(z2)) < 1e-12


def test_random_star_32768_chooses_dense_w():
    # 173 segments couple all-to-all through E: the ordering predicts ~6e6 factor
    # entries, so floor(W) (N_W = 6829) is factored densely on the device
    b, om, eta, kind = config_boundary("randstar1", 32768)
    p = problem(b, om, eta, kind)
    dp.dp_precond_build(p)
    info = dp.dp_precond_get_info(p)
    assert info["dense_w"] == 1 and info["m"] > 100
    F = np.exp(1j * om * b.x[:, 0])[:, None] * -1.0
    q = empty(b.n, 1)
    res = dp.dp_solve(p, to_dev(F), q, tol=1e-8, use_precond=True)
    assert res["converged"] and res["relres_max"] <= 1e-8
    q2 = empty(b.n, 1)
    res2 = dp.dp_solve(p, to_dev(F), q2, tol=1e-8, use_precond=False, max_iters=400)
    assert res["iters_max"] < res2["iters_max"]
    assert relerr(to_host(q), to_host(q2)) < 1e-6


@pytest.mark.parametrize("cfg,n,kind,ws", [("disk", 1024, 1, dp.W_AUTO), ("kite", 4096, 1, dp.W_DENSE)])
def test_apply_graph_replays_match_eager(cfg, n, kind, ws):
    # the apply is replayed from a captured HIP graph from its second call on:
    # every replay, with eager work and host synchronisation in between, gives
    # the bits of the apply launched kernel by kernel
    b, om, eta, _ = config_boundary(cfg, n)
    pg = problem(b, om, eta, kind)
    dp.dp_precond_build(pg, w_solver=ws, graphs=True)
    pe = problem(b, om, eta, kind)
    dp.dp_precond_build(pe, w_solver=ws, graphs=False)
    vs = [random_density(b.n, 5, seed=s) for s in range(4)]
    refs = []
    for v in vs:
        z = empty(b.n, 5)
        dp.dp_precond_apply(pe, to_dev(v), z)
        refs.append(to_host(z))
    for rep in range(3):
        for k, v in enumerate(vs):
            z = empty(b.n, 5)
            dp.dp_precond_apply(pg, to_dev(v), z)
            assert np.array_equal(to_host(z), refs[k]), (rep, k)
            y = empty(b.n, 5)
            dp.dp_matvec(pg, to_dev(v), y)
    # another column count: captured again
    v = random_density(b.n, 2, seed=9)
    z2 = empty(b.n, 2)
    dp.dp_precond_apply(pe, to_dev(v), z2)
    for _ in range(3):
        z1 = empty(b.n, 2)
        dp.dp_precond_apply(pg, to_dev(v), z1)
        assert np.array_equal(to_host(z1), to_host(z2))


@pytest.mark.parametrize("cfg,n,kind,ws", [("disk", 1024, 0, dp.W_AUTO), ("disk", 1024, 1, dp.W_AUTO),
                                           ("star", 4096, 0, dp.W_AUTO), ("kite", 4096, 1, dp.W_AUTO),
                                           ("kite", 4096, 1, dp.W_DENSE)])
def test_single_precision_apply_parity(cfg, n, kind, ws):
    # the correction solves' preconditioner: FP32 tables and vectors
    b, om, eta, _ = config_boundary(cfg, n)
    P = pc.build(b, om, eta, kind)
    p = problem(b, om, eta, kind)
    dp.dp_precond_build(p, w_solver=ws)
    for nrhs in (1, 20):
        v = random_density(b.n, nrhs, seed=nrhs + 7)
        z = empty(b.n, nrhs)
        for _ in range(3):  # eager, captured, replayed
            dp.dp_precond_apply_mixed(p, to_dev(v), z)
            err = relerr(to_host(z), pc.apply(P, v))
            assert 1e-12 < err < 2e-5


def test_graph_recaptured_after_workspace_growth():
    # a graph keeps the workspace addresses of its capture: growing the
    # workspaces through the other precision's apply must not leave it stale
    b, om, eta, kind = config_boundary("disk", 1024)
    pg = problem(b, om, eta, 1)
    dp.dp_precond_build(pg)
    pe = problem(b, om, eta, 1)
    dp.dp_precond_build(pe, graphs=False)
    v = random_density(b.n, 5, seed=3)
    ref = empty(b.n, 5)
    dp.dp_precond_apply(pe, to_dev(v), ref)
    z = empty(b.n, 5)
    for _ in range(3):
        dp.dp_precond_apply(pg, to_dev(v), z)
    assert np.array_equal(to_host(z), to_host(ref))
    w = random_density(b.n, 70, seed=4)
    for _ in range(3):
        dp.dp_precond_apply_mixed(pg, to_dev(w), empty(b.n, 70))
    for _ in range(3):
        z = empty(b.n, 5)
        dp.dp_precond_apply(pg, to_dev(v), z)
        assert np.array_equal(to_host(z), to_host(ref))
