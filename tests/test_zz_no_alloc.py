"""The preconditioner apply that allocates nothing (dp_precond_apply_noalloc):
through the C-ABI, against dp_precond_apply (same kernels: identical bits)
and the dense oracle reference (Sec. 2.2 eq. (19)), on consecutive calls
with fewer columns and on a smaller problem after a larger one, for sparse
and dense floor(W); sizes beyond the device scratch array are refused."""
import numpy as np
import pytest

import paper_1408_1578_amd as dp
from oracle import precond as pc
from synth import config_boundary, random_density
from tests.gpu_util import empty, problem, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu


def _pair(cfg, n, kind, w_solver):
    b, om, eta, _ = config_boundary(cfg, n)
    P = pc.build(b, om, eta, kind)
    p = problem(b, om, eta, kind)
    dp.dp_precond_build(p, w_solver=w_solver)
    return b, P, p


@pytest.mark.parametrize("w_solver", [dp.W_SPARSE, dp.W_DENSE])
def test_noalloc_apply_matches_apply(w_solver):
    big = _pair("kite", 4096, 1, w_solver)
    small = _pair("disk", 1024, 0, w_solver)
    for (b, P, p), nrhs in ((big, 20), (big, 5), (small, 3), (big, 64)):
        v = random_density(b.n, nrhs, seed=nrhs)
        z_ref = empty(b.n, nrhs)
        dp.dp_precond_apply(p, to_dev(v), z_ref)
        z = empty(b.n, nrhs)
        dp.dp_precond_apply_noalloc(p, to_dev(v), z)
        assert np.array_equal(to_host(z), to_host(z_ref)), (b.name, nrhs)
        assert relerr(to_host(z), pc.apply(P, v)) < 1e-10


def test_noalloc_apply_refuses_oversize():
    b, om, eta, kind = config_boundary("kite", 32768)
    p = problem(b, om, eta, kind)
    dp.dp_precond_build(p)
    nw = dp.dp_precond_get_info(p)["NW"]
    per_col = 16 * (2 * b.n + 4 * nw)
    nrhs = (128 << 20) // per_col + 1          # one column more than fits
    v = to_dev(random_density(b.n, nrhs, seed=1))
    z = empty(b.n, nrhs)
    with pytest.raises(dp.DpError) as e:
        dp.dp_precond_apply_noalloc(p, v, z)
    assert e.value.code == dp.DP_EINVAL and "scratch" in str(e.value)
    assert np.all(to_host(z) == 0)
    # the largest column count that fits runs, and matches the regular apply
    nrhs -= 1
    v = to_dev(random_density(b.n, nrhs, seed=2))
    z, z_ref = empty(b.n, nrhs), empty(b.n, nrhs)
    dp.dp_precond_apply_noalloc(p, v, z)
    dp.dp_precond_apply(p, v, z_ref)
    assert np.array_equal(to_host(z), to_host(z_ref))
