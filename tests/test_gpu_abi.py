"""C-ABI argument checks that need a device: buffers documented as device
memory are refused with DP_EINVAL (host memory, overlapping input and
output) before any kernel runs, and the binding refuses CPU tensors."""
import ctypes

import numpy as np
import pytest

import paper_1408_1578_amd as dp
from synth import config_boundary, random_density
from tests.gpu_util import empty, problem, relerr, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_host_and_short_buffers_are_refused():
    import torch
    b, om, eta, kind = config_boundary("disk", 1024)
    p = problem(b, om, eta, kind)
    L = dp.lib()
    q = to_dev(random_density(b.n, 2, seed=1))
    y = empty(b.n, 2)
    host = np.zeros(4 * b.n)
    hp = host.ctypes.data_as(ctypes.c_void_p)
    qp, yp = ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(y.data_ptr())
    calls = [
        lambda a, c: L.dp_matvec(p.h, 2, a, c),
        lambda a, c: L.dp_matvec_mixed(p.h, 2, a, c),
        lambda a, c: L.dp_layer_apply(p.h, dp.DP_OP_S, 2, a, c),
        lambda a, c: L.dp_solve(p.h, 2, a, c, None, None, None, None),
    ]
    for call in calls:
        assert call(hp, yp) == dp.DP_EINVAL and b"not device memory" in L.dp_last_error()
        assert call(qp, hp) == dp.DP_EINVAL
        # overlapping input and output
        assert call(qp, ctypes.c_void_p(q.data_ptr() + 16)) == dp.DP_EINVAL
    assert L.dp_rhs_plane_wave(p.h, 1, np.zeros(1).ctypes.data_as(ctypes.c_void_p), hp) == dp.DP_EINVAL
    # nothing above launched a kernel on the buffers: y still holds its zeros,
    # and a valid call works afterwards
    assert np.all(to_host(y) == 0)
    dp.dp_matvec(p, q, y)
    assert np.all(np.isfinite(to_host(y))) and np.any(to_host(y) != 0)
    with pytest.raises(ValueError):
        dp.dp_matvec(p, torch.zeros((2, b.n), dtype=torch.complex128), y)
