"""Host-side checks of the C-ABI library: it loads, exports every declared
symbol, validates arguments, and its host build of the Hankel code agrees
with scipy/mpmath (no GPU needed)."""
import ctypes
import os
import re

import mpmath as mp
import numpy as np
import pytest
from scipy import special as sp

import paper_1408_1578_amd as dp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "dirprec.h")).read()
    return sorted(set(re.findall(r"\b(dp_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = dp.lib()
    names = _declared()
    assert set(names) == set(dp.EXPORTED)
    for name in names:
        assert hasattr(L, name), name


def test_last_error_initially_empty_string():
    assert isinstance(dp.lib().dp_last_error(), bytes)


def test_hankel_host_build_vs_scipy():
    z = np.concatenate([np.geomspace(1e-3, 3e4, 400), np.linspace(24.0, 26.0, 41)])
    h0, h1 = dp.dp_hankel_host(z)
    tol = np.maximum(3e-15, 4 * z * 1.1e-16)
    e0 = np.abs(h0 - sp.hankel1(0, z)) / np.abs(sp.hankel1(0, z))
    e1 = np.abs(h1 - sp.hankel1(1, z)) / np.abs(sp.hankel1(1, z))
    assert np.all(e0 < tol + 2e-15) and np.all(e1 < tol + 2e-15), (e0.max(), e1.max())


def test_hankel_host_build_vs_mpmath():
    mp.mp.dps = 30
    z = np.array([0.07, 0.9, 4.3, 11.0, 19.99, 24.999, 25.0, 31.4, 250.0])
    h0, h1 = dp.dp_hankel_host(z)
    for k, zz in enumerate(z):
        r0 = complex(mp.hankel1(0, mp.mpf(zz)))
        r1 = complex(mp.hankel1(1, mp.mpf(zz)))
        assert abs(h0[k] - r0) / abs(r0) < 3e-15
        assert abs(h1[k] - r1) / abs(r1) < 3e-15


def test_hankel_host_rejects_nonpositive():
    with pytest.raises(dp.DpError):
        dp.dp_hankel_host(np.array([1.0, 0.0]))


def test_problem_create_validates_without_gpu():
    # argument validation runs before any device call
    L = dp.lib()
    n = 8  # too small
    x = np.zeros(2 * n)
    h = ctypes.c_void_p()
    rc = L.dp_problem_create(None, n, x.ctypes.data_as(ctypes.c_void_p), x.ctypes.data_as(ctypes.c_void_p),
                             x.ctypes.data_as(ctypes.c_void_p), x.ctypes.data_as(ctypes.c_void_p),
                             1.0, 1.0, 0, ctypes.byref(h))
    assert rc == dp.DP_EINVAL


def test_new_entry_points_validate_without_gpu():
    # every check below happens before any device call
    L = dp.lib()
    vp = ctypes.c_void_p
    assert L.dp_matvec_mixed(None, 1, None, None) == dp.DP_EINVAL
    assert L.dp_precond_apply_mixed(None, 1, None, None) == dp.DP_EINVAL
    assert L.dp_autotune(None, 4, 0, None) == dp.DP_EINVAL
    assert L.dp_server_create(0, None, None) == dp.DP_EINVAL
    assert L.dp_server_submit(None, None, None) == dp.DP_EINVAL
    assert L.dp_server_wait(None, 1, None, None, None) == dp.DP_EINVAL
    assert L.dp_server_get_stats(None, None) == dp.DP_EINVAL
    L.dp_server_destroy(None)  # no-op
    assert b"NULL" in L.dp_last_error() or len(L.dp_last_error()) > 0


def test_server_options_validated():
    L = dp.lib()
    out = ctypes.c_void_p()
    bad = dp.ServerOpts(0, -5)           # negative memory budget
    assert L.dp_server_create(0, ctypes.byref(bad), ctypes.byref(out)) == dp.DP_EINVAL
    assert not out.value
