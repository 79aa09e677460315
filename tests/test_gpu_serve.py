"""Request server: results alone and in a concurrent mix, memory-based
admission, failure isolation (MI355X)."""
import numpy as np
import pytest

import paper_1408_1578_amd as dp
from oracle import nystrom as ny
from synth import config_boundary, omega_for_ppw, plane_wave_angles, sample_boundary

pytestmark = pytest.mark.gpu


def _requests():
    """(boundary, omega, eta, kind, submit kwargs) of a mixed stream."""
    out = []
    b, om, eta, kind = config_boundary("disk", 1024)
    out.append((b, om, eta, kind, dict(angles=plane_wave_angles(3))))
    b = sample_boundary("kite", 2048)
    om = omega_for_ppw(2048, b.L, 10.0)
    out.append((b, om, om, 1, dict(angles=plane_wave_angles(8))))
    b = sample_boundary("star", 4096)
    om = omega_for_ppw(4096, b.L, 10.0)
    out.append((b, om, om, 0, dict(angles=plane_wave_angles(1), precision=dp.DP_PREC_MIXED)))
    b = sample_boundary("randstar1", 2048)
    om = omega_for_ppw(2048, b.L, 10.0)
    out.append((b, om, om, 0, dict(angles=plane_wave_angles(16), precision=dp.DP_PREC_MIXED)))
    b = sample_boundary("kite", 4096)
    om = omega_for_ppw(4096, b.L, 10.0)
    out.append((b, om, om, 1, dict(angles=plane_wave_angles(5), precision=dp.DP_PREC_MIXED)))
    b, om, eta, _ = config_boundary("disk", 1024)
    f = ny.point_source_data(b, om, np.array([0.2, -0.1]), 1)
    out.append((b, om, eta, 1, dict(f=f, use_precond=False)))
    b = sample_boundary("randstar4", 1000)      # sound-hard, n not a power of two
    om = omega_for_ppw(1000, b.L, 10.0)
    out.append((b, om, om, 1, dict(angles=plane_wave_angles(3), precision=dp.DP_PREC_MIXED)))
    return out


def test_serve_alone_equals_mix():
    reqs = _requests()
    alone = []
    s1 = dp.Server(slots=1)
    for b, om, eta, kind, kw in reqs:
        q, info, t, rc = s1.wait(s1.submit(b, om, eta, kind, **kw))
        assert rc == dp.DP_OK and info["relres_max"] <= 1e-8
        alone.append(q)
    s1.close()

    s4 = dp.Server(slots=4)
    ids = [s4.submit(b, om, eta, kind, **kw) for b, om, eta, kind, kw in reqs]
    res = [s4.wait(i) for i in ids]
    st = s4.stats()
    s4.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0 and st["mem_peak"] <= st["mem_budget"]
    for (q, info, t, rc), qa in zip(res, alone):
        assert rc == dp.DP_OK
        # same kernels on private buffers and stream: the same bits
        assert np.array_equal(q, qa)
    iv = sorted((t["t_admit"], t["t_done"]) for _, _, t, _ in res)
    assert any(iv[k + 1][0] < iv[k][1] for k in range(len(iv) - 1)), "no two requests overlapped"
    assert len({t["slot"] for _, _, t, _ in res}) > 1

    # one of them against the oracle's dense solve
    b, om, eta, kind, kw = reqs[0]
    A = ny.cfie_matrix(b, om, eta, kind)
    F = ny.plane_wave_rhs(b, om, kw["angles"], kind)
    Q = np.linalg.solve(A, F)
    assert np.linalg.norm(res[0][0] - Q) / np.linalg.norm(Q) < 1e-6


def test_serve_memory_admission_and_rejection():
    b = sample_boundary("kite", 2048)
    om = omega_for_ppw(2048, b.L, 10.0)
    kw = dict(angles=plane_wave_angles(4))
    probe = dp.Server(slots=1)
    _, _, t, _ = probe.wait(probe.submit(b, om, om, 1, **kw))
    probe.close()
    est = t["mem_estimate"]
    # room for one request at a time although four slots are free
    s = dp.Server(slots=4, mem_budget=int(1.5 * est))
    ids = [s.submit(b, om, om, 1, **kw) for _ in range(4)]
    res = [s.wait(i) for i in ids]
    st = s.stats()
    iv = sorted((t["t_admit"], t["t_done"]) for _, _, t, _ in res)
    assert all(iv[k + 1][0] >= iv[k][1] for k in range(len(iv) - 1))
    assert st["mem_peak"] <= st["mem_budget"] and st["completed"] == 4
    q0 = res[0][0]
    assert all(np.array_equal(r[0], q0) for r in res)
    # a request that could never fit is refused at submission
    big = sample_boundary("kite", 65536)
    with pytest.raises(dp.DpError) as e:
        s.submit(big, 1000.0, 1000.0, 1, angles=plane_wave_angles(64))
    assert e.value.code == dp.DP_ENOMEM
    s.close()


def test_serve_failure_is_isolated():
    b, om, eta, kind = config_boundary("disk", 1024)

    class Bad:  # normals of length 2: rejected by problem creation inside the worker
        x, nu, w, kappa = b.x, 2.0 * b.nu, b.w, b.kappa

    s = dp.Server(slots=2)
    good1 = s.submit(b, om, eta, kind, angles=plane_wave_angles(2))
    bad = s.submit(Bad, om, eta, kind, angles=plane_wave_angles(2))
    good2 = s.submit(b, om, eta, kind, angles=plane_wave_angles(2))
    with pytest.raises(dp.DpError) as e:
        s.wait(bad)
    assert e.value.code == dp.DP_EINVAL and "normal" in str(e.value).lower()
    q1 = s.wait(good1)[0]
    q2 = s.wait(good2)[0]
    assert np.array_equal(q1, q2)
    st = s.stats()
    assert st["failed"] == 1 and st["completed"] == 3
    with pytest.raises(dp.DpError):
        s.wait(12345)
    s.close()
