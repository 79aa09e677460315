"""Pin of the oracle on non-circular curves: the exterior field of an interior
point source is reproduced from its own boundary data (Green's representation
is unique), to quadrature accuracy."""
import numpy as np
import pytest

from oracle import nystrom as ny
from synth import omega_for_ppw, sample_boundary


@pytest.mark.parametrize("curve,n", [("kite", 1024), ("star", 1024), ("randstar3", 1024)])
@pytest.mark.parametrize("kind", [0, 1])
def test_point_source(curve, n, kind):
    b = sample_boundary(curve, n)
    om = omega_for_ppw(n, b.L, 10.0)          # 10 points per wavelength
    z0 = np.array([0.1, 0.2])
    f = ny.point_source_data(b, om, z0, kind)
    A = ny.cfie_matrix(b, om, om, kind)
    q = np.linalg.solve(A, f)
    th = np.linspace(0, 2 * np.pi, 7, endpoint=False)
    pts = np.stack([2.6 * np.cos(th), 2.6 * np.sin(th)], 1)
    u = ny.field(b, om, om, kind, q, pts)
    ue = ny.green(om, pts, z0)
    assert np.max(np.abs(u - ue)) / np.max(np.abs(ue)) < 1e-11


def test_point_source_catches_wrong_hard_sign():
    # the literal operator form 1/2 + D' - N/(i eta) does not reproduce the field
    b = sample_boundary("kite", 256)
    om = 20.0
    z0 = np.array([0.1, 0.2])
    f = ny.point_source_data(b, om, z0, 1)
    A = ny.cfie_matrix(b, om, om, 1)
    Aflip = np.eye(b.n) - A            # = 1/2 I + D' - N/(i eta)
    q = np.linalg.solve(Aflip, f)
    pts = np.array([[2.6, 0.0], [0.0, 2.6]])
    u = ny.field(b, om, om, 1, q, pts)
    ue = ny.green(om, pts, z0)
    assert np.max(np.abs(u - ue)) / np.max(np.abs(ue)) > 1e-3
