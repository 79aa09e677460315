"""Pins of the oracle's Nystrom matrices against unit-disk closed forms."""
import numpy as np
import pytest

from oracle import disk, nystrom as ny
from synth import sample_boundary


@pytest.fixture(scope="module")
def disk_case():
    b = sample_boundary("disk", 1024)
    om = 100.0
    return b, om, om, {k: ny.cfie_matrix(b, om, om, k) for k in (0, 1)}


@pytest.mark.parametrize("kind", [0, 1])
def test_density_vs_series(disk_case, kind):
    b, om, eta, A = disk_case
    theta = 2 * np.pi * np.arange(b.n) / b.n
    f = ny.plane_wave_rhs(b, om, 0.0, kind)[:, 0]
    q = np.linalg.solve(A[kind], f)
    qe = disk.density(theta, om, eta, kind)
    assert np.linalg.norm(q - qe) / np.linalg.norm(qe) < 1e-12


@pytest.mark.parametrize("kind", [0, 1])
def test_circulant_eigenvalues(disk_case, kind):
    b, om, eta, A = disk_case
    theta = 2 * np.pi * np.arange(b.n) / b.n
    m = np.arange(-b.n // 4, b.n // 4 + 1)
    ev = np.exp(1j * np.outer(m, theta)) @ A[kind][0]
    lam = disk.cfie_eigs(m, om, eta, kind)
    assert np.max(np.abs(ev - lam) / np.abs(lam)) < 1e-12
    # circulant structure
    assert np.max(np.abs(np.roll(A[kind][0], 5) - A[kind][5])) < 1e-13


@pytest.mark.parametrize("kind", [0, 1])
def test_field_vs_series(disk_case, kind):
    b, om, eta, A = disk_case
    f = ny.plane_wave_rhs(b, om, 0.0, kind)[:, 0]
    q = np.linalg.solve(A[kind], f)
    pts = np.array([[1.5, 0.3], [-2.0, 1.0], [0.2, -3.0], [1.1, 0.0]])
    u = ny.field(b, om, eta, kind, q, pts)
    r = np.linalg.norm(pts, axis=1)
    th = np.arctan2(pts[:, 1], pts[:, 0])
    ue = disk.scattered_field(r, th, om, kind)
    assert np.max(np.abs(u - ue)) / np.max(np.abs(ue)) < 1e-11


def test_layer_eigenvalues(disk_case):
    b, om, eta, _ = disk_case
    lay = ny.layer_rows(b, om, np.array([0]))
    theta = 2 * np.pi * np.arange(b.n) / b.n
    m = np.arange(-200, 201)
    Sm, Dm, _ = disk.layer_eigs(m, om)
    E = np.exp(1j * np.outer(m, theta))
    for name, ref in (("S", Sm), ("D", Dm), ("Dp", Dm)):
        ev = E @ lay[name][0]
        assert np.max(np.abs(ev - ref)) / np.max(np.abs(ref)) < 1e-12
