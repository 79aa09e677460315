"""Pins of the oracle's GMRES against a dense direct solve."""
import numpy as np
import pytest

from oracle.gmres import gmres


def _system(n, seed):
    rng = np.random.default_rng(seed)
    A = 2 * np.eye(n) + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    f = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, f


@pytest.mark.parametrize("restart", [5, 20, 80])
def test_gmres_solves(restart):
    A, f = _system(50, 1)
    x, its, hist = gmres(A, f, tol=1e-12, restart=restart, maxiter=2000)
    xe = np.linalg.solve(A, f)
    assert np.linalg.norm(x - xe) / np.linalg.norm(xe) < 1e-10
    assert np.linalg.norm(f - A @ x) / np.linalg.norm(f) < 1e-11


def test_gmres_exact_termination_and_monotone():
    A, f = _system(24, 2)
    x, its, hist = gmres(A, f, tol=1e-13, restart=80)
    assert its <= 24
    h = np.array(hist[1:])
    assert np.all(np.diff(h) <= 1e-14)


def test_gmres_right_preconditioned():
    A, f = _system(40, 3)
    M = np.linalg.inv(A + 0.05 * np.eye(40))
    x, its, _ = gmres(A, f, tol=1e-12, restart=80, M=M)
    assert its < 10
    assert np.linalg.norm(A @ x - f) / np.linalg.norm(f) < 1e-11


def test_zero_rhs():
    A, _ = _system(10, 4)
    x, its, _ = gmres(A, np.zeros(10, complex))
    assert its == 0 and not np.any(x)
