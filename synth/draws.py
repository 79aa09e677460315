"""Seeded random draws: incident-wave angles and test densities."""
from __future__ import annotations

import numpy as np


def plane_wave_angles(nrhs: int, mode: str = "uniform", seed: int = 0) -> np.ndarray:
    """Incidence angles theta_k (direction d_k = (cos theta_k, sin theta_k)).

    mode 'uniform': theta_k = 2*pi*k/nrhs (k = 0 gives the +x direction used in
    the paper's experiments, Sec. 3); mode 'random': U(0, 2*pi) from
    default_rng(seed).
    """
    if mode == "uniform":
        return 2 * np.pi * np.arange(nrhs, dtype=np.float64) / nrhs
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2 * np.pi, nrhs)


def random_density(n: int, nrhs: int = 1, seed: int = 0) -> np.ndarray:
    """Complex128 array (n, nrhs), column-major friendly, entries ~ CN(0, 1)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, nrhs)) + 1j * rng.standard_normal((n, nrhs))
    return np.asfortranarray(z / np.sqrt(2.0))
