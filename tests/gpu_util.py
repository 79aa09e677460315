"""Shared helpers for the GPU parity tests (no oracle arithmetic here)."""
import numpy as np

import paper_1408_1578_amd as dp


def to_dev(a):
    import torch
    a = np.asarray(a, dtype=np.complex128)
    if a.ndim == 2:        # (n, nrhs) column-major -> (nrhs, n)
        a = a.T
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def to_host(t):
    a = t.cpu().numpy()
    return a.T if a.ndim == 2 else a


def empty(n, nrhs=None):
    import torch
    shape = (n,) if nrhs is None else (nrhs, n)
    return torch.zeros(shape, dtype=torch.complex128, device="cuda:0")


def relerr(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        _CTX = dp.Context(0)
    return _CTX


def problem(b, omega, eta, kind):
    return dp.Problem.from_boundary(ctx(), b, omega, eta, kind)
