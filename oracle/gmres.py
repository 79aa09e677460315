"""Textbook restarted GMRES (oracle; test infrastructure).

The paper solves its systems with GMRES, relative tolerance and restart 80
(Sec. 3).  This is the plain algorithm: Arnoldi with modified Gram-Schmidt,
Givens rotations on the Hessenberg matrix, x0 = 0, optional right
preconditioner M (the Krylov space is built for A M, the iterate is M y).
Convergence is declared on the Givens residual estimate and re-checked on the
true residual at each restart.
"""
import numpy as np


def gmres(A, f, tol=1e-8, restart=80, maxiter=2000, M=None):
    """Solve A x = f.  A, M: callables or dense arrays.  Returns (x, iters, hist)."""
    mv = A if callable(A) else (lambda v: A @ v)
    pc = (lambda v: v) if M is None else (M if callable(M) else (lambda v: M @ v))
    f = np.asarray(f, dtype=np.complex128)
    n = f.size
    x = np.zeros(n, np.complex128)
    fn = np.linalg.norm(f)
    hist = []
    if fn == 0:
        return x, 0, hist
    its = 0
    while its < maxiter:
        r = f - mv(x)
        beta = np.linalg.norm(r)
        hist.append(beta / fn)
        if beta / fn <= tol:
            break
        V = np.zeros((restart + 1, n), np.complex128)
        H = np.zeros((restart + 1, restart), np.complex128)
        cs = np.zeros(restart, np.complex128)
        sn = np.zeros(restart, np.complex128)
        g = np.zeros(restart + 1, np.complex128)
        g[0] = beta
        V[0] = r / beta
        k_done = 0
        for k in range(restart):
            w = mv(pc(V[k]))
            its += 1
            for i in range(k + 1):
                H[i, k] = np.vdot(V[i], w)
                w = w - H[i, k] * V[i]
            H[k + 1, k] = np.linalg.norm(w)
            if H[k + 1, k] != 0:
                V[k + 1] = w / H[k + 1, k]
            for i in range(k):   # previous rotations Q_i = [[c*, s*], [-s, c]]
                t = np.conj(cs[i]) * H[i, k] + np.conj(sn[i]) * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            a, bb = H[k, k], H[k + 1, k]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            cs[k] = a / den if den else 1.0
            sn[k] = bb / den if den else 0.0
            H[k, k] = den
            H[k + 1, k] = 0
            g[k + 1] = -sn[k] * g[k]
            g[k] = np.conj(cs[k]) * g[k]
            k_done = k + 1
            hist.append(abs(g[k + 1]) / fn)
            if abs(g[k + 1]) / fn <= tol or its >= maxiter:
                break
        y = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done])
        x = x + pc(V[:k_done].T @ y)
    return x, its, hist
