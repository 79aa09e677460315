"""Closed smooth curves and their arclength-equispaced samples.

The paper (Sec. 2, opening paragraphs) assumes the boundary is C^2, of length
L = Theta(1), and sampled at n equally spaced points in the arclength
parametrisation rho.  The paper's own ellipse and bean (Sec. 3, Fig. 3) are
not given analytically, so seeded synthetic curves of the same size class
stand in: the unit disk, the five-petal star r = 1 + 0.3 cos 5t, the kite
(cos t + 0.65 cos 2t - 0.65, 1.5 sin t), and a seeded random star
r = 1 + sum_{k=1..16} (a_k cos kt + b_k sin kt), a_k, b_k ~ U(-0.02, 0.02).

Everything here is input preparation: positions, outward unit normals,
signed curvature and the trapezoid weight L/n at the nodes.  Nodes are placed
at arclength j*L/n (j = 0..n-1), counter-clockwise, so the outward normal is
(x2', -x1')/|x'|.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


# ---------------------------------------------------------------- curve defs
def _polar(r, dr, ddr):
    """Return (x, x', x'') for a polar curve given r(t), r'(t), r''(t) callables."""
    def ev(t):
        c, s = np.cos(t), np.sin(t)
        R, R1, R2 = r(t), dr(t), ddr(t)
        x = np.stack([R * c, R * s], -1)
        x1 = np.stack([R1 * c - R * s, R1 * s + R * c], -1)
        x2 = np.stack([R2 * c - 2 * R1 * s - R * c, R2 * s + 2 * R1 * c - R * s], -1)
        return x, x1, x2
    return ev


def _disk(t):
    c, s = np.cos(t), np.sin(t)
    return (np.stack([c, s], -1), np.stack([-s, c], -1), np.stack([-c, -s], -1))


def _kite(t):
    x = np.stack([np.cos(t) + 0.65 * np.cos(2 * t) - 0.65, 1.5 * np.sin(t)], -1)
    x1 = np.stack([-np.sin(t) - 1.3 * np.sin(2 * t), 1.5 * np.cos(t)], -1)
    x2 = np.stack([-np.cos(t) - 2.6 * np.cos(2 * t), -1.5 * np.sin(t)], -1)
    return x, x1, x2


_star = _polar(lambda t: 1 + 0.3 * np.cos(5 * t),
               lambda t: -1.5 * np.sin(5 * t),
               lambda t: -7.5 * np.cos(5 * t))


def random_star_coeffs(seed: int):
    """a_k, b_k ~ U(-0.02, 0.02), k = 1..16, from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-0.02, 0.02, 16)
    b = rng.uniform(-0.02, 0.02, 16)
    return a, b


def _random_star(seed: int):
    a, b = random_star_coeffs(seed)
    k = np.arange(1, 17, dtype=np.float64)

    def trig(t):
        # cos kt, sin kt for k = 1..16 from the powers of e^{it}
        e = np.exp(1j * np.asarray(t))[..., None]
        p = np.cumprod(np.broadcast_to(e, e.shape[:-1] + (16,)), axis=-1)
        return p.real, p.imag

    def ev(t):
        C, S = trig(t)
        R = 1 + C @ a + S @ b
        R1 = -S @ (a * k) + C @ (b * k)
        R2 = -C @ (a * k * k) - S @ (b * k * k)
        return _polar(lambda _: R, lambda _: R1, lambda _: R2)(t)

    return ev


CURVES = {"disk": _disk, "star": _star, "kite": _kite}


def curve_by_name(name: str):
    """'disk', 'star', 'kite' or 'randstar<seed>' -> callable t -> (x, x', x'')."""
    if name in CURVES:
        return CURVES[name]
    if name.startswith("randstar"):
        return _random_star(int(name[len("randstar"):] or 0))
    raise ValueError(f"unknown curve {name!r}")


# ------------------------------------------------------- arclength sampling
_GL_X, _GL_W = np.polynomial.legendre.leggauss(10)  # exact to rounding on intervals <= 2 pi/4096


def _speed(curve, t):
    return np.linalg.norm(curve(t)[1], axis=-1)


def _gl_integral(curve, a, b):
    """Integral of |x'| over [a, b] (arrays), 10-point Gauss-Legendre."""
    half = 0.5 * (b - a)
    mid = 0.5 * (b + a)
    tt = mid[..., None] + half[..., None] * _GL_X
    return half * (_speed(curve, tt) @ _GL_W)


@dataclass
class Boundary:
    """Arclength-equispaced samples of a closed curve (counter-clockwise).

    x      (n, 2)  node positions
    nu     (n, 2)  outward unit normals
    kappa  (n,)    signed curvature (positive on convex parts)
    speed  (n,)    |dx/dsigma| for sigma = 2*pi*s/L, i.e. L/(2*pi) everywhere
    w      (n,)    trapezoid weights (2*pi/n)*speed = L/n
    """
    name: str
    n: int
    L: float
    x: np.ndarray
    nu: np.ndarray
    kappa: np.ndarray
    speed: np.ndarray
    w: np.ndarray

    @property
    def ds(self) -> float:
        return self.L / self.n


def sample_boundary(name: str, n: int, intervals: int = 4096) -> Boundary:
    """n nodes at arclength j*L/n along curve `name` (float64 throughout)."""
    if n < 2:
        raise ValueError("n must be >= 2")
    curve = curve_by_name(name)
    tg = np.linspace(0.0, 2 * np.pi, intervals + 1)
    seg = _gl_integral(curve, tg[:-1], tg[1:])
    S = np.concatenate([[0.0], np.cumsum(seg)])
    L = float(S[-1])
    target = np.arange(n, dtype=np.float64) * (L / n)
    m = np.clip(np.searchsorted(S, target, side="right") - 1, 0, intervals - 1)
    t = tg[m] + (target - S[m]) / _speed(curve, tg[m])
    for _ in range(8):
        s_t = S[m] + _gl_integral(curve, tg[m], t)
        step = (s_t - target) / _speed(curve, t)
        t = t - step
        if np.max(np.abs(step)) < 1e-15:
            break
    x, x1, x2 = curve(t)
    sp = np.linalg.norm(x1, axis=-1)
    nu = np.stack([x1[:, 1], -x1[:, 0]], -1) / sp[:, None]
    kappa = (x1[:, 0] * x2[:, 1] - x1[:, 1] * x2[:, 0]) / sp ** 3
    speed = np.full(n, L / (2 * np.pi))
    w = np.full(n, L / n)
    return Boundary(name, n, L, np.ascontiguousarray(x), np.ascontiguousarray(nu),
                    kappa, speed, w)


def omega_for_ppw(n: int, L: float, ppw: float) -> float:
    """Frequency giving `ppw` points per wavelength: n = ppw * L / (2*pi/omega)."""
    return 2 * np.pi * n / (ppw * L)


def config_boundary(cfg: str, n: int | None = None):
    """(Boundary, omega, eta, kind) for the named workloads.

    disk    : unit disk, n = 1024, omega = 100, sound-soft
    star    : r = 1 + 0.3 cos 5t, n in {4096, 16384}, 10 points/wavelength, soft
    kite    : kite, n = 32768, 10 points/wavelength, sound-hard
    randstar: seeded random star (seed 0), n = 131072, 10 points/wavelength, soft
    eta = omega everywhere.
    """
    if cfg == "disk":
        b = sample_boundary("disk", n or 1024)
        om = 100.0
        return b, om, om, 0
    if cfg == "star":
        b = sample_boundary("star", n or 4096)
        om = omega_for_ppw(b.n, b.L, 10.0)
        return b, om, om, 0
    if cfg == "kite":
        b = sample_boundary("kite", n or 32768)
        om = omega_for_ppw(b.n, b.L, 10.0)
        return b, om, om, 1
    if cfg.startswith("randstar"):
        b = sample_boundary(cfg if cfg != "randstar" else "randstar0", n or 131072)
        om = omega_for_ppw(b.n, b.L, 10.0)
        return b, om, om, 0
    raise ValueError(cfg)
