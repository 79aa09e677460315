"""Special functions for the oracle.

The Green's function of Sec. 1 is G(x, y) = (i/4) H_0^(1)(omega |x - y|).
Hankel functions of the first kind come from scipy.special (a library
primitive); tests pin them against mpmath and the Wronskian.
"""
import numpy as np
from scipy import special as _sp

EULER_GAMMA = 0.57721566490153286060651209008240243104215933593992


def h0(z):
    """H_0^(1)(z) for real z > 0."""
    return _sp.hankel1(0, z)


def h1(z):
    """H_1^(1)(z) for real z > 0."""
    return _sp.hankel1(1, z)


def hankel01(z):
    z = np.asarray(z, dtype=np.float64)
    return h0(z), h1(z)
