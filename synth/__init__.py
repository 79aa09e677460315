"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package holds no arithmetic of the scattering method: it only produces
boundary samples (points, outward normals, curvature, quadrature weights),
frequencies, incident-wave angles and random densities.  Both the CPU oracle
and the HIP library receive these arrays as plain inputs.
"""
from .geometry import (Boundary, CURVES, curve_by_name, sample_boundary,
                       random_star_coeffs, config_boundary, omega_for_ppw)
from .draws import plane_wave_angles, random_density

__all__ = ["Boundary", "CURVES", "curve_by_name", "sample_boundary",
           "random_star_coeffs", "config_boundary", "omega_for_ppw",
           "plane_wave_angles", "random_density"]
