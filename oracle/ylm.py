"""Complex spherical harmonics for the oracle (test infrastructure only).

Y_l^m is orthonormal on the sphere with the Condon-Shortley phase, and obeys
Y_l^m(-x) = (-1)^l Y_l^m(x), Y_l^{m*} = (-1)^m Y_l^{-m}  (Appendix A, addition
theorem and orthonormality).  Evaluated with scipy's ``sph_harm_y``; the zero
vector is mapped to the +z direction (callers mask it where it matters).
"""
from __future__ import annotations

import numpy as np
from scipy.special import sph_harm_y


def unit_angles(v):
    """Polar and azimuthal angles of the vectors v[..., 3] (zero vector -> theta = 0)."""
    v = np.asarray(v, dtype=np.float64)
    x, y, z = v[..., 0], v[..., 1], v[..., 2]
    r = np.sqrt(x * x + y * y + z * z)
    with np.errstate(invalid="ignore", divide="ignore"):
        ct = np.where(r > 0, z / np.where(r > 0, r, 1.0), 1.0)
    ct = np.clip(ct, -1.0, 1.0)
    theta = np.arccos(ct)
    phi = np.arctan2(y, x)
    return theta, phi, r


def Ylm(l: int, m: int, v) -> np.ndarray:
    """Y_l^m(v^) for vectors v[..., 3]."""
    if abs(m) > l:
        return np.zeros(np.shape(v)[:-1], dtype=np.complex128)
    theta, phi, _ = unit_angles(v)
    return sph_harm_y(l, m, theta, phi)


def Ylm_angles(l: int, m: int, theta, phi) -> np.ndarray:
    if abs(m) > l:
        return np.zeros(np.shape(theta), dtype=np.complex128)
    return sph_harm_y(l, m, theta, phi)


def legendre(l: int, mu) -> np.ndarray:
    """Legendre polynomial L_l(mu)."""
    from scipy.special import eval_legendre
    return eval_legendre(l, mu)
