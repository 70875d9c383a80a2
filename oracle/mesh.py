"""Mesh conventions for the oracle (test infrastructure only).

* Nodes sit at x_n = b0 + n H, H = L / N, n = 0..N-1 on each axis; the observer
  is at the origin of the coordinate system the positions are given in.
* Painting (mass assignment, the nbodykit step of Section 7.2): node masses
  m_n = sum_p w_p W(u_p - n), u = (x - b0)/H, periodic node indices.
  CIC: i0 = floor(u), weights (1-d, d) at (i0, i0+1), d = u - i0.
  TSC: i0 = floor(u + 1/2), d = u - i0, weights (1/2 (1/2 - d)^2, 3/4 - d^2, 1/2 (1/2 + d)^2)
  at (i0-1, i0, i0+1).
* The density of Section 2.1, w (n_g - alpha_r n_r), is carried as node masses
  (painted weight, not divided by H^3); every estimator below is written for
  node masses, so that a pair sum sum_ij w_i w_j (...) over particles and the mesh
  form agree term by term.
* DFT: X~(k) = sum_n X_n exp(-i k . n H) (numpy ``fftn``); the box-origin phase
  cancels in every product used.  Wavevector of index n on an axis:
  (2 pi / L) * s(n), s(n) = n for n < N/2 else n - N.  The mode -k has index
  (-n) mod N.  Real-space separations use the same signed index (minimum image).
* Assignment window (the compensation of the footnote in Section 2.1):
  W(k) = prod_i sinc(k_i H / 2)^p, p = 2 (CIC) or 3 (TSC), sinc(x) = sin x / x.
"""
from __future__ import annotations

import numpy as np

CIC = 2
TSC = 3


def signed_index(N: int) -> np.ndarray:
    n = np.arange(N)
    return np.where(n < N // 2, n, n - N)


def paint(pos, w, N: int, L: float, b0, assign: int) -> np.ndarray:
    """Node masses m[ix, iy, iz] = sum_p w_p W(u_p - n) (periodic)."""
    pos = np.asarray(pos, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    H = L / N
    u = (pos - np.asarray(b0, dtype=np.float64)[None, :]) / H
    mesh = np.zeros(N * N * N, dtype=np.float64)
    if assign == CIC:
        i0 = np.floor(u).astype(np.int64)
        d = u - i0
        taps = [(0, 1.0 - d), (1, d)]
    elif assign == TSC:
        i0 = np.floor(u + 0.5).astype(np.int64)
        d = u - i0
        taps = [(-1, 0.5 * (0.5 - d) ** 2), (0, 0.75 - d * d), (1, 0.5 * (0.5 + d) ** 2)]
    else:
        raise ValueError("assign must be CIC (2) or TSC (3)")
    for ox, wx in taps:
        ix = (i0[:, 0] + ox) % N
        for oy, wy in taps:
            iy = (i0[:, 1] + oy) % N
            for oz, wz in taps:
                iz = (i0[:, 2] + oz) % N
                flat = (ix * N + iy) * N + iz
                mesh += np.bincount(flat, weights=w * wx[:, 0] * wy[:, 1] * wz[:, 2],
                                    minlength=N * N * N)
    return mesh.reshape(N, N, N)


def node_positions(N: int, L: float, b0) -> np.ndarray:
    """x_n = b0 + n H as an array [N, N, N, 3]."""
    H = L / N
    g = np.arange(N) * H
    b0 = np.asarray(b0, dtype=np.float64)
    X, Y, Z = np.meshgrid(g + b0[0], g + b0[1], g + b0[2], indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def kgrid(N: int, L: float):
    """Integer signed indices (sx, sy, sz) [N,N,N] each, and the k vectors [N,N,N,3]."""
    s = signed_index(N)
    SX, SY, SZ = np.meshgrid(s, s, s, indexing="ij")
    kf = 2.0 * np.pi / L
    return (SX, SY, SZ), np.stack([SX, SY, SZ], axis=-1) * kf


def separation_grid(N: int, L: float) -> np.ndarray:
    """Minimum-image separation vectors Delta_n = H s(n)  [N,N,N,3]."""
    s = signed_index(N) * (L / N)
    X, Y, Z = np.meshgrid(s, s, s, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def window(N: int, assign: int) -> np.ndarray:
    """W(k) = prod_i sinc(k_i H/2)^p on the FFT grid, k_i H / 2 = pi s_i / N."""
    s = signed_index(N)
    x = np.pi * s / N
    with np.errstate(invalid="ignore", divide="ignore"):
        sn = np.where(x == 0, 1.0, np.sin(x) / np.where(x == 0, 1.0, x))
    w1 = sn ** assign
    return w1[:, None, None] * w1[None, :, None] * w1[None, None, :]


def neg_k(X: np.ndarray) -> np.ndarray:
    """X(-k): the value at index (-n) mod N on every axis."""
    Y = X[::-1, ::-1, ::-1]
    return np.roll(Y, 1, axis=(0, 1, 2))


def k_bin_index(N: int, L: float, kmin: float, dk: float, nbins: int) -> np.ndarray:
    """Bin of every mode from its integer |s|^2 (FP64): b = floor((2pi/L sqrt(s2) - kmin)/dk);
    -1 outside [0, nbins)."""
    (SX, SY, SZ), _ = kgrid(N, L)
    s2 = (SX * SX + SY * SY + SZ * SZ).astype(np.float64)
    kmag = (2.0 * np.pi / L) * np.sqrt(s2)
    t = kmag - kmin
    b = np.floor(t / dk)
    b = np.where((b >= 0) & (b < nbins), b, -1).astype(np.int64)
    return b, kmag


def r_bin_index(N: int, L: float, rmin: float, dr: float, nbins: int) -> np.ndarray:
    """Bin of every grid separation: b = floor((H sqrt(s2) - rmin)/dr); the zero separation and
    separations outside [0, nbins) get -1."""
    s = signed_index(N)
    SX, SY, SZ = np.meshgrid(s, s, s, indexing="ij")
    s2 = (SX * SX + SY * SY + SZ * SZ).astype(np.float64)
    rmag = (L / N) * np.sqrt(s2)
    t = rmag - rmin
    b = np.floor(t / dr)
    b = np.where((b >= 0) & (b < nbins) & (s2 > 0), b, -1).astype(np.int64)
    return b, rmag
