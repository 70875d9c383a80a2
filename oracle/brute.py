"""O(N^2) pair sums for tiny catalogs (oracle pins; test infrastructure only).

The estimator definitions of Section 2 are double integrals over pairs; for a
catalog of point masses they are pair sums

  P_l(k_b) + d_l0 S/I = (4pi / (I N_b)) sum_{k in b} Re sum_m Y_l^{m*}(k^)
                         sum_{ij} w_i w_j exp(-i k.(x_j - x_i)) W^{lm}(i, j)

  xi_l(r_a) = (4pi / (I v_a)) sum_{ij, |x_j - x_i| in a, i != j-position}
                         w_i w_j Re sum_m Y_l^{m*}(D^_ij) W^{lm}(i, j)

with signed weights (w for galaxies, -alpha_r w for randoms) and W^{lm}(i,j) the
angular weight of the pair:

  exact midpoint  Y_l^m((x_i + x_j)^)                     (Section 2.1 definitions)
  exact bisector  Y_l^m((x_i^ + x_j^)^)
  series midpoint (1/2) sum_{even alpha<=K} Phi Y_J1^M(D^)[eps_i^alpha Y_J2^{m-M}(x_i^) + eps_j^alpha Y_J2^{m-M}(x_j^)]
                  (Section 3.3 boxed expansion; D = x_j - x_i, eps = |D|/(2r))
  series bisector sum_{beta<=K/2} B Y_J1^M(x_i^) Y_J2^{m-M}(x_j^)   (Section 5.1 boxed expansion)
  yamamoto        Y_l^m(x_j^)                               (Section 2.1)

For particles placed exactly on mesh nodes and CIC assignment the FFT estimators
equal the series pair sums to rounding, provided no separation reaches the
Nyquist index on any axis (the box is at least twice the catalog's extent and the
k-bins stay below the Nyquist wavenumber).  The sum over k in b is done on the
periodic separation grid: C_{b,lm}[d] = sum_{k in b} Y_l^{m*}(k^) exp(2 pi i s_k . d / N),
computed as an explicit (matrix) discrete Fourier sum.
"""
from __future__ import annotations

import math

import numpy as np

from . import coeffs
from .mesh import kgrid, k_bin_index, signed_index
from .ylm import Ylm, legendre

FOURPI = 4.0 * math.pi


def _particles(gal, ran, alpha_r):
    pos = np.concatenate([gal["pos"], ran["pos"]], axis=0).astype(np.float64)
    w = np.concatenate([gal["w"], -alpha_r * np.asarray(ran["w"])]).astype(np.float64)
    return pos, w


def _node_index(pos, cfg):
    H = cfg.L / cfg.N
    u = (pos - np.asarray(cfg.b0, dtype=np.float64)[None, :]) / H
    n = np.rint(u).astype(np.int64)
    if not np.allclose(u, n, atol=1e-9):
        raise ValueError("brute-force pins need particles exactly on mesh nodes")
    return n


def _dft_kernel(values, N):
    """sum_k values[k] exp(+2 pi i s_k . d / N) for every d (explicit matrix DFT on each axis)."""
    s = signed_index(N)
    d = np.arange(N)
    E = np.exp(2j * np.pi * np.outer(d, s) / N)          # [d, k]
    out = np.tensordot(E, values, axes=([1], [0]))       # d0, k1, k2
    out = np.tensordot(out, E, axes=([1], [1]))          # d0, k2, d1
    out = np.tensordot(out, E, axes=([1], [1]))          # d0, d1, d2
    return out


def pair_weight(kind: str, l: int, m: int, xi, xj, K: int, K_lo: int = 0):
    """W^{lm}(i, j) for arrays of pair endpoints xi, xj [P, 3]; the series kinds keep the
    terms of order K_lo .. K in the opening angle.  mid_series is the parity-even midpoint
    expansion (Phi, even alpha, Section 3.3); mid_series_all the symmetrised all-parity one
    (Section 3.1: phi, every alpha, the r2 half carrying (-1)^J1)."""
    D = xj - xi
    if kind == "mid_exact":
        return Ylm(l, m, xi + xj)
    if kind == "bis_exact":
        ui = xi / np.linalg.norm(xi, axis=-1, keepdims=True)
        uj = xj / np.linalg.norm(xj, axis=-1, keepdims=True)
        return Ylm(l, m, ui + uj)
    if kind == "yamamoto":
        return Ylm(l, m, xj)
    if kind == "mid_series":
        Dn = np.linalg.norm(D, axis=-1)
        ei = Dn / (2.0 * np.linalg.norm(xi, axis=-1))
        ej = Dn / (2.0 * np.linalg.norm(xj, axis=-1))
        out = np.zeros(len(xi), dtype=np.complex128)
        for a in range(K_lo + K_lo % 2, K + 1, 2):
            for (J1, J2, M), c in coeffs.Phi_table(a, l, m).items():
                out += 0.5 * c * Ylm(J1, M, D) * (ei ** a * Ylm(J2, m - M, xi) + ej ** a * Ylm(J2, m - M, xj))
        return out
    if kind == "mid_series_all":
        Dn = np.linalg.norm(D, axis=-1)
        ei = Dn / (2.0 * np.linalg.norm(xi, axis=-1))
        ej = Dn / (2.0 * np.linalg.norm(xj, axis=-1))
        out = np.zeros(len(xi), dtype=np.complex128)
        for a in range(K_lo, K + 1):
            for (J1, J2, M), c in coeffs.phi_table(a, l, m).items():
                out += 0.5 * c * Ylm(J1, M, D) * (ei ** a * Ylm(J2, m - M, xi)
                                                  + (-1) ** J1 * ej ** a * Ylm(J2, m - M, xj))
        return out
    if kind == "bis_series":
        out = np.zeros(len(xi), dtype=np.complex128)
        for (J1, J2, M), c in coeffs.B_table(K // 2, l, m, (K_lo + 1) // 2).items():
            out += c * Ylm(J1, M, xi) * Ylm(J2, m - M, xj)
        return out
    raise ValueError(kind)


def pk_pairs(gal, ran, cfg, kind: str, norm):
    """Pair-sum P_l(k_b) (shot noise S/I subtracted from l = 0) for node-placed particles."""
    alpha_r, I, S = norm
    pos, w = _particles(gal, ran, alpha_r)
    n = _node_index(pos, cfg)
    N = cfg.N
    b, _ = k_bin_index(N, cfg.L, cfg.bin_lo, cfg.bin_width, cfg.n_bins)
    _, kvec = kgrid(N, cfg.L)
    P = len(pos)
    ii, jj = np.meshgrid(np.arange(P), np.arange(P), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    d = (n[ii] - n[jj]) % N
    ww = w[ii] * w[jj]
    counts = np.array([(b == q).sum() for q in range(cfg.n_bins)], dtype=np.float64)
    out = np.zeros((len(cfg.ells), cfg.n_bins))
    for li, l in enumerate(cfg.ells):
        for m in range(-l, l + 1):
            Wp = pair_weight(kind, l, m, pos[ii], pos[jj], cfg.order, cfg.order_lo)
            Ystar = np.conj(Ylm(l, m, kvec))
            for q in range(cfg.n_bins):
                if counts[q] == 0:
                    continue
                C = _dft_kernel(np.where(b == q, Ystar, 0.0), N)
                out[li, q] += np.real(np.sum(ww * C[d[:, 0], d[:, 1], d[:, 2]] * Wp))
    with np.errstate(invalid="ignore", divide="ignore"):
        out = FOURPI / I * np.where(counts > 0, out / np.where(counts > 0, counts, 1), 0.0)
    for li, l in enumerate(cfg.ells):
        if l == 0 and cfg.order_lo == 0:
            out[li] -= np.where(counts > 0, S / I, 0.0)
    return out, counts


def xi_pairs(gal, ran, cfg, kind: str, norm):
    """Pair-sum xi_l(r_a) for node-placed particles (zero separations excluded)."""
    alpha_r, I, S = norm
    pos, w = _particles(gal, ran, alpha_r)
    n = _node_index(pos, cfg)
    N = cfg.N
    H = cfg.L / N
    P = len(pos)
    ii, jj = np.meshgrid(np.arange(P), np.arange(P), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    dn = n[jj] - n[ii]
    s2 = np.sum(dn * dn, axis=1).astype(np.float64)
    rmag = H * np.sqrt(s2)
    bq = np.floor((rmag - cfg.bin_lo) / cfg.bin_width)
    keep = (s2 > 0) & (bq >= 0) & (bq < cfg.n_bins)
    ii, jj, bq = ii[keep], jj[keep], bq[keep].astype(np.int64)
    xi_, xj_ = pos[ii], pos[jj]
    D = xj_ - xi_
    ww = w[ii] * w[jj]
    # grid-separation counts per bin (bin volume v_a = N_a H^3)
    s = signed_index(N)
    SX, SY, SZ = np.meshgrid(s, s, s, indexing="ij")
    g2 = (SX * SX + SY * SY + SZ * SZ).astype(np.float64)
    gb = np.floor((H * np.sqrt(g2) - cfg.bin_lo) / cfg.bin_width)
    counts = np.array([((gb == q) & (g2 > 0)).sum() for q in range(cfg.n_bins)], dtype=np.float64)
    out = np.zeros((len(cfg.ells), cfg.n_bins))
    for li, l in enumerate(cfg.ells):
        if kind in ("mid_series", "mid_series_all"):
            allp = kind == "mid_series_all"
            Dn = np.linalg.norm(D, axis=-1)
            Du = D / Dn[:, None]
            ri = np.linalg.norm(xi_, axis=-1)
            rj = np.linalg.norm(xj_, axis=-1)
            mui = np.sum(Du * xi_, axis=-1) / ri
            muj = np.sum(Du * xj_, axis=-1) / rj
            V = np.zeros(len(D))
            alphas = (range(cfg.order_lo, cfg.order + 1) if allp
                      else range(cfg.order_lo + cfg.order_lo % 2, cfg.order + 1, 2))
            for a in alphas:
                for J in range(a % 2, l + a + 1, 2):
                    Fv = coeffs.f(a, l, J) if allp else coeffs.F(a, l, J)
                    if Fv == 0.0:
                        continue
                    # Section 4.1 symmetrised form: the r2 half carries (-1)^(l+J)
                    V += 0.5 * (2 * J + 1) / (2 * l + 1) * Fv * ((Dn / (2 * ri)) ** a * legendre(J, mui)
                                                                  + (-1) ** ((l + J) % 2) * (Dn / (2 * rj)) ** a
                                                                  * legendre(J, muj))
            V = V * (2 * l + 1) / FOURPI
        else:
            V = np.zeros(len(D), dtype=np.complex128)
            for m in range(-l, l + 1):
                V += np.conj(Ylm(l, m, D)) * pair_weight(kind, l, m, xi_, xj_, cfg.order, cfg.order_lo)
            V = np.real(V)
        out[li] = np.bincount(bq, weights=ww * V, minlength=cfg.n_bins)
    with np.errstate(invalid="ignore", divide="ignore"):
        out = FOURPI / I * np.where(counts > 0, out / np.where(counts > 0, counts * H ** 3, 1), 0.0)
    return out, counts
