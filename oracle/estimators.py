"""FFT-based P_ell(k) and xi_ell(r) estimators, plain FP64 (oracle; test infrastructure only).

Each function follows the paper's boxed estimator step by step on full complex
grids, summing over every m and M:

* ``pk_bisector``  Section 5.2 boxed estimator (``pk_bisector_shells``: the same, keeping
  only the modes of the k-bins of every transform, for large meshes):
  P_l(k) = (4pi/I) <Re sum_m Y_l^{m*}(k^) sum_{beta J1 J2 M} B F[Y_J1^M d](-k) F[Y_J2^{m-M} d](k)> - d_l0 S/I.
* ``pk_midpoint``  Section 3.3 boxed parity-even estimator:
  g^alpha_{JM} = (-1)^J IFT[d*(k) F[(2r)^-alpha Y_J^M d](k)]   (Section 3.2),
  P_l(k) = (4pi/I) <Re sum_m Y_l^{m*}(k^) sum_{even alpha} sum Phi F[Y_J1^M(D^) D^alpha g^alpha_{J2,m-M}](k)> - d_l0 S/I.
* ``pk_yamamoto``  Section 2.1 Yamamoto estimator,
  P_l(k) = (4pi/I) <Re sum_m Y_l^{m*}(k^) F[Y_l^m d](k) d*(k)> - d_l0 S/I.
* ``pk_midpoint(parity="all")``  Section 3.2 boxed all-parity estimator: every alpha <= K
  (odd ones too) with the shift-theorem coefficients phi of Section 3.1 in place of Phi.
* ``xi_midpoint``  Section 4.3 boxed parity-even estimator,
  xi_l(r_a) = (4pi/I) (1/v_a) sum_{D in a} Re sum_{even alpha, J, M} F^{alpha,l}_J Y_J^{M*}(D^) D^alpha g^alpha_{JM}(D).
* ``xi_midpoint(parity="all")``  Section 4.2 boxed all-parity estimator: every alpha <= K
  with the Legendre shift coefficients f in place of F.
* ``xi_normalized``  optional, not in the paper (which divides xi_l by I and the bin volume and
  leaves the survey window): the random-pair normalisation and window correction below.
* ``xi_bisector``  Section 6 boxed estimator,
  h = IFT[F[Y_J1^M d](-k) F[Y_J2^{m-M} d](k)],
  xi_l(r_a) = (4pi/I) (1/v_a) sum_{D in a} Re sum_m Y_l^{m*}(D^) sum B h
  (``xi_bisector_streamed``: the same, with the transforms held on disk and the k-space sums
  formed slab by slab, for meshes whose transforms do not fit in host memory together).

Normalisation (reading of Section 2.1): the substitution d -> w (n_g - alpha_r n_r) / I^{1/2}
makes the 1/V of the definition inconsistent, so every estimator is divided by
I = alpha_r sum_r w_r^2 nbar_r; alpha_r = sum w_g / sum w_r (the ratio that makes the
weighted field vanish on average); the shot noise S/I, S = sum_g w_g^2 + alpha_r^2 sum_r w_r^2,
is subtracted from the monopole only.  k-shell averages are means over the modes of
the bin (the angular integral); r-bins divide by v_a = N_a H^3, the bin's volume on
the grid, and exclude the zero separation.

Series order K: midpoint keeps even alpha <= K; bisector keeps beta <= K // 2
(the beta-th bisector term is O(theta^{2 beta})).  ``Config.order_lo`` drops the terms below
a given order: the estimate then holds the terms of order order_lo .. K only (midpoint
alpha >= order_lo, bisector 2 beta >= order_lo), so order_lo = K gives the contribution of
order K alone; the shot noise belongs to order 0 and is subtracted only when order_lo = 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.fft

from . import coeffs
from .mesh import (paint, node_positions, kgrid, separation_grid, window, neg_k,
                   k_bin_index, r_bin_index, signed_index)
from .ylm import Ylm

FOURPI = 4.0 * math.pi


@dataclass
class Config:
    N: int
    L: float
    b0: tuple
    assign: int = 3
    ells: tuple = (0, 2, 4)
    order: int = 4
    compensate: bool = True
    bin_lo: float = 0.01
    bin_width: float = 0.01
    n_bins: int = 20
    order_lo: int = 0
    parity: str = "even"   # midpoint series: "even" (Sections 3.3, 4.3) or "all" (3.2, 4.2)


@dataclass
class Result:
    values: np.ndarray          # [n_ell, n_bins]
    bin_mean: np.ndarray        # mean |k| or |r| per bin
    counts: np.ndarray          # modes / separations per bin
    alpha_r: float = 0.0
    I: float = 0.0
    S: float = 0.0
    extra: dict = field(default_factory=dict)


def scalars(w_g, w_r, nbar_r):
    """alpha_r, I, S (Section 2.1 with the readings listed in the module docstring)."""
    w_g = np.asarray(w_g, dtype=np.float64)
    w_r = np.asarray(w_r, dtype=np.float64)
    nbar_r = np.asarray(nbar_r, dtype=np.float64)
    alpha_r = w_g.sum() / w_r.sum()
    I = alpha_r * np.sum(w_r * w_r * nbar_r)
    S = np.sum(w_g * w_g) + alpha_r * alpha_r * np.sum(w_r * w_r)
    return float(alpha_r), float(I), float(S)


def density_masses(gal, ran, cfg: Config, alpha_r: float) -> np.ndarray:
    """Node masses of w (n_g - alpha_r n_r)."""
    mg = paint(gal["pos"], gal["w"], cfg.N, cfg.L, cfg.b0, cfg.assign)
    mr = paint(ran["pos"], ran["w"], cfg.N, cfg.L, cfg.b0, cfg.assign)
    return mg - alpha_r * mr


def _prepare(gal, ran, cfg: Config, norm=None):
    if norm is None:
        alpha_r, I, S = scalars(gal["w"], ran["w"], ran["nbar"])
    else:
        alpha_r, I, S = norm
    m = density_masses(gal, ran, cfg, alpha_r)
    return m, alpha_r, I, S


def _compensation(cfg: Config):
    if cfg.compensate:
        return 1.0 / window(cfg.N, cfg.assign)
    return None


def fftn(x):
    """Unnormalised forward n-D DFT, numpy's sign convention (pocketfft, every host core)."""
    return scipy.fft.fftn(x, workers=-1)


def ifftn(x):
    """Inverse n-D DFT with the 1/N^3 factor, numpy's convention."""
    return scipy.fft.ifftn(x, workers=-1)


def _fft(x, comp):
    X = fftn(x)
    if comp is not None:
        X *= comp
    return X


def _bin_k(E_list, cfg: Config):
    """Shell means of Re E for each ell; k-bin from the integer |s|^2."""
    b, kmag = k_bin_index(cfg.N, cfg.L, cfg.bin_lo, cfg.bin_width, cfg.n_bins)
    bf = b.ravel()
    sel = bf >= 0
    counts = np.bincount(bf[sel], minlength=cfg.n_bins).astype(np.float64)
    ksum = np.bincount(bf[sel], weights=kmag.ravel()[sel], minlength=cfg.n_bins)
    vals = []
    for E in E_list:
        s = np.bincount(bf[sel], weights=np.real(E).ravel()[sel], minlength=cfg.n_bins)
        with np.errstate(invalid="ignore", divide="ignore"):
            vals.append(np.where(counts > 0, s / np.where(counts > 0, counts, 1), 0.0))
    with np.errstate(invalid="ignore", divide="ignore"):
        kmean = np.where(counts > 0, ksum / np.where(counts > 0, counts, 1), 0.0)
    return np.array(vals), kmean, counts


def _finish_pk(sums, kmean, counts, cfg, alpha_r, I, S, extra=None):
    """An empty bin has no estimate and is reported as 0 for every ell (no shot-noise term)."""
    P = FOURPI / I * sums
    for i, l in enumerate(cfg.ells):
        if l == 0 and cfg.order_lo == 0:
            P[i] -= np.where(counts > 0, S / I, 0.0)
    return Result(P, kmean, counts.astype(np.int64), alpha_r, I, S, extra or {})


# ----------------------------------------------------------------------------
# Power spectrum
# ----------------------------------------------------------------------------

def _alphas(cfg: Config):
    """Midpoint series orders kept: alpha in [order_lo, order], even ones only for the
    parity-even form."""
    step = 1 if cfg.parity == "all" else 2
    return [a for a in range(0, cfg.order + 1, step) if a >= cfg.order_lo]


def _mid_table(cfg: Config, alpha: int, l: int, m: int) -> dict:
    """Coupling of the midpoint P_l at order alpha: phi (all-parity) or Phi (parity-even)."""
    if cfg.parity == "all":
        return coeffs.phi_table(alpha, l, m)
    return coeffs.Phi_table(alpha, l, m)


def _beta_lo(cfg: Config) -> int:
    """Lowest bisector order kept: the beta-th term is of order theta^(2 beta)."""
    return (cfg.order_lo + 1) // 2


def pk_bisector(gal, ran, cfg: Config, norm=None, beta_max=None) -> Result:
    m, alpha_r, I, S = _prepare(gal, ran, cfg, norm)
    if beta_max is None:
        beta_max = cfg.order // 2
    comp = _compensation(cfg)
    xn = node_positions(cfg.N, cfg.L, cfg.b0)
    _, kvec = kgrid(cfg.N, cfg.L)
    Jmax = max(cfg.ells) + beta_max
    Qt = {}
    for J in range(Jmax + 1):
        for M in range(-J, J + 1):
            Qt[(J, M)] = _fft(m * Ylm(J, M, xn), comp)
    Qneg = {key: neg_k(v) for key, v in Qt.items()}
    E_list = []
    for l in cfg.ells:
        E = np.zeros_like(m, dtype=np.complex128)
        for mm in range(-l, l + 1):
            tab = coeffs.B_table(beta_max, l, mm, _beta_lo(cfg))
            inner = np.zeros_like(E)
            for (J1, J2, M), c in tab.items():
                inner += c * Qneg[(J1, M)] * Qt[(J2, mm - M)]
            E += np.conj(Ylm(l, mm, kvec)) * inner
        E_list.append(E)
    sums, kmean, counts = _bin_k(E_list, cfg)
    return _finish_pk(sums, kmean, counts, cfg, alpha_r, I, S)


def pk_bisector_shells(gal, ran, cfg: Config, norm=None, beta_max=None) -> Result:
    """pk_bisector with the memory of the retained modes only: the same steps (Section 5.2
    boxed estimator), but each transform is reduced to the modes of the k-bins right after it
    is computed.  Q(-k) of a retained mode is read at the index (-n) mod N, which is retained
    too (same |k|).  For meshes whose full set of transforms does not fit in host memory."""
    m, alpha_r, I, S = _prepare(gal, ran, cfg, norm)
    if beta_max is None:
        beta_max = cfg.order // 2
    N = cfg.N
    b, kmag = k_bin_index(N, cfg.L, cfg.bin_lo, cfg.bin_width, cfg.n_bins)
    sel = np.flatnonzero(b.ravel() >= 0)
    b_sel = b.ravel()[sel]
    k_sel = kmag.ravel()[sel]
    del b, kmag
    ix, iy, iz = np.unravel_index(sel, (N, N, N))
    neg = np.ravel_multi_index(((-ix) % N, (-iy) % N, (-iz) % N), (N, N, N))
    perm = np.searchsorted(sel, neg)          # Q(-k) of retained mode i is Q_sel[perm[i]]
    assert np.array_equal(sel[perm], neg)
    s = signed_index(N)
    kf = 2.0 * np.pi / cfg.L
    kvec_sel = np.stack([s[ix], s[iy], s[iz]], axis=-1) * kf
    del ix, iy, iz, neg
    comp_sel = None
    if cfg.compensate:
        comp_sel = (1.0 / window(N, cfg.assign)).ravel()[sel]
    xn = node_positions(N, cfg.L, cfg.b0)
    Jmax = max(cfg.ells) + beta_max
    Qs = {}
    for J in range(Jmax + 1):
        for M in range(-J, J + 1):
            X = fftn(m * Ylm(J, M, xn)).ravel()[sel]
            Qs[(J, M)] = X * comp_sel if comp_sel is not None else X
    del xn
    E_list = []
    for l in cfg.ells:
        E = np.zeros(len(sel), dtype=np.complex128)
        for mm in range(-l, l + 1):
            tab = coeffs.B_table(beta_max, l, mm, _beta_lo(cfg))
            inner = np.zeros(len(sel), dtype=np.complex128)
            for (J1, J2, M), c in tab.items():
                inner += c * Qs[(J1, M)][perm] * Qs[(J2, mm - M)]
            E += np.conj(Ylm(l, mm, kvec_sel)) * inner
        E_list.append(E)
    counts = np.bincount(b_sel, minlength=cfg.n_bins).astype(np.float64)
    ksum = np.bincount(b_sel, weights=k_sel, minlength=cfg.n_bins)
    vals = []
    for E in E_list:
        sm = np.bincount(b_sel, weights=np.real(E), minlength=cfg.n_bins)
        with np.errstate(invalid="ignore", divide="ignore"):
            vals.append(np.where(counts > 0, sm / np.where(counts > 0, counts, 1), 0.0))
    with np.errstate(invalid="ignore", divide="ignore"):
        kmean = np.where(counts > 0, ksum / np.where(counts > 0, counts, 1), 0.0)
    return _finish_pk(np.array(vals), kmean, counts, cfg, alpha_r, I, S)


def g_field(m, dtil, xn, alpha: int, J: int, M: int, comp):
    """g^alpha_{JM}(D) = (-1)^J IFT[d*(k) F[(2r)^-alpha Y_J^M d](k)]  (Section 3.2), on the
    separation grid (index n <-> D = H s(n)).  (2r)^-alpha is set to 0 at r = 0."""
    r = np.sqrt(np.sum(xn * xn, axis=-1))
    if alpha == 0:
        rw = np.ones_like(r)
    else:
        with np.errstate(divide="ignore"):
            rw = np.where(r > 0, (2.0 * r) ** (-float(alpha)), 0.0)
    Q = m * rw * Ylm(J, M, xn)
    Qt = _fft(Q, comp)
    g = ifftn(np.conj(dtil) * Qt)
    return (-1) ** J * g


def pk_midpoint(gal, ran, cfg: Config, norm=None) -> Result:
    m, alpha_r, I, S = _prepare(gal, ran, cfg, norm)
    comp = _compensation(cfg)
    xn = node_positions(cfg.N, cfg.L, cfg.b0)
    _, kvec = kgrid(cfg.N, cfg.L)
    Dvec = separation_grid(cfg.N, cfg.L)
    Dmag = np.sqrt(np.sum(Dvec * Dvec, axis=-1))
    dtil = _fft(m, comp)
    alphas = _alphas(cfg)
    # Phi tables per (l, m, alpha), and the g fields they need
    tabs = {(l, mm, a): _mid_table(cfg, a, l, mm)
            for l in cfg.ells for mm in range(-l, l + 1) for a in alphas}
    need = {}
    for (l, mm, a), tab in tabs.items():
        for (J1, J2, M), c in tab.items():
            need.setdefault((a, J2, mm - M), []).append((l, mm, J1, M, c))
    Ycache = {}

    def YD(J, M):
        if (J, M) not in Ycache:
            Ycache[(J, M)] = Ylm(J, M, Dvec)
        return Ycache[(J, M)]

    A = {(l, mm): np.zeros(m.shape, dtype=np.complex128) for l in cfg.ells for mm in range(-l, l + 1)}
    for (a, J2, M2), users in sorted(need.items()):
        g = g_field(m, dtil, xn, a, J2, M2, comp)
        Da = Dmag ** a if a > 0 else 1.0
        for (l, mm, J1, M, c) in users:
            A[(l, mm)] += c * YD(J1, M) * Da * g
    E_list = []
    for l in cfg.ells:
        E = np.zeros(m.shape, dtype=np.complex128)
        for mm in range(-l, l + 1):
            E += np.conj(Ylm(l, mm, kvec)) * fftn(A[(l, mm)])
        E_list.append(E)
    sums, kmean, counts = _bin_k(E_list, cfg)
    return _finish_pk(sums, kmean, counts, cfg, alpha_r, I, S)


def pk_yamamoto(gal, ran, cfg: Config, norm=None) -> Result:
    m, alpha_r, I, S = _prepare(gal, ran, cfg, norm)
    comp = _compensation(cfg)
    xn = node_positions(cfg.N, cfg.L, cfg.b0)
    _, kvec = kgrid(cfg.N, cfg.L)
    dtil = _fft(m, comp)
    E_list = []
    for l in cfg.ells:
        E = np.zeros(m.shape, dtype=np.complex128)
        for mm in range(-l, l + 1):
            E += np.conj(Ylm(l, mm, kvec)) * _fft(m * Ylm(l, mm, xn), comp) * np.conj(dtil)
        E_list.append(E)
    sums, kmean, counts = _bin_k(E_list, cfg)
    return _finish_pk(sums, kmean, counts, cfg, alpha_r, I, S)


# ----------------------------------------------------------------------------
# Correlation function
# ----------------------------------------------------------------------------

def _bin_r(X_list, cfg: Config):
    b, rmag = r_bin_index(cfg.N, cfg.L, cfg.bin_lo, cfg.bin_width, cfg.n_bins)
    bf = b.ravel()
    sel = bf >= 0
    counts = np.bincount(bf[sel], minlength=cfg.n_bins).astype(np.float64)
    rsum = np.bincount(bf[sel], weights=rmag.ravel()[sel], minlength=cfg.n_bins)
    vals = []
    for X in X_list:
        vals.append(np.bincount(bf[sel], weights=np.real(X).ravel()[sel], minlength=cfg.n_bins))
    with np.errstate(invalid="ignore", divide="ignore"):
        rmean = np.where(counts > 0, rsum / np.where(counts > 0, counts, 1), 0.0)
    return np.array(vals), rmean, counts


def _finish_xi(sums, rmean, counts, cfg, alpha_r, I, S):
    H3 = (cfg.L / cfg.N) ** 3
    with np.errstate(invalid="ignore", divide="ignore"):
        vol = np.where(counts > 0, counts * H3, 1.0)
    xi = FOURPI / I * sums / vol[None, :]
    xi[:, counts == 0] = 0.0
    return Result(xi, rmean, counts.astype(np.int64), alpha_r, I, S)


def xi_midpoint(gal, ran, cfg: Config, norm=None) -> Result:
    m, alpha_r, I, S = _prepare(gal, ran, cfg, norm)
    comp = _compensation(cfg)
    xn = node_positions(cfg.N, cfg.L, cfg.b0)
    Dvec = separation_grid(cfg.N, cfg.L)
    Dmag = np.sqrt(np.sum(Dvec * Dvec, axis=-1))
    dtil = _fft(m, comp)
    X = {l: np.zeros(m.shape, dtype=np.complex128) for l in cfg.ells}
    for a in _alphas(cfg):
        Da = Dmag ** a if a > 0 else 1.0
        # J has the parity of alpha (even l): f^{alpha,l}_J vanishes unless alpha + l + J is even
        for J in range(a % 2, max(cfg.ells) + a + 1, 2):
            if cfg.parity == "all":
                Fs = {l: coeffs.f(a, l, J) for l in cfg.ells}
            else:
                Fs = {l: coeffs.F(a, l, J) for l in cfg.ells}
            if all(v == 0.0 for v in Fs.values()):
                continue
            for M in range(-J, J + 1):
                g = g_field(m, dtil, xn, a, J, M, comp)
                t = np.conj(Ylm(J, M, Dvec)) * Da * g
                for l, Fv in Fs.items():
                    if Fv != 0.0:
                        X[l] += Fv * t
    sums, rmean, counts = _bin_r([X[l] for l in cfg.ells], cfg)
    return _finish_xi(sums, rmean, counts, cfg, alpha_r, I, S)


def xi_bisector(gal, ran, cfg: Config, norm=None, beta_max=None) -> Result:
    m, alpha_r, I, S = _prepare(gal, ran, cfg, norm)
    if beta_max is None:
        beta_max = cfg.order // 2
    comp = _compensation(cfg)
    xn = node_positions(cfg.N, cfg.L, cfg.b0)
    Dvec = separation_grid(cfg.N, cfg.L)
    Jmax = max(cfg.ells) + beta_max
    Qt = {}
    for J in range(Jmax + 1):
        for M in range(-J, J + 1):
            Qt[(J, M)] = _fft(m * Ylm(J, M, xn), comp)
    Qneg = {key: neg_k(v) for key, v in Qt.items()}
    X_list = []
    for l in cfg.ells:
        X = np.zeros(m.shape, dtype=np.complex128)
        for mm in range(-l, l + 1):
            tab = coeffs.B_table(beta_max, l, mm, _beta_lo(cfg))
            Kprod = np.zeros(m.shape, dtype=np.complex128)
            for (J1, J2, M), c in tab.items():
                Kprod += c * Qneg[(J1, M)] * Qt[(J2, mm - M)]
            Hlm = ifftn(Kprod)
            X += np.conj(Ylm(l, mm, Dvec)) * Hlm
        X_list.append(X)
    sums, rmean, counts = _bin_r(X_list, cfg)
    return _finish_xi(sums, rmean, counts, cfg, alpha_r, I, S)


def xi_bisector_streamed(gal, ran, cfg: Config, workdir: str, norm=None, beta_max=None,
                         slab: int = 16) -> Result:
    """xi_bisector for meshes whose transforms do not fit in host memory together (Section 6
    boxed estimator, the same steps).

    * Each transform F[Y_J^M d] with M >= 0 is computed once and written to a disk-backed array
      (np.memmap under `workdir`).  Those with M < 0 follow from Y_J^{-M} = (-1)^M conj(Y_J^M)
      and the reality of the density: F[Y_J^{-M} d](k) = (-1)^M conj(F[Y_J^M d](-k)).
    * The k-space sums K_lm = sum_{beta J1 J2 M} B Q(-k) Q(k) are formed for one slab of the
      first k index at a time (rows k and, for Q(-k), the mirrored rows (-n) mod N).
    * The inverse DFT is separable: each slab is transformed over the last two axes, the
      separations |D| > r_max (beyond the last bin) are dropped on those axes, and the first
      axis is transformed once every slab is in.  The 1/N^3 factor is split 1/N^2, 1/N.
    * Binning is the full-grid rule (r_bin_index) restricted to the kept separations, which
      hold every binned one."""
    import os
    m, alpha_r, I, S = _prepare(gal, ran, cfg, norm)
    if beta_max is None:
        beta_max = cfg.order // 2
    N = cfg.N
    H = cfg.L / N
    comp = _compensation(cfg)
    Jmax = max(cfg.ells) + beta_max
    xn = node_positions(N, cfg.L, cfg.b0)
    files = {}
    for J in range(Jmax + 1):
        for M in range(0, J + 1):
            path = os.path.join(workdir, f"spectrum_J{J}_M{M}.c128")
            arr = np.memmap(path, dtype=np.complex128, mode="w+", shape=(N, N, N))
            arr[...] = _fft(m * Ylm(J, M, xn), comp)
            arr.flush()
            del arr
            files[(J, M)] = path
    del xn, m
    spec = {key: np.memmap(p, dtype=np.complex128, mode="r", shape=(N, N, N)) for key, p in files.items()}

    # separations kept on each axis: signed index s with |s| H < r_max
    r_max = cfg.bin_lo + cfg.n_bins * cfg.bin_width
    w = min(int(math.ceil(r_max / H)), N // 2 - 1)
    keep_s = np.arange(-w, w + 1)
    keep = keep_s % N
    targets = [(l, mm) for l in cfg.ells for mm in range(-l, l + 1)]
    tabs = {(l, mm): coeffs.B_table(beta_max, l, mm, _beta_lo(cfg)) for (l, mm) in targets}
    acc = {t: np.zeros((N, len(keep), len(keep)), dtype=np.complex128) for t in targets}

    def neg_yz(X):
        # X at index (-n) mod N on the last two axes
        return np.roll(X[:, ::-1, ::-1], 1, axis=(1, 2))

    for a in range(0, N, slab):
        rows = np.arange(a, min(a + slab, N))
        mirror = (-rows) % N
        Qk, Qmk = {}, {}
        for (J, M), arr in spec.items():
            at_k = np.array(arr[rows])                 # F[Y_J^M d](k), k in the slab
            at_mk = neg_yz(np.array(arr[mirror]))      # F[Y_J^M d](-k)
            Qk[(J, M)], Qmk[(J, M)] = at_k, at_mk
            if M > 0:
                sgn = -1.0 if M % 2 else 1.0
                Qk[(J, -M)] = sgn * np.conj(at_mk)
                Qmk[(J, -M)] = sgn * np.conj(at_k)
        for t in targets:
            Kp = np.zeros((len(rows), N, N), dtype=np.complex128)
            for (J1, J2, M), c in tabs[t].items():
                Kp += c * Qmk[(J1, M)] * Qk[(J2, t[1] - M)]
            h = scipy.fft.ifft2(Kp, axes=(1, 2), workers=-1)
            acc[t][rows] = h[:, keep][:, :, keep]
        del Qk, Qmk
    del spec
    for p in files.values():
        os.remove(p)

    s1 = keep_s * H
    D = np.stack(np.meshgrid(s1, s1, s1, indexing="ij"), axis=-1)
    b_full, r_full = r_bin_index(N, cfg.L, cfg.bin_lo, cfg.bin_width, cfg.n_bins)
    b = b_full[np.ix_(keep, keep, keep)]
    rmag = r_full[np.ix_(keep, keep, keep)]
    counts = np.bincount(b[b >= 0], minlength=cfg.n_bins).astype(np.float64)
    assert np.array_equal(counts, np.bincount(b_full[b_full >= 0], minlength=cfg.n_bins)), \
        "kept separations must hold every binned one"
    del b_full, r_full
    sel = b >= 0
    X_vals = []
    for l in cfg.ells:
        X = np.zeros(b.shape, dtype=np.complex128)
        for mm in range(-l, l + 1):
            Hlm = scipy.fft.ifft(acc[(l, mm)], axis=0, workers=-1)[keep]
            X += np.conj(Ylm(l, mm, D)) * Hlm
        X_vals.append(np.bincount(b[sel], weights=np.real(X)[sel], minlength=cfg.n_bins))
    rsum = np.bincount(b[sel], weights=rmag[sel], minlength=cfg.n_bins)
    with np.errstate(invalid="ignore", divide="ignore"):
        rmean = np.where(counts > 0, rsum / np.where(counts > 0, counts, 1), 0.0)
    return _finish_xi(np.array(X_vals), rmean, counts, cfg, alpha_r, I, S)


# ----------------------------------------------------------------------------
# Correlation function: random-pair normalisation and window (edge) correction
# ----------------------------------------------------------------------------
# The paper normalises xi_l by I and the bin volume and leaves the survey window alone.  The
# optional normalisation below divides by the random-pair count of the bin instead (as
# Landy-Szalay pair counts do) and removes the window's mixing of multipoles:
#   N_l(a)  = sum over separations in bin a of the estimator's pair sum (the same quantity
#             xi_l holds before its 1/(I v_a)), i.e. xi_l(a) * I * v_a;
#   R_L(a)  = the same pair sum for the randoms alone, w alpha_r n_r (L = 0 is the weighted
#             random-pair count RR of the bin), i.e. xi_L^R(a) * I * v_a;
#   writing RR(mu) = sum_L R_L L_L(mu) and xi(mu) = sum_l' xi_l' L_l'(mu), the data pair sum
#   N_l = (2l+1) < L_l RR xi > gives
#     N_l / R_0 = sum_l' M_{l l'} xi_l',  M_{l l'} = (2l+1) sum_L (l L l'; 0 0 0)^2 f_L,
#   with f_L = R_L / R_0 (f_0 = 1); the window-corrected multipoles solve this system in
#   every bin, and N_l / R_0 alone is the random-pair normalised estimate.

def _empty(gal):
    return {k: np.zeros((0,) + np.asarray(v).shape[1:]) for k, v in gal.items()}


def xi_window(gal, ran, cfg: Config, estimator, norm=None, L_max=None) -> Result:
    """Random-pair multipoles xi_L^R (L = 0, 2, .., L_max; default 2 ell_max): `estimator`
    (xi_midpoint or xi_bisector) on the randoms alone, alpha_r w n_r, with the data's
    alpha_r, I, S, so that the results share the data's 1 / (I v_a)."""
    if norm is None:
        norm = scalars(gal["w"], ran["w"], ran["nbar"])
    if L_max is None:
        L_max = 2 * max(cfg.ells)
    wcfg = Config(**{**cfg.__dict__, "ells": tuple(range(0, L_max + 1, 2))})
    return estimator(_empty(gal), ran, wcfg, norm)


def xi_window_matrix(ells, f):
    """M_{l l'} = (2l+1) sum_L (l L l'; 0 0 0)^2 f_L for one bin; f maps even L to f_L."""
    M = np.zeros((len(ells), len(ells)))
    for i, l in enumerate(ells):
        for j, lp in enumerate(ells):
            tot = 0.0
            for L, fL in f.items():
                w = coeffs.wigner3j(l, L, lp, 0, 0, 0)
                tot += w * w * fL
            M[i, j] = (2 * l + 1) * tot
    return M


def xi_normalized(gal, ran, cfg: Config, estimator, norm=None, L_max=None):
    """(xi_RR, xi_edge, f): xi_RR[l][a] = N_l / R_0, xi_edge[l][a] the window-corrected
    multipoles (M^-1 N / R_0, windows f_L up to L_max), f[L][a] = R_L / R_0.  Bins without
    random pairs are 0."""
    if norm is None:
        norm = scalars(gal["w"], ran["w"], ran["nbar"])
    data = estimator(gal, ran, cfg, norm).values
    win = xi_window(gal, ran, cfg, estimator, norm, L_max).values
    Ls = list(range(0, win.shape[0] * 2, 2))
    nb = data.shape[1]
    xr = np.zeros_like(data)
    xe = np.zeros_like(data)
    f = np.zeros_like(win)
    for a in range(nb):
        R0 = win[0, a]
        if R0 == 0.0:
            continue
        xr[:, a] = data[:, a] / R0
        f[:, a] = win[:, a] / R0
        M = xi_window_matrix(list(cfg.ells), {L: f[i, a] for i, L in enumerate(Ls)})
        xe[:, a] = np.linalg.solve(M, xr[:, a])
    return xr, xe, f
