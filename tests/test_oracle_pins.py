"""Pins of the oracle's normalisation, painting, compensation window and binning against what
Section 2.1 and plain mathematics fix, independently of the oracle's own formulas:

* alpha_r (Section 2.1): the weighted density w (n_g - alpha_r n_r) carries zero total mass;
* I (Section 2.1, the integral of w^2 nbar^2): for a survey of constant density and weight it is
  w^2 nbar^2 V;
* S (the shot noise Section 2.1 sets aside): it is the self-pair part of the pair sum, so the
  monopole with S/I subtracted equals a brute-force sum over pairs i != j;
* the painting kernel and the compensation window of the footnote in Section 2.1 together:
  averaged over the particle's position inside its cell, the DFT of a particle's painted masses,
  phase-referenced to the particle, is the Fourier transform of the assignment kernel,
  prod_i sinc(k_i H / 2)^p (p-fold convolution of the cell's top hat);
* k- and r-bins: modes and separations counted by direct enumeration of integer vectors.

Each pin also runs against patched copies of the oracle, each carrying one plausible mistake
(named in the parametrisation), and must reject every one of them."""
import inspect
import itertools
import math
import sys
import textwrap

import numpy as np
import pytest

from oracle import estimators as est
from oracle import mesh
from oracle.estimators import Config, scalars, density_masses, pk_yamamoto, xi_midpoint
from oracle.mesh import CIC, TSC
from synthetic import tiny_node_catalog


def _patched(func, old, new):
    """A copy of `func` with the source text `old` replaced by `new` (exactly one occurrence),
    executed in a copy of its module's namespace."""
    src = textwrap.dedent(inspect.getsource(func))
    assert src.count(old) == 1, (func.__name__, old)
    ns = dict(vars(sys.modules[func.__module__]))
    exec(compile(src.replace(old, new), f"<patched {func.__name__}>", "exec"), ns)
    return ns[func.__name__]


# ---------------------------------------------------------------- alpha_r: zero total mass

def _mass_residual(scalars_fn=scalars, masses_fn=density_masses):
    """max over CIC/TSC of |sum_n m_n| / sum |w|, m = w (n_g - alpha_r n_r) in node masses."""
    rng = np.random.default_rng(41)
    c = np.array([0.0, 0.0, 1200.0])
    gal = {"pos": c + rng.uniform(-300, 300, (500, 3)), "w": rng.uniform(0.2, 1.8, 500)}
    ran = {"pos": c + rng.uniform(-300, 300, (2100, 3)), "w": rng.uniform(0.5, 3.0, 2100),
           "nbar": np.full(2100, 3e-5)}
    alpha_r, _, _ = scalars_fn(gal["w"], ran["w"], ran["nbar"])
    worst = 0.0
    for assign in (CIC, TSC):
        cfg = Config(N=32, L=1000.0, b0=(-500.0, -500.0, 700.0), assign=assign)
        m = masses_fn(gal, ran, cfg, alpha_r)
        worst = max(worst, abs(m.sum()) / (gal["w"].sum() + alpha_r * ran["w"].sum()))
    return worst


def test_density_has_zero_mass():
    assert _mass_residual() < 1e-13


@pytest.mark.parametrize("mistake", ["alpha_r inverted (randoms over galaxies)",
                                     "alpha_r unweighted (count ratio)",
                                     "randoms added instead of subtracted"])
def test_density_mass_pin_rejects(mistake):
    if mistake.startswith("alpha_r inverted"):
        r = _mass_residual(scalars_fn=_patched(scalars, "alpha_r = w_g.sum() / w_r.sum()",
                                               "alpha_r = w_r.sum() / w_g.sum()"))
    elif mistake.startswith("alpha_r unweighted"):
        r = _mass_residual(scalars_fn=_patched(scalars, "alpha_r = w_g.sum() / w_r.sum()",
                                               "alpha_r = len(w_g) / len(w_r)"))
    else:
        r = _mass_residual(masses_fn=_patched(density_masses, "return mg - alpha_r * mr",
                                              "return mg + alpha_r * mr"))
    assert r > 1e-3, mistake


# ---------------------------------------------------------------- I: closed form

def _I_gap(scalars_fn=scalars):
    """max relative |I - w^2 nbar^2 V| over uniform surveys of constant weight (every particle
    carries w and nbar = N_g / V)."""
    worst = 0.0
    for n_g, n_r, side, w in ((1000, 5000, 400.0, 0.3), (777, 12000, 900.0, 2.5), (50, 51, 100.0, 0.7)):
        V = side ** 3
        nbar = n_g / V
        _, I, _ = scalars_fn(np.full(n_g, w), np.full(n_r, w), np.full(n_r, nbar))
        ref = w * w * nbar * nbar * V
        worst = max(worst, abs(I - ref) / ref)
    return worst


def test_normalisation_I_is_integral_of_w2_nbar2():
    assert _I_gap() < 1e-13


@pytest.mark.parametrize("old,new", [
    ("alpha_r = w_g.sum() / w_r.sum()", "alpha_r = w_r.sum() / w_g.sum()"),
    ("I = alpha_r * np.sum(w_r * w_r * nbar_r)", "I = alpha_r * np.sum(w_r * nbar_r)"),
    ("I = alpha_r * np.sum(w_r * w_r * nbar_r)", "I = alpha_r * alpha_r * np.sum(w_r * w_r * nbar_r)"),
    ("I = alpha_r * np.sum(w_r * w_r * nbar_r)", "I = alpha_r * np.sum(w_r * w_r * nbar_r * nbar_r)"),
], ids=["alpha inverted", "w not squared", "alpha squared", "nbar squared"])
def test_normalisation_I_pin_rejects(old, new):
    assert _I_gap(_patched(scalars, old, new)) > 1e-3


# ---------------------------------------------------------------- S: self pairs

NS, LS, B0S = 16, 1000.0, (-500.0, -500.0, 1000.0)


def _modes_by_bin(N, L, lo, width, n_bins):
    """Integer mode vectors of every k-bin, by enumeration: lo + q w <= |k| < lo + (q+1) w."""
    kf = 2.0 * math.pi / L
    out = [[] for _ in range(n_bins)]
    half = N // 2
    for s in itertools.product(range(-half, half), repeat=3):
        kk = kf * math.sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2])
        for q in range(n_bins):
            if lo + q * width <= kk < lo + (q + 1) * width:
                out[q].append(s)
    return [np.array(v, dtype=np.int64).reshape(-1, 3) for v in out]


def _shot_noise_gap(scalars_fn=scalars):
    """Monopole of node-placed particles (CIC, no compensation) against
    (1 / (I N_b)) sum_{k in b} sum_{i != j} w_i w_j cos(k . (x_i - x_j)), signed weights
    (w for galaxies, -alpha_r w for randoms); self pairs left out term by term."""
    gal, ran = tiny_node_catalog(31, NS, LS, B0S, n_gal=40, n_ran=160)
    norm = scalars_fn(gal["w"], ran["w"], ran["nbar"])
    alpha_r, I, _ = norm
    cfg = Config(N=NS, L=LS, b0=B0S, assign=CIC, ells=(0,), order=0, compensate=False,
                 bin_lo=0.005, bin_width=0.01, n_bins=4)
    got = pk_yamamoto(gal, ran, cfg, norm).values[0]
    pos = np.concatenate([gal["pos"], ran["pos"]])
    w = np.concatenate([gal["w"], -alpha_r * ran["w"]])
    n = np.rint((pos - np.asarray(B0S)) / (LS / NS)).astype(np.int64)
    P = len(w)
    off = ~np.eye(P, dtype=bool)
    D = (n[:, None, :] - n[None, :, :])[off]          # [pairs, 3], i != j
    ww = (w[:, None] * w[None, :])[off]
    ref = np.zeros(cfg.n_bins)
    for q, modes in enumerate(_modes_by_bin(NS, LS, cfg.bin_lo, cfg.bin_width, cfg.n_bins)):
        tot = 0.0
        for s in modes:
            tot += np.sum(ww * np.cos(2.0 * math.pi / NS * (D @ s)))
        ref[q] = tot / (I * len(modes))
    return np.max(np.abs(got - ref)) / np.max(np.abs(ref))


def test_shot_noise_is_the_self_pair_sum():
    assert _shot_noise_gap() < 1e-12


@pytest.mark.parametrize("new", ["S = np.sum(w_g * w_g) + alpha_r * np.sum(w_r * w_r)",
                                 "S = np.sum(w_g * w_g) + np.sum(w_r * w_r)",
                                 "S = np.sum(w_g * w_g)"],
                         ids=["alpha not squared", "alpha left out", "randoms left out"])
def test_shot_noise_pin_rejects(new):
    bad = _patched(scalars, "S = np.sum(w_g * w_g) + alpha_r * alpha_r * np.sum(w_r * w_r)", new)
    assert _shot_noise_gap(bad) > 1e-4


# ---------------------------------------------------------------- paint kernel + window

NW, LW, B0W, N0W = 8, 800.0, (-400.0, -400.0, 300.0), np.array([3, 4, 2])
S_SAMPLE = (0, 1, -2, 3, -4)        # signed k indices per axis, Nyquist (-4) included


def _window_gap(assign, paint_fn=mesh.paint, window_fn=mesh.window, nq=10):
    """max_k |A(k) - W(k)|, A(k) = int_[0,1)^3 d^3u sum_n m_n(u) exp(-i k.(n - n0 - u) H), the
    painted masses m(u) of a unit particle at b0 + (n0 + u) H; the cell average is taken by
    Gauss-Legendre quadrature on [0, 1/2] and [1/2, 1] per axis (the kernels are polynomial on
    each piece), and the phase-weighted sum over quadrature points is painted in one go (painting
    is linear in the weights)."""
    x, wq = np.polynomial.legendre.leggauss(nq)
    u1 = np.concatenate([0.25 + 0.25 * x, 0.75 + 0.25 * x])
    w1 = np.concatenate([0.25 * wq, 0.25 * wq])
    U = np.stack(np.meshgrid(u1, u1, u1, indexing="ij"), axis=-1).reshape(-1, 3)
    Wq = (w1[:, None, None] * w1[None, :, None] * w1[None, None, :]).ravel()
    H = LW / NW
    pos = np.asarray(B0W)[None, :] + (N0W[None, :] + U) * H
    W = window_fn(NW, assign)
    n = np.arange(NW)
    worst = 0.0
    for s in itertools.product(S_SAMPLE, repeat=3):
        kH = 2.0 * math.pi * np.array(s, dtype=np.float64) / NW
        phase = np.exp(1j * ((N0W[None, :] + U) @ kH))
        M = (paint_fn(pos, Wq * phase.real, NW, LW, B0W, assign)
             + 1j * paint_fn(pos, Wq * phase.imag, NW, LW, B0W, assign))
        e = [np.exp(-1j * kH[a] * n) for a in range(3)]
        A = np.einsum("abc,a,b,c->", M, e[0], e[1], e[2])
        worst = max(worst, abs(A - W[s[0] % NW, s[1] % NW, s[2] % NW]))
    return worst


@pytest.mark.parametrize("assign", [CIC, TSC], ids=["CIC", "TSC"])
def test_window_is_cell_average_of_painted_phase(assign):
    assert _window_gap(assign) < 1e-13


PAINT_TSC = "taps = [(-1, 0.5 * (0.5 - d) ** 2), (0, 0.75 - d * d), (1, 0.5 * (0.5 + d) ** 2)]"
MISTAKES = {
    "TSC outer taps swapped": (TSC, "paint", PAINT_TSC,
                               "taps = [(-1, 0.5 * (0.5 + d) ** 2), (0, 0.75 - d * d), (1, 0.5 * (0.5 - d) ** 2)]"),
    "TSC anchored at floor(u)": (TSC, "paint", "i0 = np.floor(u + 0.5).astype(np.int64)",
                                 "i0 = np.floor(u).astype(np.int64)"),
    "CIC taps swapped": (CIC, "paint", "taps = [(0, 1.0 - d), (1, d)]", "taps = [(0, d), (1, 1.0 - d)]"),
    "CIC anchored at round(u)": (CIC, "paint", "i0 = np.floor(u).astype(np.int64)",
                                 "i0 = np.rint(u).astype(np.int64)"),
    "window sinc(kH)": (TSC, "window", "x = np.pi * s / N", "x = 2.0 * np.pi * s / N"),
    "window p swapped (CIC)": (CIC, "window", "w1 = sn ** assign", "w1 = sn ** (5 - assign)"),
    "window p swapped (TSC)": (TSC, "window", "w1 = sn ** assign", "w1 = sn ** (5 - assign)"),
}


@pytest.mark.parametrize("mistake", list(MISTAKES))
def test_window_pin_rejects(mistake):
    assign, which, old, new = MISTAKES[mistake]
    if which == "paint":
        gap = _window_gap(assign, paint_fn=_patched(mesh.paint, old, new))
    else:
        gap = _window_gap(assign, window_fn=_patched(mesh.window, old, new))
    assert gap > 1e-3, mistake


# ---------------------------------------------------------------- k- and r-bins by enumeration

KB = dict(N=16, L=1000.0, lo=0.004, width=0.0071, n_bins=7)     # last bins straddle k_Nyq


def _k_bins_enumerated(N, L, lo, width, n_bins):
    modes = _modes_by_bin(N, L, lo, width, n_bins)
    kf = 2.0 * math.pi / L
    counts = np.array([len(m) for m in modes])
    mean = np.array([np.mean(kf * np.sqrt(np.sum(m * m, axis=1))) if len(m) else 0.0 for m in modes])
    return counts, mean


def _k_bin_gap(bin_fn=mesh.k_bin_index):
    N, L, lo, width, nb = KB["N"], KB["L"], KB["lo"], KB["width"], KB["n_bins"]
    counts, mean = _k_bins_enumerated(N, L, lo, width, nb)
    b, kmag = bin_fn(N, L, lo, width, nb)
    c2 = np.bincount(b[b >= 0], minlength=nb)
    m2 = np.bincount(b[b >= 0], weights=kmag[b >= 0], minlength=nb) / np.maximum(c2, 1)
    return int(np.sum(np.abs(c2 - counts))), float(np.max(np.abs(m2 - mean)))


def test_k_bins_by_enumeration():
    dc, dm = _k_bin_gap()
    assert dc == 0 and dm < 1e-15
    # the estimators report the same counts and mean |k|
    N, L = KB["N"], KB["L"]
    counts, mean = _k_bins_enumerated(N, L, KB["lo"], KB["width"], KB["n_bins"])
    gal, ran = tiny_node_catalog(3, N, L, (-500.0, -500.0, 1000.0))
    r = pk_yamamoto(gal, ran, Config(N=N, L=L, b0=(-500.0, -500.0, 1000.0), assign=CIC, ells=(0,),
                                     order=0, bin_lo=KB["lo"], bin_width=KB["width"],
                                     n_bins=KB["n_bins"]))
    assert np.array_equal(r.counts, counts)
    assert np.allclose(r.bin_mean, mean, rtol=1e-14, atol=0)


@pytest.mark.parametrize("old,new", [
    ("b = np.floor(t / dk)", "b = np.rint(t / dk)"),
    ("kmag = (2.0 * np.pi / L) * np.sqrt(s2)", "kmag = (np.pi / L) * np.sqrt(s2)"),
    ("(SX, SY, SZ), _ = kgrid(N, L)",
     "SX, SY, SZ = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing='ij')"),
    ("b = np.where((b >= 0) & (b < nbins), b, -1)", "b = np.where((b >= 0) & (b <= nbins), b, -1)"),
], ids=["rounded bin", "half k", "unsigned indices", "one bin too many"])
def test_k_bin_pin_rejects(old, new):
    bad = _patched(mesh.k_bin_index, old, new)
    try:
        dc, dm = _k_bin_gap(bad)
    except (ValueError, IndexError):
        return                      # a bin index outside the bins: rejected as well
    assert dc > 0 or dm > 1e-9


RB = dict(N=16, L=1000.0, lo=30.0, width=73.0, n_bins=6)


def _r_bins_enumerated(N, L, lo, width, n_bins):
    H = L / N
    counts = np.zeros(n_bins, dtype=np.int64)
    tot = np.zeros(n_bins)
    half = N // 2
    for s in itertools.product(range(-half, half), repeat=3):
        if s == (0, 0, 0):
            continue
        rr = H * math.sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2])
        for q in range(n_bins):
            if lo + q * width <= rr < lo + (q + 1) * width:
                counts[q] += 1
                tot[q] += rr
    return counts, tot / np.maximum(counts, 1)


def _r_bin_gap(bin_fn=mesh.r_bin_index, lo=RB["lo"]):
    N, L, width, nb = RB["N"], RB["L"], RB["width"], RB["n_bins"]
    counts, mean = _r_bins_enumerated(N, L, lo, width, nb)
    b, rmag = bin_fn(N, L, lo, width, nb)
    c2 = np.bincount(b[b >= 0], minlength=nb)
    m2 = np.bincount(b[b >= 0], weights=rmag[b >= 0], minlength=nb) / np.maximum(c2, 1)
    return int(np.sum(np.abs(c2 - counts))), float(np.max(np.abs(m2 - mean)))


def test_r_bins_by_enumeration():
    for lo in (RB["lo"], 0.0):           # lo = 0: the zero separation stays out of bin 0
        dc, dm = _r_bin_gap(lo=lo)
        assert dc == 0 and dm < 1e-12
    N, L = RB["N"], RB["L"]
    counts, mean = _r_bins_enumerated(N, L, RB["lo"], RB["width"], RB["n_bins"])
    gal, ran = tiny_node_catalog(4, N, L, (-500.0, -500.0, 1000.0))
    r = xi_midpoint(gal, ran, Config(N=N, L=L, b0=(-500.0, -500.0, 1000.0), assign=CIC, ells=(0,),
                                     order=0, bin_lo=RB["lo"], bin_width=RB["width"], n_bins=RB["n_bins"]))
    assert np.array_equal(r.counts, counts)
    assert np.allclose(r.bin_mean, mean, rtol=1e-13, atol=0)


@pytest.mark.parametrize("old,new", [
    ("rmag = (L / N) * np.sqrt(s2)", "rmag = (L / (N - 1)) * np.sqrt(s2)"),
    ("b = np.where((b >= 0) & (b < nbins) & (s2 > 0), b, -1)", "b = np.where((b >= 0) & (b < nbins), b, -1)"),
    ("s = signed_index(N)", "s = np.arange(N)"),
], ids=["wrong cell size", "zero separation binned", "no minimum image"])
def test_r_bin_pin_rejects(old, new):
    bad = _patched(mesh.r_bin_index, old, new)
    gaps = [_r_bin_gap(bad, lo=lo) for lo in (RB["lo"], 0.0)]
    assert any(dc > 0 or dm > 1e-9 for dc, dm in gaps)
