"""Synthetic catalogs standing in for the paper's MultiDark-Patchy BOSS DR12 mocks.

The mocks of Section 7.2 are not available; these seeded generators produce
catalogs with the shapes, sizes, weights and clustering statistics of the
workloads the estimator is measured on.  Recipe (all host numpy, FP64, PCG64):

* Geometry: observer at the origin.  "1/8-sky cap" = a cone about +z with
  half-angle arccos(3/4) (solid angle pi/2), radial shell [r_min, r_max].
* Lognormal clustering: a Gaussian field G on a generation mesh spanning the
  workload's box, power spectrum P_G(k) ~ k^-1.5 (P_G(0) = 0, modes up to the
  generation mesh's Nyquist), scaled to cell-level sigma_G = 0.8;
  rho = exp(G - sigma^2/2).  Galaxies: exactly N_g draws of cells with
  probability ~ rho inside the footprint, uniform within the cell; draws that
  fall outside the exact cone/shell are redrawn.
* Randoms: exactly 5 N_g (or the stated ratio) uniform in the same volume
  (r from the r^2 law, cos(theta) uniform in [3/4, 1], phi uniform).
* Weights: w = 1/(1 + nbar * 1e4) with nbar = N_g / V constant (uniform within a
  catalog); nbar is returned for the randoms (it enters the normalisation I).
* Seeds: seed = 1000 * workload_id + catalog_index, with independent substreams
  for the field, the galaxies and the randoms.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

COS_CAP = 0.75                       # cos of the cone half-angle (1/8 of the sky)
SIN_CAP = math.sqrt(1.0 - COS_CAP ** 2)


@dataclass(frozen=True)
class Workload:
    """A named workload: catalog recipe + estimator configuration."""
    wid: int
    kind: str              # "uniform_cube" or "lognormal_cone"
    n_gal: int
    ran_ratio: float
    rmin: float            # cone shell (lognormal) or cube centre distance (uniform)
    rmax: float            # cone shell outer radius, or cube side (uniform)
    N: int
    L: float
    b0: tuple
    assign: int            # 2 CIC, 3 TSC
    ells: tuple
    order: int
    stat: str              # "pk" or "xi"
    los: str               # "midpoint" / "bisector"
    bin_lo: float
    bin_width: float
    n_bins: int
    n_gen: int             # generation mesh for the lognormal field
    weight_fkp: bool


def _cone_box(rmin, rmax, L):
    """Box of side L centred on the cone/shell's bounding box: returns the corner b0."""
    xy = rmax * SIN_CAP
    zlo, zhi = rmin * COS_CAP, rmax
    c = np.array([0.0, 0.0, 0.5 * (zlo + zhi)])
    assert 2 * xy <= L and (zhi - zlo) <= L
    return tuple(float(v) for v in (c - 0.5 * L))


WORKLOADS = {
    # plain method, FP64, midpoint P_l: uniform cube of side 500 at distance 1000
    "C1": Workload(1, "uniform_cube", 10_000, 5.0, 1000.0, 500.0, 64, 1000.0,
                   (-500.0, -500.0, 500.0), 2, (0, 2), 2, "pk", "midpoint",
                   0.01, 0.01, 29, 0, False),
    # midpoint P_l, lognormal cone r in [500,1500], box doubled (L = 4000)
    "C2": Workload(2, "lognormal_cone", 1_000_000, 5.0, 500.0, 1500.0, 256, 4000.0,
                   _cone_box(500.0, 1500.0, 4000.0), 3, (0, 2, 4), 4, "pk", "midpoint",
                   0.01, 0.01, 19, 256, True),
    # bisector P_l, the headline workload
    "C3": Workload(3, "lognormal_cone", 4_000_000, 5.0, 400.0, 2000.0, 512, 2700.0,
                   _cone_box(400.0, 2000.0, 2700.0), 3, (0, 2, 4), 4, "pk", "bisector",
                   0.005, 0.005, 79, 512, True),
    # xi_l via the inverse FFT (midpoint and bisector), 25 bins over 0-200
    "C4": Workload(4, "lognormal_cone", 4_000_000, 5.0, 400.0, 2000.0, 512, 2900.0,
                   _cone_box(400.0, 2000.0, 2900.0), 2, (0, 2, 4), 4, "xi", "midpoint",
                   0.0, 8.0, 25, 512, True),
    # the same catalog (same workload id, same seeds) with the bisector xi_l (Section 6)
    "C4B": Workload(4, "lognormal_cone", 4_000_000, 5.0, 400.0, 2000.0, 512, 2900.0,
                    _cone_box(400.0, 2000.0, 2900.0), 2, (0, 2, 4), 4, "xi", "bisector",
                    0.0, 8.0, 25, 512, True),
}


def uniform_cube(n, center, side, rng):
    return np.asarray(center)[None, :] + rng.uniform(-0.5 * side, 0.5 * side, size=(n, 3))


def cone_shell_uniform(n, rmin, rmax, rng):
    u = rng.uniform(size=n)
    r = np.cbrt(rmin ** 3 + u * (rmax ** 3 - rmin ** 3))
    ct = rng.uniform(COS_CAP, 1.0, size=n)
    st = np.sqrt(1.0 - ct * ct)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=n)
    return np.stack([r * st * np.cos(ph), r * st * np.sin(ph), r * ct], axis=1)


def cone_volume(rmin, rmax):
    return (2.0 * np.pi * (1.0 - COS_CAP)) / 3.0 * (rmax ** 3 - rmin ** 3)


def _in_footprint(p, rmin, rmax):
    r = np.sqrt(np.sum(p * p, axis=1))
    with np.errstate(invalid="ignore", divide="ignore"):
        ct = np.where(r > 0, p[:, 2] / np.where(r > 0, r, 1), -1)
    return (r >= rmin) & (r < rmax) & (ct >= COS_CAP)


def gaussian_field(n_gen, L, rng, slope=-1.5, sigma=0.8):
    """Gaussian random field on an n_gen^3 mesh with P(k) ~ k^slope, unit-free, scaled to sigma."""
    kf = 2.0 * np.pi / L
    kx = np.fft.fftfreq(n_gen, d=1.0 / n_gen) * kf
    kz = np.fft.rfftfreq(n_gen, d=1.0 / n_gen) * kf
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (slope / 4.0), 0.0)
    white = rng.standard_normal((n_gen, n_gen, n_gen))
    G = np.fft.irfftn(np.fft.rfftn(white) * amp, s=(n_gen,) * 3, axes=(0, 1, 2))
    G *= sigma / G.std()
    return G


def lognormal_catalog(n_gal, rmin, rmax, L, b0, n_gen, seed_seq, ran_ratio=5.0, sigma=0.8):
    """Galaxies Poisson-sampled (multinomially, exactly n_gal) from a lognormal field inside the
    cone/shell, plus uniform randoms in the same volume.  Returns float64 pos arrays."""
    s_field, s_gal, s_ran = seed_seq.spawn(3)
    rng_f, rng_g, rng_r = (np.random.Generator(np.random.PCG64(s)) for s in (s_field, s_gal, s_ran))
    G = gaussian_field(n_gen, L, rng_f, sigma=sigma)
    rho = np.exp(G - 0.5 * sigma * sigma).ravel()
    H = L / n_gen
    b0 = np.asarray(b0, dtype=np.float64)
    # cells whose extent can touch the footprint: test the cell centre with a margin of one cell diagonal
    idx = np.arange(n_gen)
    cx = b0[0] + (idx + 0.5) * H
    cy = b0[1] + (idx + 0.5) * H
    cz = b0[2] + (idx + 0.5) * H
    X, Y, Z = np.meshgrid(cx, cy, cz, indexing="ij")
    R = np.sqrt(X * X + Y * Y + Z * Z).ravel()
    marg = H * math.sqrt(3.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        CT = np.where(R > 0, Z.ravel() / np.where(R > 0, R, 1), -1)
    near = (R >= rmin - marg) & (R < rmax + marg) & (CT >= COS_CAP - marg / np.maximum(R, 1.0))
    prob = np.where(near, rho, 0.0)
    cdf = np.cumsum(prob)
    cdf /= cdf[-1]
    out = np.empty((0, 3))
    need = n_gal
    while need > 0:
        u = rng_g.uniform(size=need)
        cells = np.searchsorted(cdf, u, side="right")
        cells = np.minimum(cells, cdf.size - 1)
        i = cells // (n_gen * n_gen)
        j = (cells // n_gen) % n_gen
        k = cells % n_gen
        p = np.stack([i, j, k], axis=1).astype(np.float64)
        p = b0[None, :] + (p + rng_g.uniform(size=(need, 3))) * H
        ok = _in_footprint(p, rmin, rmax)
        out = np.concatenate([out, p[ok]], axis=0)
        need = n_gal - len(out)
    gal_pos = out[:n_gal]
    ran_pos = cone_shell_uniform(int(round(ran_ratio * n_gal)), rmin, rmax, rng_r)
    return gal_pos, ran_pos


def make_workload_catalog(name: str, index: int = 0, n_gal: int | None = None):
    """(gal, ran) dicts with float64 'pos' [n,3], 'w' [n], 'nbar' [n] for a named workload.
    n_gal overrides the galaxy count (randoms keep the workload's ratio)."""
    wl = WORKLOADS[name]
    ng = wl.n_gal if n_gal is None else int(n_gal)
    seed = np.random.SeedSequence(1000 * wl.wid + index)
    if wl.kind == "uniform_cube":
        s_g, s_r = seed.spawn(2)
        rg = np.random.Generator(np.random.PCG64(s_g))
        rr = np.random.Generator(np.random.PCG64(s_r))
        center = np.array([0.0, 0.0, wl.rmin])
        gpos = uniform_cube(ng, center, wl.rmax, rg)
        rpos = uniform_cube(int(round(wl.ran_ratio * ng)), center, wl.rmax, rr)
        V = wl.rmax ** 3
    else:
        gpos, rpos = lognormal_catalog(ng, wl.rmin, wl.rmax, wl.L, wl.b0, wl.n_gen, seed,
                                       ran_ratio=wl.ran_ratio)
        V = cone_volume(wl.rmin, wl.rmax)
    nbar = ng / V
    wv = 1.0 / (1.0 + nbar * 1e4) if wl.weight_fkp else 1.0
    gal = {"pos": gpos, "w": np.full(len(gpos), wv), "nbar": np.full(len(gpos), nbar)}
    ran = {"pos": rpos, "w": np.full(len(rpos), wv), "nbar": np.full(len(rpos), nbar)}
    return gal, ran


def tiny_node_catalog(seed, N, L, b0, n_gal=20, n_ran=60, lo=2, hi=10, nbar=1e-4):
    """Particles placed exactly on mesh nodes with index in [lo, hi) on every axis
    (for pair-sum pins), with random positive weights."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H = L / N

    def snap(n):
        return np.asarray(b0, dtype=np.float64)[None, :] + rng.integers(lo, hi, size=(n, 3)) * H

    gal = {"pos": snap(n_gal), "w": rng.uniform(0.5, 1.5, n_gal)}
    ran = {"pos": snap(n_ran), "w": rng.uniform(0.5, 1.5, n_ran)}
    gal["nbar"] = np.full(n_gal, nbar)
    ran["nbar"] = np.full(n_ran, nbar)
    return gal, ran


def serving_stream(n_requests=256, seed=5000, pool=None):
    """The serving mix: per request (n_gal in U[1e5, 4e6], mesh in {128,256,512}, LOS coin flip).
    Returns a list of dicts; catalogs are drawn later by subsampling a pool."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for i in range(n_requests):
        reqs.append({
            "n_gal": int(rng.integers(100_000, 4_000_001)),
            "N": int(rng.choice([128, 256, 512])),
            "los": "bisector" if rng.uniform() < 0.5 else "midpoint",
            "pool_index": int(rng.integers(0, 1 << 30)),
        })
    return reqs


def to_xyzw(cat, dtype=np.float32):
    """Pack a catalog as an [n, 4] array (x, y, z, w)."""
    out = np.empty((len(cat["pos"]), 4), dtype=dtype)
    out[:, :3] = cat["pos"]
    out[:, 3] = cat["w"]
    return out
