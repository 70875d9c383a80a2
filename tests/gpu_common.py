"""Helpers shared by the GPU parity tests (inputs, oracle calls, tolerances)."""
import sys

import numpy as np

from oracle.estimators import Config as OConfig
from synthetic import to_xyzw


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def rounded(cat, dtype):
    """The catalog exactly as the GPU sees it (positions / weights rounded to dtype)."""
    xyzw = to_xyzw(cat, dtype=dtype)
    out = {"pos": xyzw[:, :3].astype(np.float64), "w": xyzw[:, 3].astype(np.float64),
           "nbar": np.asarray(cat["nbar"], dtype=dtype).astype(np.float64)}
    return xyzw, out


def oracle_cfg(pcfg):
    return OConfig(N=pcfg.n_mesh, L=pcfg.box_len, b0=tuple(pcfg.box_origin), assign=pcfg.assign,
                   ells=tuple(range(0, pcfg.ell_max + 1, 2)), order=pcfg.order,
                   compensate=bool(pcfg.compensate), bin_lo=pcfg.bin_lo, bin_width=pcfg.bin_width,
                   n_bins=pcfg.n_bins)


def max_err_per_ell(gpu, ref):
    """Per multipole: max_b |gpu - ref| / max_b |ref_0| (the monopole scale)."""
    scale = np.max(np.abs(ref[0]))
    return np.max(np.abs(gpu - ref), axis=1) / scale


def uniform_catalog(seed, n_gal, n_ran, center, side, w_range=(0.5, 1.5)):
    rng = np.random.default_rng(seed)
    c = np.asarray(center, dtype=np.float64)
    gal = {"pos": c + rng.uniform(-side / 2, side / 2, (n_gal, 3)),
           "w": rng.uniform(*w_range, n_gal)}
    ran = {"pos": c + rng.uniform(-side / 2, side / 2, (n_ran, 3)),
           "w": rng.uniform(*w_range, n_ran)}
    nbar = n_gal / side ** 3
    gal["nbar"] = np.full(n_gal, nbar)
    ran["nbar"] = np.full(n_ran, nbar)
    return gal, ran
