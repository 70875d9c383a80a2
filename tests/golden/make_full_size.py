"""Write the full-size expected values of the parity tests with the FP64 oracle.

    python tests/golden/make_full_size.py {c3_bisector_pk,c2_midpoint_pk,c4_midpoint_xi,c4_bisector_xi,
                                           c4_bisector_xi_256}

Each case takes the seeded synthetic catalog of its workload (catalog index 0), rounds the
positions, weights and nbar to FP32 exactly as the GPU receives them, runs the oracle
(``oracle.estimators``) at the workload's full configuration and writes
tests/golden/full_<case>.json.  Nothing here calls the library.

  c3_bisector_pk       bisector P_l (Section 5.2), 512^3 TSC, 4e6 + 2e7, l <= 4, order 4,
                       79 k-bins 0.005-0.40 (memory-lean path: retained modes only)
  c2_midpoint_pk       midpoint P_l (Section 3.3), 256^3 TSC, 1e6 + 5e6, l <= 4, order 4,
                       19 k-bins 0.01-0.20
  c4_midpoint_xi       midpoint xi_l (Section 4.3), 512^3 CIC, 4e6 + 2e7, l <= 4, order 4,
                       25 r-bins 0-200
  c4_bisector_xi       bisector xi_l (Section 6), 512^3 CIC, 4e6 + 2e7, l <= 4, order 4,
                       25 r-bins 0-200 (streamed oracle: the 28 transforms with M >= 0, ~60 GB,
                       are held on disk under $PW_ORACLE_SCRATCH, default <repo>/_oracle_scratch)
  c4_bisector_xi_256   bisector xi_l (Section 6) on the same catalog at 256^3 (full-grid oracle)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.estimators import (Config, pk_bisector_shells, pk_midpoint, xi_midpoint,  # noqa: E402
                               xi_bisector, xi_bisector_streamed)
from synthetic import WORKLOADS, make_workload_catalog, to_xyzw  # noqa: E402



def xi_bisector_on_disk(g, r, cfg):
    """xi_bisector_streamed with its transforms in the scratch folder."""
    scratch = os.environ.get("PW_ORACLE_SCRATCH", os.path.join(ROOT, "_oracle_scratch"))
    os.makedirs(scratch, exist_ok=True)
    return xi_bisector_streamed(g, r, cfg, scratch, slab=32)


CASES = {
    "c3_bisector_pk": ("C3", None, pk_bisector_shells),
    "c2_midpoint_pk": ("C2", None, pk_midpoint),
    "c4_midpoint_xi": ("C4", None, xi_midpoint),
    "c4_bisector_xi": ("C4", None, xi_bisector_on_disk),
    "c4_bisector_xi_256": ("C4", 256, xi_bisector),
}


def fp32_catalog(cat):
    xyzw = to_xyzw(cat, dtype=np.float32)
    return {"pos": xyzw[:, :3].astype(np.float64), "w": xyzw[:, 3].astype(np.float64),
            "nbar": np.asarray(cat["nbar"], dtype=np.float32).astype(np.float64)}


def config(name, n_mesh=None):
    wl = WORKLOADS[name]
    return Config(N=n_mesh or wl.N, L=wl.L, b0=wl.b0, assign=wl.assign, ells=wl.ells, order=wl.order,
                  compensate=True, bin_lo=wl.bin_lo, bin_width=wl.bin_width, n_bins=wl.n_bins)


def main(case):
    name, n_mesh, fn = CASES[case]
    t_cat = time.time()
    gal, ran = make_workload_catalog(name, index=0)
    g, r = fp32_catalog(gal), fp32_catalog(ran)
    del gal, ran
    t_cat = time.time() - t_cat
    cfg = config(name, n_mesh)
    print(f"[golden] {case}: {len(g['w'])} + {len(r['w'])} particles, N={cfg.N}", flush=True)
    t0 = time.time()
    res = fn(g, r, cfg)
    seconds = time.time() - t0
    out = {
        "case": case, "workload": name, "n_mesh": cfg.N, "box_len": cfg.L, "box_origin": list(cfg.b0),
        "assign": cfg.assign, "ells": list(cfg.ells), "order": cfg.order, "bin_lo": cfg.bin_lo,
        "bin_width": cfg.bin_width, "n_bins": cfg.n_bins, "catalog_index": 0,
        "values": res.values.tolist(), "bin_mean": res.bin_mean.tolist(),
        "counts": res.counts.tolist(), "norm": [res.alpha_r, res.I, res.S],
        "oracle": fn.__name__, "command": f"python tests/golden/make_full_size.py {case}",
        "seconds": seconds, "catalog_seconds": t_cat, "host_cores": len(os.sched_getaffinity(0)),
        "host": f"{len(os.sched_getaffinity(0))}-core host without a GPU (the build container)",
    }
    path = os.path.join(HERE, f"full_{case}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"[golden] wrote {path}: oracle {seconds:.0f}s, catalog {t_cat:.0f}s", flush=True)


if __name__ == "__main__":
    for c in sys.argv[1:] or list(CASES):
        main(c)
