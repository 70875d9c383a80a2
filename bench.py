"""Benchmark: bisector P_l on the 512^3 headline workload, one catalog per step.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--workload C3]

A step is one pass of the whole hot path (FP64 scalars, paint, weighted fields, pruned forward
FFTs, contraction and FP64 binning) over one synthetic catalog already resident in HBM, through
the C ABI (pw_estimate).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bisector P_ℓ 512³ catalogs/s, served vs plain; p50/p99 latency; HBM GB/s"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def workload_config(pw, name):
    from synthetic import WORKLOADS
    wl = WORKLOADS[name]
    return pw.Config(stat=pw.PW_PK if wl.stat == "pk" else pw.PW_XI,
                     los=pw.PW_BISECTOR if wl.los == "bisector" else pw.PW_MIDPOINT,
                     assign=wl.assign, prec=pw.PW_FP32, n_mesh=wl.N, box_len=wl.L,
                     box_origin=wl.b0, ell_max=max(wl.ells), order=wl.order, compensate=1,
                     bin_lo=wl.bin_lo, bin_width=wl.bin_width, n_bins=wl.n_bins)


def cpu_baseline(name, frac=0.25, n_mesh=96):
    """The oracle as it stands, on a bounded sample of the workload: the same catalog
    subsampled to `frac` of its particles, on an n_mesh^3 mesh with the same bins/orders."""
    from oracle.estimators import Config as OConfig, pk_bisector
    from synthetic import WORKLOADS, make_workload_catalog
    wl = WORKLOADS[name]
    gal, ran = make_workload_catalog(name, index=0)
    rng = np.random.default_rng(0)
    sel_g = rng.random(len(gal["pos"])) < frac
    sel_r = rng.random(len(ran["pos"])) < frac
    g = {k: v[sel_g] for k, v in gal.items()}
    r = {k: v[sel_r] for k, v in ran.items()}
    cfg = OConfig(N=n_mesh, L=wl.L, b0=wl.b0, assign=wl.assign, ells=wl.ells, order=wl.order,
                  compensate=True, bin_lo=wl.bin_lo, bin_width=wl.bin_width, n_bins=wl.n_bins)
    t0 = time.perf_counter()
    pk_bisector(g, r, cfg)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "catalogs/s", "cores": 1, "kind": "oracle",
            "seconds": dt,
            "sample": f"{name} catalog subsampled to {frac:g} of its particles "
                      f"({len(g['pos'])} galaxies + {len(r['pos'])} randoms) on a {n_mesh}^3 mesh "
                      f"(full workload: {wl.N}^3), same l<=4, order {wl.order}, bins; numpy FP64, "
                      f"single-threaded FFTs"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)

    import torch
    from paper_2102_08384_amd import pw
    from synthetic import WORKLOADS, make_workload_catalog, to_xyzw

    wl = WORKLOADS[a.workload]
    log("generating", a.workload, "catalog")
    t0 = time.time()
    gal, ran = make_workload_catalog(a.workload, index=0)
    log(f"catalog ready ({len(gal['pos'])} gal, {len(ran['pos'])} ran) in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    gx = torch.from_numpy(to_xyzw(gal, np.float32)).to(dev)
    rx = torch.from_numpy(to_xyzw(ran, np.float32)).to(dev)
    rn = torch.from_numpy(ran["nbar"].astype(np.float32)).to(dev)
    cfg = workload_config(pw, a.workload)
    stream = torch.cuda.current_stream(dev)
    ctx = pw.Context(0, stream=stream.cuda_stream)
    ctx.set_timing(True)
    log("warmup", a.warmup)
    for _ in range(a.warmup):
        ctx.estimate(cfg, gx, rx, ran_nbar=rn)
    torch.cuda.synchronize()
    lat = []
    stage_ms = {}
    stage_bytes = {}
    log("timing", a.steps, "steps")
    t_start = time.perf_counter()
    for _ in range(a.steps):
        t1 = time.perf_counter()
        res = ctx.estimate(cfg, gx, rx, ran_nbar=rn)
        lat.append((time.perf_counter() - t1) * 1e3)
        for name, ms, by in ctx.stages():
            stage_ms.setdefault(name, []).append(ms)
            stage_bytes[name] = by
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    log(f"timed {a.steps} steps in {elapsed:.3f}s")
    value = a.steps / elapsed
    stages = {n: {"ms": float(np.mean(v)), "GB": stage_bytes[n] / 1e9,
                  "GBps": (stage_bytes[n] / 1e9) / (np.mean(v) / 1e3) if np.mean(v) > 0 else None}
              for n, v in stage_ms.items()}
    dom = max(stages, key=lambda n: stages[n]["ms"])
    ach = stages[dom]["GBps"]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                "algorithmic_GB_per_launch": stages[dom]["GB"], "avg_ms": stages[dom]["ms"]}
    out = {
        "metric": METRIC, "value": value, "unit": "catalogs/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": elapsed * 1e3 / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{a.workload}: bisector P_l, {wl.N}^3 TSC, {wl.n_gal:.0e} lognormal "
                               f"galaxies + {wl.n_gal * wl.ran_ratio:.0e} randoms in a 1/8-sky cone "
                               f"r in [{wl.rmin:g},{wl.rmax:g}], l<=4, order {wl.order} (beta<=2), "
                               f"k {wl.bin_lo}-{wl.bin_lo + wl.n_bins * wl.bin_width:.3f} dk {wl.bin_width}",
                   "mode": "plain (one pw_estimate per catalog, inputs resident in HBM)"},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "roofline": roofline,
        "stages": stages,
        "monopole_first_bins": res["values"][0][:3].tolist(),
    }
    ctx.close()
    if not a.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(a.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
