"""Benchmark: bisector P_l on the 512^3 headline workload (catalogs/s, served vs plain), and the
serving stream (p50/p99 latency under Poisson arrivals).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--lanes 2] [--workload C3]
                [--no-cpu-baseline] [--no-served] [--no-serving] [--serving-requests 256]
                [--copy-calibration] [--stream N] [--figures]

A step is one pass of the whole hot path (FP64 scalars, paint, weighted fields, pruned forward
FFTs, contraction and FP64 binning) over one synthetic catalog already resident in HBM,
through the C ABI.
  plain    one synchronous pw_estimate per catalog on one stream, stage timing off
  stages   a separate pass with stage timing on (HIP events on the library's stream): the
           per-stage times and the roofline of the dominant kernel
  served   K catalogs submitted at once to the serving loop (pw_submit), which runs them on
           `--lanes` concurrent lanes: saturated throughput
  serving  the serving workload: a stream of mixed requests (galaxies ~ U[1e5, 4e6] with 5x
           randoms, meshes 128/256/512, midpoint or bisector) whose catalogs sit in pinned host
           memory; capacity from a plain pass, then Poisson arrivals at 0.7x and 1.5x of it;
           latency = pw_submit -> result on the host (includes the copy to the device)
`value` is the served throughput of the headline workload; `latency_ms` is the serving
stream's at 0.7x load.  --stream N prints only a serving stream of N requests.  --figures
writes the per-order and convergence analogues of the paper's figures to figures/.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bisector P_ℓ 512³ catalogs/s, served vs plain; p50/p99 latency; HBM GB/s"
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30   # calibration copy: 1 GiB read + 1 GiB written
KERNEL_NAMES = {"fx": "k_fx", "fy": "k_fy", "fz": "k_fz", "contract": "k_contract_bis_reg"}
# midpoint P_l: forward passes, product + inverse z pass, inverse y/x passes, re-weighting, the
# forward passes of the A fields and the k-space contraction
KERNEL_NAMES_MID = {"fx": "k_fx", "fy": "k_fy", "fziz": "k_fziz", "iy": "k_fy", "ix": "k_ix", "ix_bin": "k_ix",
                    "reweight": "k_reweight", "afx": "k_fx", "afy": "k_fy", "afz": "k_fz",
                    "contract": "k_contract_mid"}
# bisector xi_l: forward passes, per-mode targets, inverse z / y passes, c2r x pass with r-binning
KERNEL_NAMES_BXI = {"fx": "k_fx", "fy": "k_fy", "fz": "k_fz", "targets": "k_targets", "iz": "k_iz",
                    "iy": "k_fy", "ix_bin": "k_ix"}
GOLDEN_CASE = {"C3": "c3_bisector_pk", "C2": "c2_midpoint_pk", "C4": "c4_midpoint_xi", "C4B": "c4_bisector_xi"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def workload_config(pw, name, parity=0):
    from synthetic import WORKLOADS
    wl = WORKLOADS[name]
    return pw.Config(stat=pw.PW_PK if wl.stat == "pk" else pw.PW_XI,
                     los=pw.PW_BISECTOR if wl.los == "bisector" else pw.PW_MIDPOINT,
                     assign=wl.assign, prec=pw.PW_FP32, n_mesh=wl.N, box_len=wl.L,
                     box_origin=wl.b0, ell_max=max(wl.ells), order=wl.order, compensate=1,
                     bin_lo=wl.bin_lo, bin_width=wl.bin_width, n_bins=wl.n_bins, midpoint_parity=parity)


def describe(wl, name, cfg):
    est = ("bisector" if wl.los == "bisector" else
           "midpoint" + (" all-parity" if cfg.midpoint_parity else "")) + (" P_l" if wl.stat == "pk" else " xi_l")
    series = f"order {wl.order} (beta<=2)" if wl.los == "bisector" else f"order {wl.order} (alpha<={wl.order})"
    unit = "k" if wl.stat == "pk" else "r"
    return (f"{name}: {est}, {wl.N}^3 {'TSC' if wl.assign == 3 else 'CIC'}, {wl.n_gal:.0e} lognormal "
            f"galaxies + {wl.n_gal * wl.ran_ratio:.0e} randoms in a 1/8-sky cone r in [{wl.rmin:g},{wl.rmax:g}], "
            f"l<={max(wl.ells)}, {series}, {unit} {wl.bin_lo}-{wl.bin_lo + wl.n_bins * wl.bin_width:.3f} "
            f"d{unit} {wl.bin_width}")


def cpu_baseline(name, frac=0.25, n_mesh=96):
    """The oracle as it stands, on a bounded sample of the workload: the same catalog
    subsampled to `frac` of its particles, on an n_mesh^3 mesh with the same bins/orders; plus
    the oracle's recorded time on the full workload (tests/golden)."""
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
    cores = len(os.sched_getaffinity(0))
    out = {"value": 1.0 / dt, "unit": "catalogs/s", "cores": cores, "kind": "oracle",
           "seconds": dt, "fft_threads": os.cpu_count(),
           "sample": f"{name} catalog subsampled to {frac:g} of its particles "
                     f"({len(g['pos'])} galaxies + {len(r['pos'])} randoms) on a {n_mesh}^3 mesh "
                     f"(full workload: {wl.N}^3), same l<=4, order {wl.order}, bins; numpy/scipy FP64, "
                     f"FFTs on os.cpu_count() threads over the {cores} cores this process may use"}
    gold = os.path.join(ROOT, "tests", "golden", f"full_{GOLDEN_CASE.get(name, '')}.json")
    if os.path.exists(gold):
        with open(gold) as fh:
            gd = json.load(fh)
        if "seconds" in gd:
            out["full_size"] = {"value": 1.0 / gd["seconds"], "seconds": gd["seconds"], "oracle": gd["oracle"],
                                "where": gd.get("host", "the build container (8 cores, no GPU), when the "
                                                        "expected values were written"),
                                "cores": gd.get("host_cores", 8),
                                "timed": ("the oracle call alone" if "catalog_seconds" in gd
                                          else "the oracle call and the catalog's generation")}
    return out


def oracle_check(workload, midpoint_parity, cfg, values):
    """Per-multipole error of the measured estimate against the FP64 oracle's values for the
    same catalog (catalog 0 of the workload, FP32-rounded inputs) and configuration, stored by
    tests/golden/make_full_size.py; in units of the oracle's monopole scale.  None when no
    stored values match the configuration."""
    case = GOLDEN_CASE.get(workload)
    path = os.path.join(ROOT, "tests", "golden", f"full_{case}.json")
    if case is None or midpoint_parity != "even" or not os.path.exists(path):
        return None
    with open(path) as fh:
        gold = json.load(fh)
    same = (gold["n_mesh"] == cfg.n_mesh and gold["n_bins"] == cfg.n_bins and gold["order"] == cfg.order
            and max(gold["ells"]) == cfg.ell_max and abs(gold["bin_lo"] - cfg.bin_lo) < 1e-12
            and abs(gold["bin_width"] - cfg.bin_width) < 1e-12 and gold["assign"] == cfg.assign)
    if not same:
        return None
    ref = np.asarray(gold["values"])
    err = np.max(np.abs(np.asarray(values) - ref), axis=1) / np.max(np.abs(ref[0]))
    return {"max_err_per_ell": err.tolist(), "ells": gold["ells"], "tolerance": 1e-4,
            "reference": f"FP64 oracle on the same catalog, stored in tests/golden/full_{case}.json"}


def source_digest():
    """Digest of the sources of every kernel the bisector P_l workload runs and of their launch
    code (all of csrc/ but inverse.hip, which holds only the inverse-transform and midpoint
    kernels); counter-based traffic is reported only for this digest."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2102_08384_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".cpp")) and f != "inverse.hip":
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_text(name):
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None, path
    return open(path).read(), path


def copy_bandwidth(torch, dev, nbytes=COPY_BYTES, reps=10):
    """Rate of torch's device-to-device copy (bytes read + written per second, in GB/s) on a
    1 GiB buffer, four times the Infinity Cache: what a plain library streaming kernel reaches
    on this device, reported beside the 8 TB/s peak (context, not the roofline's peak).  Timed
    with events on torch's current stream, outside every timed region of the estimates."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = None
    for _ in range(3):   # the best of three batches
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def counter_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None when the
    summary is missing or was taken on other kernel sources."""
    txt, path = _profile_text("bisector_pk_512_traffic.txt")
    if txt is None:
        return None, None
    m = re.search(r"^source_digest\s*=\s*(\S+)", txt, re.M)
    if not m or m.group(1) != source_digest():
        return None, "counters taken on other kernel sources"
    m = re.search(rf"^{re.escape(kernel)}\s+traffic_bytes_per_launch\s*=\s*(\S+)", txt, re.M)
    if not m:
        return None, None
    return float(m.group(1)), os.path.relpath(path, ROOT)


def rocprof_avg_us(kernel):
    """Average duration of `kernel` from the committed kernel-trace summary, when it was taken
    on these kernel sources; else None."""
    txt, path = _profile_text("bisector_pk_512_kernels.md")
    if txt is None:
        return None, None
    m = re.search(r"source_digest\s*=\s*(\S+)", txt)
    if not m or m.group(1) != source_digest():
        return None, "kernel trace taken on other kernel sources"
    m = re.search(rf"^\|\s*pw::{re.escape(kernel)}<[^|]*\|\s*\d+\s*\|\s*([0-9.]+)\s*\|", txt, re.M)
    if not m:
        return None, None
    return float(m.group(1)), os.path.relpath(path, ROOT)


def plain_run(ctx, cfg, gx, rx, rn, steps, warmup, torch):
    for _ in range(warmup):
        ctx.estimate(cfg, gx, rx, ran_nbar=rn)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    res = None
    for _ in range(steps):
        t1 = time.perf_counter()
        res = ctx.estimate(cfg, gx, rx, ran_nbar=rn)
        lat.append((time.perf_counter() - t1) * 1e3)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return elapsed, lat, res


def stage_run(ctx, cfg, gx, rx, rn, steps):
    """Per-stage GPU times from HIP events on the library's stream (timing on for this pass only)."""
    ctx.set_timing(True)
    stage_ms, stage_bytes = {}, {}
    for _ in range(steps):
        ctx.estimate(cfg, gx, rx, ran_nbar=rn)
        for name, ms, by in ctx.stages():
            stage_ms.setdefault(name, []).append(ms)
            stage_bytes[name] = by
    ctx.set_timing(False)
    return stage_ms, stage_bytes


def served_run(ctx, cfg, gx, rx, rn, steps, warmup, torch):
    for t in [ctx.submit(cfg, gx, rx, ran_nbar=rn) for _ in range(warmup)]:
        t.wait()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sub, tickets = [], []
    for _ in range(steps):
        sub.append(time.perf_counter())
        tickets.append(ctx.submit(cfg, gx, rx, ran_nbar=rn))
    done = [None] * steps
    res = None
    while any(d is None for d in done):
        for i, t in enumerate(tickets):
            if done[i] is None:
                r = t.poll()
                if r is not None:
                    done[i] = time.perf_counter()
                    res = r
        time.sleep(2e-4)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lat = [(d - s) * 1e3 for s, d in zip(sub, done)]
    return elapsed, lat, res


# ------------------------------------------------------------------------------ serving stream

def stream_requests(pw, torch, n_req, seed=5):
    """The serving workload: P_l requests with galaxy counts uniform in [1e5, 4e6] and 5x
    randoms, a mesh of 128, 256 or 512, the midpoint or the bisector by a fair coin, l <= 4,
    order 4, k-bins 0.005 .. min(0.40, k_Nyq) by 0.005.  Catalogs are windows of one shuffled
    lognormal cone per geometry (bisector: r in [400, 2000], L = 2700; midpoint: r in
    [500, 1500], box doubled, L = 4000) held in pinned host memory, so any window is a uniform
    subsample; nbar scales with the subsampled count (one pinned array holds every request's).
    Returns (label, cfg, gal, ran, nbar) tuples of pinned host tensors."""
    from synthetic import WORKLOADS, make_workload_catalog, to_xyzw
    rng = np.random.default_rng(seed)
    pools = {}
    for los, name in ((pw.PW_BISECTOR, "C3"), (pw.PW_MIDPOINT, "C2")):
        g, r = make_workload_catalog(name, index=1, n_gal=4_000_000)
        gx = torch.from_numpy(to_xyzw(g, np.float32)[rng.permutation(len(g["pos"]))]).pin_memory()
        rx = torch.from_numpy(to_xyzw(r, np.float32)[rng.permutation(len(r["pos"]))]).pin_memory()
        pools[los] = (gx, rx, float(r["nbar"][0]), WORKLOADS[name])
    spec = []
    for i in range(n_req):
        los = pw.PW_BISECTOR if rng.random() < 0.5 else pw.PW_MIDPOINT
        N = int(rng.choice([128, 256, 512]))
        ng = int(rng.uniform(1e5, 4e6))
        gx = pools[los][0]
        rx = pools[los][1]
        g0 = int(rng.integers(0, len(gx) - ng + 1))
        r0 = int(rng.integers(0, len(rx) - 5 * ng + 1))
        spec.append((los, N, ng, g0, r0))
    nbar_all = torch.empty(sum(5 * s[2] for s in spec), dtype=torch.float32).pin_memory()
    out, off = [], 0
    for los, N, ng, g0, r0 in spec:
        gx, rx, nbar, wl = pools[los]
        nbar_all[off:off + 5 * ng] = nbar * ng / len(gx)
        kny = np.pi * N / wl.L
        nbins = int((min(0.40, kny) - 0.005) / 0.005)
        cfg = pw.Config(stat=pw.PW_PK, los=los, assign=pw.PW_TSC, prec=pw.PW_FP32, n_mesh=N, box_len=wl.L,
                        box_origin=wl.b0, ell_max=4, order=4, compensate=1, bin_lo=0.005, bin_width=0.005,
                        n_bins=nbins)
        out.append((f"{'bis' if los == pw.PW_BISECTOR else 'mid'}{N} ng={ng}", cfg, gx[g0:g0 + ng],
                    rx[r0:r0 + 5 * ng], nbar_all[off:off + 5 * ng]))
        off += 5 * ng
    return out


def _pct(v):
    return {"p50": float(np.percentile(v, 50)), "p99": float(np.percentile(v, 99))} if len(v) else None


def batch_gain(pw, torch, ctx, reqs, n=8):
    """Batched launches against one estimate after another: n bisector catalogs of one mesh, as
    n pw_estimate calls and as one pw_estimate_batch call (each forward pass and the contraction
    once over the n catalogs).  Cases: the stream's own requests at 128^3 and 256^3 (pinned host
    inputs, so every catalog is copied to the device), the same catalogs device-resident, and
    small device-resident catalogs (windows of 1e5 galaxies) at 64^3 and 128^3."""
    out = {}
    cases = []
    for N in (128, 256):
        sel = [q for q in reqs if q[1].los == pw.PW_BISECTOR and q[1].n_mesh == N][:n]
        if len(sel) >= 2:
            cats = [(g, r, nb) for _, _, g, r, nb in sel]
            cases.append((f"bisector_{N}_host_inputs", sel[0][1], cats))
            cases.append((f"bisector_{N}_device_inputs", sel[0][1], [tuple(a.cuda() for a in c) for c in cats]))
    bis = [q for q in reqs if q[1].los == pw.PW_BISECTOR]
    if bis:
        g, r, nb = bis[0][2], bis[0][3], bis[0][4]
        small = [(g[i * 100_000:(i + 1) * 100_000].cuda(), r[i * 500_000:(i + 1) * 500_000].cuda(),
                  nb[i * 500_000:(i + 1) * 500_000].cuda()) for i in range(n)
                 if (i + 1) * 100_000 <= len(g) and (i + 1) * 500_000 <= len(r)]
        for N in (64, 128):
            cfg = pw.Config(**{**bis[0][1].__dict__, "n_mesh": N,
                               "n_bins": int((min(0.40, np.pi * N / bis[0][1].box_len) - 0.005) / 0.005)})
            if len(small) >= 2:
                cases.append((f"bisector_{N}_small_device_inputs", cfg, small))
    for name, cfg, cats in cases:
        ctx.estimate_batch(cfg, cats)        # warm: batch plans and workspace
        reps = 3
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for g, r, nb in cats:
                ctx.estimate(cfg, g, r, ran_nbar=nb)
        seq = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.estimate_batch(cfg, cats)
        bat = (time.perf_counter() - t0) / reps
        out[name] = {"catalogs": len(cats), "n_mesh": cfg.n_mesh, "one_after_another_ms": seq * 1e3,
                     "batched_ms": bat * 1e3, "speedup": seq / bat,
                     "galaxies": [int(g.shape[0]) for g, _, _ in cats]}
        log(f"batched {name}: {seq * 1e3:.1f} ms one after another, {bat * 1e3:.1f} ms batched")
        del cats
    return out


def serving_stream(pw, torch, n_req, lanes, loads=(0.7, 1.5)):
    """Capacity from one plain pass over the stream (one pw_estimate after another), then, after
    one untimed served pass that warms the lanes, the same requests at exponential
    inter-arrival times at each load x capacity; latency from pw_submit to the result on the
    host.  Failed requests are counted, not retried."""
    log("building a serving stream of", n_req, "requests (catalogs in pinned host memory)")
    t0 = time.perf_counter()
    reqs = stream_requests(pw, torch, n_req)
    log(f"stream ready in {time.perf_counter() - t0:.1f}s")
    ctx = pw.Context(0)
    ctx.set_lanes(lanes)
    seen = set()
    for lab, cfg, g, r, n in reqs:         # every configuration once: plans built, kernels loaded
        key = (cfg.los, cfg.n_mesh)
        if key not in seen:
            seen.add(key)
            ctx.estimate(cfg, g, r, ran_nbar=n)
    t0 = time.perf_counter()
    plain_lat = []
    for lab, cfg, g, r, n in reqs:
        t1 = time.perf_counter()
        ctx.estimate(cfg, g, r, ran_nbar=n)
        plain_lat.append((time.perf_counter() - t1) * 1e3)
    cap = len(reqs) / (time.perf_counter() - t0)
    log(f"serving: plain pass {cap:.2f} requests/s")
    mix = {}
    for lab, *_ in reqs:
        k = lab.split()[0]
        mix[k] = mix.get(k, 0) + 1
    out = {"requests": len(reqs), "lanes": lanes, "mix_counts": mix,
           "mix": "N_g ~ U[1e5, 4e6] + 5 N_g randoms; mesh 128/256/512; midpoint (L = 4000) or bisector "
                  "(L = 2700) by a fair coin; l <= 4, order 4; FP32; catalogs in pinned host memory "
                  "(copied to the device inside each request)",
           "plain": {"value": cap, "unit": "requests/s", "latency_ms": _pct(plain_lat)}}
    warm = [ctx.submit(cfg, g, r, ran_nbar=n) for lab, cfg, g, r, n in reqs]
    for t in warm:
        t.wait()
    rng = np.random.default_rng(11)
    for load in loads:
        gaps = rng.exponential(1.0 / (load * cap), len(reqs))
        arrivals = np.cumsum(gaps) - gaps[0]
        torch.cuda.synchronize()
        l0, q0 = ctx.serving_stats()
        t0 = time.perf_counter()
        tickets, sub = [], []
        done = [None] * len(reqs)
        failed = []

        def poll_all():
            # completion times are taken while later requests are still being submitted
            for i, t in enumerate(tickets):
                if done[i] is None:
                    try:
                        if t.poll() is None:
                            continue
                    except pw.PwError as e:
                        failed.append(f"{reqs[i][0]}: {e}")
                    done[i] = time.perf_counter()

        for i, (lab, cfg, g, r, n) in enumerate(reqs):
            while time.perf_counter() - t0 < arrivals[i]:
                poll_all()
                time.sleep(5e-5)
            sub.append(time.perf_counter())
            try:
                tickets.append(ctx.submit(cfg, g, r, ran_nbar=n))
            except pw.PwError as e:        # refused at submission (queue full)
                failed.append(f"{lab}: {e}")
                tickets.append(None)
                done[i] = time.perf_counter()
        while any(d is None for d in done):
            poll_all()
            time.sleep(1e-4)
        el = max(done) - t0
        lat = [(d - s_) * 1e3 for s_, d, t in zip(sub, done, tickets) if t is not None]
        l1, q1 = ctx.serving_stats()
        out[f"at_{load}x"] = {"offered": load * cap, "value": (len(reqs) - len(failed)) / el,
                              "unit": "requests/s", "failed": len(failed), "failures": failed[:5],
                              "latency_ms": _pct(lat), "launches": l1 - l0, "requests_launched": q1 - q0}
        log(f"serving at {load}x: {(len(reqs) - len(failed)) / el:.2f} requests/s, p50 {np.percentile(lat, 50):.1f} "
            f"ms, p99 {np.percentile(lat, 99):.1f} ms, {len(failed)} failed")
    out["batched"] = batch_gain(pw, torch, ctx, reqs)
    ctx.close()
    return out


# ------------------------------------------------------------------------------ figures

def _mock_tensors(torch, name, index, shift_z=0.0):
    """Catalog `index` of a workload on the device, optionally translated along +z (the cone's
    axis) by shift_z: (gal, ran, nbar) tensors."""
    from synthetic import make_workload_catalog, to_xyzw
    gal, ran = make_workload_catalog(name, index=index)
    gx, rx = to_xyzw(gal, np.float32), to_xyzw(ran, np.float32)
    if shift_z:
        gx[:, 2] += shift_z
        rx[:, 2] += shift_z
    return (torch.from_numpy(gx).cuda(), torch.from_numpy(rx).cuda(),
            torch.from_numpy(ran["nbar"].astype(np.float32)).cuda())


def _orders_over_mocks(ctx, cfgs, name, n_mocks, torch, shift_z=0.0):
    """Per-order outputs (pw_estimate_orders) of each configuration over n_mocks catalogs: mean
    and standard deviation over the mocks, [order][l][bin]."""
    acc = {k: [] for k in cfgs}
    centers = None
    for i in range(n_mocks):
        g, r, n = _mock_tensors(torch, name, 100 + i, shift_z)
        for key, cfg in cfgs.items():
            res = ctx.estimate_orders(cfg, g, r, ran_nbar=n)
            acc[key].append(res["values"])
            centers = res["bin_mean"]
        del g, r, n
    out = {}
    for key, v in acc.items():
        v = np.asarray(v)
        out[key] = {"mean": v.mean(axis=0).tolist(), "std": v.std(axis=0, ddof=1).tolist()}
    return out, centers


def figures_leg(pw, torch, n_mocks=8, n_mocks_xi=4):
    """Analogues of the paper's Figs 2-5 (Sections 7.1 and 7.2) from the GPU path, on synthetic
    lognormal mocks in place of the Patchy BOSS mocks; written to figures/figures.json.
      fig2  truncation error of the estimators against the survey's opening angle: a compact
            survey (cube of side 300) placed at distances D, |X(K) - X(K_ref)| / |X(K_ref)|
            for each series order K (bisector P_l: K_ref = 8; midpoint P_l, parity-even and
            all-parity: K_ref = 4), max over the k-bins, l = 2 and 4
      fig3  per-order contributions to P_l (orders theta^0, theta^2, theta^4) of the BOSS-like
            mocks (r in [500, 1500], 1e6 galaxies, box doubled, 256^3 TSC): midpoint all-parity,
            midpoint parity-even, bisector; mean over the mocks and the ratio to the standard
            deviation of the Yamamoto spectra (the midpoint's order 0)
      fig4  the same mocks translated outward by 2000 along the line of sight (z)
      fig5  per-order contributions to xi_l of the 512^3 mocks (r in [400, 2000], 4e6
            galaxies, CIC), midpoint parity-even and bisector, 25 r-bins of 8"""
    from synthetic import WORKLOADS
    t0 = time.perf_counter()
    out = {"note": "synthetic lognormal mocks stand in for the Patchy mocks; see bench.figures_leg",
           "sections": {"fig2": "Section 7.1", "fig3": "Section 7.2", "fig4": "Section 7.2",
                        "fig5": "Section 7.2"}}
    ctx = pw.Context(0)
    # ---- fig2: truncation scan against the opening angle
    rng = np.random.default_rng(7)
    side, n_g = 300.0, 20000
    scan = []
    for D in (600.0, 1200.0, 2400.0, 4800.0):
        c = np.array([0.0, 0.0, D])
        gx = np.empty((n_g, 4), np.float32)
        rx = np.empty((3 * n_g, 4), np.float32)
        gx[:, :3] = c + rng.uniform(-side / 2, side / 2, (n_g, 3))
        rx[:, :3] = c + rng.uniform(-side / 2, side / 2, (3 * n_g, 3))
        gx[:, 3] = 1.0
        rx[:, 3] = 1.0
        nb = np.full(3 * n_g, n_g / side ** 3, np.float32)
        L = 2.0 * side + 40.0
        b0 = (-L / 2, -L / 2, D - L / 2)
        theta = float(np.sqrt(3.0) * side / 2 / (D - side / 2))
        row = {"distance": D, "theta_max": theta}
        for label, los, par, kref, ks in (("bisector", pw.PW_BISECTOR, 0, 8, (0, 2, 4, 6)),
                                          ("midpoint_even", pw.PW_MIDPOINT, 0, 4, (0, 2)),
                                          ("midpoint_all", pw.PW_MIDPOINT, 1, 4, (0, 1, 2, 3))):
            base = dict(stat=pw.PW_PK, los=los, assign=pw.PW_TSC, prec=pw.PW_FP32, n_mesh=128, box_len=L,
                        box_origin=b0, ell_max=4, compensate=1, bin_lo=0.02, bin_width=0.02, n_bins=10,
                        midpoint_parity=par)
            ref = ctx.estimate(pw.Config(order=kref, **base), gx, rx, ran_nbar=nb)["values"]
            errs = {}
            for K in ks:
                v = ctx.estimate(pw.Config(order=K, **base), gx, rx, ran_nbar=nb)["values"]
                errs[str(K)] = [float(np.max(np.abs(v[i] - ref[i])) / np.max(np.abs(ref[i]))) for i in (1, 2)]
            row[label] = {"K_ref": kref, "max_frac_err_l2_l4": errs}
        scan.append(row)
    out["fig2"] = scan
    log(f"figures: convergence scan done ({time.perf_counter() - t0:.0f}s)")
    # ---- fig3 / fig4: per-order P_l of the BOSS-like mocks, and translated by +2000
    wl = WORKLOADS["C2"]
    pk = dict(stat=pw.PW_PK, assign=pw.PW_TSC, prec=pw.PW_FP32, n_mesh=wl.N, box_len=wl.L, ell_max=4, order=4,
              compensate=1, bin_lo=wl.bin_lo, bin_width=wl.bin_width, n_bins=wl.n_bins)
    for fig, shift in (("fig3", 0.0), ("fig4", 2000.0)):
        b0 = (wl.b0[0], wl.b0[1], wl.b0[2] + shift)
        cfgs = {"midpoint_all": pw.Config(los=pw.PW_MIDPOINT, midpoint_parity=1, box_origin=b0, **pk),
                "midpoint_even": pw.Config(los=pw.PW_MIDPOINT, box_origin=b0, **pk),
                "bisector": pw.Config(los=pw.PW_BISECTOR, box_origin=b0, **pk)}
        res, kc = _orders_over_mocks(ctx, cfgs, "C2", n_mocks, torch, shift)
        yam_std = np.asarray(res["midpoint_even"]["std"])[0]   # order 0 of the midpoint = Yamamoto
        for key, r in res.items():
            m = np.asarray(r["mean"])
            # the all-parity midpoint's slices are alpha = 0..4: orders theta^0, theta^2, theta^4
            # are alpha 0, 1 + 2, 3 + 4
            if key == "midpoint_all":
                m = np.stack([m[0], m[1] + m[2], m[3] + m[4]])
            r["mean_by_theta_order"] = m.tolist()
            with np.errstate(divide="ignore", invalid="ignore"):
                r["ratio_to_yamamoto_std"] = np.where(yam_std > 0, np.abs(m) / yam_std, 0.0).tolist()
            del r["std"]
        out[fig] = {"k": np.asarray(kc).tolist(), "ells": [0, 2, 4], "n_mocks": n_mocks,
                    "translation_z": shift, "catalog": "C2 geometry: 1e6 lognormal galaxies + 5e6 randoms, "
                    "r in [500, 1500] (+ translation), box 4000 (doubled), 256^3 TSC", "estimators": res}
        log(f"figures: {fig} done ({time.perf_counter() - t0:.0f}s)")
    # ---- fig5: per-order xi_l of the 512^3 mocks
    wl = WORKLOADS["C4"]
    xi = dict(stat=pw.PW_XI, assign=wl.assign, prec=pw.PW_FP32, n_mesh=wl.N, box_len=wl.L, box_origin=wl.b0,
              ell_max=4, order=4, compensate=1, bin_lo=wl.bin_lo, bin_width=wl.bin_width, n_bins=wl.n_bins)
    cfgs = {"midpoint_even": pw.Config(los=pw.PW_MIDPOINT, **xi), "bisector": pw.Config(los=pw.PW_BISECTOR, **xi)}
    res, rc = _orders_over_mocks(ctx, cfgs, "C4", n_mocks_xi, torch)
    yam_std = np.asarray(res["midpoint_even"]["std"])[0]
    for key, r in res.items():
        m = np.asarray(r["mean"])
        r["mean_by_theta_order"] = m.tolist()
        with np.errstate(divide="ignore", invalid="ignore"):
            r["ratio_to_yamamoto_std"] = np.where(yam_std > 0, np.abs(m) / yam_std, 0.0).tolist()
        del r["std"]
    out["fig5"] = {"r": np.asarray(rc).tolist(), "ells": [0, 2, 4], "n_mocks": n_mocks_xi,
                   "catalog": "C4: 4e6 lognormal galaxies + 2e7 randoms, r in [400, 2000], box 2900, 512^3 CIC",
                   "estimators": res}
    ctx.close()
    out["seconds"] = time.perf_counter() - t0
    path = os.path.join(ROOT, "figures", "figures.json")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    log(f"figures written to {path} in {out['seconds']:.0f}s")
    return {"figures": os.path.relpath(path, ROOT), "seconds": out["seconds"],
            "fig2": [{"theta_max": r["theta_max"], "bisector": r["bisector"]["max_frac_err_l2_l4"]} for r in scan]}


# ------------------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--lanes", type=int, default=2)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-orders", action="store_true")
    ap.add_argument("--midpoint-parity", choices=["even", "all"], default="even",
                    help="midpoint series form (the headline workload is the bisector)")
    ap.add_argument("--memory-lean", action="store_true",
                    help="bisector P_l: forward transforms in groups of fields (less device memory)")
    ap.add_argument("--stream", type=int, default=0,
                    help="only a serving stream of this many requests (throughput and latency)")
    ap.add_argument("--figures", action="store_true",
                    help="write the analogues of the paper's per-order and convergence figures")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": a.gpus}), flush=True)
        sys.exit(2)
    import torch
    from paper_2102_08384_amd import pw
    if a.figures:
        print(json.dumps(figures_leg(pw, torch)), flush=True)
        return
    if a.stream > 0:
        out = {"metric": "serving stream (mixed P_l requests) requests/s and latency", "n_gpus": 1}
        out.update(serving_stream(pw, torch, a.stream, a.lanes))
        print(json.dumps(out), flush=True)
        return

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
    cfg = workload_config(pw, a.workload, 1 if a.midpoint_parity == "all" else 0)
    cfg.memory_lean = 1 if a.memory_lean else 0
    knames = (KERNEL_NAMES if wl.stat == "pk" else KERNEL_NAMES_BXI) if wl.los == "bisector" else KERNEL_NAMES_MID
    stream = torch.cuda.current_stream(dev)
    if a.copy_calibration:
        src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {COPY_BYTES} bytes done")
        del src, dst
    ctx = pw.Context(0, stream=stream.cuda_stream)
    ctx.set_lanes(a.lanes)

    log("plain: warmup", a.warmup, "then", a.steps, "steps (stage timing off)")
    p_el, p_lat, res = plain_run(ctx, cfg, gx, rx, rn, a.steps, a.warmup, torch)
    plain_value = a.steps / p_el
    log(f"plain {plain_value:.2f} catalogs/s")
    n_stage = max(3, a.steps // 4)
    stage_ms, stage_bytes = stage_run(ctx, cfg, gx, rx, rn, n_stage)
    served = None
    if not a.no_served:
        log("served:", a.lanes, "lanes, warmup", a.warmup, "then", a.steps, "catalogs")
        s_el, s_lat, s_res = served_run(ctx, cfg, gx, rx, rn, a.steps, a.warmup, torch)
        served = {"value": a.steps / s_el, "ms_per_catalog": s_el * 1e3 / a.steps, "lanes": a.lanes,
                  "latency_ms_saturated": _pct(s_lat),
                  "arrivals": f"{a.steps} catalogs submitted at once (saturated queue: the latency is queue depth)",
                  "max_abs_diff_vs_plain": float(np.max(np.abs(s_res["values"] - res["values"])))}
        log(f"served {served['value']:.2f} catalogs/s")

    orders = None
    if not a.no_orders and wl.stat == "pk":
        # each series order's terms separately (one pass for the bisector P_l)
        for _ in range(max(1, a.warmup)):
            ctx.estimate_orders(cfg, gx, rx, ran_nbar=rn)
        torch.cuda.synchronize()
        n_o = max(3, a.steps // 4)
        t0 = time.perf_counter()
        for _ in range(n_o):
            o_res = ctx.estimate_orders(cfg, gx, rx, ran_nbar=rn)
        torch.cuda.synchronize()
        o_el = time.perf_counter() - t0
        orders = {"value": n_o / o_el, "unit": "catalogs/s", "ms_per_catalog": o_el * 1e3 / n_o,
                  "steps": n_o, "n_orders": int(o_res["values"].shape[0]),
                  "max_abs_sum_minus_plain": float(np.max(np.abs(o_res["values"].sum(axis=0) - res["values"])))}
        log(f"per-order outputs {orders['value']:.2f} catalogs/s")

    stages = {n: {"ms": float(np.mean(v)), "GB": stage_bytes[n] / 1e9,
                  "GBps": (stage_bytes[n] / 1e9) / (np.mean(v) / 1e3) if np.mean(v) > 0 else None}
              for n, v in stage_ms.items()}
    dom = max((n for n in stages if n in knames), key=lambda n: stages[n]["ms"])
    ach = stages[dom]["GBps"]
    headline = a.workload == "C3" and not a.memory_lean
    traffic, tsrc = counter_traffic(knames[dom]) if headline else (None, None)
    rp_us, rp_src = rocprof_avg_us(knames[dom]) if headline else (None, None)
    roofline = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": knames[dom], "algorithmic_bytes_per_launch": stage_bytes[dom],
                "avg_ms": stages[dom]["ms"], "timing": f"HIP events on the library's stream, {n_stage} estimates",
                "traffic_source": tsrc}
    if headline:
        roofline["copy_GBps"] = copy_bandwidth(torch, dev)
        roofline["frac_of_copy"] = ach / roofline["copy_GBps"]
    if rp_us:
        roofline["rocprof"] = {"avg_ms": rp_us / 1e3, "frac": stage_bytes[dom] / (rp_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                               "source": rp_src}
    serving = None
    if not a.no_serving and a.workload == "C3":
        ctx.close()
        del gx, rx, rn
        torch.cuda.empty_cache()
        serving = serving_stream(pw, torch, a.serving_requests, a.lanes)
    value = served["value"] if served else plain_value
    elapsed = (a.steps / value)
    latency = (serving["at_0.7x"]["latency_ms"] if serving else _pct(p_lat))
    out = {
        "metric": METRIC, "value": value, "unit": "catalogs/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": elapsed * 1e3 / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": describe(wl, a.workload, cfg),
                   "mode": "served" if served else "plain",
                   "memory_lean": bool(a.memory_lean),
                   "inputs": "resident in HBM (device pointers)"},
        "plain": {"value": plain_value, "ms_per_catalog": p_el * 1e3 / a.steps, "latency_ms": _pct(p_lat)},
        "served": served,
        "serving": serving,
        "latency_ms": latency,
        "latency_source": ("serving stream at 0.7x of its plain capacity (Poisson arrivals, pinned host inputs)"
                           if serving else "plain pw_estimate calls"),
        "orders": orders,
        "roofline": roofline,
        "stages": stages,
        "monopole_first_bins": res["values"][0][:3].tolist(),
        # launch shapes the autotuner picked during the warm-up (candidate 0 = default shape)
        "autotune": pw.tune_entries(),
        # error of the measured estimate against the FP64 oracle, per multipole
        "oracle_check": oracle_check(a.workload, a.midpoint_parity, cfg, res["values"]),
    }
    if serving is None:
        ctx.close()
    if a.workload != "C3":
        out["metric"] = f"{a.workload} catalogs/s (secondary workload; the headline metric is C3's)"
    if not a.no_cpu_baseline and a.workload == "C3":
        log("timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(a.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
