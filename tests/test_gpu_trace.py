"""Per-request tracing (PW_TRACE, the tracing subsystem): a context created with PW_TRACE set
writes one JSON line per completed estimate, for pw_estimate, pw_estimate_batch and served
requests, with stage times from the lane's HIP events.  Run in a process of its own, since the
variable is read at pw_create."""
import json
import os
import subprocess
import sys

import pytest

from gpu_common import say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CODE = r'''
import numpy as np
import torch
from paper_2102_08384_amd import pw
from gpu_common import rounded, uniform_catalog
gal, ran = uniform_catalog(931, 20000, 60000, (0, 0, 1000), 420)
gx, _ = rounded(gal, np.float32); rx, _ = rounded(ran, np.float32)
nb = ran["nbar"].astype(np.float32)
dev = [torch.from_numpy(a).cuda() for a in (gx, rx, nb)]
cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=pw.PW_FP32, n_mesh=64, box_len=1000.0,
                box_origin=(-500.0, -500.0, 600.0), ell_max=4, order=4, compensate=1, bin_lo=0.005,
                bin_width=0.02, n_bins=9)
mid = pw.Config(stat=pw.PW_XI, los=pw.PW_MIDPOINT, assign=pw.PW_CIC, prec=pw.PW_FP32, n_mesh=32, box_len=1000.0,
                box_origin=(-500.0, -500.0, 500.0), ell_max=2, order=2, compensate=1, bin_lo=0.0,
                bin_width=40.0, n_bins=5)
with pw.Context(0) as ctx:
    ctx.estimate(cfg, *dev[:2], ran_nbar=dev[2])
    ctx.estimate_batch(cfg, [tuple(dev), tuple(dev)])
    ts = [ctx.submit(cfg, *dev[:2], ran_nbar=dev[2]) for _ in range(3)] + [ctx.submit(mid, gx, rx, ran_nbar=nb)]
    for t in ts:
        t.wait()
'''


def test_trace_lines(tmp_path):
    say("tracing: PW_TRACE lines for estimate, batch and served requests")
    path = tmp_path / "trace.jsonl"
    env = dict(os.environ, PW_TRACE=str(path), PYTHONPATH=os.pathsep.join([ROOT, os.path.join(ROOT, "tests")]))
    r = subprocess.run([sys.executable, "-c", CODE], env=env, cwd=ROOT, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [json.loads(x) for x in path.read_text().splitlines() if x.strip()]
    say("trace kinds", [x["kind"] for x in lines])
    kinds = [x["kind"] for x in lines]
    assert kinds.count("estimate") == 1 and kinds.count("batch") == 2 and kinds.count("served") == 4
    est = next(x for x in lines if x["kind"] == "estimate")
    assert est["lane"] == 0 and est["status"] == 0 and est["n_gal"] == 20000 and est["n_ran"] == 60000
    assert {"paint", "fx", "fy", "fz", "contract"} <= set(est["stages_ms"])
    assert all(v >= 0 for v in est["stages_ms"].values()) and est["stages_ms"]["fy"] > 0
    assert sum(est["stages_ms"].values()) <= est["run_ms"] + 1e-6
    served = [x for x in lines if x["kind"] == "served"]
    assert sorted(x["ticket"] for x in served) == sorted({x["ticket"] for x in served})
    for x in served:
        assert x["status"] == 0 and x["lane"] >= 1 and x["queued_ms"] >= 0 and x["run_ms"] > 0
        if x["batch"] == 1:
            assert x["stages_ms"], x
    xi = [x for x in served if x["stat"] == "xi"]
    assert len(xi) == 1 and xi[0]["los"] == "midpoint" and xi[0]["n_mesh"] == 32
    assert all(a["t_ms"] <= b["t_ms"] for a, b in zip(lines, lines[1:]))
