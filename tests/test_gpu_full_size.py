"""Full-size parity: the workloads at their real sizes (FP32 path, the configuration bench.py
times) against expected values the FP64 oracle wrote (tests/golden/make_full_size.py)."""
import json
import os

import numpy as np
import pytest

from synthetic import WORKLOADS, make_workload_catalog, to_xyzw

from gpu_common import say, max_err_per_ell

pytestmark = pytest.mark.gpu

pw = pytest.importorskip("paper_2102_08384_amd.pw")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CASES = ["c3_bisector_pk", "c2_midpoint_pk", "c4_midpoint_xi", "c4_bisector_xi", "c4_bisector_xi_256"]
STAT = {"c3_bisector_pk": (pw.PW_PK, pw.PW_BISECTOR), "c2_midpoint_pk": (pw.PW_PK, pw.PW_MIDPOINT),
        "c4_midpoint_xi": (pw.PW_XI, pw.PW_MIDPOINT), "c4_bisector_xi": (pw.PW_XI, pw.PW_BISECTOR),
        "c4_bisector_xi_256": (pw.PW_XI, pw.PW_BISECTOR)}


@pytest.fixture(scope="module")
def ctx():
    c = pw.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("case", CASES)
def test_full_size_matches_oracle(ctx, case):
    path = os.path.join(GOLDEN, f"full_{case}.json")
    if not os.path.exists(path):
        pytest.skip(f"expected values not generated: python tests/golden/make_full_size.py {case}")
    with open(path) as fh:
        gold = json.load(fh)
    say("full-size", case, "N =", gold["n_mesh"])
    gal, ran = make_workload_catalog(gold["workload"], index=gold["catalog_index"])
    gx = to_xyzw(gal, np.float32)
    rx = to_xyzw(ran, np.float32)
    rn = np.asarray(ran["nbar"], dtype=np.float32)
    stat, los = STAT[case]
    cfg = pw.Config(stat=stat, los=los, assign=gold["assign"], prec=pw.PW_FP32, n_mesh=gold["n_mesh"],
                    box_len=gold["box_len"], box_origin=tuple(gold["box_origin"]),
                    ell_max=max(gold["ells"]), order=gold["order"], compensate=1, bin_lo=gold["bin_lo"],
                    bin_width=gold["bin_width"], n_bins=gold["n_bins"])
    res = ctx.estimate(cfg, gx, rx, ran_nbar=rn)
    ref = np.asarray(gold["values"])
    err = max_err_per_ell(res["values"], ref)
    say("per-ell err (units of the monopole scale)", err)
    assert np.array_equal(res["counts"], np.asarray(gold["counts"]))
    # Mean |k| (or r) sums `count` positive FP64 terms in a different order on each side:
    # each sum is within (count-1)*2^-53 relative of exact, so they agree within count*2^-52.
    cnt = np.maximum(np.asarray(gold["counts"], dtype=np.float64), 1.0)
    rel = np.abs(res["bin_mean"] - np.asarray(gold["bin_mean"])) / np.maximum(np.abs(gold["bin_mean"]), 1e-300)
    say("bin_mean max relative diff", rel.max(), "bound", (cnt * 2.0**-52).max())
    assert np.all(rel <= cnt * 2.0**-52 + 1e-15)
    a, I, S = res["norm"]
    assert np.allclose([a, I, S], gold["norm"], rtol=1e-10)
    assert np.all(err < 1e-4)
