"""GPU parity of the all-parity midpoint estimators (midpoint_parity = PW_PARITY_ALL, through the
C ABI) against the FP64 oracle: Section 3.2's P_l (every alpha <= K, coefficients phi) and
Section 4.2's xi_l (coefficients f)."""
import dataclasses

import numpy as np
import pytest

from oracle.estimators import pk_midpoint, xi_midpoint

from gpu_common import say, rounded, oracle_cfg, max_err_per_ell, uniform_catalog

pytestmark = pytest.mark.gpu

pw = pytest.importorskip("paper_2102_08384_amd.pw")


@pytest.fixture(scope="module")
def ctx():
    c = pw.Context(0)
    yield c
    c.close()


def _cfg(stat, prec, order, ell_max=4, n_mesh=32):
    if stat == pw.PW_PK:
        bins = dict(bin_lo=0.004, bin_width=0.012, n_bins=8)
    else:
        bins = dict(bin_lo=20.0, bin_width=40.0, n_bins=8)
    return pw.Config(stat=stat, los=pw.PW_MIDPOINT, assign=pw.PW_TSC, prec=prec, n_mesh=n_mesh,
                     box_len=800.0, box_origin=(-400.0, -400.0, 700.0), ell_max=ell_max, order=order,
                     compensate=1, midpoint_parity=pw.PW_PARITY_ALL, **bins)


def _ocfg(cfg, **kw):
    return dataclasses.replace(oracle_cfg(cfg), parity="all", **kw)


@pytest.mark.parametrize("stat", [pw.PW_PK, pw.PW_XI])
@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_allparity_fp64(ctx, stat, order):
    say("all-parity", "pk" if stat == pw.PW_PK else "xi", "fp64 N=32 ell<=4 order", order)
    gal, ran = uniform_catalog(40 + order, 3000, 9000, (0, 0, 1100), 400)
    cfg = _cfg(stat, pw.PW_FP64, order)
    gx, g64 = rounded(gal, np.float64)
    rx, r64 = rounded(ran, np.float64)
    res = ctx.estimate(cfg, gx, rx, ran_nbar=ran["nbar"])
    est = pk_midpoint if stat == pw.PW_PK else xi_midpoint
    ref = est(g64, r64, _ocfg(cfg))
    err = max_err_per_ell(res["values"], ref.values)
    say("per-ell err", err)
    assert np.array_equal(res["counts"], ref.counts)
    assert np.all(err < 1e-10)
    # the odd orders are really there: the all-parity estimate differs from the parity-even one
    even = est(g64, r64, dataclasses.replace(oracle_cfg(cfg), order=order - order % 2)).values
    assert np.max(np.abs(ref.values[1:] - even[1:])) > 1e3 * np.max(err) * np.max(np.abs(ref.values[0]))


@pytest.mark.parametrize("stat", [pw.PW_PK, pw.PW_XI])
def test_allparity_fp32_cone(ctx, stat):
    """FP32 path on a clustered cone catalog at reduced mesh, order 3, against the oracle."""
    from synthetic import WORKLOADS, make_workload_catalog
    say("all-parity", "pk" if stat == pw.PW_PK else "xi", "fp32 cone N=64 order 3")
    if stat == pw.PW_PK:
        gal, ran = make_workload_catalog("C2", index=3, n_gal=30000)
        cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_MIDPOINT, assign=pw.PW_TSC, prec=pw.PW_FP32, n_mesh=64,
                        box_len=WORKLOADS["C2"].L, box_origin=WORKLOADS["C2"].b0, ell_max=4, order=3,
                        compensate=1, bin_lo=0.005, bin_width=0.01, n_bins=8,
                        midpoint_parity=pw.PW_PARITY_ALL)
    else:
        gal, ran = make_workload_catalog("C4", index=3, n_gal=30000)
        cfg = pw.Config(stat=pw.PW_XI, los=pw.PW_MIDPOINT, assign=pw.PW_CIC, prec=pw.PW_FP32, n_mesh=64,
                        box_len=WORKLOADS["C4"].L, box_origin=WORKLOADS["C4"].b0, ell_max=4, order=3,
                        compensate=1, bin_lo=0.0, bin_width=90.0, n_bins=12,
                        midpoint_parity=pw.PW_PARITY_ALL)
    gx, g64 = rounded(gal, np.float32)
    rx, r64 = rounded(ran, np.float32)
    res = ctx.estimate(cfg, gx, rx, ran_nbar=ran["nbar"].astype(np.float32))
    est = pk_midpoint if stat == pw.PW_PK else xi_midpoint
    ref = est(g64, r64, _ocfg(cfg))
    err = max_err_per_ell(res["values"], ref.values)
    say("per-ell err", err)
    assert np.all(err < 1e-4)


def test_allparity_orders(ctx):
    """pw_estimate_orders for the all-parity midpoint: one slice per alpha, each equal to the
    oracle restricted to that alpha."""
    say("all-parity orders: xi fp64 N=32 order 3")
    gal, ran = uniform_catalog(47, 3000, 9000, (0, 0, 1100), 400)
    cfg = _cfg(pw.PW_XI, pw.PW_FP64, 3)
    gx, g64 = rounded(gal, np.float64)
    rx, r64 = rounded(ran, np.float64)
    res = ctx.estimate_orders(cfg, gx, rx, ran_nbar=ran["nbar"])
    assert res["values"].shape == (4, 3, 8)
    ref = np.array([xi_midpoint(g64, r64, _ocfg(cfg, order=a, order_lo=a)).values for a in range(4)])
    scale = np.max(np.abs(ref[0, 0]))
    err = np.max(np.abs(res["values"] - ref)) / scale
    say("max err (monopole scale)", err)
    assert err < 1e-10


def test_allparity_validation(ctx):
    """Odd orders are accepted only for the all-parity midpoint; shapes without a generated
    re-weighting are refused."""
    gal, ran = uniform_catalog(48, 500, 1500, (0, 0, 1100), 400)
    gx, _ = rounded(gal, np.float64)
    rx, _ = rounded(ran, np.float64)
    bad = [dataclasses.replace(_cfg(pw.PW_PK, pw.PW_FP64, 3), midpoint_parity=pw.PW_PARITY_EVEN),
           dataclasses.replace(_cfg(pw.PW_PK, pw.PW_FP64, 3), los=pw.PW_BISECTOR),
           _cfg(pw.PW_PK, pw.PW_FP64, 5),
           dataclasses.replace(_cfg(pw.PW_PK, pw.PW_FP64, 2), midpoint_parity=2)]
    for cfg in bad:
        with pytest.raises(pw.PwError) as e:
            ctx.estimate(cfg, gx, rx, ran_nbar=ran["nbar"])
        assert e.value.code == pw.PW_EINVAL
