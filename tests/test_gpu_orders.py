"""GPU parity of the per-order outputs (pw_estimate_orders through the C ABI): slice o holds
the terms of order theta^(2o) alone (midpoint alpha = 2o, bisector beta = o), compared with
the FP64 oracle restricted to that order's terms (Config.order_lo = order = 2o)."""
import dataclasses

import numpy as np
import pytest

from oracle.estimators import pk_bisector, pk_midpoint, xi_bisector, xi_midpoint

from gpu_common import say, rounded, oracle_cfg, uniform_catalog

pytestmark = pytest.mark.gpu

pw = pytest.importorskip("paper_2102_08384_amd.pw")

ORACLE = {(pw.PW_PK, pw.PW_BISECTOR): pk_bisector, (pw.PW_PK, pw.PW_MIDPOINT): pk_midpoint,
          (pw.PW_XI, pw.PW_BISECTOR): xi_bisector, (pw.PW_XI, pw.PW_MIDPOINT): xi_midpoint}


@pytest.fixture(scope="module")
def ctx():
    c = pw.Context(0)
    yield c
    c.close()


def _cfg(stat, los, prec, order=4, ell_max=4):
    if stat == pw.PW_PK:
        bins = dict(bin_lo=0.004, bin_width=0.012, n_bins=8)
    else:
        bins = dict(bin_lo=20.0, bin_width=40.0, n_bins=8)
    return pw.Config(stat=stat, los=los, assign=pw.PW_TSC, prec=prec, n_mesh=32, box_len=800.0,
                     box_origin=(-400.0, -400.0, 700.0), ell_max=ell_max, order=order, compensate=1,
                     **bins)


def _oracle_orders(cfg, g64, r64):
    est = ORACLE[(cfg.stat, cfg.los)]
    out = []
    for o in range(cfg.order // 2 + 1):
        oc = dataclasses.replace(oracle_cfg(cfg), order=2 * o, order_lo=2 * o)
        out.append(est(g64, r64, oc).values)
    return np.array(out)


@pytest.mark.parametrize("stat,los", [(pw.PW_PK, pw.PW_BISECTOR), (pw.PW_PK, pw.PW_MIDPOINT),
                                      (pw.PW_XI, pw.PW_BISECTOR), (pw.PW_XI, pw.PW_MIDPOINT)])
@pytest.mark.parametrize("prec", [pw.PW_FP64, pw.PW_FP32])
def test_orders_match_oracle(ctx, stat, los, prec):
    dtype = np.float64 if prec == pw.PW_FP64 else np.float32
    say("orders", "pk" if stat == pw.PW_PK else "xi", "bis" if los == pw.PW_BISECTOR else "mid",
        "fp64" if prec == pw.PW_FP64 else "fp32", "N=32 ell<=4 order 4")
    gal, ran = uniform_catalog(21 + stat + 2 * los, 3000, 9000, (0, 0, 1100), 400)
    cfg = _cfg(stat, los, prec)
    gx, g64 = rounded(gal, dtype)
    rx, r64 = rounded(ran, dtype)
    nb = ran["nbar"].astype(dtype)
    res = ctx.estimate_orders(cfg, gx, rx, ran_nbar=nb)
    ref = _oracle_orders(cfg, g64, r64)
    assert res["values"].shape == ref.shape == (3, 3, 8)
    scale = np.max(np.abs(ref[0, 0]))
    err = np.max(np.abs(res["values"] - ref), axis=2) / scale      # [order, ell]
    say("per-order, per-ell error (monopole scale)", err.tolist())
    tol = 1e-10 if prec == pw.PW_FP64 else 1e-4
    assert np.all(err < tol)
    # beyond zeroth order the monopole vanishes (and carries no shot noise)
    assert np.max(np.abs(res["values"][1:, 0])) <= tol * scale
    if prec == pw.PW_FP64:
        # each order against its own size: the small higher-order terms are resolved too
        for o in (1, 2):
            own = np.max(np.abs(ref[o, 1:]))
            rel = np.max(np.abs(res["values"][o, 1:] - ref[o, 1:])) / own
            say("order", 2 * o, "error relative to its own size", rel)
            assert rel < 1e-6
    # the slices add up to the plain estimate
    full = ctx.estimate(cfg, gx, rx, ran_nbar=nb)
    assert np.array_equal(res["counts"], full["counts"])
    sum_err = np.max(np.abs(res["values"].sum(axis=0) - full["values"])) / scale
    say("sum of orders vs estimate", sum_err)
    assert sum_err < (1e-12 if prec == pw.PW_FP64 else 1e-5)


def test_bisector_orders_headline_shape(ctx):
    """The one-pass path at the headline couplings (ell <= 4, order 4, 79 k-bins) on a
    clustered cone at reduced mesh: every order against the oracle."""
    from synthetic import make_workload_catalog
    say("orders bisector cone N=64 79 bins")
    gal, ran = make_workload_catalog("C3", index=0, n_gal=20000)
    cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=pw.PW_FP32, n_mesh=64,
                    box_len=2700.0, box_origin=(-1350.0, -1350.0, 300.0), ell_max=4, order=4,
                    compensate=1, bin_lo=0.005, bin_width=0.005, n_bins=79)
    gx, g64 = rounded(gal, np.float32)
    rx, r64 = rounded(ran, np.float32)
    res = ctx.estimate_orders(cfg, gx, rx, ran_nbar=ran["nbar"].astype(np.float32))
    ref = _oracle_orders(cfg, g64, r64)
    scale = np.max(np.abs(ref[0, 0]))
    err = np.max(np.abs(res["values"] - ref), axis=2) / scale
    say("per-order, per-ell error (monopole scale)", err.tolist())
    assert np.all(err < 1e-4)


def test_wide_angle_orders_shrink_when_survey_moves_out(ctx):
    """The paper's shifted-survey check on synthetic data: moving the same catalog 2000 Mpc/h
    further out shrinks the opening angles, so the beta = 1 (theta^2) bisector contribution to
    the quadrupole falls roughly as the square of the distance ratio, while the zeroth order
    barely changes."""
    say("orders bisector: shift by +2000")
    gal, ran = uniform_catalog(31, 4000, 12000, (0, 0, 900), 500)
    out = []
    for shift in (0.0, 2000.0):
        g = {k: (v + np.array([0, 0, shift]) if k == "pos" else v) for k, v in gal.items()}
        r = {k: (v + np.array([0, 0, shift]) if k == "pos" else v) for k, v in ran.items()}
        cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=pw.PW_FP64, n_mesh=32,
                        box_len=1000.0, box_origin=(-500.0, -500.0, 400.0 + shift), ell_max=2, order=2,
                        compensate=1, bin_lo=0.006, bin_width=0.012, n_bins=6)
        gx, _ = rounded(g, np.float64)
        rx, _ = rounded(r, np.float64)
        out.append(ctx.estimate_orders(cfg, gx, rx, ran_nbar=r["nbar"])["values"])
    near, far = out
    q1 = np.max(np.abs(far[1, 1])) / np.max(np.abs(near[1, 1]))
    ratio2 = (900.0 / 2900.0) ** 2
    say("beta=1 quadrupole: far/near", q1, "(distance ratio squared", ratio2, ")")
    assert q1 < 3 * ratio2
    assert np.allclose(far[0, 0], near[0, 0], rtol=1e-6, atol=1e-9 * np.max(np.abs(near[0, 0])))
