"""GPU parity of the random-pair normalised and window-corrected xi_l
(pw_estimate_xi_normalized through the C ABI) against the FP64 oracle (xi_normalized)."""
import numpy as np
import pytest

from oracle.estimators import xi_bisector, xi_midpoint, xi_normalized

from gpu_common import say, rounded, oracle_cfg, uniform_catalog

pytestmark = pytest.mark.gpu

pw = pytest.importorskip("paper_2102_08384_amd.pw")


@pytest.fixture(scope="module")
def ctx():
    c = pw.Context(0)
    yield c
    c.close()


def _check(res, ref, tol):
    xr, xe, f = ref
    assert res["window"].shape == f.shape
    s0 = np.max(np.abs(xr[0]))
    for name, got, want in (("xi_rr", res["xi_rr"], xr), ("xi_edge", res["xi_edge"], xe)):
        err = np.max(np.abs(got - want), axis=1) / s0
        say(name, "err per ell (monopole scale)", err)
        assert np.all(err < tol)
    ferr = np.max(np.abs(res["window"] - f))
    say("window err", ferr)
    assert ferr < tol


@pytest.mark.parametrize("los", [pw.PW_MIDPOINT, pw.PW_BISECTOR])
def test_xi_normalized_fp64(ctx, los):
    say("xi normalized fp64 N=32", "midpoint" if los == pw.PW_MIDPOINT else "bisector")
    gal, ran = uniform_catalog(71 + los, 3000, 9000, (0, 0, 1100), 400)
    cfg = pw.Config(stat=pw.PW_XI, los=los, assign=pw.PW_TSC, prec=pw.PW_FP64, n_mesh=32, box_len=800.0,
                    box_origin=(-400.0, -400.0, 700.0), ell_max=4, order=2, compensate=1, bin_lo=20.0,
                    bin_width=40.0, n_bins=8)
    gx, g64 = rounded(gal, np.float64)
    rx, r64 = rounded(ran, np.float64)
    res = ctx.estimate_xi_normalized(cfg, gx, rx, ran_nbar=ran["nbar"])
    est = xi_midpoint if los == pw.PW_MIDPOINT else xi_bisector
    ref = xi_normalized(g64, r64, oracle_cfg(cfg), est, L_max=8 if los == pw.PW_MIDPOINT else 6)
    _check(res, ref, 1e-10)
    plain = ctx.estimate(cfg, gx, rx, ran_nbar=ran["nbar"])
    assert np.array_equal(res["counts"], plain["counts"])


def test_xi_normalized_fp32_cone(ctx):
    """FP32 path on a clustered cone in the C4 geometry at reduced mesh (midpoint, order 4)."""
    from synthetic import WORKLOADS, make_workload_catalog
    say("xi normalized fp32 cone N=64 midpoint order 4")
    gal, ran = make_workload_catalog("C4", index=5, n_gal=30000)
    cfg = pw.Config(stat=pw.PW_XI, los=pw.PW_MIDPOINT, assign=pw.PW_CIC, prec=pw.PW_FP32, n_mesh=64,
                    box_len=WORKLOADS["C4"].L, box_origin=WORKLOADS["C4"].b0, ell_max=4, order=4, compensate=1,
                    bin_lo=0.0, bin_width=90.0, n_bins=12)
    gx, g64 = rounded(gal, np.float32)
    rx, r64 = rounded(ran, np.float32)
    res = ctx.estimate_xi_normalized(cfg, gx, rx, ran_nbar=ran["nbar"].astype(np.float32))
    ref = xi_normalized(g64, r64, oracle_cfg(cfg), xi_midpoint, L_max=8)
    _check(res, ref, 1e-4)


def test_xi_normalized_needs_xi(ctx):
    gal, ran = uniform_catalog(79, 300, 900, (0, 0, 1100), 400)
    gx, _ = rounded(gal, np.float64)
    rx, _ = rounded(ran, np.float64)
    cfg = pw.Config(stat=pw.PW_PK, n_mesh=32, box_len=800.0, box_origin=(-400.0, -400.0, 700.0), n_bins=4)
    with pytest.raises(pw.PwError) as e:
        ctx.estimate_xi_normalized(cfg, gx, rx, ran_nbar=ran["nbar"])
    assert e.value.code == pw.PW_EINVAL
