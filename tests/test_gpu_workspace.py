"""Plans cached on one lane share the lane's workspace (mesh, spectrum buffers, paint tiles):
every estimate re-points its plan into the workspace, which grows to the largest plan run on
the lane.  Alternating configurations, growing the workspace under a cached plan, and a
served stream alternating between sizes must all give the results of fresh contexts."""
import numpy as np
import pytest

from gpu_common import say, rounded, uniform_catalog

pytestmark = pytest.mark.gpu

pw = pytest.importorskip("paper_2102_08384_amd.pw")


def _close(a, b, tol=1e-12):
    """Same arithmetic, FP64 shell sums in another order."""
    return np.max(np.abs(a - b)) <= tol * np.max(np.abs(b))


def _case(N, los, seed, prec=pw.PW_FP64):
    dt = np.float64 if prec == pw.PW_FP64 else np.float32
    gal, ran = uniform_catalog(seed, 3000, 9000, (0, 0, 1000), 440)
    gx, _ = rounded(gal, dt)
    rx, _ = rounded(ran, dt)
    cfg = pw.Config(stat=pw.PW_PK, los=los, assign=pw.PW_TSC, prec=prec, n_mesh=N, box_len=1000.0,
                    box_origin=(-500.0, -500.0, 600.0), ell_max=4, order=4 if los == pw.PW_MIDPOINT else 2,
                    compensate=1, bin_lo=0.005, bin_width=0.02, n_bins=6)
    return cfg, gx, rx, ran["nbar"].astype(dt)


def _buffer(ctx, cfg):
    """What the estimate left in the workspace: the k-sphere spectra (bisector P_l) or the mesh."""
    what = 1 if cfg.los == pw.PW_BISECTOR else 0
    return ctx.inspect(what, np.float64 if cfg.prec == pw.PW_FP64 else np.float32).copy()


def _fresh(case):
    cfg, gx, rx, nb = case
    with pw.Context(0) as c:
        res = c.estimate(cfg, gx, rx, ran_nbar=nb)
        buf = _buffer(c, cfg)
    return res, buf


def test_workspace_grows_under_cached_plans():
    """small, large, small, large on one context: the large plan grows the workspace after the
    small plan was bound to the old one; the small plan must follow it to the new one."""
    say("workspace: N=32 bisector, N=64 midpoint, alternating on one lane")
    small = _case(32, pw.PW_BISECTOR, 201)
    large = _case(64, pw.PW_MIDPOINT, 202)
    ref = {id(small): _fresh(small), id(large): _fresh(large)}
    with pw.Context(0) as ctx:
        for case in (small, large, small, large, small):
            cfg, gx, rx, nb = case
            res = ctx.estimate(cfg, gx, rx, ran_nbar=nb)
            want, buf = ref[id(case)]
            assert _close(res["values"], want["values"])
            assert np.array_equal(res["counts"], want["counts"])
            assert np.array_equal(_buffer(ctx, cfg), buf)


def test_workspace_budget_holds_tables_of_both():
    """A budget that holds the larger plan's footprint and half the smaller one's, not two
    whole plans: both configurations run alternately and match fresh contexts."""
    say("workspace: two N=64 configurations under a budget below two whole plans")
    a = _case(64, pw.PW_BISECTOR, 203, pw.PW_FP32)
    b = _case(64, pw.PW_MIDPOINT, 204, pw.PW_FP32)
    fa = pw.footprint(a[0], len(a[1]), len(a[2]))
    fb = pw.footprint(b[0], len(b[1]), len(b[2]))
    budget = max(fa, fb) + min(fa, fb) // 2
    assert budget < fa + fb
    ra, rb = _fresh(a)[0], _fresh(b)[0]
    with pw.Context(0, hbm_budget=budget) as ctx:
        for case, want in ((a, ra), (b, rb), (a, ra), (b, rb)):
            cfg, gx, rx, nb = case
            got = ctx.estimate(cfg, gx, rx, ran_nbar=nb)
            assert _close(got["values"], want["values"], 1e-6)


def test_served_lanes_alternate_sizes():
    """Two serving lanes fed alternating sizes: each lane's workspace is re-bound per request."""
    say("workspace: served stream alternating N=32 / N=64 over 2 lanes")
    cases = [_case(32, pw.PW_BISECTOR, 205), _case(64, pw.PW_BISECTOR, 206), _case(64, pw.PW_MIDPOINT, 207),
             _case(32, pw.PW_MIDPOINT, 208)]
    refs = [_fresh(c)[0] for c in cases]
    order = [0, 1, 2, 3, 1, 0, 3, 2, 0, 2]
    with pw.Context(0) as ctx:
        ctx.set_lanes(2)
        tickets = [ctx.submit(cases[i][0], cases[i][1], cases[i][2], ran_nbar=cases[i][3]) for i in order]
        for i, t in zip(order, tickets):
            got = t.wait()
            assert _close(got["values"], refs[i]["values"])
        # lane 0 after the served stream: its own workspace is intact (or re-made)
        cfg, gx, rx, nb = cases[1]
        again = ctx.estimate(cfg, gx, rx, ran_nbar=nb)
        assert _close(again["values"], refs[1]["values"])
