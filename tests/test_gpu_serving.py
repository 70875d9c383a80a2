"""Serving loop (pw_submit / pw_poll / pw_wait / pw_cancel): every request's result in a mixed,
concurrent stream equals its result alone (pw_estimate), and the stream matches the oracle."""
import dataclasses

import numpy as np
import pytest

from oracle.estimators import pk_bisector, pk_midpoint, xi_bisector, xi_midpoint

from gpu_common import say, rounded, oracle_cfg, max_err_per_ell, uniform_catalog

pytestmark = pytest.mark.gpu

pw = pytest.importorskip("paper_2102_08384_amd.pw")
torch = pytest.importorskip("torch")


def _requests():
    """A mix of estimators, meshes, precisions and catalog sizes."""
    reqs = []
    specs = [
        # (stat, los, N, prec, n_gal, seed, bins)
        (pw.PW_PK, pw.PW_BISECTOR, 64, pw.PW_FP32, 12000, 101, (0.005, 0.02, 9)),
        (pw.PW_PK, pw.PW_MIDPOINT, 64, pw.PW_FP32, 7000, 102, (0.005, 0.02, 9)),
        (pw.PW_XI, pw.PW_BISECTOR, 32, pw.PW_FP32, 4000, 103, (0.0, 40.0, 10)),
        (pw.PW_XI, pw.PW_MIDPOINT, 64, pw.PW_FP32, 9000, 104, (0.0, 25.0, 12)),
        (pw.PW_PK, pw.PW_BISECTOR, 32, pw.PW_FP64, 3000, 105, (0.005, 0.02, 9)),
        (pw.PW_PK, pw.PW_BISECTOR, 64, pw.PW_FP32, 15000, 106, (0.005, 0.02, 9)),
        (pw.PW_PK, pw.PW_MIDPOINT, 32, pw.PW_FP32, 5000, 107, (0.005, 0.02, 9)),
        # all-parity midpoint at an odd order, and the memory-lean bisector plan
        (pw.PW_PK, pw.PW_MIDPOINT, 32, pw.PW_FP32, 6000, 108, (0.005, 0.02, 9),
         dict(midpoint_parity=pw.PW_PARITY_ALL, order=3)),
        (pw.PW_PK, pw.PW_BISECTOR, 64, pw.PW_FP32, 11000, 109, (0.005, 0.02, 9), dict(memory_lean=1)),
    ]
    for i, spec in enumerate(specs):
        stat, los, N, prec, ng, seed, (lo, w, nb) = spec[:7]
        extra = spec[7] if len(spec) > 7 else {}
        gal, ran = uniform_catalog(seed, ng, 3 * ng, (0, 0, 1000), 440)
        cfg = pw.Config(stat=stat, los=los, assign=pw.PW_TSC, prec=prec, n_mesh=N, box_len=1000.0,
                        box_origin=(-500.0, -500.0, 600.0), ell_max=4, order=4 if los == pw.PW_MIDPOINT else 2,
                        compensate=1, bin_lo=lo, bin_width=w, n_bins=nb)
        cfg = dataclasses.replace(cfg, **extra)
        dt = np.float64 if prec == pw.PW_FP64 else np.float32
        gx, g64 = rounded(gal, dt)
        rx, r64 = rounded(ran, dt)
        nb_ = ran["nbar"].astype(dt)
        on_dev = i % 2 == 0   # alternate device-resident and host inputs
        if on_dev:
            gx, rx, nb_ = (torch.from_numpy(gx).cuda(), torch.from_numpy(rx).cuda(),
                           torch.from_numpy(nb_).cuda())
        reqs.append(dict(cfg=cfg, gx=gx, rx=rx, nbar=nb_, g64=g64, r64=r64))
    return reqs


def _oracle(cfg, g64, r64):
    oc = oracle_cfg(cfg)
    if cfg.midpoint_parity == pw.PW_PARITY_ALL:
        oc = dataclasses.replace(oc, parity="all")
    if cfg.stat == pw.PW_PK:
        return (pk_bisector if cfg.los == pw.PW_BISECTOR else pk_midpoint)(g64, r64, oc)
    return (xi_bisector if cfg.los == pw.PW_BISECTOR else xi_midpoint)(g64, r64, oc)


def test_mixed_stream_equals_alone_and_oracle():
    say("serving: 9 mixed requests on 3 lanes vs alone vs oracle")
    reqs = _requests()
    with pw.Context(0) as ctx:
        ctx.set_lanes(3)
        alone = [ctx.estimate(r["cfg"], r["gx"], r["rx"], ran_nbar=r["nbar"]) for r in reqs]
        # the same requests twice over, all in flight together
        tickets = [ctx.submit(r["cfg"], r["gx"], r["rx"], ran_nbar=r["nbar"]) for r in reqs + reqs]
        mixed = [t.wait() for t in tickets]
    for i, r in enumerate(reqs):
        a = alone[i]["values"]
        for m in (mixed[i], mixed[i + len(reqs)]):
            assert np.array_equal(m["counts"], alone[i]["counts"])
            e = max_err_per_ell(m["values"], a)
            assert np.all(e < 1e-10), (i, e)
        ref = _oracle(r["cfg"], r["g64"], r["r64"])
        e = max_err_per_ell(mixed[i]["values"], ref.values)
        say("request", i, "stat", r["cfg"].stat, "los", r["cfg"].los, "err vs oracle", e)
        assert np.all(e < 1e-4)


def test_budget_admission_serialises_requests():
    """With a budget that holds one request at a time, every request still completes."""
    say("serving: budget-limited admission (one request at a time)")
    reqs = _requests()[:4]
    need = max(pw.footprint(r["cfg"], len(r["gx"]), len(r["rx"])) for r in reqs)
    with pw.Context(0, hbm_budget=int(need * 1.3)) as ctx:
        ctx.set_lanes(3)
        tickets = [ctx.submit(r["cfg"], r["gx"], r["rx"], ran_nbar=r["nbar"]) for r in reqs]
        outs = [t.wait() for t in tickets]
        alone = [ctx.estimate(r["cfg"], r["gx"], r["rx"], ran_nbar=r["nbar"]) for r in reqs[:1]]
    assert np.all(max_err_per_ell(outs[0]["values"], alone[0]["values"]) < 1e-10)
    for r, o in zip(reqs, outs):
        ref = _oracle(r["cfg"], r["g64"], r["r64"])
        assert np.all(max_err_per_ell(o["values"], ref.values) < 1e-4)


def test_cancel_errors_and_never_fitting():
    say("serving: cancel, per-request error, request larger than the budget")
    reqs = _requests()
    with pw.Context(0) as ctx:
        ctx.set_lanes(1)
        # a request with a particle outside the box fails alone, the others are unaffected
        r0 = reqs[1]
        bad = np.array(r0["gx"] if isinstance(r0["gx"], np.ndarray) else r0["gx"].cpu().numpy())
        bad[0, 2] = 5000.0
        t_bad = ctx.submit(r0["cfg"], bad, r0["rx"], ran_nbar=r0["nbar"])
        ts = [ctx.submit(r["cfg"], r["gx"], r["rx"], ran_nbar=r["nbar"]) for r in reqs]
        # the last request has a configuration of its own: the serving loop batches pending
        # requests of one configuration, so with reqs[0]'s it could join their batch and be
        # running already; on its own it waits behind every earlier request
        last_cfg = dataclasses.replace(reqs[0]["cfg"], order=4)
        t_last = ctx.submit(last_cfg, reqs[0]["gx"], reqs[0]["rx"], ran_nbar=reqs[0]["nbar"])
        try:
            t_last.cancel()
            cancelled = True
        except pw.PwError as e:   # a request that has started runs to the end
            assert e.code == pw.PW_EBUSY
            cancelled = False
        with pytest.raises(pw.PwError) as ei:
            t_bad.wait()
        assert ei.value.code == pw.PW_ERANGE
        for t in ts:
            t.wait()
        if cancelled:
            with pytest.raises(pw.PwError) as ei:
                t_last.wait()
            assert ei.value.code == pw.PW_ECANCELED
        else:
            assert np.all(np.isfinite(t_last.wait()["values"]))
    with pw.Context(0, hbm_budget=1 << 20) as small:
        with pytest.raises(pw.PwError) as ei:
            small.submit(reqs[0]["cfg"], reqs[0]["gx"], reqs[0]["rx"], ran_nbar=reqs[0]["nbar"])
        assert ei.value.code == pw.PW_ENOMEM


def test_served_request_evicts_idle_estimate_plans():
    """Plans cached by pw_estimate (lane 0) give way to a served request when the budget is
    tight: with room for one plan, an estimate followed by a request of another
    configuration must still complete (it used to fail with PW_ENOMEM)."""
    say("serving: a served request evicts lane 0's cached plan")
    reqs = _requests()
    a, b = reqs[0], reqs[5]            # two bisector P_l at 64^3, different catalogs and sizes
    b = dict(b, cfg=dataclasses.replace(b["cfg"], order=4))   # a different configuration
    need = max(pw.footprint(r["cfg"], len(r["gx"]), len(r["rx"])) for r in (a, b))
    with pw.Context(0, hbm_budget=int(need * 1.4)) as ctx:
        ctx.set_lanes(1)
        ctx.estimate(a["cfg"], a["gx"], a["rx"], ran_nbar=a["nbar"])
        got = ctx.submit(b["cfg"], b["gx"], b["rx"], ran_nbar=b["nbar"]).wait()
        again = ctx.estimate(a["cfg"], a["gx"], a["rx"], ran_nbar=a["nbar"])
    ref = _oracle(b["cfg"], b["g64"], b["r64"])
    assert np.all(max_err_per_ell(got["values"], ref.values) < 1e-4)
    assert np.all(np.isfinite(again["values"]))


def test_dropped_tickets_wait_for_their_requests():
    """A ticket dropped while its request is pending or running waits for it before its
    output arrays and inputs are released; the context stays usable afterwards."""
    import gc
    say("serving: tickets dropped while pending")
    reqs = _requests()[:5]
    with pw.Context(0) as ctx:
        ctx.set_lanes(2)
        for r in reqs:
            ctx.submit(r["cfg"], r["gx"], r["rx"], ran_nbar=r["nbar"])   # ticket dropped at once
        gc.collect()
        r = reqs[0]
        alone = ctx.estimate(r["cfg"], r["gx"], r["rx"], ran_nbar=r["nbar"])
        served = ctx.submit(r["cfg"], r["gx"], r["rx"], ran_nbar=r["nbar"]).wait()
    assert np.all(max_err_per_ell(served["values"], alone["values"]) < 1e-10)
