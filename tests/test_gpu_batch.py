"""Batched launches (pw_estimate_batch and the serving loop's batching): several catalogs of one
bisector P_l configuration go through each forward pass and the contraction in one launch
(fields x catalogs).  Every catalog's result equals its pw_estimate result alone (to FP64
rounding of the shell sums, which are combined across workgroups in the order they finish) and
the oracle."""
import numpy as np
import pytest

from oracle.estimators import pk_bisector

from gpu_common import say, rounded, oracle_cfg, max_err_per_ell, uniform_catalog

pytestmark = pytest.mark.gpu

pw = pytest.importorskip("paper_2102_08384_amd.pw")
torch = pytest.importorskip("torch")


def _cfg(**kw):
    base = dict(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=pw.PW_FP32, n_mesh=64,
                box_len=1000.0, box_origin=(-500.0, -500.0, 600.0), ell_max=4, order=4, compensate=1,
                bin_lo=0.005, bin_width=0.02, n_bins=9)
    base.update(kw)
    return pw.Config(**base)


def _cat(seed, n_gal, dtype, device, side=420.0):
    gal, ran = uniform_catalog(seed, n_gal, 3 * n_gal, (0, 0, 1000), side)
    gx, g64 = rounded(gal, dtype)
    rx, r64 = rounded(ran, dtype)
    nb = ran["nbar"].astype(dtype)
    arrs = (gx, rx, nb)
    if device:
        arrs = tuple(torch.from_numpy(a).cuda() for a in arrs)
    return arrs, (g64, r64)


def _same(a, b, tol):
    assert np.array_equal(a["counts"], b["counts"])
    assert np.allclose(a["bin_mean"], b["bin_mean"], rtol=1e-14, atol=0)
    assert np.allclose(a["norm"], b["norm"], rtol=1e-13, atol=0)
    err = max_err_per_ell(a["values"], b["values"])
    assert np.all(err < tol), err


@pytest.mark.parametrize("prec", [pw.PW_FP64, pw.PW_FP32])
def test_batch_equals_alone_and_oracle(prec):
    dt = np.float64 if prec == pw.PW_FP64 else np.float32
    say("batch: 3 catalogs of different sizes, 64^3, prec", prec)
    cats = [_cat(401 + i, n, dt, device=(i != 1)) for i, n in enumerate((9000, 3000, 15000))]
    cfg = _cfg(prec=prec)
    with pw.Context(0) as ctx:
        batch = ctx.estimate_batch(cfg, [c[0] for c in cats])
        alone = [ctx.estimate(cfg, *c[0][:2], ran_nbar=c[0][2]) for c in cats]
    for b, a in zip(batch, alone):
        _same(b, a, 1e-12)
    tol = 1e-10 if prec == pw.PW_FP64 else 1e-4
    for b, c in zip(batch, cats):
        ref = pk_bisector(*c[1], oracle_cfg(cfg))
        err = max_err_per_ell(b["values"], ref.values)
        say("batch vs oracle per ell", err)
        assert np.all(err < tol)


def test_batch_of_eight_at_128_and_reuse():
    """The largest batch at 128^3 (FP32, device inputs), then a smaller batch on the same context
    (the batch plans and workspace are reused)."""
    say("batch: 8 catalogs at 128^3, then 3")
    cats = [_cat(501 + i, 4000 + 1500 * i, np.float32, device=True)[0] for i in range(8)]
    cfg = _cfg(n_mesh=128)
    with pw.Context(0) as ctx:
        b8 = ctx.estimate_batch(cfg, cats)
        b3 = ctx.estimate_batch(cfg, cats[5:])
        alone = [ctx.estimate(cfg, *c[:2], ran_nbar=c[2]) for c in cats]
    for b, a in zip(b8, alone):
        _same(b, a, 1e-12)
    for b, a in zip(b3, alone[5:]):
        _same(b, a, 1e-12)


def test_batch_of_other_estimators_runs_one_after_another():
    say("batch: midpoint P_l (no batched path) and the memory-lean bisector")
    cats = [_cat(601 + i, 5000, np.float32, device=True)[0] for i in range(2)]
    for cfg in (_cfg(los=pw.PW_MIDPOINT, n_mesh=32, box_origin=(-500.0, -500.0, 500.0)), _cfg(memory_lean=1)):
        with pw.Context(0) as ctx:
            batch = ctx.estimate_batch(cfg, cats)
            alone = [ctx.estimate(cfg, *c[:2], ran_nbar=c[2]) for c in cats]
        for b, a in zip(batch, alone):
            _same(b, a, 1e-12)


def test_batch_errors_write_nothing():
    say("batch: argument errors and a particle outside the box")
    good = _cat(701, 3000, np.float32, device=False)[0]
    bad_g = good[0].copy()
    bad_g[7, 0] = 5000.0  # outside [box_origin, box_origin + box_len)
    with pw.Context(0) as ctx:
        with pytest.raises(pw.PwError) as ei:
            ctx.estimate_batch(_cfg(), [good] * 9)
        assert ei.value.code == pw.PW_EINVAL
        with pytest.raises(pw.PwError) as ei:
            ctx.estimate_batch(_cfg(), [good, (bad_g, good[1], good[2])])
        assert ei.value.code == pw.PW_ERANGE
        # the context still works
        r = ctx.estimate_batch(_cfg(), [good, good])
        a = ctx.estimate(_cfg(), *good[:2], ran_nbar=good[2])
    for b in r:
        _same(b, a, 1e-12)


def test_serving_batches_pending_requests_of_one_configuration():
    """One serving lane: while the first request runs, the next ones of the same 128^3
    configuration wait and are then admitted together in batched launches; a 64^3 request in
    between is not batched with them.  Every result equals the request alone."""
    say("serving: batched admission of same-configuration requests")
    cfg128 = _cfg(n_mesh=128)
    cfg64 = _cfg()
    cats = [_cat(801 + i, 6000 + 500 * i, np.float32, device=True)[0] for i in range(7)]
    with pw.Context(0) as ctx:
        ctx.set_lanes(1)
        order = [(cfg128, c) for c in cats[:4]] + [(cfg64, cats[4])] + [(cfg128, c) for c in cats[4:]]
        tickets = [ctx.submit(cfg, *c[:2], ran_nbar=c[2]) for cfg, c in order]
        res = [t.wait() for t in tickets]
        launches, requests = ctx.serving_stats()
        alone = [ctx.estimate(cfg, *c[:2], ran_nbar=c[2]) for cfg, c in order]
    say("serving launches", launches, "requests", requests)
    assert requests == len(order)
    assert launches < requests
    for r, a in zip(res, alone):
        _same(r, a, 1e-12)
