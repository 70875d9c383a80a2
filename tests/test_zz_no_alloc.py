"""pw_estimate_noalloc (the estimate in the library's static device scratch) against
pw_estimate on the same inputs: two calls in a row with the second on a smaller catalog, then
another estimator in the same scratch; the refusals (host catalogs, an estimate too large for
the scratch) come before anything runs."""
import numpy as np
import pytest

from oracle.estimators import pk_bisector

from gpu_common import say, rounded, oracle_cfg, max_err_per_ell, uniform_catalog

pytestmark = pytest.mark.gpu

pw = pytest.importorskip("paper_2102_08384_amd.pw")
torch = pytest.importorskip("torch")

SAME = 1e-12   # the two entry points run the same kernels; FP64 shell sums differ in order only


def _cfg(**kw):
    base = dict(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=pw.PW_FP32, n_mesh=64,
                box_len=1000.0, box_origin=(-500.0, -500.0, 600.0), ell_max=4, order=4, compensate=1,
                bin_lo=0.005, bin_width=0.02, n_bins=9)
    base.update(kw)
    return pw.Config(**base)


def _dev(seed, n_gal, n_ran, side):
    gal, ran = uniform_catalog(seed, n_gal, n_ran, (0, 0, 1000), side)
    gx, g64 = rounded(gal, np.float32)
    rx, r64 = rounded(ran, np.float32)
    nb = ran["nbar"].astype(np.float32)
    return [torch.from_numpy(a).cuda() for a in (gx, rx, nb)], (g64, r64)


def _same(a, b):
    assert np.array_equal(a["counts"], b["counts"])
    # FP64 sums over a bin's modes: the two calls may run the contraction with different
    # workgroup counts (the estimate's autotuned choice, the scratch call's settled one or the
    # default), which adds the same terms in another order
    assert np.allclose(a["bin_mean"], b["bin_mean"], rtol=1e-13, atol=0)
    assert np.allclose(a["norm"], b["norm"], rtol=1e-14, atol=0)
    err = max_err_per_ell(a["values"], b["values"])
    assert np.all(err < SAME), err


def test_noalloc_equals_estimate_twice_then_smaller_and_other_estimator():
    big, _ = _dev(301, 60000, 180000, 420)
    small, (g64, r64) = _dev(302, 9000, 23000, 380)
    cfg = _cfg()
    mid = _cfg(los=pw.PW_MIDPOINT, n_mesh=32, box_origin=(-500.0, -500.0, 500.0))
    with pw.Context(0) as ctx:
        say("noalloc: bisector 64^3, 2.4e5 particles")
        a1 = ctx.estimate_noalloc(cfg, *big[:2], ran_nbar=big[2])
        say("noalloc: bisector 64^3, 3.2e4 particles (second call, smaller)")
        a2 = ctx.estimate_noalloc(cfg, *small[:2], ran_nbar=small[2])
        say("noalloc: midpoint 32^3 in the same scratch")
        a3 = ctx.estimate_noalloc(mid, *small[:2], ran_nbar=small[2])
        say("pw_estimate on the same inputs")
        e1 = ctx.estimate(cfg, *big[:2], ran_nbar=big[2])
        e2 = ctx.estimate(cfg, *small[:2], ran_nbar=small[2])
        e3 = ctx.estimate(mid, *small[:2], ran_nbar=small[2])
        # and once more after pw_estimate has run on the context
        a4 = ctx.estimate_noalloc(cfg, *small[:2], ran_nbar=small[2])
    for a, e in ((a1, e1), (a2, e2), (a3, e3), (a4, e2)):
        _same(a, e)
    ref = pk_bisector(g64, r64, oracle_cfg(cfg))
    err = max_err_per_ell(a2["values"], ref.values)
    say("noalloc vs oracle per ell", err)
    assert np.all(err < 1e-4)


def test_noalloc_refusals():
    small, _ = _dev(303, 2000, 6000, 300)
    with pw.Context(0) as ctx:
        with pytest.raises(pw.PwError) as ei:
            ctx.estimate_noalloc(_cfg(), small[0].cpu().numpy(), small[1].cpu().numpy(),
                                 ran_nbar=small[2].cpu().numpy())
        assert ei.value.code == pw.PW_EINVAL and "device-resident" in ctx.last_error()
        with pytest.raises(pw.PwError) as ei:
            ctx.estimate_noalloc(_cfg(n_mesh=256), *small[:2], ran_nbar=small[2])
        assert ei.value.code == pw.PW_ENOMEM and "static scratch" in ctx.last_error()
        # the context is still usable afterwards
        r = ctx.estimate_noalloc(_cfg(n_mesh=32), *small[:2], ran_nbar=small[2])
        e = ctx.estimate(_cfg(n_mesh=32), *small[:2], ran_nbar=small[2])
    _same(r, e)
