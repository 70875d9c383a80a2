"""The memory-lean bisector P_l (memory_lean = 1): the forward transforms run in groups of
fields through group-sized work buffers.  Every field's transforms are computed by the same
kernels as before, so the k-sphere spectra the contraction reads must equal the default path's
bit for bit, at a fraction of its device memory.  The shell sums accumulate with FP64 atomics
in no fixed order, so the binned multipoles of any two runs agree to rounding, not bitwise."""
import dataclasses

import numpy as np
import pytest

from oracle.estimators import pk_bisector
from synthetic import make_workload_catalog

from gpu_common import say, rounded, oracle_cfg, max_err_per_ell, uniform_catalog

pytestmark = pytest.mark.gpu

pw = pytest.importorskip("paper_2102_08384_amd.pw")


@pytest.fixture(scope="module")
def ctx():
    c = pw.Context(0)
    yield c
    c.close()


def _close(a, b):
    """Two runs of the same arithmetic: equal up to the order of the FP64 shell sums."""
    return np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def _cone_cfg(prec, n_mesh=128, **kw):
    return pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=prec, n_mesh=n_mesh,
                     box_len=2700.0, box_origin=(-1350.0, -1350.0, -200.0), ell_max=4, order=4, compensate=1,
                     bin_lo=0.005, bin_width=0.005, n_bins=29, **kw)


@pytest.mark.parametrize("prec", [pw.PW_FP32, pw.PW_FP64])
def test_lean_equals_default_bitwise_and_oracle(ctx, prec):
    dtype = np.float64 if prec == pw.PW_FP64 else np.float32
    say("lean bisector", "fp64" if prec == pw.PW_FP64 else "fp32", "N=128 cone: lean vs default vs oracle")
    gal, ran = make_workload_catalog("C3", index=9, n_gal=150_000)
    gx, g64 = rounded(gal, dtype)
    rx, r64 = rounded(ran, dtype)
    nb = ran["nbar"].astype(dtype)
    cfg = _cone_cfg(prec)
    base = ctx.estimate(cfg, gx, rx, ran_nbar=nb)
    sph_base = ctx.inspect(1, dtype).copy()
    lean = ctx.estimate(dataclasses.replace(cfg, memory_lean=1), gx, rx, ran_nbar=nb)
    sph_lean = ctx.inspect(1, dtype)
    assert np.array_equal(sph_lean, sph_base)
    assert _close(lean["values"], base["values"])
    assert np.array_equal(lean["counts"], base["counts"])
    ref = pk_bisector(g64, r64, oracle_cfg(cfg))
    err = max_err_per_ell(lean["values"], ref.values)
    say("lean err per ell", err)
    assert np.all(err < (1e-10 if prec == pw.PW_FP64 else 1e-4))


def test_lean_orders_and_high_order(ctx):
    """The one-pass per-order contraction and the table-driven high-order contraction read the
    lean path's k-sphere exactly as the default one's."""
    say("lean bisector: per-order outputs, and ell_max 4 order 8 (fp64 N=32)")
    gal, ran = uniform_catalog(61, 3000, 9000, (0, 0, 1100), 400)
    gx, _ = rounded(gal, np.float64)
    rx, _ = rounded(ran, np.float64)
    cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=pw.PW_FP64, n_mesh=32,
                    box_len=800.0, box_origin=(-400.0, -400.0, 700.0), ell_max=4, order=4, compensate=1,
                    bin_lo=0.004, bin_width=0.012, n_bins=8)
    a = ctx.estimate_orders(cfg, gx, rx, ran_nbar=ran["nbar"])
    b = ctx.estimate_orders(dataclasses.replace(cfg, memory_lean=1), gx, rx, ran_nbar=ran["nbar"])
    assert _close(b["values"], a["values"])
    hi = dataclasses.replace(cfg, order=8)
    a = ctx.estimate(hi, gx, rx, ran_nbar=ran["nbar"])
    sph_a = ctx.inspect(1, np.float64).copy()
    b = ctx.estimate(dataclasses.replace(hi, memory_lean=1), gx, rx, ran_nbar=ran["nbar"])
    assert np.array_equal(ctx.inspect(1, np.float64), sph_a)
    assert _close(b["values"], a["values"])


def test_lean_fits_where_default_does_not():
    """A budget between the two footprints: the default plan is refused (PW_ENOMEM), the lean
    one runs and matches a default run on an unconstrained context."""
    say("lean bisector: N=256 under a budget only the lean plan fits")
    gal, ran = make_workload_catalog("C3", index=11, n_gal=100_000)
    gx, _ = rounded(gal, np.float32)
    rx, _ = rounded(ran, np.float32)
    nb = ran["nbar"].astype(np.float32)
    cfg = _cone_cfg(pw.PW_FP32, n_mesh=256)
    lean_cfg = dataclasses.replace(cfg, memory_lean=1)
    need_default = pw.footprint(cfg, len(gx), len(rx))
    need_lean = pw.footprint(lean_cfg, len(gx), len(rx))
    say("footprints: default", need_default, "lean", need_lean)
    assert need_lean < 0.6 * need_default
    budget = (need_lean + need_default) // 2
    with pw.Context(0, hbm_budget=budget) as small:
        with pytest.raises(pw.PwError) as e:
            small.estimate(cfg, gx, rx, ran_nbar=nb)
        assert e.value.code == pw.PW_ENOMEM
        got = small.estimate(lean_cfg, gx, rx, ran_nbar=nb)
    with pw.Context(0) as big:
        ref = big.estimate(cfg, gx, rx, ran_nbar=nb)
    assert _close(got["values"], ref["values"])
