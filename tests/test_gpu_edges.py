"""Edge cases of the C-ABI path against the FP64 oracle: an empty galaxy catalog under an
imposed normalisation, catalogs of 1 and of ragged sizes around the sort kernels' workgroup
and chunk sizes, and the smallest mesh (N = 16, a single paint tile) for every estimator."""
import dataclasses

import numpy as np
import pytest

from oracle.estimators import pk_bisector, pk_midpoint, xi_bisector, xi_midpoint

from gpu_common import say, rounded, oracle_cfg, max_err_per_ell, uniform_catalog

pytestmark = pytest.mark.gpu

pw = pytest.importorskip("paper_2102_08384_amd.pw")

ORACLE = {(pw.PW_PK, pw.PW_BISECTOR): pk_bisector, (pw.PW_PK, pw.PW_MIDPOINT): pk_midpoint,
          (pw.PW_XI, pw.PW_BISECTOR): xi_bisector, (pw.PW_XI, pw.PW_MIDPOINT): xi_midpoint}
CASES = [(pw.PW_PK, pw.PW_BISECTOR), (pw.PW_PK, pw.PW_MIDPOINT), (pw.PW_XI, pw.PW_BISECTOR),
         (pw.PW_XI, pw.PW_MIDPOINT)]


@pytest.fixture(scope="module")
def ctx():
    c = pw.Context(0)
    yield c
    c.close()


def _cfg(stat, los, n_mesh=32, box=800.0):
    if stat == pw.PW_PK:
        kny = np.pi * n_mesh / box
        width = 0.012
        bins = dict(bin_lo=0.004, bin_width=width, n_bins=int((kny - 0.004) / width))
    else:
        bins = dict(bin_lo=20.0, bin_width=40.0, n_bins=8)
    return pw.Config(stat=stat, los=los, assign=pw.PW_TSC, prec=pw.PW_FP64, n_mesh=n_mesh, box_len=box,
                     box_origin=(-box / 2, -box / 2, 1100.0 - box / 2), ell_max=4,
                     order=4 if los == pw.PW_MIDPOINT else 2, compensate=1, **bins)


def _scale_err(got, ref):
    return np.max(np.abs(got - ref)) / np.max(np.abs(ref[0]))


@pytest.mark.parametrize("stat,los", CASES)
def test_empty_galaxy_catalog_with_given_norm(ctx, stat, los):
    """No galaxies: the field is the randoms' -alpha_r w n_r alone; with the normalisation
    imposed the estimate is finite and equals the oracle's under the same normalisation."""
    say("edges: empty galaxy catalog", stat, los)
    gal, ran = uniform_catalog(301 + stat + 2 * los, 0, 4000, (0, 0, 1100), 400)
    cfg = _cfg(stat, los)
    gx, g64 = rounded(gal, np.float64)
    rx, r64 = rounded(ran, np.float64)
    assert len(gx) == 0
    norm = (0.25, 3.5e-4, 180.0)
    res = ctx.estimate(cfg, gx, rx, ran_nbar=ran["nbar"], norm=norm)
    ref = ORACLE[(stat, los)](g64, r64, oracle_cfg(cfg), norm=norm)
    assert np.all(np.isfinite(res["values"]))
    assert np.array_equal(res["counts"], ref.counts)
    err = _scale_err(res["values"], ref.values)
    say("err (monopole scale)", err)
    assert err < 1e-10


@pytest.mark.parametrize("n_gal", [1, 1023, 1025, 4097])
def test_tiny_and_ragged_catalogs(ctx, n_gal):
    """Catalog sizes around the sort kernels' 1024-thread workgroups and 4096-particle chunks,
    and a single galaxy; randoms of a prime count."""
    say("edges: bisector P, n_gal =", n_gal)
    gal, ran = uniform_catalog(320 + n_gal, n_gal, 7919, (0, 0, 1100), 400)
    cfg = _cfg(pw.PW_PK, pw.PW_BISECTOR)
    gx, g64 = rounded(gal, np.float64)
    rx, r64 = rounded(ran, np.float64)
    res = ctx.estimate(cfg, gx, rx, ran_nbar=ran["nbar"])
    ref = pk_bisector(g64, r64, oracle_cfg(cfg))
    assert np.array_equal(res["counts"], ref.counts)
    a, I, S = res["norm"]
    assert np.allclose([a, I, S], [ref.alpha_r, ref.I, ref.S], rtol=1e-12)
    err = max_err_per_ell(res["values"], ref.values)
    say("per-ell err", err)
    assert np.all(err < 1e-10)


@pytest.mark.parametrize("stat,los", CASES)
def test_smallest_mesh(ctx, stat, los):
    """N = 16: one paint tile holds the whole mesh, and every transform is one short pencil."""
    say("edges: N = 16", stat, los)
    gal, ran = uniform_catalog(340 + stat + 2 * los, 1500, 4500, (0, 0, 1100), 380)
    cfg = _cfg(stat, los, n_mesh=16)
    gx, g64 = rounded(gal, np.float64)
    rx, r64 = rounded(ran, np.float64)
    res = ctx.estimate(cfg, gx, rx, ran_nbar=ran["nbar"])
    ref = ORACLE[(stat, los)](g64, r64, oracle_cfg(cfg))
    assert np.array_equal(res["counts"], ref.counts)
    err = max_err_per_ell(res["values"], ref.values)
    say("per-ell err", err)
    assert np.all(err < 1e-10)
    # FP32 on the same mesh, to the FP32 tolerance
    c32 = dataclasses.replace(cfg, prec=pw.PW_FP32)
    gx32, _ = rounded(gal, np.float32)
    rx32, _ = rounded(ran, np.float32)
    r32 = ctx.estimate(c32, gx32, rx32, ran_nbar=ran["nbar"].astype(np.float32))
    ref32 = ORACLE[(stat, los)](rounded(gal, np.float32)[1], rounded(ran, np.float32)[1], oracle_cfg(c32))
    assert np.all(max_err_per_ell(r32["values"], ref32.values) < 1e-4)
