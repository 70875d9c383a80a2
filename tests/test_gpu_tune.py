"""Autotuned launch shapes (pw_set_tuning, pw_tune_entry) of the x pass, the column passes, the
tile paint and gather and the bisector contraction: every candidate shape computes the same
values as the default one, bit for bit on the mesh and the transforms, and the autotuner's first
launch (which times every candidate on the estimate's own data) leaves a correct estimate and a
table entry per pass."""
import numpy as np
import pytest

from oracle.estimators import pk_bisector, pk_midpoint, xi_midpoint

from gpu_common import say, rounded, oracle_cfg, max_err_per_ell, uniform_catalog

pytestmark = pytest.mark.gpu

pw = pytest.importorskip("paper_2102_08384_amd.pw")


def _close(a, b, tol=1e-12):
    """Same arithmetic, FP64 shell sums in another order."""
    return np.max(np.abs(a - b)) <= tol * np.max(np.abs(b))


def _cfg(stat, los, prec, n_mesh):
    bins = (dict(bin_lo=0.004, bin_width=0.012, n_bins=8) if stat == pw.PW_PK
            else dict(bin_lo=20.0, bin_width=40.0, n_bins=8))
    return pw.Config(stat=stat, los=los, assign=pw.PW_TSC, prec=prec, n_mesh=n_mesh, box_len=800.0,
                     box_origin=(-400.0, -400.0, 700.0), ell_max=4, order=4 if los == pw.PW_MIDPOINT else 2,
                     compensate=1, **bins)


@pytest.mark.parametrize("prec", [pw.PW_FP32, pw.PW_FP64])
def test_bisector_every_shape_same_spectra(prec):
    """Bisector P_l: the forward y and z passes under every candidate shape give the default's
    k-sphere spectra bit for bit."""
    dt = np.float32 if prec == pw.PW_FP32 else np.float64
    say("tune: bisector P N=64 every shape", "fp32" if prec == pw.PW_FP32 else "fp64")
    gal, ran = uniform_catalog(401, 6000, 18000, (0, 0, 1100), 400)
    gx, g64 = rounded(gal, dt)
    rx, r64 = rounded(ran, dt)
    nb = ran["nbar"].astype(dt)
    cfg = _cfg(pw.PW_PK, pw.PW_BISECTOR, prec, 64)
    with pw.Context(0) as ctx:
        ctx.set_tuning(0)
        base = ctx.estimate(cfg, gx, rx, ran_nbar=nb)
        sph = ctx.inspect(1, dt).copy()
        for mode in range(2, 8):   # candidates 0..5 (past the last one: the default)
            ctx.set_tuning(mode)
            res = ctx.estimate(cfg, gx, rx, ran_nbar=nb)
            assert np.array_equal(ctx.inspect(1, dt), sph), mode
            assert _close(res["values"], base["values"]), mode
        ctx.set_tuning(1)
        tuned = ctx.estimate(cfg, gx, rx, ran_nbar=nb)   # first launch: times the candidates
        assert np.array_equal(ctx.inspect(1, dt), sph)
        again = ctx.estimate(cfg, gx, rx, ran_nbar=nb)   # the cached choice
        assert np.array_equal(ctx.inspect(1, dt), sph)
    assert _close(tuned["values"], base["values"]) and _close(again["values"], base["values"])
    ref = pk_bisector(g64, r64, oracle_cfg(cfg))
    assert np.all(max_err_per_ell(base["values"], ref.values) < (1e-4 if prec == pw.PW_FP32 else 1e-10))
    entries = {e["key"].split(":")[0]: e for e in pw.tune_entries()}
    say("tuning table", pw.tune_entries())
    for k in ("fy", "fz"):
        assert k in entries
        assert entries[k]["choice"] >= 0


@pytest.mark.parametrize("stat", [pw.PW_PK, pw.PW_XI])
def test_midpoint_every_shape_same_values(stat):
    """Midpoint: the forward y pass, the fused z pass and the inverse y pass under every
    candidate shape give the default's multipoles, and the oracle's."""
    say("tune: midpoint N=32 fp64 every shape", "pk" if stat == pw.PW_PK else "xi")
    gal, ran = uniform_catalog(411 + stat, 3000, 9000, (0, 0, 1100), 400)
    gx, g64 = rounded(gal, np.float64)
    rx, r64 = rounded(ran, np.float64)
    cfg = _cfg(stat, pw.PW_MIDPOINT, pw.PW_FP64, 32)
    with pw.Context(0) as ctx:
        ctx.set_tuning(0)
        base = ctx.estimate(cfg, gx, rx, ran_nbar=ran["nbar"])
        for mode in (2, 3, 4, 5, 1):
            ctx.set_tuning(mode)
            res = ctx.estimate(cfg, gx, rx, ran_nbar=ran["nbar"])
            assert _close(res["values"], base["values"]), mode
    ref = (pk_midpoint if stat == pw.PW_PK else xi_midpoint)(g64, r64, oracle_cfg(cfg))
    assert np.all(max_err_per_ell(base["values"], ref.values) < 1e-10)


def test_bisector_512_every_shape_same_mesh_and_spectra():
    """FP32 bisector P_l at N = 512, where the x pass has its row-count candidates: under every
    candidate shape (x pass rows, paint threads, gather tiles per workgroup, contraction
    workgroups, column passes) the painted mesh and the k-sphere spectra equal the default's bit
    for bit, and the multipoles agree to FP64 rounding of the shell sums.  (The default path is
    held to the oracle at N = 512 by the full-size tests; an oracle run here would take minutes.)"""
    say("tune: bisector P N=512 fp32 every shape (x pass, paint, gather, contraction)")
    gal, ran = uniform_catalog(421, 60000, 180000, (0, 0, 1100), 400)
    gx, _ = rounded(gal, np.float32)
    rx, _ = rounded(ran, np.float32)
    nb = ran["nbar"].astype(np.float32)
    # a small k-sphere (|n| <= 5) keeps the spectra copied to the host small
    cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=pw.PW_FP32, n_mesh=512,
                    box_len=800.0, box_origin=(-400.0, -400.0, 700.0), ell_max=4, order=2, compensate=1,
                    bin_lo=0.004, bin_width=0.008, n_bins=4)
    with pw.Context(0) as ctx:
        ctx.set_tuning(0)
        base = ctx.estimate(cfg, gx, rx, ran_nbar=nb)
        mesh = ctx.inspect(0, np.float32).copy()
        sph = ctx.inspect(1, np.float32).copy()
        for mode in range(2, 8):   # candidates 0..5 of every pass (past a pass's last: its default)
            say("shape candidate", mode - 2)
            ctx.set_tuning(mode)
            res = ctx.estimate(cfg, gx, rx, ran_nbar=nb)
            assert np.array_equal(ctx.inspect(0, np.float32), mesh), mode
            assert np.array_equal(ctx.inspect(1, np.float32), sph), mode
            assert _close(res["values"], base["values"]), mode
        say("autotuned")
        ctx.set_tuning(1)
        tuned = ctx.estimate(cfg, gx, rx, ran_nbar=nb)
        assert np.array_equal(ctx.inspect(1, np.float32), sph)
    assert _close(tuned["values"], base["values"])
    entries = {e["key"].split(":")[0] for e in pw.tune_entries()}
    say("tuned passes", sorted(entries))
    assert {"fx", "fy", "fz", "paint", "gather", "contract"} <= entries


def test_tuning_mode_validation():
    with pw.Context(0) as ctx:
        with pytest.raises(pw.PwError):
            ctx.set_tuning(-1)


def test_stale_cache_choice_falls_back_to_default(tmp_path):
    """A PW_TUNE_CACHE entry whose choice no longer exists selects the default shape, once,
    without re-timing the candidates on every launch (run in a process of its own, since the
    cache file is read at first use)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    say("tune: stale cache entry")
    code = r'''
import numpy as np
from paper_2102_08384_amd import pw
from gpu_common import rounded, uniform_catalog
gal, ran = uniform_catalog(431, 3000, 9000, (0, 0, 1100), 400)
gx, _ = rounded(gal, np.float32); rx, _ = rounded(ran, np.float32)
cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=pw.PW_FP32, n_mesh=32, box_len=800.0,
                box_origin=(-400.0, -400.0, 700.0), ell_max=4, order=2, compensate=1, bin_lo=0.004,
                bin_width=0.012, n_bins=8)
with pw.Context(0) as ctx:
    a = ctx.estimate(cfg, gx, rx, ran_nbar=ran["nbar"].astype(np.float32))
    b = ctx.estimate(cfg, gx, rx, ran_nbar=ran["nbar"].astype(np.float32))
    ctx.set_tuning(0)
    c = ctx.estimate(cfg, gx, rx, ran_nbar=ran["nbar"].astype(np.float32))
assert np.max(np.abs(a["values"] - c["values"])) <= 1e-5 * np.max(np.abs(c["values"]))
assert np.max(np.abs(b["values"] - c["values"])) <= 1e-5 * np.max(np.abs(c["values"]))
print(pw.tune_entries())
'''
    f = tmp_path / "tune.txt"
    env = dict(os.environ, PW_TUNE_CACHE=str(f), PYTHONPATH=os.pathsep.join([root, os.path.join(root, "tests")]))
    f.write_text("")
    first = subprocess.run([sys.executable, "-c", code], env=env, cwd=root, capture_output=True, text=True,
                           timeout=240)
    assert first.returncode == 0, first.stderr[-2000:]
    keys = [line.split()[0] for line in f.read_text().splitlines() if line.strip()]
    assert keys
    f.write_text("".join(f"{k} 99\n" for k in keys))   # choices that do not exist
    second = subprocess.run([sys.executable, "-c", code], env=env, cwd=root, capture_output=True, text=True,
                            timeout=240)
    assert second.returncode == 0, second.stderr[-2000:]
    assert f.read_text().count("\n") == len(keys)       # nothing re-tuned, nothing appended
