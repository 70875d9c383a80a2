"""GPU parity of the bisector P_l path (libpw through the C ABI) against the FP64 oracle."""
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


def _run(ctx, cfg, gal, ran, dtype):
    gx, g64 = rounded(gal, dtype)
    rx, r64 = rounded(ran, dtype)
    res = ctx.estimate(cfg, gx, rx, ran_nbar=ran["nbar"].astype(dtype))
    ref = pk_bisector(g64, r64, oracle_cfg(cfg))
    return res, ref


def _real_sh(J, mu, v):
    """y_J^mu from the oracle's complex harmonics: y^0 = Y^0, y^m = sqrt2 (-1)^m Re Y^m,
    y^-m = sqrt2 (-1)^m Im Y^m."""
    from oracle.ylm import Ylm
    if mu == 0:
        return Ylm(J, 0, v).real
    Y = Ylm(J, abs(mu), v)
    f = np.sqrt(2.0) * (-1) ** abs(mu)
    return f * (Y.real if mu > 0 else Y.imag)


def test_bisector_stages_fp64(ctx):
    """Painted mesh and retained spectra against the oracle's paint and numpy FFTs."""
    from oracle.estimators import density_masses, scalars
    from oracle.mesh import node_positions
    say("bisector stages fp64 N=32: paint + spectra")
    gal, ran = uniform_catalog(11, 2000, 6000, (0, 0, 1100), 400)
    cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=pw.PW_FP64,
                    n_mesh=32, box_len=800.0, box_origin=(-400.0, -400.0, 700.0), ell_max=2,
                    order=2, compensate=0, bin_lo=0.004, bin_width=0.02, n_bins=6)
    gx, g64 = rounded(gal, np.float64)
    rx, r64 = rounded(ran, np.float64)
    ctx.estimate(cfg, gx, rx, ran_nbar=ran["nbar"])
    oc = oracle_cfg(cfg)
    a, I, S = scalars(g64["w"], r64["w"], r64["nbar"])
    m = density_masses(g64, r64, oc, a)                     # [ix, iy, iz]
    mesh = ctx.inspect(0, np.float64).reshape(32, 32, 32)    # [z, y, x]
    err = np.max(np.abs(mesh - np.transpose(m, (2, 1, 0)))) / np.max(np.abs(m))
    say("paint rel err", err)
    assert err < 1e-12
    spec = ctx.inspect(1, np.float64).view(np.complex128)
    mc = ctx.inspect(2)
    nf = 16
    spec = spec.reshape(nf, -1)
    keep = mc != 0xFFFFFFFF                                  # padding slots carry no mode
    spec, mc = spec[:, keep], mc[keep]
    kx, ky, kz = mc & 0x7FF, (mc >> 11) & 0x7FF, (mc >> 22) & 0x3FF
    # the retained modes are distinct and are every half-spectrum mode up to the largest |n|^2
    assert len(np.unique(mc)) == len(mc)
    sg = lambda k: np.where(k < 16, k, k - 32)
    s2 = sg(kx) ** 2 + sg(ky) ** 2 + sg(kz) ** 2
    g = np.arange(32)
    ax, ay, az = np.meshgrid(g[:17], g, g, indexing="ij")
    full_s2 = np.where(ax == 16, 16, ax) ** 2 + sg(ay) ** 2 + sg(az) ** 2
    assert len(mc) == np.count_nonzero(full_s2 <= s2.max())
    xn = node_positions(32, 800.0, cfg.box_origin)
    for J in range(3):
        for mu in range(-J, J + 1):
            f = m * _real_sh(J, mu, xn)                   # [ix, iy, iz]
            ref = np.fft.fftn(f)                          # [kx, ky, kz]
            p = J * J + J + mu
            e = np.max(np.abs(spec[p] - ref[kx, ky, kz])) / np.max(np.abs(ref))
            say("spectrum", J, mu, "rel err", e)
            assert e < 1e-12


def test_bisector_fp64_small_mesh(ctx):
    say("bisector P fp64 N=32 TSC uniform cube, ell<=4 order 4")
    gal, ran = uniform_catalog(1, 3000, 9000, (0, 0, 1100), 400)
    cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=pw.PW_FP64,
                    n_mesh=32, box_len=800.0, box_origin=(-400.0, -400.0, 700.0), ell_max=4,
                    order=4, compensate=1, bin_lo=0.004, bin_width=0.02, n_bins=12)
    res, ref = _run(ctx, cfg, gal, ran, np.float64)
    assert np.array_equal(res["counts"], ref.counts)
    assert np.allclose(res["bin_mean"], ref.bin_mean, rtol=1e-12)
    err = max_err_per_ell(res["values"], ref.values)
    say("fp64 err per ell", err)
    assert np.all(err < 1e-10)
    a, I, S = res["norm"]
    assert a == pytest.approx(ref.alpha_r, rel=1e-12)
    assert I == pytest.approx(ref.I, rel=1e-12)
    assert S == pytest.approx(ref.S, rel=1e-12)


@pytest.mark.parametrize("assign", [pw.PW_CIC, pw.PW_TSC] if hasattr(pw, "PW_CIC") else [])
def test_bisector_fp32_ragged_bins(ctx, assign):
    say("bisector P fp32 N=64 assign", assign, "bins past Nyquist (ragged pruning)")
    gal, ran = uniform_catalog(2, 20000, 60000, (0, 0, 1200), 600)
    cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=assign, prec=pw.PW_FP32,
                    n_mesh=64, box_len=1000.0, box_origin=(-500.0, -500.0, 700.0), ell_max=4,
                    order=4, compensate=1, bin_lo=0.003, bin_width=0.0117, n_bins=27)
    res, ref = _run(ctx, cfg, gal, ran, np.float32)
    assert np.array_equal(res["counts"], ref.counts)
    err = max_err_per_ell(res["values"], ref.values)
    say("fp32 err per ell", err)
    assert np.all(err < 1e-4)


@pytest.mark.parametrize("ell_max,order", [(0, 0), (2, 0), (2, 2), (4, 2)])
def test_bisector_orders(ctx, ell_max, order):
    say("bisector P fp32 N=32 ell_max", ell_max, "order", order)
    gal, ran = uniform_catalog(3, 5000, 15000, (100, -50, 900), 300)
    cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=pw.PW_FP32,
                    n_mesh=32, box_len=700.0, box_origin=(-250.0, -400.0, 550.0), ell_max=ell_max,
                    order=order, compensate=0, bin_lo=0.0, bin_width=0.025, n_bins=10)
    res, ref = _run(ctx, cfg, gal, ran, np.float32)
    err = max_err_per_ell(res["values"], ref.values)
    say("err", err)
    assert np.all(err < 1e-4)


@pytest.mark.parametrize("ell_max,order,prec", [(4, 6, pw.PW_FP32), (4, 8, pw.PW_FP64), (6, 6, pw.PW_FP64),
                                                (8, 8, pw.PW_FP32), (8, 8, pw.PW_FP64)])
def test_bisector_high_orders(ctx, ell_max, order, prec):
    """beta_max up to 4 and ell_max up to 8 (up to 169 real fields): the table-driven
    contraction with smaller blocks so that every field value of a block fits in LDS."""
    dtype = np.float64 if prec == pw.PW_FP64 else np.float32
    say("bisector P", "fp64" if prec == pw.PW_FP64 else "fp32", "N=32 ell_max", ell_max, "order", order)
    gal, ran = uniform_catalog(51, 2000, 6000, (0, 0, 1100), 400)
    cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=prec, n_mesh=32,
                    box_len=800.0, box_origin=(-400.0, -400.0, 700.0), ell_max=ell_max, order=order,
                    compensate=1, bin_lo=0.004, bin_width=0.012, n_bins=8)
    res, ref = _run(ctx, cfg, gal, ran, dtype)
    assert np.array_equal(res["counts"], ref.counts)
    err = max_err_per_ell(res["values"], ref.values)
    say("err", err)
    assert np.all(err < (1e-10 if prec == pw.PW_FP64 else 1e-4))


def test_bisector_lognormal_cone_n128(ctx):
    say("bisector P fp32 N=128 lognormal cone (C3 geometry, 2e5 galaxies)")
    gal, ran = make_workload_catalog("C3", index=7, n_gal=200_000)
    cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=pw.PW_FP32,
                    n_mesh=128, box_len=2700.0, box_origin=(-1350.0, -1350.0, -200.0),
                    ell_max=4, order=4, compensate=1, bin_lo=0.005, bin_width=0.005, n_bins=29)
    res, ref = _run(ctx, cfg, gal, ran, np.float32)
    assert np.array_equal(res["counts"], ref.counts)
    err = max_err_per_ell(res["values"], ref.values)
    say("err", err)
    assert np.all(err < 1e-4)


def test_out_of_box_particle_is_rejected(ctx):
    say("bisector P out-of-box particle -> PW_ERANGE")
    gal, ran = uniform_catalog(4, 100, 300, (0, 0, 1000), 200)
    gal["pos"][5] = (0.0, 0.0, 5000.0)
    cfg = pw.Config(n_mesh=16, box_len=400.0, box_origin=(-200.0, -200.0, 800.0), n_bins=4,
                    bin_lo=0.01, bin_width=0.02)
    gx, _ = rounded(gal, np.float32)
    rx, _ = rounded(ran, np.float32)
    with pytest.raises(pw.PwError) as e:
        ctx.estimate(cfg, gx, rx, ran_nbar=ran["nbar"].astype(np.float32))
    assert e.value.code == pw.PW_ERANGE
