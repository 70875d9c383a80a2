"""Pins of the oracle's estimators: pair sums on node-placed tiny catalogs (exact equality),
zeroth order = Yamamoto, monopole invariance, convergence to the exact line of sight,
painting invariants."""
import numpy as np
import pytest

from oracle import brute
from oracle.estimators import (Config, scalars, pk_bisector, pk_midpoint, pk_yamamoto,
                               xi_bisector, xi_midpoint)
from oracle.mesh import paint, CIC, TSC
from synthetic import tiny_node_catalog

N, L, B0 = 16, 1000.0, (-500.0, -500.0, 1000.0)


def _tiny(seed=5, **kw):
    return tiny_node_catalog(seed, N, L, B0, **kw)


def _cfg_pk(order, ells=(0, 2, 4)):
    # 4 bins up to 0.045 < k_Nyq = 0.0503: no Nyquist-plane modes
    return Config(N=N, L=L, b0=B0, assign=CIC, ells=ells, order=order, compensate=False,
                  bin_lo=0.005, bin_width=0.01, n_bins=4)


def _cfg_xi(order, ells=(0, 2, 4)):
    return Config(N=N, L=L, b0=B0, assign=CIC, ells=ells, order=order, compensate=False,
                  bin_lo=0.0, bin_width=100.0, n_bins=4)


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


# ---------------------------------------------------------------- painting

def test_paint_conserves_mass_and_node_particles_hit_one_node():
    rng = np.random.default_rng(0)
    pos = rng.uniform(-400, 400, size=(500, 3)) + np.array([0, 0, 1500.0])
    w = rng.uniform(0.2, 2.0, 500)
    for a in (CIC, TSC):
        m = paint(pos, w, 32, 1000.0, (-500, -500, 1000), a)
        assert m.sum() == pytest.approx(w.sum(), rel=1e-13)
    gal, _ = _tiny()
    m = paint(gal["pos"], gal["w"], N, L, B0, CIC)
    idx = np.rint((gal["pos"] - np.array(B0)) / (L / N)).astype(int)
    ref = np.zeros((N, N, N))
    np.add.at(ref, (idx[:, 0], idx[:, 1], idx[:, 2]), gal["w"])
    assert np.allclose(m, ref, atol=1e-14)
    # TSC of a node particle: (1/8, 3/4, 1/8) per axis
    one = {"pos": np.array([[B0[0] + 5 * L / N, B0[1] + 6 * L / N, B0[2] + 7 * L / N]])}
    mt = paint(one["pos"], [1.0], N, L, B0, TSC)
    k1 = np.array([0.125, 0.75, 0.125])
    assert np.allclose(mt[4:7, 5:8, 6:9], k1[:, None, None] * k1[None, :, None] * k1[None, None, :])
    assert mt.sum() == pytest.approx(1.0)


def test_paint_periodic_wrap():
    # a particle just below L - H/2 from b0 spreads onto node 0 (TSC) and node N-1
    u = N - 0.3
    pos = np.array([[B0[0] + u * L / N, B0[1] + 3 * L / N, B0[2] + 3 * L / N]])
    m = paint(pos, [1.0], N, L, B0, TSC)
    assert m[0].sum() > 0 and m[N - 1].sum() > 0 and m.sum() == pytest.approx(1.0)


# ---------------------------------------------------------------- pair sums (exact)

@pytest.mark.parametrize("order", [0, 2, 4])
def test_bisector_pk_equals_series_pair_sum(order):
    gal, ran = _tiny()
    cfg = _cfg_pk(order)
    norm = scalars(gal["w"], ran["w"], ran["nbar"])
    r = pk_bisector(gal, ran, cfg, norm)
    bp, counts = brute.pk_pairs(gal, ran, cfg, "bis_series", norm)
    assert np.array_equal(r.counts, counts.astype(int))
    assert _rel(r.values, bp) < 1e-12


@pytest.mark.parametrize("order", [0, 2, 4])
def test_midpoint_pk_equals_series_pair_sum(order):
    gal, ran = _tiny(seed=7)
    cfg = _cfg_pk(order)
    norm = scalars(gal["w"], ran["w"], ran["nbar"])
    r = pk_midpoint(gal, ran, cfg, norm)
    bp, _ = brute.pk_pairs(gal, ran, cfg, "mid_series", norm)
    assert _rel(r.values, bp) < 1e-12


def test_yamamoto_pk_equals_pair_sum():
    gal, ran = _tiny(seed=8)
    cfg = _cfg_pk(0)
    norm = scalars(gal["w"], ran["w"], ran["nbar"])
    r = pk_yamamoto(gal, ran, cfg, norm)
    bp, _ = brute.pk_pairs(gal, ran, cfg, "yamamoto", norm)
    assert _rel(r.values, bp) < 1e-12


@pytest.mark.parametrize("order", [2, 4])
def test_bisector_xi_equals_series_pair_sum(order):
    gal, ran = _tiny(seed=9)
    cfg = _cfg_xi(order)
    norm = scalars(gal["w"], ran["w"], ran["nbar"])
    r = xi_bisector(gal, ran, cfg, norm)
    bp, counts = brute.xi_pairs(gal, ran, cfg, "bis_series", norm)
    assert np.array_equal(r.counts, counts.astype(int))
    assert _rel(r.values, bp) < 1e-12


@pytest.mark.parametrize("order", [2, 4])
def test_midpoint_xi_equals_series_pair_sum(order):
    gal, ran = _tiny(seed=10)
    cfg = _cfg_xi(order)
    norm = scalars(gal["w"], ran["w"], ran["nbar"])
    r = xi_midpoint(gal, ran, cfg, norm)
    bp, _ = brute.xi_pairs(gal, ran, cfg, "mid_series", norm)
    assert _rel(r.values, bp) < 1e-12


# ---------------------------------------------------------------- all-parity midpoint

@pytest.mark.parametrize("order", [1, 2, 3])
def test_midpoint_allparity_pk_equals_series_pair_sum(order):
    """Section 3.2 all-parity estimator (every alpha <= K, coefficients phi) against the pair
    sum of the symmetrised shift-theorem series, exactly."""
    gal, ran = _tiny(seed=15)
    cfg = _cfg_pk(order)
    cfg.parity = "all"
    norm = scalars(gal["w"], ran["w"], ran["nbar"])
    r = pk_midpoint(gal, ran, cfg, norm)
    bp, _ = brute.pk_pairs(gal, ran, cfg, "mid_series_all", norm)
    assert _rel(r.values, bp) < 1e-12


@pytest.mark.parametrize("order", [1, 3])
def test_midpoint_allparity_xi_equals_series_pair_sum(order):
    """Section 4.2 all-parity estimator (coefficients f) against the pair sum of the
    symmetrised Legendre shift series, exactly."""
    gal, ran = _tiny(seed=16)
    cfg = _cfg_xi(order)
    cfg.parity = "all"
    norm = scalars(gal["w"], ran["w"], ran["nbar"])
    r = xi_midpoint(gal, ran, cfg, norm)
    bp, _ = brute.xi_pairs(gal, ran, cfg, "mid_series_all", norm)
    assert _rel(r.values, bp) < 1e-12


def test_midpoint_allparity_zeroth_order_and_monopole():
    """At K = 0 both forms are Yamamoto (phi^0 = Phi^0, f^0 = F^0 = delta); the monopole has
    no alpha > 0 term in either form (phi^{alpha,00} = sqrt(4pi) delta_alpha0)."""
    gal, ran = _generic(seed=17)
    base = dict(N=32, L=1000.0, b0=(-500, -500, 700), assign=TSC, compensate=True, bin_lo=0.01,
                bin_width=0.02, n_bins=6)
    e0 = pk_midpoint(gal, ran, Config(ells=(0, 2, 4), order=0, **base)).values
    a0 = pk_midpoint(gal, ran, Config(ells=(0, 2, 4), order=0, parity="all", **base)).values
    assert _rel(a0, e0) < 1e-13
    for K in (1, 2, 3):
        aK = pk_midpoint(gal, ran, Config(ells=(0,), order=K, parity="all", **base)).values[0]
        assert _rel(aK, e0[0]) < 1e-12


def test_midpoint_allparity_converges_to_exact_line_of_sight():
    """The all-parity series approaches the exact midpoint pair sum as K grows (Section 3.1:
    truncating at alpha = K leaves O(theta^{K+1})); at equal order it is at least as close as
    the parity-even form, which needs 2 eps << 1 rather than eps << 1 (Section 3.3)."""
    gal, ran = _tiny(seed=18)
    norm = scalars(gal["w"], ran["w"], ran["nbar"])
    cfg = _cfg_pk(0, ells=(2,))
    exact, _ = brute.pk_pairs(gal, ran, cfg, "mid_exact", norm)
    errs = []
    for K in range(0, 5):
        c = _cfg_pk(K, ells=(2,))
        c.parity = "all"
        errs.append(np.max(np.abs(pk_midpoint(gal, ran, c, norm).values - exact)))
    assert errs[2] < 0.5 * errs[0] and errs[4] < 0.5 * errs[2]
    c = _cfg_pk(4, ells=(2,))
    even4 = np.max(np.abs(pk_midpoint(gal, ran, c, norm).values - exact))
    assert errs[4] <= 1.5 * even4


# ---------------------------------------------------------------- terms of one order

@pytest.mark.parametrize("los,order", [("bis", 2), ("bis", 4), ("mid", 2), ("mid", 4)])
def test_single_order_pk_equals_series_pair_sum(los, order):
    """order_lo = order keeps one order's terms alone (midpoint alpha = order, bisector
    beta = order/2, Sections 3.3 and 5.2): it equals the pair sum over those terms only, its
    monopole vanishes (no shot noise: the monopole has no term beyond zeroth order), and the
    single-order pieces add up to the full truncated estimate."""
    gal, ran = _tiny(seed=11 if los == "bis" else 12)
    norm = scalars(gal["w"], ran["w"], ran["nbar"])
    est = pk_bisector if los == "bis" else pk_midpoint
    kind = "bis_series" if los == "bis" else "mid_series"
    one = _cfg_pk(order)
    one.order_lo = order
    r = est(gal, ran, one, norm)
    bp, _ = brute.pk_pairs(gal, ran, one, kind, norm)
    assert _rel(r.values, bp) < 1e-10
    assert np.max(np.abs(r.values[0])) < 1e-12 * np.max(np.abs(r.values))
    parts = [est(gal, ran, _cfg_pk(0), norm).values]
    for o in range(2, order + 1, 2):
        c = _cfg_pk(order)
        c.order_lo, c.order = o, o
        parts.append(est(gal, ran, c, norm).values)
    full = est(gal, ran, _cfg_pk(order), norm).values
    assert _rel(np.sum(parts, axis=0), full) < 1e-12


@pytest.mark.parametrize("los", ["bis", "mid"])
def test_single_order_xi_equals_series_pair_sum(los):
    gal, ran = _tiny(seed=13 if los == "bis" else 14)
    norm = scalars(gal["w"], ran["w"], ran["nbar"])
    est = xi_bisector if los == "bis" else xi_midpoint
    kind = "bis_series" if los == "bis" else "mid_series"
    cfg = _cfg_xi(4)
    cfg.order_lo = 4
    r = est(gal, ran, cfg, norm)
    bp, _ = brute.xi_pairs(gal, ran, cfg, kind, norm)
    # one order's terms are small against the products they are summed from (FP64 rounding
    # of the cancellation), hence 1e-10 rather than 1e-12
    assert _rel(r.values, bp) < 1e-10


# ---------------------------------------------------------------- structural identities

def _generic(seed=3, n_gal=300, n_ran=900):
    rng = np.random.default_rng(seed)
    c = np.array([0.0, 0.0, 1200.0])
    gal = {"pos": c + rng.uniform(-200, 200, (n_gal, 3)), "w": rng.uniform(0.5, 1.5, n_gal)}
    ran = {"pos": c + rng.uniform(-200, 200, (n_ran, 3)), "w": rng.uniform(0.5, 1.5, n_ran)}
    ran["nbar"] = np.full(n_ran, 2e-5)
    gal["nbar"] = np.full(n_gal, 2e-5)
    return gal, ran


def test_midpoint_zeroth_order_is_yamamoto():
    gal, ran = _generic()
    cfg = Config(N=32, L=1000.0, b0=(-500, -500, 700), assign=TSC, ells=(0, 2, 4), order=0,
                 compensate=True, bin_lo=0.005, bin_width=0.02, n_bins=7)
    a = pk_midpoint(gal, ran, cfg)
    b = pk_yamamoto(gal, ran, cfg)
    assert np.max(np.abs(a.values - b.values)) < 1e-10 * np.max(np.abs(b.values))


def test_monopole_identical_across_lines_of_sight_and_orders():
    gal, ran = _generic(seed=4)
    base = dict(N=32, L=1000.0, b0=(-500, -500, 700), assign=TSC, compensate=True,
                bin_lo=0.005, bin_width=0.02, n_bins=7)
    ref = pk_yamamoto(gal, ran, Config(ells=(0,), order=0, **base)).values[0]
    for K in (0, 2, 4):
        m = pk_midpoint(gal, ran, Config(ells=(0,), order=K, **base)).values[0]
        b = pk_bisector(gal, ran, Config(ells=(0,), order=K, **base)).values[0]
        assert np.max(np.abs(m - ref)) < 1e-10 * np.max(np.abs(ref))
        assert np.max(np.abs(b - ref)) < 1e-10 * np.max(np.abs(ref))
    xbase = dict(base, bin_lo=0.0, bin_width=60.0, n_bins=5)
    x0 = xi_midpoint(gal, ran, Config(ells=(0,), order=0, **xbase)).values[0]
    for K in (2, 4):
        xm = xi_midpoint(gal, ran, Config(ells=(0,), order=K, **xbase)).values[0]
        xb = xi_bisector(gal, ran, Config(ells=(0,), order=K, **xbase)).values[0]
        assert np.max(np.abs(xm - x0)) < 1e-10 * np.max(np.abs(x0))
        assert np.max(np.abs(xb - x0)) < 1e-10 * np.max(np.abs(x0))


def test_bisector_zeroth_order_is_not_yamamoto():
    gal, ran = _generic(seed=5)
    cfg = Config(N=32, L=1000.0, b0=(-500, -500, 700), assign=TSC, ells=(2,), order=0,
                 compensate=True, bin_lo=0.005, bin_width=0.02, n_bins=7)
    a = pk_bisector(gal, ran, cfg).values
    b = pk_yamamoto(gal, ran, cfg).values
    assert np.max(np.abs(a - b)) > 1e-6 * np.max(np.abs(b))


# ---------------------------------------------------------------- convergence to the exact LOS

def test_series_converge_to_exact_line_of_sight():
    """Tiny far catalog (theta_max ~ 0.1): the difference to the exact-LOS pair sum
    shrinks by ~theta^2 per step of the series order."""
    Nl, Ll = 16, 800.0
    b0 = (-400.0, -400.0, 1800.0)
    gal, ran = tiny_node_catalog(21, Nl, Ll, b0, n_gal=15, n_ran=45, lo=4, hi=11)
    cfg0 = Config(N=Nl, L=Ll, b0=b0, assign=CIC, ells=(2,), order=0, compensate=False,
                  bin_lo=0.005, bin_width=0.012, n_bins=4)
    norm = scalars(gal["w"], ran["w"], ran["nbar"])
    for kind, fn, exact in (("mid", pk_midpoint, "mid_exact"), ("bis", pk_bisector, "bis_exact")):
        ex, _ = brute.pk_pairs(gal, ran, cfg0, exact, norm)
        errs = []
        for K in (0, 2, 4):
            cfg = Config(**{**cfg0.__dict__, "order": K})
            errs.append(np.max(np.abs(fn(gal, ran, cfg, norm).values - ex)))
        assert errs[1] < 0.1 * errs[0] and errs[2] < 0.1 * errs[1], (kind, errs)


def test_wide_angle_correction_shrinks_with_distance():
    """Moving a catalog outward by a factor s shrinks the correction beyond zeroth order,
    P_l(K=4) - P_l(K=0), roughly as s^-2 for both lines of sight (Section 7.2 shift test).
    (The midpoint and bisector directions of one pair differ by an angle ~ theta^2, so their
    difference is not used as a fourth-order pin.)"""
    Nl, Ll = 16, 800.0
    out = {"mid": [], "bis": []}
    for shift in (1000.0, 2000.0):
        b0 = (-400.0, -400.0, shift)
        gal, ran = tiny_node_catalog(23, Nl, Ll, b0, n_gal=15, n_ran=45, lo=4, hi=11)
        cfg = Config(N=Nl, L=Ll, b0=b0, assign=CIC, ells=(2,), order=4, compensate=False,
                     bin_lo=0.005, bin_width=0.012, n_bins=4)
        c0 = Config(**{**cfg.__dict__, "order": 0})
        norm = scalars(gal["w"], ran["w"], ran["nbar"])
        for kind, fn in (("mid", pk_midpoint), ("bis", pk_bisector)):
            out[kind].append(np.max(np.abs(fn(gal, ran, cfg, norm).values - fn(gal, ran, c0, norm).values)))
    s2 = ((2000.0 + 600.0) / (1000.0 + 600.0)) ** 2   # catalog centre distance ratio, squared
    for kind, v in out.items():
        ratio = v[0] / v[1]
        assert 0.6 * s2 < ratio < 1.6 * s2, (kind, ratio, s2)


def test_bisector_shell_path_equals_full_grid_path():
    """The memory-lean bisector (retained modes only) is the full-grid estimator."""
    from oracle.estimators import pk_bisector_shells
    rng = np.random.default_rng(71)
    gal = {"pos": np.array([0.0, 0.0, 1000.0]) + rng.uniform(-200, 200, (400, 3)),
           "w": rng.uniform(0.5, 1.5, 400), "nbar": np.full(400, 1e-4)}
    ran = {"pos": np.array([0.0, 0.0, 1000.0]) + rng.uniform(-200, 200, (1200, 3)),
           "w": rng.uniform(0.5, 1.5, 1200), "nbar": np.full(1200, 1e-4)}
    cfg = Config(N=32, L=900.0, b0=(-450.0, -450.0, 700.0), assign=3, ells=(0, 2, 4), order=4,
                 compensate=True, bin_lo=0.01, bin_width=0.03, n_bins=7)
    a = pk_bisector(gal, ran, cfg)
    b = pk_bisector_shells(gal, ran, cfg)
    assert np.array_equal(a.counts, b.counts)
    assert np.allclose(a.bin_mean, b.bin_mean, rtol=1e-14, atol=0)
    scale = np.max(np.abs(a.values[0]))
    assert np.max(np.abs(a.values - b.values)) < 1e-12 * scale


# ---------------------------------------------------------------- random-pair normalisation

def test_xi_window_equals_random_pair_sum():
    """The randoms-only multipoles R_L / (I v_a) equal the brute-force pair sum over the randoms
    alone, with the data's normalisation (node-placed tiny catalog, both lines of sight)."""
    from oracle.estimators import xi_window
    gal, ran = _tiny(seed=19)
    norm = scalars(gal["w"], ran["w"], ran["nbar"])
    cfg = _cfg_xi(2)
    for est, kind in ((xi_midpoint, "mid_series"), (xi_bisector, "bis_series")):
        w = xi_window(gal, ran, cfg, est, norm, L_max=4)
        empty = {k: np.zeros((0,) + np.asarray(v).shape[1:]) for k, v in gal.items()}
        bp, _ = brute.xi_pairs(empty, ran, cfg, kind, norm)
        assert _rel(w.values, bp) < 1e-12


def test_xi_window_matrix_against_quadrature():
    """M_{l l'} = (2l+1) sum_L (l L l'; 000)^2 f_L is the Legendre-product integral
    (2l+1) int dmu/2 L_l(mu) L_l'(mu) sum_L f_L L_L(mu), computed here by Gauss-Legendre
    quadrature (no 3j symbols); f_0 = 1 alone gives the identity."""
    from numpy.polynomial import legendre as npl
    from oracle.estimators import xi_window_matrix
    ells = [0, 2, 4]
    assert np.allclose(xi_window_matrix(ells, {0: 1.0}), np.eye(3), atol=1e-14)
    f = {0: 1.0, 2: -0.31, 4: 0.12, 6: -0.05, 8: 0.02}
    x, wq = npl.leggauss(40)
    P = {n: npl.legval(x, [0] * n + [1]) for n in range(9)}
    RR = sum(v * P[L] for L, v in f.items())
    ref = np.array([[(2 * l + 1) * np.sum(wq * P[l] * P[lp] * RR) / 2 for lp in ells] for l in ells])
    assert np.allclose(xi_window_matrix(ells, f), ref, atol=1e-13)


def test_xi_window_correction_recovers_multipoles():
    """With pair counts that follow RR(mu) xi(mu) exactly, N_l / R_0 mixes the multipoles through
    the window and the correction recovers them: build N_l / R_0 by quadrature from a chosen
    xi_l' and window f_L, then solve."""
    from numpy.polynomial import legendre as npl
    from oracle.estimators import xi_window_matrix
    ells = [0, 2, 4]
    f = {0: 1.0, 2: 0.4, 4: -0.2, 6: 0.1, 8: -0.03}
    xi_true = np.array([2.0, -0.7, 0.3])
    x, wq = npl.leggauss(40)
    P = {n: npl.legval(x, [0] * n + [1]) for n in range(9)}
    RR = sum(v * P[L] for L, v in f.items())
    xi_mu = sum(v * P[l] for l, v in zip(ells, xi_true))
    NR = np.array([(2 * l + 1) * np.sum(wq * P[l] * RR * xi_mu) / 2 for l in ells])
    assert not np.allclose(NR, xi_true)
    assert np.allclose(np.linalg.solve(xi_window_matrix(ells, f), NR), xi_true, rtol=1e-12)


def test_xi_normalized_is_ratio_of_estimates():
    """xi_RR = N_l / R_0 bin by bin (the data estimate over the randoms-only monopole, both with
    the data's 1 / (I v_a)), f_0 = 1, and a survey window has non-zero higher multipoles."""
    from oracle.estimators import xi_normalized, xi_window
    gal, ran = _generic(seed=20, n_gal=600, n_ran=3000)
    cfg = Config(N=32, L=1000.0, b0=(-500, -500, 700), assign=TSC, ells=(0, 2, 4), order=2,
                 compensate=True, bin_lo=20.0, bin_width=60.0, n_bins=6)
    norm = scalars(gal["w"], ran["w"], ran["nbar"])
    xr, xe, f = xi_normalized(gal, ran, cfg, xi_midpoint, norm)
    data = xi_midpoint(gal, ran, cfg, norm).values
    win = xi_window(gal, ran, cfg, xi_midpoint, norm).values
    assert np.allclose(xr, data / win[0][None, :], rtol=1e-12)
    assert np.allclose(f[0], 1.0)
    assert f.shape[0] == 5 and np.max(np.abs(f[1:])) > 1e-3


@pytest.mark.parametrize("n_mesh,slab", [(32, 5), (64, 16)])
def test_bisector_xi_streamed_equals_full_grid(tmp_path, n_mesh, slab):
    """The streamed bisector xi_l (transforms on disk, k-space sums slab by slab, separable
    inverse transform kept to the binned separations) is the full-grid estimator; the slab of
    5 rows leaves a ragged last slab and slabs that hold a row and its mirror."""
    from oracle.estimators import xi_bisector_streamed
    rng = np.random.default_rng(73)
    c = np.array([0.0, 0.0, 1000.0])
    gal = {"pos": c + rng.uniform(-200, 200, (400, 3)), "w": rng.uniform(0.5, 1.5, 400),
           "nbar": np.full(400, 1e-4)}
    ran = {"pos": c + rng.uniform(-200, 200, (1200, 3)), "w": rng.uniform(0.5, 1.5, 1200),
           "nbar": np.full(1200, 1e-4)}
    cfg = Config(N=n_mesh, L=900.0, b0=(-450.0, -450.0, 700.0), assign=CIC, ells=(0, 2, 4), order=4,
                 compensate=True, bin_lo=0.0, bin_width=40.0, n_bins=6)
    a = xi_bisector(gal, ran, cfg)
    b = xi_bisector_streamed(gal, ran, cfg, str(tmp_path), slab=slab)
    assert np.array_equal(a.counts, b.counts)
    assert np.allclose(a.bin_mean, b.bin_mean, rtol=1e-14, atol=0)
    scale = np.max(np.abs(a.values[0]))
    assert np.max(np.abs(a.values - b.values)) < 1e-12 * scale
    assert not list(tmp_path.iterdir())          # the spectra files are removed
