"""Host-only checks of libpw: it loads, exports every symbol include/pw.h declares, rejects
malformed configurations without touching a device, and its C++ coupling tables (rotated to the
real-harmonic basis) equal the oracle's complex tables rotated here independently."""
import ctypes
import math

import numpy as np
import pytest

from oracle import coeffs

pw = pytest.importorskip("paper_2102_08384_amd.pw")


def test_library_exports_every_declared_symbol():
    names = pw.declared_symbols()
    assert len(names) >= 10
    lib = ctypes.CDLL(pw.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def _U(l):
    """Y_l^m = sum_nu U[m, nu] y_l^nu for y_l^0 = Y_l^0, y_l^m = sqrt2 (-1)^m Re Y_l^m,
    y_l^-m = sqrt2 (-1)^m Im Y_l^m (m > 0)."""
    u = np.zeros((2 * l + 1, 2 * l + 1), dtype=complex)
    s = 1 / math.sqrt(2)
    for m in range(-l, l + 1):
        if m == 0:
            u[l, l] = 1
        elif m > 0:
            u[m + l, m + l] = (-1) ** m * s
            u[m + l, -m + l] = (-1) ** m * 1j * s
        else:
            u[m + l, -m + l] = s
            u[m + l, m + l] = -1j * s
    return u


def _idx(J, mu):
    return J * J + J + mu


def _rows_to_dict(rows, sym):
    d = {}
    for l, nu, J1, mu1, J2, mu2, v in rows:
        k = (int(l), int(nu), _idx(int(J1), int(mu1)), _idx(int(J2), int(mu2)))
        if sym:
            k = (k[0], k[1], min(k[2], k[3]), max(k[2], k[3]))
        d[k] = d.get(k, 0.0) + v
    return d


def test_real_harmonic_basis_reproduces_scipy():
    from oracle.ylm import Ylm
    rng = np.random.default_rng(0)
    v = rng.normal(size=(6, 3))
    for l in range(0, 7):
        U = _U(l)
        # y = U^-1 Y must be real
        Y = np.array([Ylm(l, m, v) for m in range(-l, l + 1)])
        y = np.linalg.solve(U, Y)
        assert np.max(np.abs(y.imag)) < 1e-13


@pytest.mark.parametrize("ell_max,order", [(2, 2), (4, 4), (4, 2)])
def test_bisector_table_matches_oracle(ell_max, order):
    bmax = order // 2
    exp = {}
    for l in range(0, ell_max + 1, 2):
        Ul = _U(l)
        for m in range(-l, l + 1):
            for (J1, J2, M), c in coeffs.B_table(bmax, l, m).items():
                U1 = _U(J1)[M + J1]
                U2 = _U(J2)[m - M + J2]
                for nu in range(-l, l + 1):
                    cl = np.conj(Ul[m + l, nu + l])
                    if cl == 0:
                        continue
                    for n1 in range(-J1, J1 + 1):
                        if U1[n1 + J1] == 0:
                            continue
                        for n2 in range(-J2, J2 + 1):
                            if U2[n2 + J2] == 0:
                                continue
                            p1, p2 = _idx(J1, n1), _idx(J2, n2)
                            k = (l, nu, min(p1, p2), max(p1, p2))
                            exp[k] = exp.get(k, 0) + cl * c * U1[n1 + J1] * U2[n2 + J2]
    exp = {k: v for k, v in exp.items() if abs(v) > 1e-12}
    assert max(abs(v.imag) for v in exp.values()) < 1e-12
    got = _rows_to_dict(pw.coupling_table(0, ell_max, order), True)
    assert set(got) == set(exp)
    for k in exp:
        assert got[k] == pytest.approx(exp[k].real, rel=1e-11, abs=1e-12)


@pytest.mark.parametrize("alpha", [2, 4])
def test_midpoint_table_matches_oracle(alpha):
    ell_max = 4
    exp = {}
    for l in range(0, ell_max + 1, 2):
        Ul = _U(l)
        for m in range(-l, l + 1):
            for (J1, J2, M), c in coeffs.Phi_table(alpha, l, m).items():
                U1 = _U(J1)[M + J1]
                U2 = _U(J2)[m - M + J2]
                for nu in range(-l, l + 1):
                    cl = np.conj(Ul[m + l, nu + l])
                    if cl == 0:
                        continue
                    for n1 in range(-J1, J1 + 1):
                        for n2 in range(-J2, J2 + 1):
                            val = cl * c * U1[n1 + J1] * U2[n2 + J2]
                            if val == 0:
                                continue
                            k = (l, nu, _idx(J1, n1), _idx(J2, n2))
                            exp[k] = exp.get(k, 0) + val
    exp = {k: v for k, v in exp.items() if abs(v) > 1e-12}
    assert max(abs(v.imag) for v in exp.values()) < 1e-11
    got = _rows_to_dict(pw.coupling_table(1, ell_max, 4, alpha), False)
    assert set(got) == set(exp)
    for k in exp:
        assert got[k] == pytest.approx(exp[k].real, rel=1e-10, abs=1e-11)


def test_legendre_F_table_matches_oracle():
    for alpha in (0, 2, 4):
        rows = pw.coupling_table(2, 4, 4, alpha)
        got = {(int(r[0]), int(r[2])): r[6] for r in rows}
        for l in (0, 2, 4):
            for J in range(0, l + alpha + 1, 2):
                v = coeffs.F(alpha, l, J)
                if abs(v) > 1e-12:
                    assert got[(l, J)] == pytest.approx(v, rel=1e-11)


@pytest.mark.parametrize("alpha", [1, 2, 3])
def test_midpoint_allparity_table_matches_oracle(alpha):
    """Real-basis all-parity coupling: the oracle's phi (Appendix B) with the (-1)^J2 of
    g^alpha_J2 (Section 3.2) folded in."""
    ell_max = 4
    exp = {}
    for l in range(0, ell_max + 1, 2):
        Ul = _U(l)
        for m in range(-l, l + 1):
            for (J1, J2, M), c in coeffs.phi_table(alpha, l, m).items():
                c = c * (-1) ** J2
                U1 = _U(J1)[M + J1]
                U2 = _U(J2)[m - M + J2]
                for nu in range(-l, l + 1):
                    cl = np.conj(Ul[m + l, nu + l])
                    if cl == 0:
                        continue
                    for n1 in range(-J1, J1 + 1):
                        for n2 in range(-J2, J2 + 1):
                            val = cl * c * U1[n1 + J1] * U2[n2 + J2]
                            if val == 0:
                                continue
                            k = (l, nu, _idx(J1, n1), _idx(J2, n2))
                            exp[k] = exp.get(k, 0) + val
    exp = {k: v for k, v in exp.items() if abs(v) > 1e-12}
    assert max(abs(v.imag) for v in exp.values()) < 1e-11
    got = _rows_to_dict(pw.coupling_table(3, ell_max, 4, alpha), False)
    assert set(got) == set(exp)
    for k in exp:
        assert got[k] == pytest.approx(exp[k].real, rel=1e-10, abs=1e-11)


def test_legendre_f_table_matches_oracle():
    for alpha in (0, 1, 2, 3, 4):
        rows = pw.coupling_table(4, 4, 4, alpha)
        got = {(int(r[0]), int(r[2])): r[6] for r in rows}
        n = 0
        for l in (0, 2, 4):
            for J in range(0, l + alpha + 1):
                v = coeffs.f(alpha, l, J)
                if abs(v) > 1e-12:
                    assert got[(l, J)] == pytest.approx(v, rel=1e-11)
                    n += 1
        assert n == len(got)


def test_memory_lean_footprint():
    """The memory-lean bisector keeps the k-sphere of every field plus one field group's x- and
    y-pass buffers: at the 512^3 headline configuration about a third of the default."""
    cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, n_mesh=512, box_len=2700.0,
                    box_origin=(-1350.0, -1350.0, -200.0), ell_max=4, order=4, bin_lo=0.005,
                    bin_width=0.005, n_bins=79)
    full = pw.footprint(cfg, 4_000_000, 20_000_000)
    cfg.memory_lean = 1
    lean = pw.footprint(cfg, 4_000_000, 20_000_000)
    assert lean < 0.4 * full
    cfg.memory_lean = 2
    with pytest.raises(pw.PwError):
        pw.footprint(cfg, 1000, 1000)


def test_footprint_and_validation_need_no_device():
    cfg = pw.Config(n_mesh=64, los=pw.PW_BISECTOR, stat=pw.PW_PK, ell_max=4, order=4,
                    bin_lo=0.01, bin_width=0.01, n_bins=20)
    b = pw.footprint(cfg, 10000, 50000)
    assert b > 64 ** 3 * 4
    bad = pw.Config(n_mesh=48)
    with pytest.raises(pw.PwError) as e:
        pw.footprint(bad, 1, 1)
    assert e.value.code == pw.PW_EINVAL
    bad = pw.Config(ell_max=3)
    with pytest.raises(pw.PwError):
        pw.footprint(bad, 1, 1)
    bad = pw.Config(bin_width=0.0)
    with pytest.raises(pw.PwError):
        pw.footprint(bad, 1, 1)


def test_tune_cache_file_is_loaded(tmp_path):
    """PW_TUNE_CACHE: the launch-shape choices a file holds make up the tuning table, without a
    device; malformed choices are skipped."""
    import ast
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    f = tmp_path / "tune.txt"
    f.write_text("fy:p0:N512:f28:a173:b93216 3\nfz:p0:N512:f28:a93216:b1 1\nbad -1\n")
    code = "from paper_2102_08384_amd import pw; print(pw.tune_entries())"
    env = dict(os.environ, PW_TUNE_CACHE=str(f))
    out = subprocess.run([sys.executable, "-c", code], env=env, cwd=root, capture_output=True, text=True,
                         check=True).stdout
    entries = ast.literal_eval(out.strip().splitlines()[-1])
    assert [(e["key"], e["choice"]) for e in entries] == [("fy:p0:N512:f28:a173:b93216", 3),
                                                          ("fz:p0:N512:f28:a93216:b1", 1)]
    assert all(e["ms_best"] == -1.0 and e["ms_default"] == -1.0 for e in entries)


def test_footprint_counts_records_and_staging_per_particle():
    """pw_footprint grows per particle by the tile-sorted record (4 values in the mesh
    precision) plus the host staging of its (x, y, z, w) record, and per random also by its
    nbar staging (steps of 16 particles keep the records' 256-byte padding and the sort's
    chunk count unchanged)."""
    for prec, rsz in ((pw.PW_FP32, 4), (pw.PW_FP64, 8)):
        cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, prec=prec, n_mesh=64, box_len=1000.0,
                        box_origin=(-500.0, -500.0, 500.0), ell_max=4, order=4, bin_lo=0.01,
                        bin_width=0.01, n_bins=10)
        base = pw.footprint(cfg, 1000, 5000)
        assert pw.footprint(cfg, 1016, 5000) - base == 16 * 8 * rsz
        assert pw.footprint(cfg, 1000, 5016) - base == 16 * 9 * rsz
