"""Pins of the oracle's coupling coefficients against what the paper and the mathematics fix:
printed worked examples (complete term lists), closed-form special cases, selection rules,
and series truncation slopes on random geometry."""
import math

import numpy as np
import pytest

from oracle import coeffs
from oracle.ylm import Ylm, legendre

SQ4PI = math.sqrt(4 * math.pi)


# ---------------------------------------------------------------- 3j / Gaunt

def test_wigner3j_known_values():
    # (1 1 0; 0 0 0) = -1/sqrt(3); (1 1 2; 1 -1 0) = 1/sqrt(30); (2 2 2; 0 0 0) = -sqrt(2/35)
    assert coeffs.wigner3j(1, 1, 0, 0, 0, 0) == pytest.approx(-1 / math.sqrt(3), rel=1e-15)
    assert coeffs.wigner3j(1, 1, 2, 1, -1, 0) == pytest.approx(1 / math.sqrt(30), rel=1e-15)
    assert coeffs.wigner3j(2, 2, 2, 0, 0, 0) == pytest.approx(-math.sqrt(2 / 35), rel=1e-15)
    # orthogonality: sum_{m1 m2} (j1 j2 j3; m1 m2 m3)^2 = 1/(2 j3 + 1)
    for j1, j2, j3 in [(2, 3, 4), (3, 3, 2), (4, 2, 6)]:
        s = sum(coeffs.wigner3j(j1, j2, j3, m1, -m1 - 1, 1) ** 2
                for m1 in range(-j1, j1 + 1))
        assert s == pytest.approx(1 / (2 * j3 + 1), rel=1e-13)


def test_gaunt_is_integral_of_three_harmonics():
    # G^{m1 m2 m3}_{l1 l2 l3} = int dOmega Y Y Y, checked by Gauss-Legendre x trapezoid quadrature
    nth, nph = 40, 80
    x, wx = np.polynomial.legendre.leggauss(nth)
    th = np.arccos(x)
    ph = np.arange(nph) * 2 * np.pi / nph
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    v = np.stack([np.sin(TH) * np.cos(PH), np.sin(TH) * np.sin(PH), np.cos(TH)], axis=-1)
    W = wx[:, None] * (2 * np.pi / nph)
    for (l1, l2, l3, m1, m2) in [(2, 2, 2, 1, -2), (1, 3, 2, 1, 0), (4, 2, 2, -1, 2), (3, 1, 2, 2, -1)]:
        m3 = -m1 - m2
        integ = np.sum(W * Ylm(l1, m1, v) * Ylm(l2, m2, v) * Ylm(l3, m3, v))
        assert coeffs.gaunt(l1, l2, l3, m1, m2, m3) == pytest.approx(integ.real, abs=1e-12)
        assert abs(integ.imag) < 1e-12


def test_ctilde_inverts_legendre_powers():
    mu = np.linspace(-1, 1, 7)
    for n in range(0, 9):
        rec = sum(coeffs.ctilde(n, L) * legendre(L, mu) for L in range(n, -1, -2))
        assert np.allclose(rec, mu ** n, atol=1e-14)


def test_gegenbauer_coefficients_reproduce_generating_function():
    # [1 - 2 s t + t^2]^-a = sum_N C_N^(a)(s) t^N
    for a2 in (1, 2, 3, 4, 6):
        a = a2 / 2
        s, t = 0.3, 0.05
        lhs = (1 - 2 * s * t + t * t) ** (-a)
        rhs = 0.0
        for N in range(0, 30):
            rhs += sum(float(coeffs.gegenbauer_coef(N, k, a2)) * (2 * s) ** (N - 2 * k)
                       for k in range(N // 2 + 1)) * t ** N
        assert rhs == pytest.approx(lhs, rel=1e-13)


# ---------------------------------------------------------------- harmonics

def test_ylm_addition_theorem_and_orthonormality():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(5, 3))
    y = rng.normal(size=(5, 3))
    mu = np.sum(x * y, 1) / np.linalg.norm(x, axis=1) / np.linalg.norm(y, axis=1)
    for l in range(0, 9):
        s = sum(Ylm(l, m, x) * np.conj(Ylm(l, m, y)) for m in range(-l, l + 1))
        assert np.allclose(s, (2 * l + 1) / (4 * np.pi) * legendre(l, mu), atol=1e-13)
        for m in range(-l, l + 1):
            # Y^* = (-1)^m Y^{-m};  Y(-x) = (-1)^l Y(x)
            assert np.allclose(np.conj(Ylm(l, m, x)), (-1) ** m * Ylm(l, -m, x), atol=1e-14)
            assert np.allclose(Ylm(l, m, -x), (-1) ** l * Ylm(l, m, x), atol=1e-14)


# ---------------------------------------------------------------- printed worked examples

def _complete(table_fn, printed, tol=1e-13):
    """printed: {(idx): value}; table_fn(idx) -> value; also checks no printed-index-set gaps."""
    for key, val in printed.items():
        assert table_fn(*key) == pytest.approx(val, rel=tol, abs=tol), key


def test_phi_matches_printed_Y21_all_parity(golden):
    rows = golden("phi_Y21_all_parity.txt")
    printed = {(a, J1, J2, M): v for (a, J1, M, J2), v in rows}
    for (a, J1, J2, M), v in printed.items():
        assert coeffs.phi(a, 2, 1, J1, J2, M) == pytest.approx(v, rel=1e-13)
    # completeness: no other non-zero phi^{alpha,21} for alpha <= 2
    for a in range(3):
        for J1 in range(0, a + 1):
            for J2 in range(0, 2 + a + 1):
                for M in range(-J1, J1 + 1):
                    if (a, J1, J2, M) not in printed:
                        assert abs(coeffs.phi(a, 2, 1, J1, J2, M)) < 1e-14, (a, J1, J2, M)


def test_Phi_matches_printed_Y21_parity_even(golden):
    rows = golden("Phi_Y21_parity_even.txt")
    printed = {(a, J1, J2, M): v for (a, J1, M, J2), v in rows}
    for a in (0, 2):
        tab = coeffs.Phi_table(a, 2, 1)
        got = {(a,) + k: v for k, v in tab.items() if abs(v) > 1e-14}
        exp = {k: v for k, v in printed.items() if k[0] == a}
        assert set(got) == set(exp)
        for k, v in exp.items():
            assert got[k] == pytest.approx(v, rel=1e-13)


def test_f_matches_printed_L2_all_parity(golden):
    for (l, a, J), v in golden("f_L2_all_parity.txt"):
        assert (2 * J + 1) / (2 * l + 1) * coeffs.f(a, l, J) == pytest.approx(v, rel=1e-13, abs=1e-14)
    printed = {(l, a, J) for (l, a, J), _ in golden("f_L2_all_parity.txt")}
    for a in range(5):
        for J in range(0, 2 + a + 1):
            if (2, a, J) not in printed:
                assert abs(coeffs.f(a, 2, J)) < 1e-14


def test_F_matches_printed_L2_L4_parity_even(golden):
    rows = golden("F_L2_L4_parity_even.txt")
    printed = {k for k, _ in rows}
    for (l, a, J), v in rows:
        assert (2 * J + 1) / (2 * l + 1) * coeffs.F(a, l, J) == pytest.approx(v, rel=1e-12)
    for l in (2, 4):
        for a in (0, 2, 4):
            for J in range(0, l + a + 1):
                if (l, a, J) not in printed:
                    assert abs(coeffs.F(a, l, J)) < 1e-12, (l, a, J)


def test_B_matches_printed_Y21_bisector(golden):
    rows = golden("B_Y21_bisector.txt")
    printed = {(b, J1, J2, M): v for (b, J1, M, J2), v in rows}
    for b in (0, 1):
        got = {}
        for J1 in range(0, 2 + b + 1):
            for J2 in range(0, 2 + b + 1):
                for M in range(-J1, J1 + 1):
                    val = coeffs.B(b, 2, 1, J1, J2, M)
                    if abs(val) > 1e-14:
                        got[(b, J1, J2, M)] = val
        exp = {k: v for k, v in printed.items() if k[0] == b}
        assert set(got) == set(exp)
        for k, v in exp.items():
            assert got[k] == pytest.approx(v, rel=1e-13)


# ---------------------------------------------------------------- closed-form special cases

@pytest.mark.parametrize("l", [0, 1, 2, 3, 4, 6])
def test_zeroth_order_and_monopole_special_cases(l):
    for m in range(-l, l + 1):
        for J1 in range(0, 3):
            for J2 in range(0, l + 3):
                for M in range(-J1, J1 + 1):
                    exp = SQ4PI if (J1 == 0 and J2 == l and M == 0) else 0.0
                    assert coeffs.phi(0, l, m, J1, J2, M) == pytest.approx(exp, abs=1e-14)
    for a in range(0, 6):
        for J1 in range(0, a + 1):
            for J2 in range(0, a + 1):
                for M in range(-J1, J1 + 1):
                    exp = SQ4PI if (a == 0 and J1 == 0 and J2 == 0 and M == 0) else 0.0
                    assert coeffs.phi(a, 0, 0, J1, J2, M) == pytest.approx(exp, abs=1e-13)
    # f^{0,l}_J = d_{lJ};  f^{alpha,0}_J = d_{alpha0} d_{J0}
    for J in range(0, l + 4):
        assert coeffs.f(0, l, J) == pytest.approx(1.0 if J == l else 0.0, abs=1e-14)
    for a in range(0, 6):
        for J in range(0, a + 1):
            assert coeffs.f(a, 0, J) == pytest.approx(1.0 if (a == 0 and J == 0) else 0.0, abs=1e-13)


@pytest.mark.parametrize("l", [0, 2, 3, 4])
def test_bisector_zeroth_order_and_monopole(l):
    for m in range(-l, l + 1):
        for J1 in range(0, l + 1):
            for J2 in range(0, l + 1):
                for M in range(-J1, J1 + 1):
                    exp = 2.0 ** (-l) * coeffs.A_coef(l, m, J1, M) if J2 == l - J1 else 0.0
                    assert coeffs.B(0, l, m, J1, J2, M) == pytest.approx(exp, abs=1e-13)
    # B^{beta,00} = sqrt(4pi) d d d d_{beta 0}
    for b in range(0, 4):
        for J1 in range(0, b + 1):
            for J2 in range(0, b + 1):
                exp = SQ4PI if (b == 0 and J1 == 0 and J2 == 0) else 0.0
                assert coeffs.B(b, 0, 0, J1, J2, 0) == pytest.approx(exp, abs=1e-13)


def test_selection_rules():
    for l in (2, 3, 4):
        for m in range(0, l + 1):
            for a in range(0, 5):
                for J1 in range(0, a + 1):
                    for J2 in range(0, l + a + 1):
                        for M in range(-J1, J1 + 1):
                            if (a + J1) % 2 or (l + a + J2) % 2:
                                assert coeffs.phi(a, l, m, J1, J2, M) == 0.0
            for b in range(0, 3):
                for J1 in range(0, l + b + 1):
                    for J2 in range(0, l + b + 1):
                        if (l + J1 + J2) % 2:
                            for M in range(-J1, J1 + 1):
                                assert coeffs.B(b, l, m, J1, J2, M) == 0.0


def test_full_legendre_coefficients_sum_to_zero_beyond_zeroth_order():
    # L_l(1) = 1 forces sum_J (2J+1)/(2l+1) f^{alpha,l}_J = d_{alpha 0} (reading of Appendix E:
    # the sum vanishes for the full coefficients, not for f itself)
    for l in range(0, 7):
        for a in range(0, 7):
            s = sum((2 * J + 1) / (2 * l + 1) * coeffs.f(a, l, J) for J in range(0, l + a + 1))
            assert s == pytest.approx(1.0 if a == 0 else 0.0, abs=1e-11)
    assert coeffs.f(1, 2, 1) + coeffs.f(1, 2, 3) != pytest.approx(0.0)


def test_Phi4_recursion_equals_appendix_D_explicit_form():
    for l in (2, 4):
        for m in (0, 1, l):
            tab = coeffs.Phi_table(4, l, m)
            for J1 in range(0, 5, 2):
                for J2 in range(0, l + 5, 2):
                    for M in range(-J1, J1 + 1):
                        assert tab.get((J1, J2, M), 0.0) == pytest.approx(
                            coeffs.Phi4_explicit(l, m, J1, J2, M), abs=1e-12)


def test_parity_even_legendre_F4_is_five_f4_for_quadrupole_and_hexadecapole():
    # a consequence visible in the printed numbers of Section 4.3
    for l in (2, 4):
        for J in range(0, l + 5, 2):
            assert coeffs.F(4, l, J) == pytest.approx(5 * coeffs.f(4, l, J), rel=1e-12, abs=1e-13)


# ---------------------------------------------------------------- truncation slopes

def _rand_geometry(seed):
    rng = np.random.default_rng(seed)
    R = rng.normal(size=3)
    R /= np.linalg.norm(R)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    return R, d


def _slope(errs, ratio=2.0):
    return [math.log(errs[i] / errs[i + 1]) / math.log(ratio) for i in range(len(errs) - 1)]


@pytest.mark.parametrize("l,m", [(2, 1), (4, 3), (2, 0), (4, 0)])
def test_shift_theorem_all_parity_truncation_slope(l, m):
    R, d = _rand_geometry(11)
    for K in (0, 1, 2, 3):
        errs = []
        for eps in (0.02, 0.01, 0.005):
            A = R
            a = d * eps
            approx = sum(coeffs.phi(al, l, m, J1, J2, M) * eps ** al * Ylm(J1, M, a) * Ylm(J2, m - M, A)
                         for al in range(K + 1) for J1 in range(al + 1) for J2 in range(max(0, l - al), l + al + 1)
                         for M in range(-J1, J1 + 1))
            errs.append(abs(approx - Ylm(l, m, a + A)))
        assert all(abs(s - (K + 1)) < 0.1 for s in _slope(errs)), (K, errs)


@pytest.mark.parametrize("l,m", [(2, 1), (4, 3), (4, 0)])
def test_midpoint_parity_even_truncation_slope(l, m):
    R, d = _rand_geometry(1)
    for K in (0, 2, 4):
        errs = []
        for th in (0.04, 0.02, 0.01) if K == 4 else (0.02, 0.01, 0.005):
            r1 = 1000 * (R - d * th / 2)
            r2 = 1000 * (R + d * th / 2)
            D = r2 - r1
            e1 = np.linalg.norm(D) / (2 * np.linalg.norm(r1))
            e2 = np.linalg.norm(D) / (2 * np.linalg.norm(r2))
            s = 0.0
            for a in range(0, K + 1, 2):
                for (J1, J2, M), c in coeffs.Phi_table(a, l, m).items():
                    s += 0.5 * c * Ylm(J1, M, D) * (e1 ** a * Ylm(J2, m - M, r1) + e2 ** a * Ylm(J2, m - M, r2))
            errs.append(abs(s - Ylm(l, m, r1 + r2)))
        assert all(abs(x - (K + 2)) < 0.1 for x in _slope(errs)), (K, errs)


@pytest.mark.parametrize("l,m", [(2, 1), (4, 3), (2, 0)])
def test_bisector_truncation_slope(l, m):
    R, d = _rand_geometry(2)
    for bmax in (0, 1, 2):
        errs = []
        for th in (0.16, 0.08, 0.04) if bmax == 2 else (0.04, 0.02, 0.01):
            r1 = 1300 * (R - d * th / 2)
            r2 = 1000 * (R + d * th / 2)
            bis = r1 / np.linalg.norm(r1) + r2 / np.linalg.norm(r2)
            s = sum(c * Ylm(J1, M, r1) * Ylm(J2, m - M, r2) for (J1, J2, M), c in coeffs.B_table(bmax, l, m).items())
            errs.append(abs(s - Ylm(l, m, bis)))
        assert all(abs(x - (2 * bmax + 2)) < 0.1 for x in _slope(errs)), (bmax, errs)


@pytest.mark.parametrize("l", [2, 4])
def test_legendre_parity_even_truncation_slope(l):
    R, d = _rand_geometry(4)
    for K in (0, 2, 4):
        errs = []
        for th in (0.02, 0.01, 0.005):
            r1 = 1000 * (R - d * th / 2)
            r2 = 1000 * (R + d * th / 2)
            D = r2 - r1
            Dn = np.linalg.norm(D)
            Du = D / Dn
            mu1 = Du @ r1 / np.linalg.norm(r1)
            mu2 = Du @ r2 / np.linalg.norm(r2)
            e1 = Dn / (2 * np.linalg.norm(r1))
            e2 = Dn / (2 * np.linalg.norm(r2))
            s = 0.0
            for a in range(0, K + 1, 2):
                for J in range(0, l + a + 1, 2):
                    s += 0.5 * (2 * J + 1) / (2 * l + 1) * coeffs.F(a, l, J) * (
                        e1 ** a * legendre(J, mu1) + e2 ** a * legendre(J, mu2))
            Ru = (r1 + r2) / np.linalg.norm(r1 + r2)
            errs.append(abs(s - legendre(l, Du @ Ru)))
        assert all(abs(x - (K + 2)) < 0.15 for x in _slope(errs)), (K, errs)
