"""Coupling coefficients of the series expansions (oracle; test infrastructure only).

Everything here is written from the formulas of the paper's appendices:

* Wigner 3j (Racah's closed form) and the Gaunt integral, Appendix A
  (Gaunt written through 3j symbols).
* Legendre inverse coefficients c~_n^L, Appendix A (inverse power relation).
* Gegenbauer expansion coefficients C_{Nk}^{(a)}, Appendix A.
* Solid-harmonic addition coefficients A_{lm}^{lambda mu}, Appendix B
  (definition of A in the solid-harmonic form of the shift theorem).
* phi^{alpha,lm}_{J1J2M}, the spherical-harmonic shift coefficients,
  Appendix B, boxed equation "shift-coeff-def".
* omega^{beta,lm,alpha}: phi with the Gegenbauer index l/2 -> (l+alpha)/2,
  Appendix C.  Omega^{beta,alpha J1 J2 m M}_{S1 S2 T}: Appendix C, boxed
  generalised shift theorem (omega contracted with one Gaunt factor).
* Phi^{alpha,lm}_{J1J2M}, parity-even midpoint coefficients, Appendix D:
  Phi^0 = sqrt(4 pi) delta delta delta, Phi^2 = -phi^2,
  Phi^4 = -phi^4 + sum phi^2 Omega^{2,2}; higher even orders follow the same
  order-by-order inversion (``Phi`` below implements that inversion).
* f^{alpha,l}_J, Legendre shift coefficients, Appendix E, boxed "f-alpha-def";
  h^{beta,alpha l}_J = f with C^{l/2} -> C^{(l+alpha)/2}; F^{alpha,l}_J, the
  parity-even Legendre coefficients, Appendix E ("F-coeff-def" and the explicit
  F^0, F^2, F^4 list).
* B^{beta,lm}_{J1J2M}, bisector coefficients, Appendix F, boxed "B-def".

Readings taken where the text is garbled (each pinned by a test against the
printed worked examples):
* In the explicit form of phi the upper k limit prints as floor(alpha - lambda/2);
  it is floor((alpha-lambda)/2) (N = alpha - lambda, k <= N/2), which is what the
  Gaunt form of the definition implies.
* The parity-even Legendre theorem (Section 4.3 boxed form) omits the factor
  (2J+1)/(2l+1) that the all-parity theorem carries.  The printed numbers are
  the full coefficients (2J+1)/(2l+1) F, so F enters exactly like f.
* The l=m=0 bisector coefficient carries an implicit delta_{beta 0}
  (binom(0, beta) = delta_{beta0}, Appendix F).

Precision: factorial ratios are exact Python integers / Fractions; each 3j is
rounded to float once, so tables are accurate to a few ulp in FP64.
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache

SQRT4PI = math.sqrt(4.0 * math.pi)
FOURPI = 4.0 * math.pi


# ----------------------------------------------------------------------------
# Appendix A building blocks
# ----------------------------------------------------------------------------

@lru_cache(maxsize=None)
def wigner3j(j1: int, j2: int, j3: int, m1: int, m2: int, m3: int) -> float:
    """Wigner 3j symbol (j1 j2 j3; m1 m2 m3) for integer arguments (Racah formula)."""
    if m1 + m2 + m3 != 0:
        return 0.0
    if j3 < abs(j1 - j2) or j3 > j1 + j2:
        return 0.0
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0.0
    f = math.factorial
    tri = Fraction(f(j1 + j2 - j3) * f(j1 - j2 + j3) * f(-j1 + j2 + j3), f(j1 + j2 + j3 + 1))
    pre2 = tri * (f(j1 + m1) * f(j1 - m1) * f(j2 + m2) * f(j2 - m2) * f(j3 + m3) * f(j3 - m3))
    kmin = max(0, j2 - j3 - m1, j1 - j3 + m2)
    kmax = min(j1 + j2 - j3, j1 - m1, j2 + m2)
    s = Fraction(0)
    for k in range(kmin, kmax + 1):
        den = (f(k) * f(j3 - j2 + k + m1) * f(j3 - j1 + k - m2) * f(j1 + j2 - j3 - k)
               * f(j1 - k - m1) * f(j2 - k + m2))
        s += Fraction((-1) ** k, den)
    if s == 0:
        return 0.0
    sign = (-1) ** (j1 - j2 - m3)
    if s < 0:
        sign = -sign
    return sign * math.sqrt(float(pre2 * s * s))


@lru_cache(maxsize=None)
def gaunt(l1: int, l2: int, l3: int, m1: int, m2: int, m3: int) -> float:
    """Gaunt integral G^{m1 m2 m3}_{l1 l2 l3} = int dOmega Y_l1^m1 Y_l2^m2 Y_l3^m3
    written through 3j symbols (Appendix A)."""
    if (l1 + l2 + l3) % 2:
        return 0.0
    w0 = wigner3j(l1, l2, l3, 0, 0, 0)
    if w0 == 0.0:
        return 0.0
    wm = wigner3j(l1, l2, l3, m1, m2, m3)
    if wm == 0.0:
        return 0.0
    return math.sqrt((2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1) / FOURPI) * wm * w0


def _binom_int(n: int, k: int) -> int:
    if k < 0 or k > n or n < 0:
        return 0
    return math.comb(n, k)


@lru_cache(maxsize=None)
def ctilde(n: int, L: int) -> float:
    """c~_n^L: mu^n = sum_{L = n, n-2, ...} c~_n^L L_L(mu)  (Appendix A)."""
    if L < 0 or L > n or (n - L) % 2:
        return 0.0

    def dfact(x: int) -> int:
        r = 1
        while x > 1:
            r *= x
            x -= 2
        return r

    num = (2 * L + 1) * math.factorial(n) * dfact(L + n + 2)
    den = math.factorial(L + n + 2) * dfact(n - L)
    return float(Fraction(num, den))


@lru_cache(maxsize=None)
def gegenbauer_coef(N: int, k: int, a2: int) -> Fraction:
    """C_{Nk}^{(a)} with a = a2/2 (Appendix A explicit Gegenbauer form):
    C_N^{(a)}(s) = sum_k C_{Nk}^{(a)} (2s)^{N-2k},
    C_{Nk}^{(a)} = (-1)^k Gamma(a+N-k) / (Gamma(a) k! (N-2k)!),  C^{(0)}_{Nk} = delta_{N0}."""
    a = Fraction(a2, 2)
    if a == 0:
        return Fraction(1) if (N == 0 and k == 0) else Fraction(0)
    # Gamma(a+N-k)/Gamma(a) = rising factorial (a)_{N-k}
    poch = Fraction(1)
    for i in range(N - k):
        poch *= (a + i)
    return Fraction((-1) ** k) * poch / (math.factorial(k) * math.factorial(N - 2 * k))


@lru_cache(maxsize=None)
def A_coef(l: int, m: int, lam: int, mu: int) -> float:
    """A_{lm}^{lambda mu} (Appendix B, solid-harmonic addition written for Y_lm)."""
    b1 = _binom_int(l + m, lam + mu)
    b2 = _binom_int(l - m, lam - mu)
    if b1 == 0 or b2 == 0:
        return 0.0
    return math.sqrt(FOURPI * (2 * l + 1) / ((2 * lam + 1) * (2 * l - 2 * lam + 1)) * b1 * b2)


# ----------------------------------------------------------------------------
# Appendix B / C: spherical-harmonic shift theorem
# ----------------------------------------------------------------------------

@lru_cache(maxsize=None)
def omega(beta: int, l: int, m: int, alpha: int, J1: int, J2: int, M: int) -> float:
    """omega^{beta,lm,alpha}_{J1J2M}: the shift coefficient phi^{beta,lm}_{J1J2M}
    (boxed "shift-coeff-def") with the Gegenbauer index l/2 replaced by
    (l+alpha)/2 (Appendix C).  omega(beta, l, m, 0, ...) == phi(beta, l, m, ...).

    Expands (a/|a+A|)^alpha Y_l^m((a+A)^) = sum eps^{alpha+beta} omega Y_J1^M(a^) Y_J2^{m-M}(A^)."""
    if abs(m) > l or abs(M) > J1 or abs(m - M) > J2:
        return 0.0
    if (J1 + beta) % 2 or (l + beta + J2) % 2:
        return 0.0
    total = 0.0
    for lam in range(0, min(l, beta) + 1):
        N = beta - lam
        for mu in range(-lam, lam + 1):
            A = A_coef(l, m, lam, mu)
            if A == 0.0:
                continue
            for k in range(0, N // 2 + 1):
                C = gegenbauer_coef(N, k, l + alpha)
                if C == 0:
                    continue
                pw = float(C) * (-2.0) ** (N - 2 * k)
                n = N - 2 * k
                for Lp in range(n, -1, -2):
                    ct = ctilde(n, Lp)
                    if ct == 0.0:
                        continue
                    g1 = gaunt(lam, Lp, J1, mu, M - mu, -M)
                    if g1 == 0.0:
                        continue
                    g2 = gaunt(l - lam, Lp, J2, m - mu, mu - M, M - m)
                    if g2 == 0.0:
                        continue
                    sign = (-1) ** ((m + M - mu) % 2)
                    total += A * pw * ct * FOURPI / (2 * Lp + 1) * g1 * g2 * sign
    return total


def phi(alpha: int, l: int, m: int, J1: int, J2: int, M: int) -> float:
    """phi^{alpha,lm}_{J1J2M}: spherical-harmonic shift theorem coefficients,
    Y_l^m((a+A)^) = sum phi (a/A)^alpha Y_J1^M(a^) Y_J2^{m-M}(A^)  (Appendix B)."""
    return omega(alpha, l, m, 0, J1, J2, M)


@lru_cache(maxsize=None)
def Omega(beta: int, alpha: int, J1: int, J2: int, m: int, M: int,
          S1: int, S2: int, T: int) -> float:
    """Omega^{beta, alpha J1 J2 m M}_{S1 S2 T} (Appendix C, boxed generalised shift theorem):
    (a/|A+a|)^alpha Y_J1^M(a^) Y_J2^{m-M}((a+A)^)
        = sum_{beta S1 S2 T} Omega eps^{alpha+beta} Y_S1^T(a^) Y_S2^{m-T}(A^),
    Omega = sum_J' omega^{beta, J2 (m-M) alpha}_{J' S2 (T-M)} G^{M (T-M) (-T)}_{J1 J' S1} (-1)^T."""
    total = 0.0
    for Jp in range(0, beta + 1):
        w = omega(beta, J2, m - M, alpha, Jp, S2, T - M)
        if w == 0.0:
            continue
        g = gaunt(J1, Jp, S1, M, T - M, -T)
        if g == 0.0:
            continue
        total += w * g * (-1) ** (T % 2)
    return total


def _y_product(J1: int, M1: int, J2: int, M2: int):
    """Y_J1^M1(x) Y_J2^M2(x) = sum_{L} G^{M1 M2 (-M3)}_{J1 J2 L} (-1)^{M3} Y_L^{M3}(x),
    M3 = M1 + M2 (Appendix A product-to-sum rule).  Yields (L, M3, coefficient)."""
    M3 = M1 + M2
    for L in range(abs(J1 - J2), J1 + J2 + 1):
        if abs(M3) > L:
            continue
        g = gaunt(J1, J2, L, M1, M2, -M3)
        if g != 0.0:
            yield L, M3, g * (-1) ** (M3 % 2)


@lru_cache(maxsize=None)
def _psi(a0: int, a1: int, l: int, m: int):
    """Order-by-order inversion of Appendix D.

    theta^a0 Y_l^m(R^) = sum_{a1 >= a0, even} sum Psi^{a0->a1}_{lm; J1 J2 M} Y_J1^M(D^) z^{a1, m-M}_{J2},
    with z^{a,m}_J = [eps1^a Y_J^m(r1^) + eps2^a Y_J^m(r2^)] / 2 and the recursion
    theta^a Y_l^m(R^) = z^{a,m}_l - sum_{even beta > 0} omega^{beta,lm,a}_{J1J2M} Y_J1^M(D^) theta^{a+beta} Y_J2^{m-M}(R^).
    Returns a dict {(J1, J2, M): value} for the target order a1."""
    out: dict = {}
    if a1 == a0:
        out[(0, l, 0)] = SQRT4PI
        return out
    for beta in range(2, a1 - a0 + 1, 2):
        for J1 in range(0, beta + 1, 2):
            for J2 in range(max(0, l - beta), l + beta + 1, 2):
                for M in range(-J1, J1 + 1):
                    if abs(m - M) > J2:
                        continue
                    w = omega(beta, l, m, a0, J1, J2, M)
                    if w == 0.0:
                        continue
                    sub = _psi(a0 + beta, a1, J2, m - M)
                    for (S1, S2, T), c in sub.items():
                        for Q, MQ, gcoef in _y_product(J1, M, S1, T):
                            key = (Q, S2, MQ)
                            out[key] = out.get(key, 0.0) - w * c * gcoef
    return {k: v for k, v in out.items() if v != 0.0}


def phi_table(alpha: int, l: int, m: int) -> dict:
    """All-parity midpoint coefficients phi^{alpha,lm}_{J1J2M} (Appendix B; the boxed shift
    theorem of Section 3.1) as {(J1, J2, M): value}: J1 = alpha, alpha-2, .. >= 0 and
    J2 = max(0, l-alpha) .. l+alpha with l + alpha + J2 even (the parity rules of Section 3.1)."""
    out = {}
    for J1 in range(alpha % 2, alpha + 1, 2):
        for J2 in range(max(0, l - alpha), l + alpha + 1):
            if (l + alpha + J2) % 2:
                continue
            for M in range(-J1, J1 + 1):
                if abs(m - M) > J2:
                    continue
                v = phi(alpha, l, m, J1, J2, M)
                if v != 0.0:
                    out[(J1, J2, M)] = v
    return out


def Phi_table(alpha: int, l: int, m: int) -> dict:
    """Parity-even midpoint coefficients Phi^{alpha,lm}_{J1J2M} as {(J1, J2, M): value}
    (Appendix D: Phi^0 = sqrt(4pi) d d d, Phi^2 = -phi^2, Phi^4 = -phi^4 + sum phi^2 Omega^{2,2};
    higher even alpha by the same inversion)."""
    if alpha % 2:
        return {}
    return dict(_psi(0, alpha, l, m))


def Phi(alpha: int, l: int, m: int, J1: int, J2: int, M: int) -> float:
    return Phi_table(alpha, l, m).get((J1, J2, M), 0.0)


def Phi4_explicit(l: int, m: int, J1: int, J2: int, M: int) -> float:
    """Phi^4 written literally as in Appendix D: -phi^4 + sum_{J1'J2'M'} phi^2_{J1'J2'M'} Omega^{2,2 J1'J2' m M'}_{J1J2M}."""
    total = -phi(4, l, m, J1, J2, M)
    for J1p in range(0, 3):
        for J2p in range(max(0, l - 2), l + 3):
            for Mp in range(-J1p, J1p + 1):
                p2 = phi(2, l, m, J1p, J2p, Mp)
                if p2 == 0.0:
                    continue
                total += p2 * Omega(2, 2, J1p, J2p, m, Mp, J1, J2, M)
    return total


# ----------------------------------------------------------------------------
# Appendix E: Legendre shift theorem
# ----------------------------------------------------------------------------

@lru_cache(maxsize=None)
def h(beta: int, alpha: int, l: int, J: int) -> float:
    """h^{beta, alpha l}_J: f^{beta,l}_J (boxed "f-alpha-def") with the Gegenbauer index
    l/2 replaced by (l+alpha)/2 (Appendix E).  h(beta, 0, l, J) == f(beta, l, J)."""
    if (beta + l + J) % 2:
        return 0.0
    total = 0.0
    for lam in range(0, min(beta, l) + 1):
        b = math.sqrt(math.comb(2 * l, 2 * lam))
        w = wigner3j(l, lam, l - lam, 0, 0, 0)
        if w == 0.0:
            continue
        N = beta - lam
        for k in range(0, N // 2 + 1):
            C = gegenbauer_coef(N, k, l + alpha)
            if C == 0:
                continue
            n = N - 2 * k
            pw = float(C) * (-2.0) ** n
            for Lp in range(n, -1, -2):
                ct = ctilde(n, Lp)
                w2 = wigner3j(l - lam, Lp, J, 0, 0, 0)
                if ct == 0.0 or w2 == 0.0:
                    continue
                total += b * w * pw * ct * w2 * w2
    return (-1) ** l * (2 * l + 1) ** 1.5 * total


def f(alpha: int, l: int, J: int) -> float:
    """f^{alpha,l}_J: L_l(a^.(a+A)^) = sum (2J+1)/(2l+1) f (a/A)^alpha L_J(a^.A^)  (Appendix E)."""
    return h(alpha, 0, l, J)


@lru_cache(maxsize=None)
def _G_leg(a0: int, a1: int, l: int, J: int) -> float:
    """Legendre analogue of the Appendix D inversion:
    theta^a0 L_l(D^.R^) = sum_{a1} sum_J (2J+1)/(2l+1) G^{a0->a1}_{l,J} zeta^{a1}_J,
    G^{a0->a0}_{l,J} = delta_{lJ},
    G^{a0->a1}_{l,J} = - sum_{even beta>0} sum_S h^{beta, a0 l}_S G^{a0+beta -> a1}_{S,J}."""
    if a1 == a0:
        return 1.0 if l == J else 0.0
    total = 0.0
    for beta in range(2, a1 - a0 + 1, 2):
        for S in range(max(0, l - beta), l + beta + 1, 2):
            hv = h(beta, a0, l, S)
            if hv == 0.0:
                continue
            total -= hv * _G_leg(a0 + beta, a1, S, J)
    return total


def F(alpha: int, l: int, J: int) -> float:
    """Parity-even Legendre coefficients F^{alpha,l}_J (Appendix E):
    F^0 = delta_{lJ}, F^2 = -f^2, F^4 = -f^4 + sum_S f^{2,l}_S h^{2,2S}_J, and so on."""
    if alpha % 2 or J % 2 != l % 2:
        return 0.0
    return _G_leg(0, alpha, l, J)


# ----------------------------------------------------------------------------
# Appendix F: bisector expansion
# ----------------------------------------------------------------------------

def _gen_binom(a: Fraction, b: int) -> Fraction:
    """Generalised binomial coefficient binom(a, b) = (a)(a-1)...(a-b+1)/b!."""
    r = Fraction(1)
    for i in range(b):
        r *= (a - i)
    return r / math.factorial(b)


@lru_cache(maxsize=None)
def B(beta: int, l: int, m: int, J1: int, J2: int, M: int) -> float:
    """B^{beta,lm}_{J1J2M} (Appendix F, boxed "B-def"):
    Y_l^m(d^) = sum_beta sum B Y_J1^M(r1^) Y_J2^{m-M}(r2^),  d = bisector."""
    if abs(m) > l or abs(M) > J1 or abs(m - M) > J2:
        return 0.0
    if (l + J1 + J2) % 2:
        return 0.0
    gb = float(_gen_binom(Fraction(-l, 2), beta)) * 2.0 ** (-beta)
    if gb == 0.0:
        return 0.0
    total = 0.0
    for lam in range(0, l + 1):
        for mu in range(-lam, lam + 1):
            A = A_coef(l, m, lam, mu)
            if A == 0.0:
                continue
            for n in range(0, beta + 1):
                bn = math.comb(beta, n) * (-1) ** (beta - n)
                for L in range(n, -1, -2):
                    ct = ctilde(n, L)
                    if ct == 0.0:
                        continue
                    g1 = gaunt(lam, L, J1, mu, M - mu, -M)
                    if g1 == 0.0:
                        continue
                    g2 = gaunt(l - lam, L, J2, m - mu, mu - M, M - m)
                    if g2 == 0.0:
                        continue
                    sign = (-1) ** ((M - mu - m) % 2)
                    total += A * bn * ct * FOURPI / (2 * L + 1) * sign * g1 * g2
    return 2.0 ** (-l) * gb * total


def B_table(beta_max: int, l: int, m: int, beta_lo: int = 0) -> dict:
    """B-bar^{lm}_{J1J2M} = sum_{beta_lo <= beta <= beta_max} B^{beta,lm}_{J1J2M} as
    {(J1, J2, M): value} (beta_lo > 0 keeps the higher-order terms only)."""
    out: dict = {}
    Jmax = l + beta_max
    for beta in range(beta_lo, beta_max + 1):
        for J1 in range(0, Jmax + 1):
            for J2 in range(0, Jmax + 1):
                if (l + J1 + J2) % 2:
                    continue
                for M in range(-J1, J1 + 1):
                    if abs(m - M) > J2:
                        continue
                    v = B(beta, l, m, J1, J2, M)
                    if v != 0.0:
                        out[(J1, J2, M)] = out.get((J1, J2, M), 0.0) + v
    return {k: v for k, v in out.items() if v != 0.0}
