// Host FP64 coupling coefficients of the pairwise line-of-sight series.
//
// Complex-basis coefficients follow the paper's appendices:
//   Wigner 3j (Racah's closed form) and the Gaunt integral through 3j symbols (Appendix A);
//   c~_n^L inverse Legendre-power coefficients and Gegenbauer C_{Nk}^{(a)} (Appendix A);
//   A_{lm}^{lambda mu} solid-harmonic addition coefficients and the shift coefficients
//   phi^{alpha,lm}_{J1J2M} (Appendix B, boxed definition); omega = phi with the Gegenbauer
//   index (l+alpha)/2 (Appendix C); parity-even Phi by the order-by-order inversion of
//   Appendix D (Phi^0 = sqrt(4pi) d d d, Phi^2 = -phi^2, Phi^4 = -phi^4 + sum phi^2 Omega^{2,2});
//   f^{alpha,l}_J (Appendix E, boxed definition), h = f with index (l+alpha)/2 and the
//   parity-even F by the same inversion (F^2 = -f^2, F^4 = -f^4 + sum_S f^2_S h^{2,2S}_J);
//   B^{beta,lm}_{J1J2M} (Appendix F, boxed definition).
// The kernels work with real spherical harmonics
//   y_l^0 = Y_l^0, y_l^m = sqrt(2)(-1)^m Re Y_l^m, y_l^{-m} = sqrt(2)(-1)^m Im Y_l^m (m>0),
// so every field is real; the tables are rotated into that basis here.  The rotated
// couplings are real (each expands a real function in a real product basis); the builder
// checks that the imaginary parts vanish.
#include "coeffs.h"

#include <cmath>
#include <complex>
#include <map>
#include <mutex>
#include <stdexcept>
#include <tuple>

namespace pw {
namespace {

typedef long double ld;
typedef std::complex<double> cd;
const double kPi = 3.14159265358979323846;
const double kFourPi = 4.0 * kPi;

ld fact(int n) {
  static ld table[171];
  static bool init = false;
  if (!init) {
    table[0] = 1;
    for (int i = 1; i < 171; ++i) table[i] = table[i - 1] * (ld)i;
    init = true;
  }
  if (n < 0 || n > 170) throw std::runtime_error("factorial out of range");
  return table[n];
}

ld dfact(int n) {  // n!!, with n!! = 1 for n <= 0
  ld r = 1;
  for (int x = n; x > 1; x -= 2) r *= (ld)x;
  return r;
}

double binom_int(int n, int k) {
  if (k < 0 || n < 0 || k > n) return 0.0;
  return (double)(fact(n) / (fact(k) * fact(n - k)));
}

int parity_sign(int n) { return (n % 2 == 0) ? 1 : -1; }  // (-1)^n for any integer n

std::mutex g_mu;  // protects the memo tables below

}  // namespace

double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3) {
  if (m1 + m2 + m3 != 0) return 0.0;
  if (j3 < std::abs(j1 - j2) || j3 > j1 + j2) return 0.0;
  if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(m3) > j3) return 0.0;
  ld tri = fact(j1 + j2 - j3) * fact(j1 - j2 + j3) * fact(-j1 + j2 + j3) / fact(j1 + j2 + j3 + 1);
  ld pre = std::sqrt(tri * fact(j1 + m1) * fact(j1 - m1) * fact(j2 + m2) * fact(j2 - m2) *
                     fact(j3 + m3) * fact(j3 - m3));
  int kmin = std::max(0, std::max(j2 - j3 - m1, j1 - j3 + m2));
  int kmax = std::min(j1 + j2 - j3, std::min(j1 - m1, j2 + m2));
  ld s = 0;
  for (int k = kmin; k <= kmax; ++k) {
    ld den = fact(k) * fact(j3 - j2 + k + m1) * fact(j3 - j1 + k - m2) * fact(j1 + j2 - j3 - k) *
             fact(j1 - k - m1) * fact(j2 - k + m2);
    s += (k % 2 ? -1.0L : 1.0L) / den;
  }
  return (double)(parity_sign(j1 - j2 - m3) * pre * s);
}

double gaunt(int l1, int l2, int l3, int m1, int m2, int m3) {
  if ((l1 + l2 + l3) % 2) return 0.0;
  double w0 = wigner3j(l1, l2, l3, 0, 0, 0);
  if (w0 == 0.0) return 0.0;
  double wm = wigner3j(l1, l2, l3, m1, m2, m3);
  if (wm == 0.0) return 0.0;
  return std::sqrt((2.0 * l1 + 1) * (2.0 * l2 + 1) * (2.0 * l3 + 1) / kFourPi) * wm * w0;
}

namespace {

// c~_n^L (mu^n = sum_L c~_n^L L_L(mu))
double ctilde(int n, int L) {
  if (L < 0 || L > n || (n - L) % 2) return 0.0;
  return (double)((ld)(2 * L + 1) * fact(n) * dfact(L + n + 2) / (fact(L + n + 2) * dfact(n - L)));
}

// C_{Nk}^{(a)}, a = a2 / 2
double gegen(int N, int k, int a2) {
  if (a2 == 0) return (N == 0 && k == 0) ? 1.0 : 0.0;
  ld a = (ld)a2 / 2.0L, poch = 1;
  for (int i = 0; i < N - k; ++i) poch *= (a + i);
  return (double)((k % 2 ? -1.0L : 1.0L) * poch / (fact(k) * fact(N - 2 * k)));
}

double Acoef(int l, int m, int lam, int mu) {
  double b1 = binom_int(l + m, lam + mu), b2 = binom_int(l - m, lam - mu);
  if (b1 == 0.0 || b2 == 0.0) return 0.0;
  return std::sqrt(kFourPi * (2.0 * l + 1) / ((2.0 * lam + 1) * (2.0 * l - 2 * lam + 1)) * b1 * b2);
}

// omega^{beta, l m, alpha}_{J1 J2 M}; omega(alpha = 0) = phi
double omega_raw(int beta, int l, int m, int alpha, int J1, int J2, int M) {
  if (std::abs(m) > l || std::abs(M) > J1 || std::abs(m - M) > J2) return 0.0;
  if ((J1 + beta) % 2 || (l + beta + J2) % 2) return 0.0;
  double total = 0.0;
  for (int lam = 0; lam <= std::min(l, beta); ++lam) {
    int N = beta - lam;
    for (int mu = -lam; mu <= lam; ++mu) {
      double A = Acoef(l, m, lam, mu);
      if (A == 0.0) continue;
      for (int k = 0; k <= N / 2; ++k) {
        double C = gegen(N, k, l + alpha);
        if (C == 0.0) continue;
        int n = N - 2 * k;
        double pw2 = C * std::pow(-2.0, n);
        for (int Lp = n; Lp >= 0; Lp -= 2) {
          double ct = ctilde(n, Lp);
          if (ct == 0.0) continue;
          double g1 = gaunt(lam, Lp, J1, mu, M - mu, -M);
          if (g1 == 0.0) continue;
          double g2 = gaunt(l - lam, Lp, J2, m - mu, mu - M, M - m);
          if (g2 == 0.0) continue;
          total += A * pw2 * ct * kFourPi / (2 * Lp + 1) * g1 * g2 * parity_sign(m + M - mu);
        }
      }
    }
  }
  return total;
}

std::map<std::tuple<int, int, int, int, int, int, int>, double> g_omega_memo;

double omega(int beta, int l, int m, int alpha, int J1, int J2, int M) {
  auto key = std::make_tuple(beta, l, m, alpha, J1, J2, M);
  auto it = g_omega_memo.find(key);
  if (it != g_omega_memo.end()) return it->second;
  double v = omega_raw(beta, l, m, alpha, J1, J2, M);
  g_omega_memo[key] = v;
  return v;
}

typedef std::map<std::tuple<int, int, int>, double> Tab3;
std::map<std::tuple<int, int, int, int>, Tab3> g_psi_memo;

// Appendix D inversion: theta^{a0} Y_l^m(R^) = sum_{a1} sum Psi^{a0->a1} Y_J1^M(D^) z^{a1, m-M}_{J2}
const Tab3 &psi(int a0, int a1, int l, int m) {
  auto key = std::make_tuple(a0, a1, l, m);
  auto it = g_psi_memo.find(key);
  if (it != g_psi_memo.end()) return it->second;
  Tab3 out;
  if (a1 == a0) {
    out[std::make_tuple(0, l, 0)] = std::sqrt(kFourPi);
  } else {
    for (int beta = 2; beta <= a1 - a0; beta += 2) {
      for (int J1 = 0; J1 <= beta; J1 += 2) {
        for (int J2 = std::max(0, l - beta); J2 <= l + beta; J2 += 2) {
          for (int M = -J1; M <= J1; ++M) {
            if (std::abs(m - M) > J2) continue;
            double w = omega(beta, l, m, a0, J1, J2, M);
            if (w == 0.0) continue;
            const Tab3 sub = psi(a0 + beta, a1, J2, m - M);  // copy: the memo may rehash
            for (const auto &kv : sub) {
              int S1 = std::get<0>(kv.first), S2 = std::get<1>(kv.first), T = std::get<2>(kv.first);
              int MQ = M + T;
              for (int Q = std::abs(J1 - S1); Q <= J1 + S1; ++Q) {
                if (std::abs(MQ) > Q) continue;
                double g = gaunt(J1, S1, Q, M, T, -MQ);
                if (g == 0.0) continue;
                out[std::make_tuple(Q, S2, MQ)] -= w * kv.second * g * parity_sign(MQ);
              }
            }
          }
        }
      }
    }
  }
  auto res = g_psi_memo.emplace(key, out);
  return res.first->second;
}

// h^{beta, alpha l}_J (f with the Gegenbauer index (l+alpha)/2); h(alpha = 0) = f
double hcoef(int beta, int alpha, int l, int J) {
  if ((beta + l + J) % 2) return 0.0;
  double total = 0.0;
  for (int lam = 0; lam <= std::min(beta, l); ++lam) {
    double b = std::sqrt(binom_int(2 * l, 2 * lam));
    double w = wigner3j(l, lam, l - lam, 0, 0, 0);
    if (w == 0.0) continue;
    int N = beta - lam;
    for (int k = 0; k <= N / 2; ++k) {
      double C = gegen(N, k, l + alpha);
      if (C == 0.0) continue;
      int n = N - 2 * k;
      double pw2 = C * std::pow(-2.0, n);
      for (int Lp = n; Lp >= 0; Lp -= 2) {
        double ct = ctilde(n, Lp);
        double w2 = wigner3j(l - lam, Lp, J, 0, 0, 0);
        if (ct == 0.0 || w2 == 0.0) continue;
        total += b * w * pw2 * ct * w2 * w2;
      }
    }
  }
  return parity_sign(l) * std::pow(2.0 * l + 1, 1.5) * total;
}

std::map<std::tuple<int, int, int, int>, double> g_fleg_memo;

// theta^{a0} L_l = sum_{a1} sum_J (2J+1)/(2l+1) G^{a0->a1}_{l J} zeta^{a1}_J
double Gleg(int a0, int a1, int l, int J) {
  if (a1 == a0) return l == J ? 1.0 : 0.0;
  auto key = std::make_tuple(a0, a1, l, J);
  auto it = g_fleg_memo.find(key);
  if (it != g_fleg_memo.end()) return it->second;
  double total = 0.0;
  for (int beta = 2; beta <= a1 - a0; beta += 2)
    for (int S = std::max(0, l - beta); S <= l + beta; S += 2) {
      double hv = hcoef(beta, a0, l, S);
      if (hv != 0.0) total -= hv * Gleg(a0 + beta, a1, S, J);
    }
  g_fleg_memo[key] = total;
  return total;
}

double gen_binom(double a, int b) {
  double r = 1.0;
  for (int i = 0; i < b; ++i) r *= (a - i);
  return r / (double)fact(b);
}

double Bcoef(int beta, int l, int m, int J1, int J2, int M) {
  if (std::abs(m) > l || std::abs(M) > J1 || std::abs(m - M) > J2) return 0.0;
  if ((l + J1 + J2) % 2) return 0.0;
  double gb = gen_binom(-0.5 * l, beta) * std::pow(2.0, -beta);
  if (gb == 0.0) return 0.0;
  double total = 0.0;
  for (int lam = 0; lam <= l; ++lam)
    for (int mu = -lam; mu <= lam; ++mu) {
      double A = Acoef(l, m, lam, mu);
      if (A == 0.0) continue;
      for (int n = 0; n <= beta; ++n) {
        double bn = binom_int(beta, n) * parity_sign(beta - n);
        for (int L = n; L >= 0; L -= 2) {
          double ct = ctilde(n, L);
          if (ct == 0.0) continue;
          double g1 = gaunt(lam, L, J1, mu, M - mu, -M);
          if (g1 == 0.0) continue;
          double g2 = gaunt(l - lam, L, J2, m - mu, mu - M, M - m);
          if (g2 == 0.0) continue;
          total += A * bn * ct * kFourPi / (2 * L + 1) * parity_sign(M - mu - m) * g1 * g2;
        }
      }
    }
  return std::pow(2.0, -l) * gb * total;
}

// Y_l^m = sum_nu U[m][nu] y_l^nu  (nonzero entries only)
void Urow(int l, int m, int nu_out[2], cd val_out[2], int *count) {
  const double s = std::sqrt(0.5);
  (void)l;
  if (m == 0) {
    nu_out[0] = 0; val_out[0] = cd(1.0, 0.0); *count = 1;
  } else if (m > 0) {
    double sg = parity_sign(m);
    nu_out[0] = m; val_out[0] = cd(sg * s, 0.0);
    nu_out[1] = -m; val_out[1] = cd(0.0, sg * s);
    *count = 2;
  } else {
    int mu = -m;
    nu_out[0] = mu; val_out[0] = cd(s, 0.0);
    nu_out[1] = -mu; val_out[1] = cd(0.0, -s);
    *count = 2;
  }
}

cd Uval(int l, int m, int nu) {
  int n[2]; cd v[2]; int c;
  Urow(l, m, n, v, &c);
  for (int i = 0; i < c; ++i) if (n[i] == nu) return v[i];
  return cd(0.0, 0.0);
}

typedef std::map<std::tuple<int, int, int, int>, cd> RealAcc;  // (l, nu, p1, p2)

std::vector<Term> finish(const RealAcc &acc, bool symmetric) {
  std::vector<Term> out;
  double scale = 0.0;
  for (const auto &kv : acc) scale = std::max(scale, std::abs(kv.second));
  for (const auto &kv : acc) {
    cd v = kv.second;
    if (std::abs(v.imag()) > 1e-10 * std::max(1.0, scale))
      throw std::runtime_error("real-basis coupling has an imaginary part");
    if (std::abs(v.real()) <= 1e-13 * std::max(1.0, scale)) continue;
    Term t;
    t.l = std::get<0>(kv.first);
    t.nu = std::get<1>(kv.first);
    int p1 = std::get<2>(kv.first), p2 = std::get<3>(kv.first);
    t.J1 = (int)std::floor(std::sqrt((double)p1) + 1e-9); t.mu1 = p1 - t.J1 * t.J1 - t.J1;
    t.J2 = (int)std::floor(std::sqrt((double)p2) + 1e-9); t.mu2 = p2 - t.J2 * t.J2 - t.J2;
    t.c = v.real();
    out.push_back(t);
  }
  (void)symmetric;
  return out;
}

}  // namespace

double shift_phi(int alpha, int l, int m, int J1, int J2, int M) {
  std::lock_guard<std::mutex> lk(g_mu);
  return omega(alpha, l, m, 0, J1, J2, M);
}

double bisector_B(int beta, int l, int m, int J1, int J2, int M) {
  return Bcoef(beta, l, m, J1, J2, M);
}

double legendre_f(int alpha, int l, int J) { return hcoef(alpha, 0, l, J); }

double legendre_F(int alpha, int l, int J) {
  if (alpha % 2 || (J % 2) != (l % 2)) return 0.0;
  std::lock_guard<std::mutex> lk(g_mu);
  return Gleg(0, alpha, l, J);
}

std::vector<Term> bisector_terms(int ell_max, int beta_max, int beta_lo) {
  RealAcc acc;
  for (int l = 0; l <= ell_max; l += 2) {
    int Jmax = l + beta_max;
    for (int m = -l; m <= l; ++m) {
      for (int J1 = 0; J1 <= Jmax; ++J1)
        for (int J2 = 0; J2 <= Jmax; ++J2) {
          if ((l + J1 + J2) % 2) continue;
          for (int M = -J1; M <= J1; ++M) {
            if (std::abs(m - M) > J2) continue;
            double b = 0.0;
            for (int beta = beta_lo; beta <= beta_max; ++beta) b += Bcoef(beta, l, m, J1, J2, M);
            if (b == 0.0) continue;
            for (int nu = -l; nu <= l; ++nu) {
              cd cl = std::conj(Uval(l, m, nu));
              if (cl == cd(0.0, 0.0)) continue;
              int n1[2], n2[2], c1, c2; cd v1[2], v2[2];
              Urow(J1, M, n1, v1, &c1);
              Urow(J2, m - M, n2, v2, &c2);
              for (int a = 0; a < c1; ++a)
                for (int bb = 0; bb < c2; ++bb) {
                  int p1 = sh_index(J1, n1[a]), p2 = sh_index(J2, n2[bb]);
                  int q1 = std::min(p1, p2), q2 = std::max(p1, p2);
                  acc[std::make_tuple(l, nu, q1, q2)] += cl * b * v1[a] * v2[bb];
                }
            }
          }
        }
    }
  }
  return finish(acc, true);
}

std::vector<Term> midpoint_terms(int ell_max, int alpha) {
  RealAcc acc;
  std::lock_guard<std::mutex> lk(g_mu);
  for (int l = 0; l <= ell_max; l += 2)
    for (int m = -l; m <= l; ++m) {
      const Tab3 tab = psi(0, alpha, l, m);
      for (const auto &kv : tab) {
        int J1 = std::get<0>(kv.first), J2 = std::get<1>(kv.first), M = std::get<2>(kv.first);
        double c = kv.second;
        if (c == 0.0) continue;
        for (int nu = -l; nu <= l; ++nu) {
          cd cl = std::conj(Uval(l, m, nu));
          if (cl == cd(0.0, 0.0)) continue;
          int n1[2], n2[2], c1, c2; cd v1[2], v2[2];
          Urow(J1, M, n1, v1, &c1);
          Urow(J2, m - M, n2, v2, &c2);
          for (int a = 0; a < c1; ++a)
            for (int bb = 0; bb < c2; ++bb)
              acc[std::make_tuple(l, nu, sh_index(J1, n1[a]), sh_index(J2, n2[bb]))] +=
                  cl * c * v1[a] * v2[bb];
        }
      }
    }
  return finish(acc, false);
}

std::vector<Term> midpoint_terms_all(int ell_max, int alpha) {
  RealAcc acc;
  std::lock_guard<std::mutex> lk(g_mu);
  for (int l = 0; l <= ell_max; l += 2)
    for (int m = -l; m <= l; ++m)
      for (int J1 = alpha % 2; J1 <= alpha; J1 += 2)
        for (int J2 = std::max(0, l - alpha); J2 <= l + alpha; ++J2) {
          if ((l + alpha + J2) % 2) continue;
          for (int M = -J1; M <= J1; ++M) {
            if (std::abs(m - M) > J2) continue;
            const double c = omega(alpha, l, m, 0, J1, J2, M) * parity_sign(J2);
            if (c == 0.0) continue;
            for (int nu = -l; nu <= l; ++nu) {
              cd cl = std::conj(Uval(l, m, nu));
              if (cl == cd(0.0, 0.0)) continue;
              int n1[2], n2[2], c1, c2; cd v1[2], v2[2];
              Urow(J1, M, n1, v1, &c1);
              Urow(J2, m - M, n2, v2, &c2);
              for (int a = 0; a < c1; ++a)
                for (int bb = 0; bb < c2; ++bb)
                  acc[std::make_tuple(l, nu, sh_index(J1, n1[a]), sh_index(J2, n2[bb]))] +=
                      cl * c * v1[a] * v2[bb];
            }
          }
        }
  return finish(acc, false);
}

}  // namespace pw
