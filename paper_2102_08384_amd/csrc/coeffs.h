// Host FP64 coupling-coefficient generator (complex basis from the paper's appendices,
// then the real spherical-harmonic basis the kernels use).
#pragma once
#include <cstdint>
#include <vector>

namespace pw {

// One term of a real-basis coupling: target (l, nu) <- coef * field p1 (x) field p2.
// Real spherical-harmonic index p = J*J + J + mu, mu in [-J, J].
struct Term {
  int l, nu;
  int J1, mu1, J2, mu2;
  double c;
};

inline int sh_index(int J, int mu) { return J * J + J + mu; }

// Bisector: S^{l nu}_{(J1mu1)(J2mu2)} with sum_{beta_lo<=beta<=beta_max} B folded in and the
// pair symmetrised ((J1,mu1) <= (J2,mu2) by index), for every even l <= ell_max.  beta_lo =
// beta_max gives the terms of one order, theta^(2 beta), alone.
std::vector<Term> bisector_terms(int ell_max, int beta_max, int beta_lo = 0);

// Midpoint parity-even real coupling Phi'^{alpha, l nu}_{(J1mu1)(J2mu2)} for one even alpha
// (l even <= ell_max).  The (J2, mu2) index refers to the real field
// (2r)^-alpha y_J2^mu2(x^) d of series order alpha.
std::vector<Term> midpoint_terms(int ell_max, int alpha);

// Midpoint all-parity real coupling for one alpha >= 0 (Section 3.2): the shift-theorem
// coefficients phi^{alpha, lm}_{J1J2M} (Appendix B) in the real basis, with the sign
// (-1)^J2 of g^alpha_{J2 M} folded in, so that
//   A_{l nu}(D) = sum phi' y_J1^mu1(D^) |D|^alpha IFT[conj(d) F[(2r)^-alpha y_J2^mu2 d]](D).
std::vector<Term> midpoint_terms_all(int ell_max, int alpha);

// Parity-even Legendre coefficients F^{alpha,l}_J (Appendix E).
double legendre_F(int alpha, int l, int J);

// Building blocks (exposed for the table self-checks).
double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3);
double gaunt(int l1, int l2, int l3, int m1, int m2, int m3);
double shift_phi(int alpha, int l, int m, int J1, int J2, int M);
double bisector_B(int beta, int l, int m, int J1, int J2, int M);
double legendre_f(int alpha, int l, int J);

}  // namespace pw
