// Planner (host).  See plan.h.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <string>

#include "coeffs.h"

namespace pw {

namespace {

int64_t isqrt64(int64_t v) {
  if (v <= 0) return 0;
  int64_t r = (int64_t)std::sqrt((double)v);
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

int signed_idx(int i, int N) { return i < N / 2 ? i : i - N; }

}  // namespace

PlanKey make_key(const pw_config &c) {
  return PlanKey(c.stat, c.los, c.assign, c.prec, c.n_mesh, c.box_len, c.box_origin[0],
                 c.box_origin[1], c.box_origin[2], c.ell_max, c.order, c.compensate, c.bin_lo,
                 c.bin_width, c.n_bins);
}

void validate_config(const pw_config &c) {
  if (c.stat != PW_PK && c.stat != PW_XI) plan_fail(PW_EINVAL, "stat must be PW_PK or PW_XI");
  if (c.los != PW_MIDPOINT && c.los != PW_BISECTOR) plan_fail(PW_EINVAL, "los must be PW_MIDPOINT or PW_BISECTOR");
  if (c.assign != PW_CIC && c.assign != PW_TSC) plan_fail(PW_EINVAL, "assign must be PW_CIC or PW_TSC");
  if (c.prec != PW_FP32 && c.prec != PW_FP64) plan_fail(PW_EINVAL, "prec must be PW_FP32 or PW_FP64");
  if (!pow2(c.n_mesh) || c.n_mesh < 16 || c.n_mesh > 512)
    plan_fail(PW_EINVAL, "n_mesh must be a power of two in [16, 512]");
  if (!(c.box_len > 0) || !std::isfinite(c.box_len)) plan_fail(PW_EINVAL, "box_len must be positive");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(c.box_origin[a])) plan_fail(PW_EINVAL, "box_origin must be finite");
  if (c.ell_max < 0 || c.ell_max > 8 || (c.ell_max & 1)) plan_fail(PW_EINVAL, "ell_max must be even, 0..8");
  if (c.order < 0 || c.order > 8 || (c.order & 1)) plan_fail(PW_EINVAL, "order must be even, 0..8");
  if (!(c.bin_width > 0) || !std::isfinite(c.bin_lo)) plan_fail(PW_EINVAL, "bins must have bin_width > 0");
  if (c.n_bins < 1 || c.n_bins > 4096) plan_fail(PW_EINVAL, "n_bins must be in 1..4096");
  if (c.stat != PW_PK || c.los != PW_BISECTOR)
    plan_fail(PW_EINVAL, "this configuration (stat/los) is not built yet");
  int Jmax = c.ell_max + c.order / 2;
  int nf = (Jmax + 1) * (Jmax + 1);
  size_t lds = (size_t)nf * (c.prec == PW_FP32 ? 128 * 8 : 64 * 16) +
               (size_t)(c.ell_max / 2 + 3) * c.n_bins * 8;
  if (lds > 65536)
    plan_fail(PW_EINVAL, "ell_max + order/2 (or n_bins) too large for the contraction kernel's LDS");
}

HostPlan build_host_plan(const pw_config &c) {
  HostPlan h;
  h.stat = c.stat; h.los = c.los; h.prec = c.prec; h.N = c.n_mesh;
  h.ell_max = c.ell_max; h.order = c.order; h.n_bins = c.n_bins;
  h.L = c.box_len; h.H = c.box_len / c.n_mesh; h.kf = 2.0 * 3.14159265358979323846 / c.box_len;
  h.nell = c.ell_max / 2 + 1;
  for (int l = 0; l <= c.ell_max; l += 2) h.ells.push_back(l);
  h.check_extent = (c.stat == PW_PK && c.los == PW_MIDPOINT && c.order > 0) ? 1 : 0;
  const int N = h.N;

  // FP64 bin decision from the integer |n|^2 (same expression order as the definition:
  // |k| = (2 pi / L) sqrt(s2), b = floor((|k| - lo) / width)).
  const int64_t smax = 3LL * (N / 2) * (N / 2);
  h.bin_of_s2.assign((size_t)smax + 1, -1);
  h.K2 = -1;
  for (int64_t s2 = 0; s2 <= smax; ++s2) {
    double kmag = (2.0 * 3.14159265358979323846 / c.box_len) * std::sqrt((double)s2);
    double t = kmag - c.bin_lo;
    double b = std::floor(t / c.bin_width);
    if (b >= 0 && b < c.n_bins) {
      h.bin_of_s2[(size_t)s2] = (int)b;
      h.K2 = s2;
    }
  }
  const int64_t K2 = std::max<int64_t>(h.K2, 0);

  // assignment window W(k) = prod_i sinc(pi s_i / N)^p, p = 2 (CIC) or 3 (TSC)
  if (c.compensate) {
    h.winv.resize(N);
    for (int i = 0; i < N; ++i) {
      double x = 3.14159265358979323846 * (double)signed_idx(i, N) / (double)N;
      double sn = (x == 0.0) ? 1.0 : std::sin(x) / x;
      h.winv[i] = 1.0 / std::pow(sn, (double)c.assign);
    }
  }

  // fields: every real harmonic (J, mu) with J <= ell_max + order/2 (bisector)
  const int Jmax = c.ell_max + c.order / 2;
  h.nfields = (Jmax + 1) * (Jmax + 1);
  for (int J = 0; J <= Jmax; J += 2) {
    FieldJob j{0, 1, J, 0, (J + 1 <= Jmax) ? J + 1 : -1, sh_index(J, 0),
               (J + 1 <= Jmax) ? sh_index(J + 1, 0) : -1, 0};
    h.jobs.push_back(j);
  }
  for (int m = 1; m <= Jmax; ++m)
    for (int J = m; J <= Jmax; ++J) {
      FieldJob j{0, 0, J, m, -1, sh_index(J, m), sh_index(J, -m), 0};
      h.jobs.push_back(j);
    }

  // pruned index sets: keep |n|^2 <= K2
  h.nkx = (int)std::min<int64_t>(N / 2 + 1, isqrt64(K2) + 1);
  h.ycnt.assign(N, 0);
  h.yoff.assign(N, 0);
  int64_t off = 0;
  for (int ky = 0; ky < N; ++ky) {
    int64_t sy = signed_idx(ky, N);
    int cnt = 0;
    if (sy * sy <= K2) cnt = (int)std::min<int64_t>(h.nkx, isqrt64(K2 - sy * sy) + 1);
    h.ycnt[ky] = cnt;
    h.yoff[ky] = off;
    off += cnt;
  }
  h.npen = off;
  int64_t moff = 0;
  h.pinfo.reserve((size_t)h.npen);
  h.moff.reserve((size_t)h.npen);
  for (int ky = 0; ky < N; ++ky) {
    int64_t sy = signed_idx(ky, N);
    for (int kx = 0; kx < h.ycnt[ky]; ++kx) {
      int64_t rem = K2 - (int64_t)kx * kx - sy * sy;
      int cnt;
      if (rem < 0) cnt = 1;  // cannot happen for retained pencils; keep kz = 0 slot
      else {
        int64_t kzm = isqrt64(rem);
        cnt = (2 * kzm + 1 >= N) ? N : (int)(2 * kzm + 1);
      }
      PencilInfo pi{kx, ky, cnt, 0};
      h.pinfo.push_back(pi);
      h.moff.push_back(moff);
      const int half = (cnt - 1) / 2;
      for (int j = 0; j < cnt; ++j) {
        int kz = (cnt == N) ? j : (j <= half ? j : N - (cnt - j));
        h.modecoord.push_back((uint32_t)kx | ((uint32_t)ky << 11) | ((uint32_t)kz << 22));
      }
      moff += cnt;
    }
  }
  h.nmodes = moff;

  // coupling terms grouped by target (l, nu)
  std::vector<Term> terms = bisector_terms(c.ell_max, c.order / 2);
  std::map<std::pair<int, int>, std::vector<Term>> by;
  for (const Term &t : terms) by[{t.l, t.nu}].push_back(t);
  h.t_start.push_back(0);
  for (auto &kv : by) {
    for (const Term &t : kv.second) {
      h.t_p1.push_back(sh_index(t.J1, t.mu1));
      h.t_p2.push_back(sh_index(t.J2, t.mu2));
      h.t_coef.push_back(t.c);
    }
    h.t_start.push_back((int)h.t_p1.size());
    h.t_sh.push_back(kv.first.first * kv.first.first + kv.first.first + kv.first.second);
    h.t_ell.push_back(kv.first.first / 2);
  }
  return h;
}

size_t footprint_bytes(const pw_config &c, int64_t n_gal, int64_t n_ran) {
  HostPlan h = build_host_plan(c);
  size_t csz = c.prec == PW_FP32 ? 8 : 16, rsz = c.prec == PW_FP32 ? 4 : 8;
  size_t x1 = (size_t)h.nfields * h.N * h.N * h.nkx * csz;
  size_t x2 = (size_t)h.nfields * h.N * h.npen * csz;
  size_t x3 = (size_t)h.nfields * h.nmodes * csz;
  size_t b = (size_t)h.N * h.N * h.N * rsz + std::max(x1, x3) + x2;
  b += h.modecoord.size() * 4 + h.bin_of_s2.size() * 4 + h.pinfo.size() * 24;
  b += (size_t)(n_gal + n_ran) * 4 * rsz + (size_t)n_ran * rsz;
  return b;
}

}  // namespace pw
