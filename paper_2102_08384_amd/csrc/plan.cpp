// Planner (host).  See plan.h.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <string>

#include "coeffs.h"

namespace pw {

namespace {

constexpr double kPi = 3.14159265358979323846;

int64_t isqrt64(int64_t v) {
  if (v <= 0) return 0;
  int64_t r = (int64_t)std::sqrt((double)v);
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

int signed_idx(int i, int N) { return i < N / 2 ? i : i - N; }

int path_of(const pw_config &c) {
  if (c.stat == PW_PK) return c.los == PW_BISECTOR ? PATH_BIS_PK : PATH_MID_PK;
  return c.los == PW_BISECTOR ? PATH_BIS_XI : PATH_MID_XI;
}

// compact index of (l, nu) over even l = 0, 2, ..: l(l-1)/2 + l + nu
int even_index(int l, int nu) { return l * (l - 1) / 2 + l + nu; }

Prune make_prune(int N, int64_t K2, bool full, bool coords, int prec) {
  Prune p;
  p.full = full;
  const int Q = prec == PW_FP32 ? 16 : 8;  // complex values per 128 bytes
  auto padq = [Q](int64_t v) { return (v + Q - 1) / Q * Q; };
  if (full) K2 = 3LL * (N / 2) * (N / 2);
  K2 = std::max<int64_t>(K2, 0);
  p.nkx = full ? N / 2 + 1 : (int)std::min<int64_t>(N / 2 + 1, isqrt64(K2) + 1);
  p.rs = row_stride(p.nkx, prec);
  p.ycnt.assign(N, 0);
  p.yoff.assign(N, 0);
  int64_t off = 0;
  for (int ky = 0; ky < N; ++ky) {
    int64_t sy = signed_idx(ky, N);
    int cnt = 0;
    if (full) cnt = p.nkx;
    else if (sy * sy <= K2) cnt = (int)std::min<int64_t>(p.nkx, isqrt64(K2 - sy * sy) + 1);
    p.ycnt[ky] = cnt;
    p.yoff[ky] = off;
    off += full ? p.rs : padq(cnt);
    p.npen_real += cnt;
  }
  p.npen = off;
  int64_t moff = 0;
  p.pinfo.reserve((size_t)p.npen);
  p.moff.reserve((size_t)p.npen);
  for (int ky = 0; ky < N; ++ky) {
    int64_t sy = signed_idx(ky, N);
    const int slots = full ? p.rs : (int)padq(p.ycnt[ky]);
    for (int kx = 0; kx < slots; ++kx) {
      int cnt;
      if (full) {
        cnt = N;  // kx >= nkx: an all-zero padding pencil, transformed like the others
      } else if (kx >= p.ycnt[ky]) {
        cnt = 0;  // padding slot: no modes
      } else {
        int64_t rem = K2 - (int64_t)kx * kx - sy * sy;
        int64_t kzm = rem < 0 ? 0 : isqrt64(rem);
        cnt = (2 * kzm + 1 >= N) ? N : (int)(2 * kzm + 1);
      }
      p.pinfo.push_back(PencilInfo{kx, ky, cnt, 0});
      p.moff.push_back(moff);
      if (coords && full && cnt > 0) {
        for (int kz = 0; kz < N; ++kz)
          p.modecoord.push_back((uint32_t)kx | ((uint32_t)ky << 11) | ((uint32_t)kz << 22));
      }
      moff += cnt;
      p.nretained += cnt;
    }
  }
  if (full) {
    p.nmodes = moff;
    p.mstride = padq(moff);
    return p;
  }
  // Sphere-pruned: groups of Q adjacent pencils (the z pass transforms Q pencils per workgroup;
  // npen is a multiple of Q), each [kz slot][pencil], so that every slot row is one 128-byte
  // line written straight from the transform's registers.
  p.grp = Q;
  const int64_t ngroups = p.npen / Q;
  p.goff.assign((size_t)ngroups + 1, 0);
  p.gsize.assign((size_t)ngroups, 0);
  int64_t soff = 0;
  for (int64_t g = 0; g < ngroups; ++g) {
    int hmax = -1;
    bool whole = false;
    for (int c = 0; c < Q; ++c) {
      const int cnt = p.pinfo[(size_t)(g * Q + c)].kzcnt;
      if (cnt == N) whole = true;
      else if (cnt > 0) hmax = std::max(hmax, (cnt - 1) / 2);
    }
    const int S = whole ? N : (hmax >= 0 ? 2 * hmax + 1 : 0);
    p.goff[(size_t)g] = soff;
    p.gsize[(size_t)g] = S;
    if (coords) {
      for (int j = 0; j < S; ++j) {
        const int kz = (S == N || j <= hmax) ? j : N - (S - j);
        const int64_t sz = signed_idx(kz, N);
        for (int c = 0; c < Q; ++c) {
          const PencilInfo &pi = p.pinfo[(size_t)(g * Q + c)];
          const bool keep = pi.kzcnt == N || (pi.kzcnt > 0 && sz * sz <= (int64_t)((pi.kzcnt - 1) / 2) * ((pi.kzcnt - 1) / 2));
          p.modecoord.push_back(keep ? ((uint32_t)pi.kx | ((uint32_t)pi.ky << 11) | ((uint32_t)kz << 22)) : kModeNone);
        }
      }
    }
    soff += (int64_t)S * Q;
  }
  p.goff[(size_t)ngroups] = soff;
  p.nmodes = soff;
  p.mstride = padq(soff);
  return p;
}

// Pair jobs of one group of real fields.  fields: (alpha, J, mu) -> index.  m > 0 fields are
// paired (J, +m) with (J, -m); the m = 0 fields are paired in order of J.
void add_jobs(const std::map<std::tuple<int, int, int>, int> &fields, std::vector<FieldJob> &jobs) {
  std::vector<std::pair<int, int>> zero;  // (J, alpha)
  for (const auto &kv : fields) {
    const int alpha = std::get<0>(kv.first), J = std::get<1>(kv.first), mu = std::get<2>(kv.first);
    if (mu > 0) {
      FieldJob j{alpha, 0, J, mu, -1, kv.second, fields.at(std::make_tuple(alpha, J, -mu)), alpha};
      jobs.push_back(j);
    } else if (mu == 0) {
      zero.push_back({J, alpha});
    }
  }
  std::stable_sort(zero.begin(), zero.end());
  for (size_t i = 0; i < zero.size(); i += 2) {
    const int Ja = zero[i].first, aa = zero[i].second;
    const int pa = fields.at(std::make_tuple(aa, Ja, 0));
    if (i + 1 < zero.size()) {
      const int Jb = zero[i + 1].first, ab = zero[i + 1].second;
      jobs.push_back(FieldJob{aa, 1, Ja, 0, Jb, pa, fields.at(std::make_tuple(ab, Jb, 0)), ab});
    } else {
      jobs.push_back(FieldJob{aa, 1, Ja, 0, -1, pa, -1, 0});
    }
  }
}

void sort_jobs(std::vector<FieldJob> &jobs) {
  std::stable_sort(jobs.begin(), jobs.end(), [](const FieldJob &a, const FieldJob &b) {
    if (a.m != b.m) return a.m < b.m;
    return a.Ja < b.Ja;
  });
}

}  // namespace

PlanKey make_key(const pw_config &c) {
  return PlanKey(c.stat, c.los, c.assign, c.prec, c.n_mesh, c.box_len, c.box_origin[0],
                 c.box_origin[1], c.box_origin[2], c.ell_max, c.order, c.compensate, c.bin_lo,
                 c.bin_width, c.n_bins, c.los == PW_MIDPOINT ? c.midpoint_parity : 0,
                 (c.los == PW_BISECTOR && c.stat == PW_PK) ? c.memory_lean : 0);
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
  if (c.memory_lean != 0 && c.memory_lean != 1) plan_fail(PW_EINVAL, "memory_lean must be 0 or 1");
  if (c.midpoint_parity != PW_PARITY_EVEN && c.midpoint_parity != PW_PARITY_ALL)
    plan_fail(PW_EINVAL, "midpoint_parity must be PW_PARITY_EVEN or PW_PARITY_ALL");
  const bool allp = c.los == PW_MIDPOINT && c.midpoint_parity == PW_PARITY_ALL;
  if (c.order < 0 || c.order > 8 || (!allp && (c.order & 1)))
    plan_fail(PW_EINVAL, "order must be in 0..8 (even except for the all-parity midpoint)");
  if (!(c.bin_width > 0) || !std::isfinite(c.bin_lo) || !std::isfinite(c.bin_width))
    plan_fail(PW_EINVAL, "bins must have a finite bin_lo and bin_width > 0");
  if (c.n_bins < 1 || c.n_bins > 4096) plan_fail(PW_EINVAL, "n_bins must be in 1..4096");
  const int path = path_of(c);
  const int nell = c.ell_max / 2 + 1;
  if (path == PATH_BIS_PK) {
    int Jmax = c.ell_max + c.order / 2;
    int nf = (Jmax + 1) * (Jmax + 1);
    bool gen = bis_contract_generated(c.ell_max, c.order / 2);
    const bool fits = gen ? (size_t)(nell + 2) * c.n_bins * 8 <= 65536
                          : contract_bis_threads(c.prec == PW_FP32 ? 0 : 1, nf, nell, c.n_bins) > 0;
    if (!fits) plan_fail(PW_EINVAL, "ell_max + order/2 (or n_bins) too large for the contraction kernel's LDS");
  } else if (path == PATH_MID_PK) {
    if (c.ell_max >= 2 && c.order >= (allp ? 1 : 2) && !mid_reweight_generated(c.ell_max, c.order, allp))
      plan_fail(PW_EINVAL, allp ? "midpoint P_l, all-parity: (ell_max, order) has no re-weighting kernel "
                                  "(built: ell_max 2..4 with order 1..4)"
                                : "midpoint P_l: (ell_max, order) has no re-weighting kernel (built: "
                                  "ell_max 2..6 with order 2..4, and order 6 for ell_max <= 4)");
    if ((size_t)(nell + 2) * c.n_bins * 8 > 65536) plan_fail(PW_EINVAL, "n_bins too large");
  } else {
    const double r_hi = c.bin_lo + c.n_bins * c.bin_width;
    if (r_hi > 0.5 * c.box_len)
      plan_fail(PW_EINVAL, "xi_l: the r-bins must end at or below box_len / 2 (periodic images beyond)");
    // the fused x pass keeps ROWS rows of N complex values and the bins in LDS
    const int T = c.n_mesh / 8;
    const int rows = (T >= 64) ? (256 / T > 0 ? 256 / T : 1) : 64 / T * 2;
    const size_t csz = c.prec == PW_FP32 ? 8 : 16;
    const size_t lds = (size_t)rows * (c.n_mesh + c.n_mesh / 8) * csz + (size_t)c.n_mesh * csz +
                       (size_t)(nell + 2) * c.n_bins * 8;
    if (lds > 65536) plan_fail(PW_EINVAL, "n_bins too large for xi_l (LDS of the fused x pass)");
    if (path == PATH_BIS_XI && !bis_contract_generated(c.ell_max, c.order / 2))
      plan_fail(PW_EINVAL, "bisector xi_l is built for ell_max <= 6 and order <= 4");
  }
}

bool one_pass_orders(const pw_config &c) {
  if (path_of(c) != PATH_BIS_PK || !bis_contract_generated(c.ell_max, c.order / 2)) return false;
  const int rows = (c.order / 2 + 1) * (c.ell_max / 2 + 1);
  return (size_t)(rows + 2) * c.n_bins * 8 <= 65536;
}

HostPlan build_host_plan(const pw_config &c) {
  HostPlan h;
  h.path = path_of(c);
  h.stat = c.stat; h.los = c.los; h.prec = c.prec; h.N = c.n_mesh;
  h.ell_max = c.ell_max; h.order = c.order; h.n_bins = c.n_bins;
  h.L = c.box_len; h.H = c.box_len / c.n_mesh; h.kf = 2.0 * kPi / c.box_len;
  {
    // (2r)^-alpha and |D|^alpha are evaluated in the unit u ~ 2 |box centre| (at least L/2):
    // fields of different alpha then have comparable magnitudes, which the two-real-fields-per-
    // complex-transform packing needs (a field 1e13 times smaller than its partner would keep
    // no significant digits).
    double cx = c.box_origin[0] + 0.5 * c.box_len, cy = c.box_origin[1] + 0.5 * c.box_len,
           cz = c.box_origin[2] + 0.5 * c.box_len;
    h.unit = std::max(2.0 * std::sqrt(cx * cx + cy * cy + cz * cz), 0.5 * c.box_len);
  }
  h.nell = c.ell_max / 2 + 1;
  for (int l = 0; l <= c.ell_max; l += 2) h.ells.push_back(l);
  h.n_orders_native = one_pass_orders(c) ? c.order / 2 + 1 : 0;
  for (int o = 0; o < std::max(h.n_orders_native, 1); ++o)
    for (int l : h.ells) h.ells_orders.push_back(o == 0 ? l : -1);
  h.check_extent = (h.path == PATH_MID_PK && c.order > 0 && c.ell_max > 0) ? 1 : 0;
  h.all_parity = (c.los == PW_MIDPOINT && c.midpoint_parity == PW_PARITY_ALL) ? 1 : 0;
  h.n0 = 0; h.n_inv = 0; h.n_inplace = 0; h.nz = 0; h.ny = 0; h.n_targets = 0; h.n_a = 0;
  const int N = h.N;
  const bool is_pk = c.stat == PW_PK;

  // FP64 bin decision from the integer |n|^2 (same expression order as the definition):
  //   P:  |k| = (2 pi / L) sqrt(s2),  b = floor((|k| - lo) / width)
  //   xi: |D| = (L / N) sqrt(s2),     b = floor((|D| - lo) / width), D = 0 excluded
  const int64_t smax = 3LL * (N / 2) * (N / 2);
  h.bin_of_s2.assign((size_t)smax + 1, -1);
  h.K2 = -1;
  for (int64_t s2 = 0; s2 <= smax; ++s2) {
    double mag = is_pk ? (2.0 * kPi / c.box_len) * std::sqrt((double)s2)
                       : (c.box_len / N) * std::sqrt((double)s2);
    double b = std::floor((mag - c.bin_lo) / c.bin_width);
    if (!is_pk && s2 == 0) continue;
    if (b >= 0 && b < c.n_bins) {
      h.bin_of_s2[(size_t)s2] = (int)b;
      h.K2 = s2;
    }
  }

  // assignment window W(k) = prod_i sinc(pi s_i / N)^p, p = 2 (CIC) or 3 (TSC)
  if (c.compensate) {
    h.winv.resize(N);
    for (int i = 0; i < N; ++i) {
      double x = kPi * (double)signed_idx(i, N) / (double)N;
      double sn = (x == 0.0) ? 1.0 : std::sin(x) / x;
      h.winv[i] = 1.0 / std::pow(sn, (double)c.assign);
    }
  }

  // ------------------------------------------------------------------ forward fields
  std::map<std::tuple<int, int, int>, int> fields;  // (alpha, J, mu) -> index
  if (c.los == PW_BISECTOR) {
    // every real harmonic (J, mu), J <= ell_max + order/2, at index J*J + J + mu
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
  } else {
    // alpha = 0: y_J^mu d, J = 0, 2, .., ell_max (index even_index(J, mu));
    // alpha > 0 (only when ell_max >= 2: the monopole has no alpha > 0 term):
    //   (2r)^-alpha y_J^mu d, J <= ell_max + alpha with the parity of alpha, in (alpha, J, mu)
    //   order after them; alpha = 2, 4, .., order (parity-even) or 1, 2, .., order (all-parity).
    std::map<std::tuple<int, int, int>, int> f0, fa;
    int p = 0;
    for (int J = 0; J <= c.ell_max; J += 2)
      for (int mu = -J; mu <= J; ++mu) f0[std::make_tuple(0, J, mu)] = p++;
    h.n0 = p;
    if (c.ell_max >= 2)
      for (int alpha = h.all_parity ? 1 : 2; alpha <= c.order; alpha += h.all_parity ? 1 : 2)
        for (int J = alpha % 2; J <= c.ell_max + alpha; J += 2)
          for (int mu = -J; mu <= J; ++mu) fa[std::make_tuple(alpha, J, mu)] = p++;
    h.nfields = p;
    add_jobs(f0, h.jobs);
    add_jobs(fa, h.jobs);
    fields = f0;
    fields.insert(fa.begin(), fa.end());
    h.n_inv = (h.path == PATH_MID_PK) ? h.nfields - h.n0 : h.nfields;
    h.n_inplace = (h.path == PATH_MID_PK) ? h.n0 : 0;
  }
  sort_jobs(h.jobs);
  h.lean = (h.path == PATH_BIS_PK && c.memory_lean) ? 1 : 0;
  if (h.lean) {
    // consecutive sorted jobs (the x pass's harmonic recurrence runs along them) in groups of
    // about kLeanFields fields, each field at a slot local to its group
    h.lean_jstart.push_back(0);
    h.lean_fstart.push_back(0);
    int nf = 0;
    for (size_t i = 0; i < h.jobs.size(); ++i) {
      FieldJob j = h.jobs[i];
      const int base = (int)h.lean_fmap.size() - h.lean_fstart.back();
      h.lean_fmap.push_back(j.pa);
      j.pa = base;
      nf = base + 1;
      if (j.pb >= 0) {
        h.lean_fmap.push_back(j.pb);
        j.pb = base + 1;
        nf = base + 2;
      }
      h.lean_jobs.push_back(j);
      if (nf >= kLeanFields || i + 1 == h.jobs.size()) {
        h.lean_maxf = std::max(h.lean_maxf, nf);
        h.lean_jstart.push_back((int)h.lean_jobs.size());
        h.lean_fstart.push_back((int)h.lean_fmap.size());
        nf = 0;
      }
    }
  }

  // ------------------------------------------------------------------ retention
  h.fwd = make_prune(N, h.K2, h.path != PATH_BIS_PK, h.path == PATH_BIS_PK, c.prec);
  if (h.path == PATH_MID_PK) h.sph = make_prune(N, h.K2, false, true, c.prec);

  // ------------------------------------------------------------------ inverse transforms
  if (h.path != PATH_BIS_PK) {
    int R;
    if (h.path == PATH_MID_PK) R = N / 2;
    else R = (int)isqrt64(std::max<int64_t>(h.K2, 0));
    const int n = std::min(N, 2 * R + 1);
    h.nz = n;
    h.ny = n;
    h.zrank.assign(N, -1);
    h.zidx.assign(n, 0);
    for (int j = 0; j < n; ++j) {
      const int half = (n - 1) / 2;
      const int z = (n == N) ? j : (j <= half ? j : N - (n - j));
      h.zidx[j] = z;
      h.zrank[z] = j;
    }
    h.yidx = h.zidx;
    const int nkx = h.fwd.nkx, rs = h.fwd.rs;
    h.iycnt.assign(N, 0);
    h.iyoff.assign(N, 0);
    for (int y = 0; y < N; ++y)
      if (h.zrank[y] >= 0) {
        h.iycnt[y] = nkx;
        h.iyoff[y] = (int64_t)h.zrank[y] * rs;
      }
  }
  if (h.path == PATH_MID_PK || h.path == PATH_MID_XI) {
    for (const FieldJob &j : h.jobs) {
      const bool a0 = j.pa < h.n0;
      if (h.path == PATH_MID_PK && a0) continue;  // alpha = 0: stays in k-space
      FieldJob k = j;
      k.pa -= h.n_inplace;
      if (k.pb >= 0) k.pb -= h.n_inplace;
      h.ijobs.push_back(k);
    }
  }
  if (h.path == PATH_BIS_XI) {
    // targets T_{l nu} at even_index(l, nu); pair jobs as for fields (alpha = 0)
    std::map<std::tuple<int, int, int>, int> tg;
    for (int l = 0; l <= c.ell_max; l += 2)
      for (int nu = -l; nu <= l; ++nu) tg[std::make_tuple(0, l, nu)] = even_index(l, nu);
    h.n_targets = (int)tg.size();
    h.n_inv = h.n_targets;
    add_jobs(tg, h.ijobs);
  }
  sort_jobs(h.ijobs);
  // xi: per-field multipole coefficients of every inverse job, [job][side][l]
  //   midpoint: F^{alpha,l}_J, or (-1)^J f^{alpha,l}_J all-parity (Appendix E; the sign is
  //   that of g^alpha_J, trivial for the even J of the parity-even form); bisector: the
  //   target's own l.
  if (h.path == PATH_MID_XI || h.path == PATH_BIS_XI) {
    for (const FieldJob &j : h.ijobs) {
      const int Jb = j.kind == 0 ? j.Ja : j.Jb;
      for (int side = 0; side < 2; ++side)
        for (int l : h.ells) {
          double F = 0.0;
          if (h.path == PATH_MID_XI) {
            auto coef = [&](int alpha, int J) {
              return h.all_parity ? ((J & 1) ? -1.0 : 1.0) * legendre_f(alpha, l, J) : legendre_F(alpha, l, J);
            };
            if (side == 0) F = coef(j.alpha, j.Ja);
            else if (j.pb >= 0) F = coef(j.alpha_b, Jb);
          } else {
            F = side == 0 ? (l == j.Ja ? 1.0 : 0.0) : (j.pb >= 0 && l == Jb ? 1.0 : 0.0);
          }
          h.icoef.push_back(F);
        }
    }
  }

  // ------------------------------------------------------------------ midpoint P: A fields
  if (h.path == PATH_MID_PK) {
    // alpha = 0 couplings: (l, nu) <- y_0^0(D^) g_{0 l nu} with coefficient sqrt(4 pi), so the
    // k-space term is conj(D) Q_{0 l nu} / W^2 with unit weight.
    for (const Term &t : midpoint_terms(c.ell_max, 0)) {
      const bool ok = t.J1 == 0 && t.mu1 == 0 && t.J2 == t.l && t.mu2 == t.nu &&
                      std::fabs(t.c - std::sqrt(4.0 * kPi)) < 1e-12;
      if (!ok) plan_fail(PW_EINVAL, "midpoint alpha = 0 coupling is not the identity");
    }
    if (h.n_inv > 0) {
      if (mid_reweight_nfields(c.ell_max, c.order, h.all_parity) != h.n_inv)
        plan_fail(PW_EINVAL, "internal: midpoint field set differs from the re-weighting kernel's");
      for (int l = 2; l <= c.ell_max; l += 2) h.n_a += 2 * l + 1;
      for (int i = 0; i < h.n_a; i += 2)
        h.ajobs.push_back(FieldJob{0, 2, i, 0, (i + 1 < h.n_a) ? i + 1 : -1, i,
                                   (i + 1 < h.n_a) ? i + 1 : -1, 0});
    }
  }

  // ------------------------------------------------------------------ bisector P tables
  if (h.path == PATH_BIS_PK) {
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
  }
  const size_t rsz = h.prec == PW_FP32 ? 4 : 8, csz = 2 * rsz;
  if (h.path == PATH_MID_PK && h.n_a > 0) {
    // buffer A: the alpha = 0 products, then a region (avail) that holds in turn the retained z
    // planes, the real g fields and the A fields' x-pass and z-pass outputs; B holds the y-pass
    // outputs and the re-weighted A fields in real space
    const size_t sfull = (size_t)N * h.fwd.npen * csz, sb = spectrum_buffer_bytes(h);
    const size_t front = (size_t)h.n_inplace * sfull, avail = sb > front ? sb - front : 0;
    if ((size_t)h.n_inv * h.nz * h.fwd.npen * csz > avail || (size_t)h.n_inv * N * N * N * rsz > avail ||
        (size_t)h.n_a * N * N * N * rsz > sb || (size_t)h.n_a * N * N * h.sph.rs * csz > avail ||
        (size_t)h.n_a * h.sph.mstride * csz > avail)
      plan_fail(PW_EINVAL, "internal: A fields do not fit the spectrum buffer");
  }
  return h;
}

size_t spectrum_buffer_bytes(const HostPlan &h) {
  const size_t csz = h.prec == PW_FP32 ? 8 : 16;
  if (h.lean) return std::max<size_t>((size_t)h.nfields * h.fwd.mstride * csz, 16);  // the k-sphere
  const size_t x1 = (size_t)h.nfields * h.N * h.N * h.fwd.rs * csz;
  const size_t x2 = (size_t)h.nfields * h.N * h.fwd.npen * csz;
  const size_t x3 = (size_t)h.nfields * h.fwd.mstride * csz;
  return std::max<size_t>(std::max(x1, std::max(x2, x3)), 16);
}

WorkLayout work_layout(const HostPlan &h) {
  const size_t rsz = h.prec == PW_FP32 ? 4 : 8;
  const int ts = tile_size(h.N), nt = h.N / ts;
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  WorkLayout w;
  size_t off = 0;
  w.mesh = off;
  off += up((size_t)h.N * h.N * h.N * rsz);
  w.bufA = off;
  off += up(spectrum_buffer_bytes(h));
  w.bufB = off;
  off += up(h.lean ? lean_x_bytes(h) : spectrum_buffer_bytes(h));
  w.bufC = off;
  if (h.lean) off += up(lean_y_bytes(h));
  w.tiles = off;
  off += up((size_t)nt * nt * nt * (ts + 2) * (ts + 2) * (ts + 2) * 8);
  w.total = off;
  return w;
}

size_t table_bytes(const HostPlan &h) {
  const size_t rsz = h.prec == PW_FP32 ? 4 : 8;
  const int ts = tile_size(h.N), nt = h.N / ts;
  size_t b = (h.fwd.modecoord.size() + h.sph.modecoord.size() + h.bin_of_s2.size()) * 4 +
             (h.fwd.pinfo.size() + h.sph.pinfo.size()) * sizeof(PencilInfo) +
             (h.fwd.moff.size() + h.sph.moff.size() + h.fwd.goff.size() + h.sph.goff.size() + h.fwd.yoff.size() +
              h.sph.yoff.size() + h.iyoff.size()) * 8 +
             (h.fwd.ycnt.size() + h.sph.ycnt.size() + h.fwd.gsize.size() + h.sph.gsize.size() + h.zrank.size() +
              h.zidx.size() + h.yidx.size() + h.iycnt.size()) * 4;
  b += (h.t_start.size() + h.t_sh.size() + h.t_ell.size() + h.t_p1.size() + h.t_p2.size()) * 4 +
       (h.t_coef.size() + h.winv.size() + h.icoef.size()) * rsz;
  b += (size_t)nt * nt * nt * 16 + (size_t)h.N * h.N * 8 + (size_t)h.N * 8;  // tile sort, occupancy
  return b + ((size_t)1 << 20);  // job lists, twiddles, result rows and scalars
}

size_t plan_bytes(const pw_config &c) {
  HostPlan h = build_host_plan(c);
  return table_bytes(h) + work_layout(h).total;
}

size_t records_bytes(int prec, int64_t n_gal, int64_t n_ran) {
  const size_t rsz = prec == PW_FP32 ? 4 : 8;
  return ((size_t)(n_gal + n_ran) * 4 * rsz + 255) & ~(size_t)255;
}

size_t catalog_bytes(const pw_config &c, int64_t n_gal, int64_t n_ran) {
  const size_t rsz = c.prec == PW_FP32 ? 4 : 8;
  // tile-sorted records and the sort's chunk histograms + staging of host catalogs (+ nbar)
  return records_bytes(c.prec, n_gal, n_ran) + sort_layout(c.n_mesh, n_gal, n_ran).hist_bytes +
         (size_t)(n_gal + n_ran) * 4 * rsz + (size_t)n_ran * rsz;
}

size_t catalog_bytes(const pw_config &c, const pw_catalog &gal, const pw_catalog &ran) {
  auto isz = [](const pw_catalog &k) -> size_t { return k.dtype == PW_FP32 ? 4 : 8; };
  size_t b = records_bytes(c.prec, gal.n, ran.n) + sort_layout(c.n_mesh, gal.n, ran.n).hist_bytes;
  if (!gal.on_device) b += (size_t)gal.n * 4 * isz(gal);
  if (!ran.on_device) b += (size_t)ran.n * 4 * isz(ran) + (ran.nbar ? (size_t)ran.n * isz(ran) : 0);
  return b;
}

size_t footprint_bytes(const pw_config &c, int64_t n_gal, int64_t n_ran) {
  return plan_bytes(c) + catalog_bytes(c, n_gal, n_ran);
}

size_t lean_x_bytes(const HostPlan &h) {
  const size_t csz = h.prec == PW_FP32 ? 8 : 16;
  return (size_t)h.lean_maxf * h.N * h.N * h.fwd.rs * csz;
}

size_t lean_y_bytes(const HostPlan &h) {
  const size_t csz = h.prec == PW_FP32 ? 8 : 16;
  return (size_t)h.lean_maxf * h.N * h.fwd.npen * csz;
}

}  // namespace pw
