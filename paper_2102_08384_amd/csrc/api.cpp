// C ABI of libpw: context, planner and the synchronous estimate pipeline.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pw.h"
#include "coeffs.h"
#include "dev_core.h"
#include "kernels.h"
#include "plan.h"

using namespace pw;

namespace {

struct Fail {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Fail{code, buf};
}

#define HIPCHECK(x)                                                                   \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) fail(PW_EDEVICE, "%s failed: %s", #x, hipGetErrorString(e_)); \
  } while (0)

}  // namespace

constexpr int kMaxStages = 16;

struct pw_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0;
  size_t used = 0;
  std::string err;
  std::map<PlanKey, std::unique_ptr<DevPlan>> plans;
  // catalog staging (host pointers are copied here)
  void *stage[2] = {nullptr, nullptr};
  size_t stage_bytes[2] = {0, 0};
  void *stage_nbar = nullptr;
  size_t stage_nbar_bytes = 0;
  size_t lds_per_block = 65536;
  void *records = nullptr;  // tile-sorted particle records of the current estimate
  size_t records_bytes = 0;
  DevPlan *last = nullptr;  // plan of the most recent estimate (pw_inspect)
  // stage timing
  bool timing = false;
  hipEvent_t ev[kMaxStages + 1] = {};
  int n_stages = 0;
  const char *st_name[kMaxStages] = {};
  double st_ms[kMaxStages] = {};
  double st_bytes[kMaxStages] = {};
};

namespace {

void *dev_alloc(pw_ctx *ctx, size_t bytes) {
  if (bytes == 0) return nullptr;
  if (ctx->used + bytes > ctx->budget)
    fail(PW_ENOMEM, "device memory budget exceeded: need %zu more bytes, %zu of %zu in use", bytes,
         ctx->used, ctx->budget);
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) fail(PW_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  ctx->used += bytes;
  return p;
}

void dev_free(pw_ctx *ctx, void *p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  ctx->used -= std::min(ctx->used, bytes);
}

template <typename T>
T *upload(pw_ctx *ctx, DevPlan *dp, const std::vector<T> &v) {
  if (v.empty()) return nullptr;
  size_t bytes = v.size() * sizeof(T);
  T *p = (T *)dev_alloc(ctx, bytes);
  dp->allocs.push_back({p, bytes});
  HIPCHECK(hipMemcpy(p, v.data(), bytes, hipMemcpyHostToDevice));
  return p;
}

void *alloc_plan(pw_ctx *ctx, DevPlan *dp, size_t bytes) {
  void *p = dev_alloc(ctx, bytes);
  dp->allocs.push_back({p, bytes});
  return p;
}

void free_plan(pw_ctx *ctx, DevPlan *dp) {
  for (auto &a : dp->allocs) dev_free(ctx, a.first, a.second);
  dp->allocs.clear();
}

ShConst make_sh_const() {
  ShConst c;
  std::memset(&c, 0, sizeof(c));
  const double pi = 3.14159265358979323846;
  for (int l = 0; l <= kMaxJ; ++l)
    for (int m = 0; m <= l; ++m) {
      double a = (l - m) > 0 ? (2.0 * l - 1) / (double)(l - m) : 0.0;
      double b = (l - m) > 0 ? (l + m - 1.0) / (double)(l - m) : 0.0;
      // (l-m)!/(l+m)!
      double ratio = 1.0;
      for (int i = l - m + 1; i <= l + m; ++i) ratio /= (double)i;
      double dfm = 1.0;
      for (int i = 2 * m - 1; i > 1; i -= 2) dfm *= (double)i;
      double nrm = std::sqrt((2.0 * l + 1) / (4.0 * pi) * ratio) * dfm * (m > 0 ? std::sqrt(2.0) : 1.0);
      c.a[l][m] = (float)a; c.b[l][m] = (float)b; c.nrm[l][m] = (float)nrm;
      c.a_d[l][m] = a; c.b_d[l][m] = b; c.nrm_d[l][m] = nrm;
    }
  return c;
}

std::mutex g_sh_mu;
std::vector<int> g_sh_uploaded;  // devices with the constant table

void ensure_sh(int device) {
  std::lock_guard<std::mutex> lk(g_sh_mu);
  if (std::find(g_sh_uploaded.begin(), g_sh_uploaded.end(), device) != g_sh_uploaded.end()) return;
  ShConst c = make_sh_const();
  upload_sh_const(c);
  HIPCHECK(hipGetLastError());
  g_sh_uploaded.push_back(device);
}

DevPlan *get_plan(pw_ctx *ctx, const pw_config *cfg) {
  PlanKey key = make_key(*cfg);
  auto it = ctx->plans.find(key);
  if (it != ctx->plans.end()) return it->second.get();
  std::unique_ptr<HostPlan> hp(new HostPlan(build_host_plan(*cfg)));
  std::unique_ptr<DevPlan> dp(new DevPlan());
  dp->host = std::move(hp);
  HostPlan &h = *dp->host;
  try {
    // twiddles exp(-2 pi i e / N)
    std::vector<double> tw(2 * h.N);
    for (int e = 0; e < h.N; ++e) {
      double ang = -2.0 * 3.14159265358979323846 * (double)e / (double)h.N;
      tw[2 * e] = std::cos(ang);
      tw[2 * e + 1] = std::sin(ang);
    }
    if (h.prec == PW_FP32) {
      std::vector<float> twf(tw.begin(), tw.end());
      dp->tw = upload(ctx, dp.get(), twf);
    } else {
      dp->tw = upload(ctx, dp.get(), tw);
    }
    dp->jobs = upload(ctx, dp.get(), h.jobs);
    dp->ijobs = upload(ctx, dp.get(), h.ijobs);
    dp->ajobs = upload(ctx, dp.get(), h.ajobs);
    auto up_prune = [&](const Prune &p, DevPrune &d) {
      d.ycnt = upload(ctx, dp.get(), p.ycnt);
      d.yoff = upload(ctx, dp.get(), p.yoff);
      d.pinfo = upload(ctx, dp.get(), p.pinfo);
      d.moff = upload(ctx, dp.get(), p.moff);
      d.modecoord = upload(ctx, dp.get(), p.modecoord);
    };
    up_prune(h.fwd, dp->fwd);
    up_prune(h.sph, dp->sph);
    dp->bin_of_s2 = upload(ctx, dp.get(), h.bin_of_s2);
    dp->ells = upload(ctx, dp.get(), h.ells);
    dp->zrank = upload(ctx, dp.get(), h.zrank);
    dp->zidx = upload(ctx, dp.get(), h.zidx);
    dp->yidx = upload(ctx, dp.get(), h.yidx);
    dp->iycnt = upload(ctx, dp.get(), h.iycnt);
    dp->iyoff = upload(ctx, dp.get(), h.iyoff);
    auto up_real = [&](const std::vector<double> &v) -> void * {
      if (h.prec == PW_FP32) {
        std::vector<float> f(v.begin(), v.end());
        return upload(ctx, dp.get(), f);
      }
      return upload(ctx, dp.get(), v);
    };
    dp->winv = up_real(h.winv);
    dp->icoef = up_real(h.icoef);
    dp->t_start = upload(ctx, dp.get(), h.t_start);
    dp->t_sh = upload(ctx, dp.get(), h.t_sh);
    dp->t_ell = upload(ctx, dp.get(), h.t_ell);
    dp->t_p1 = upload(ctx, dp.get(), h.t_p1);
    dp->t_p2 = upload(ctx, dp.get(), h.t_p2);
    dp->t_coef = up_real(h.t_coef);
    size_t rsz = h.prec == PW_FP32 ? 4 : 8;
    dp->mesh = alloc_plan(ctx, dp.get(), (size_t)h.N * h.N * h.N * rsz);
    const size_t sb = spectrum_buffer_bytes(h);
    dp->bufA = alloc_plan(ctx, dp.get(), sb);
    dp->bufB = alloc_plan(ctx, dp.get(), sb);
    dp->acc = (double *)alloc_plan(ctx, dp.get(), (size_t)(h.nell + 2) * h.n_bins * sizeof(double));
    dp->out = (double *)alloc_plan(ctx, dp.get(), (size_t)(h.nell + 2) * h.n_bins * sizeof(double));
    dp->part_g = (double *)alloc_plan(ctx, dp.get(), kScalarBlocks * kScalarCols * sizeof(double));
    dp->part_r = (double *)alloc_plan(ctx, dp.get(), kScalarBlocks * kScalarCols * sizeof(double));
    dp->norm = (DevNorm *)alloc_plan(ctx, dp.get(), sizeof(DevNorm));
    {
      const int ts = tile_size(h.N), nt = h.N / ts;
      dp->ntiles = nt * nt * nt;
      dp->tile_counts = (int *)alloc_plan(ctx, dp.get(), (size_t)dp->ntiles * sizeof(int));
      dp->tile_offsets = (int *)alloc_plan(ctx, dp.get(), (size_t)(dp->ntiles + 1) * sizeof(int));
      dp->tile_cursor = (int *)alloc_plan(ctx, dp.get(), (size_t)dp->ntiles * sizeof(int));
      dp->tile_slot = (int *)alloc_plan(ctx, dp.get(), (size_t)(dp->ntiles + 1) * sizeof(int));
      dp->tile_blocks = alloc_plan(ctx, dp.get(), (size_t)dp->ntiles * (ts + 2) * (ts + 2) * (ts + 2) * 8);
      if ((size_t)dp->ntiles * sizeof(int) > ctx->lds_per_block)
        fail(PW_EINVAL, "n_mesh too large for the tile sort on this device (%zu bytes of LDS per block)",
             ctx->lds_per_block);
    }
  } catch (...) {
    free_plan(ctx, dp.get());
    throw;
  }
  DevPlan *raw = dp.get();
  ctx->plans[key] = std::move(dp);
  return raw;
}

const void *stage_catalog(pw_ctx *ctx, const pw_catalog *c, int slot, const void **nbar_out) {
  size_t rs = c->dtype == PW_FP32 ? 4 : 8;
  *nbar_out = nullptr;
  if (c->on_device) {
    *nbar_out = c->nbar;
    return c->xyzw;
  }
  size_t bytes = (size_t)c->n * 4 * rs;
  if (ctx->stage_bytes[slot] < bytes) {
    dev_free(ctx, ctx->stage[slot], ctx->stage_bytes[slot]);
    ctx->stage[slot] = nullptr;
    ctx->stage_bytes[slot] = 0;
    ctx->stage[slot] = dev_alloc(ctx, bytes);
    ctx->stage_bytes[slot] = bytes;
  }
  if (bytes) HIPCHECK(hipMemcpyAsync(ctx->stage[slot], c->xyzw, bytes, hipMemcpyHostToDevice, ctx->stream));
  if (c->nbar && slot == 1) {
    size_t nb = (size_t)c->n * rs;
    if (ctx->stage_nbar_bytes < nb) {
      dev_free(ctx, ctx->stage_nbar, ctx->stage_nbar_bytes);
      ctx->stage_nbar = nullptr;
      ctx->stage_nbar_bytes = 0;
      ctx->stage_nbar = dev_alloc(ctx, nb);
      ctx->stage_nbar_bytes = nb;
    }
    HIPCHECK(hipMemcpyAsync(ctx->stage_nbar, c->nbar, nb, hipMemcpyHostToDevice, ctx->stream));
    *nbar_out = ctx->stage_nbar;
  }
  return ctx->stage[slot];
}

void check_catalog(const pw_catalog *c, const char *name) {
  if (!c) fail(PW_EINVAL, "%s catalog is NULL", name);
  if (c->n < 0) fail(PW_EINVAL, "%s catalog has n < 0", name);
  if (c->n > 0 && !c->xyzw) fail(PW_EINVAL, "%s catalog has no xyzw array", name);
  if (c->dtype != PW_FP32 && c->dtype != PW_FP64) fail(PW_EINVAL, "%s catalog dtype must be PW_FP32 or PW_FP64", name);
}

void run_estimate(pw_ctx *ctx, const pw_config *cfg, const pw_catalog *gal, const pw_catalog *ran,
                  pw_norm *norm, double *out, double *bin_mean, int64_t *counts) {
  validate_config(*cfg);
  check_catalog(gal, "galaxy");
  check_catalog(ran, "random");
  if (!out) fail(PW_EINVAL, "out is NULL");
  if (!(norm && norm->use_given) && !ran->nbar)
    fail(PW_EINVAL, "random catalog needs nbar when the normalisation is not given");
  HIPCHECK(hipSetDevice(ctx->device));
  ensure_sh(ctx->device);
  DevPlan *dp = get_plan(ctx, cfg);
  HostPlan &h = *dp->host;
  hipStream_t s = ctx->stream;
  ctx->last = dp;
  const void *gnb = nullptr, *rnb = nullptr;
  const void *gx = stage_catalog(ctx, gal, 0, &gnb);
  const void *rx = stage_catalog(ctx, ran, 1, &rnb);
  const bool timing = ctx->timing;
  int ns = 0;
  auto mark = [&](const char *name, double bytes) {
    if (timing) HIPCHECK(hipEventRecord(ctx->ev[ns], s));
    if (name) { ctx->st_name[ns] = name; ctx->st_bytes[ns] = bytes; }
    ++ns;
  };
  const double rsz = h.prec == PW_FP32 ? 4.0 : 8.0, csz = 2.0 * rsz;
  const double isz_g = gal->dtype == PW_FP32 ? 4.0 : 8.0, isz_r = ran->dtype == PW_FP32 ? 4.0 : 8.0;
  const double ncell = (double)h.N * h.N * h.N;
  // a1: FP64 scalars
  mark("scalars", 4.0 * isz_g * gal->n + 5.0 * isz_r * ran->n);
  launch_scalars(s, gx, nullptr, gal->n, gal->dtype, dp->part_g);
  launch_scalars(s, rx, rnb, ran->n, ran->dtype, dp->part_r);
  const bool use_given = norm && norm->use_given;
  launch_finalize_norm(s, dp->part_g, dp->part_r, dp->norm, cfg->box_origin, cfg->box_len,
                       h.check_extent, use_given ? 1 : 0, use_given ? norm->alpha_r : 0.0,
                       use_given ? norm->I : 0.0, use_given ? norm->S : 0.0);
  // a2: paint (particles read once, mesh written once)
  mark("paint", 4.0 * isz_g * gal->n + 4.0 * isz_r * ran->n + ncell * rsz);
  {
    const size_t need = (size_t)(gal->n + ran->n) * 4 * (size_t)rsz;
    if (ctx->records_bytes < need) {
      dev_free(ctx, ctx->records, ctx->records_bytes);
      ctx->records = nullptr;
      ctx->records_bytes = 0;
      ctx->records = dev_alloc(ctx, need);
      ctx->records_bytes = need;
    }
  }
  launch_fill(s, dp->tile_counts, (size_t)dp->ntiles, 0);
  launch_tile_count(s, gx, gal->n, gal->dtype, h.N, cfg->box_origin, h.H, cfg->assign, dp->tile_counts);
  launch_tile_count(s, rx, ran->n, ran->dtype, h.N, cfg->box_origin, h.H, cfg->assign, dp->tile_counts);
  launch_tile_scan(s, dp->tile_counts, dp->ntiles, dp->tile_offsets, dp->tile_cursor, dp->tile_slot);
  launch_tile_scatter(s, gx, gal->n, gal->dtype, h.prec, h.N, cfg->box_origin, h.H, cfg->assign, dp->norm, 0,
                      dp->tile_cursor, ctx->records);
  launch_tile_scatter(s, rx, ran->n, ran->dtype, h.prec, h.N, cfg->box_origin, h.H, cfg->assign, dp->norm, 1,
                      dp->tile_cursor, ctx->records);
  launch_tile_paint(s, h.prec, h.N, cfg->assign, dp->tile_offsets, dp->tile_slot, ctx->records,
                    dp->norm, dp->tile_blocks, dp->mesh);
  // a3 + a4: weighted fields and the forward transforms
  const int N = h.N;
  const Prune &F = h.fwd;
  const double x1 = (double)h.nfields * N * N * F.nkx * csz;
  const double x2 = (double)h.nfields * N * F.npen * csz;
  const double x3 = (double)h.nfields * F.nmodes * csz;
  char *A = (char *)dp->bufA, *B = (char *)dp->bufB;
  mark("fx", ncell * rsz + x1);
  launch_fx(s, h.prec, N, dp->mesh, A, dp->jobs, (int)h.jobs.size(), F.nkx, cfg->box_origin, h.H, h.unit,
            dp->tw);
  mark("fy", x1 + x2);
  if (F.npen > 0)
    launch_fy(s, h.prec, N, 0, A, B, h.nfields, N, F.nkx, dp->fwd.ycnt, dp->fwd.yoff, F.npen, dp->tw);
  mark("fz", x2 + x3);
  if (F.npen > 0)
    launch_fz(s, h.prec, N, B, A, h.nfields, F.npen, dp->fwd.pinfo, dp->fwd.moff, F.nmodes, dp->tw);
  const int64_t n_s2 = (int64_t)h.bin_of_s2.size();
  const size_t nacc = (size_t)(h.nell + 2) * h.n_bins;
  if (h.path == PATH_BIS_PK) {
    // a7: contraction and FP64 binning
    mark("contract", x3 + 4.0 * F.nmodes);
    launch_fill(s, dp->acc, nacc, 1);
    TermTable tab;
    tab.tstart = dp->t_start; tab.tsh = dp->t_sh; tab.tell = dp->t_ell;
    tab.p1 = dp->t_p1; tab.p2 = dp->t_p2; tab.coef = dp->t_coef;
    tab.ntargets = (int)h.t_sh.size();
    launch_contract_bis(s, h.prec, h.ell_max, h.order / 2, A, h.nfields, F.nmodes, dp->fwd.modecoord, N,
                        dp->bin_of_s2, n_s2, h.n_bins, h.nell, tab, h.kf, dp->winv, dp->acc);
    mark("finalize", 0.0);
    launch_finalize_pk(s, dp->acc, h.nell, h.n_bins, dp->ells, dp->norm, dp->out);
  } else {
    // Spectra after fz: full pencil-major A[p][q * N + kz], q = ky * nkx + kx.
    const double sfull = (double)N * N * F.nkx * csz;  // one full spectrum
    const size_t sfull_b = (size_t)N * N * F.nkx * (size_t)csz;
    const double inv_n3 = 1.0 / ncell;
    const int npl = h.nz;  // retained z planes (= y rows) of the inverse outputs
    const double zpart = (double)h.n_inv * npl * F.npen * csz;
    const double ypart = (double)h.n_inv * npl * h.ny * F.nkx * csz;
    const bool xi = h.path != PATH_MID_PK;
    if (xi) launch_fill(s, dp->acc, nacc, 1);
    void *zin = A, *zout = B;
    int real_in = 0;
    if (h.path == PATH_BIS_XI) {
      // a8 (bisector): T_{l nu}(k) = sum S Re(conj R_p1 R_p2) / W^2 on every mode
      mark("targets", x3 + (double)h.n_targets * F.nmodes * rsz);
      launch_targets(s, h.prec, N, h.ell_max, h.order / 2, A, F.nmodes, F.nkx, dp->winv, B);
      zin = B;
      zout = A;
      real_in = 1;
    }
    // a5: conj(D) Q / W^2 (midpoint) and the inverse z pass; D = sqrt(4 pi) Q_{0,0,0}
    const int nzf = h.path == PATH_BIS_XI ? h.n_targets : h.nfields;
    // bytes: the input spectra (+ D once), the in-place products and the retained z planes
    mark("iz", (real_in ? (double)nzf * F.nmodes * rsz : (double)(nzf + 1) * sfull) +
                   (double)h.n_inplace * sfull + zpart);
    const double sqrt4pi = std::sqrt(4.0 * 3.14159265358979323846);
    launch_iz(s, h.prec, N, zin, zout, nzf, h.n_inplace, real_in, F.npen, F.nkx,
              h.path == PATH_BIS_XI ? nullptr : A, sqrt4pi, h.path == PATH_BIS_XI ? nullptr : dp->winv,
              dp->zrank, npl, dp->tw);
    // inverse y pass into the other buffer (midpoint P: behind the alpha = 0 products)
    void *yout = (zout == B) ? (void *)(A + (size_t)h.n_inplace * sfull_b) : (void *)B;
    mark("iy", (double)h.n_inv * npl * N * F.nkx * csz + ypart);
    launch_fy(s, h.prec, N, 1, zout, yout, h.n_inv, npl, F.nkx, dp->iycnt, dp->iyoff, (int64_t)h.ny * F.nkx,
              dp->tw);
    if (xi) {
      // a8: c2r along x fused with the |D|^alpha y(D^) weighting and FP64 r-binning
      mark("ix_bin", ypart);
      launch_ix(s, h.prec, N, 1, yout, nullptr, dp->ijobs, (int)h.ijobs.size(), dp->icoef, h.nell, h.nz, h.ny,
                dp->zidx, dp->yidx, h.H, h.unit, inv_n3, dp->bin_of_s2, n_s2, h.n_bins, dp->acc, dp->tw);
      mark("finalize", 0.0);
      launch_finalize_xi(s, dp->acc, h.nell, h.n_bins, h.H * h.H * h.H, dp->norm, dp->out);
    } else {
      void *Aoff = A + (size_t)h.n_inplace * sfull_b;  // behind the alpha = 0 products
      if (h.n_inv > 0) {
        // g fields in real space (B), then a6: A_{l nu} = sum Phi' y(D^) |D|^alpha g (into Aoff)
        mark("ix", ypart + (double)h.n_inv * ncell * rsz);
        launch_ix(s, h.prec, N, 0, yout, B, dp->ijobs, (int)h.ijobs.size(), nullptr, h.nell, h.nz, h.ny,
                  dp->zidx, dp->yidx, h.H, h.unit, inv_n3, nullptr, 0, 0, nullptr, dp->tw);
        mark("reweight", (double)(h.n_inv + h.n_a) * ncell * rsz);
        launch_reweight(s, h.prec, N, h.ell_max, h.order, B, Aoff, h.H / h.unit);
        // forward transforms of A, pruned to the k-sphere of the bins
        const Prune &P = h.sph;
        const double a1 = (double)h.n_a * N * N * P.nkx * csz, a2 = (double)h.n_a * N * P.npen * csz,
                     a3 = (double)h.n_a * P.nmodes * csz;
        mark("afx", (double)h.n_a * ncell * rsz + a1);
        launch_fx(s, h.prec, N, Aoff, B, dp->ajobs, (int)h.ajobs.size(), P.nkx, cfg->box_origin, h.H, h.unit,
                  dp->tw);
        mark("afy", a1 + a2);
        if (P.npen > 0)
          launch_fy(s, h.prec, N, 0, B, Aoff, h.n_a, N, P.nkx, dp->sph.ycnt, dp->sph.yoff, P.npen, dp->tw);
        mark("afz", a2 + a3);
        if (P.npen > 0)
          launch_fz(s, h.prec, N, Aoff, B, h.n_a, P.npen, dp->sph.pinfo, dp->sph.moff, P.nmodes, dp->tw);
      }
      // a7 (midpoint): sum_nu y_l^nu(k^) Re[G_{l nu} + A_{l nu}] and FP64 k-binning
      mark("contract", (double)(h.n0 + h.n_a) * h.sph.nmodes * csz + 4.0 * h.sph.nmodes);
      launch_fill(s, dp->acc, nacc, 1);
      launch_contract_mid(s, h.prec, h.ell_max, A, F.nkx, h.n_a > 0 ? B : nullptr, h.sph.nmodes,
                          dp->sph.modecoord, N, dp->bin_of_s2, n_s2, h.n_bins, h.kf, dp->acc);
      mark("finalize", 0.0);
      launch_finalize_pk(s, dp->acc, h.nell, h.n_bins, dp->ells, dp->norm, dp->out);
    }
  }
  mark(nullptr, 0.0);
  ctx->n_stages = ns - 1;
  HIPCHECK(hipGetLastError());
  std::vector<double> res((size_t)(h.nell + 2) * h.n_bins);
  DevNorm dn;
  HIPCHECK(hipMemcpyAsync(res.data(), dp->out, res.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(&dn, dp->norm, sizeof(DevNorm), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  for (int i = 0; i < ctx->n_stages; ++i) {
    float ms = -1.0f;
    if (timing) HIPCHECK(hipEventElapsedTime(&ms, ctx->ev[i], ctx->ev[i + 1]));
    ctx->st_ms[i] = timing ? (double)ms : -1.0;
  }
  if (dn.flags & 1) fail(PW_ERANGE, "a particle lies outside [box_origin, box_origin + box_len)");
  if (dn.flags & 2)
    fail(PW_EINVAL, "midpoint P_l with order > 0 needs the catalog extent <= box_len / 2 on every axis");
  std::memcpy(out, res.data(), (size_t)h.nell * h.n_bins * sizeof(double));
  if (bin_mean) std::memcpy(bin_mean, res.data() + (size_t)h.nell * h.n_bins, h.n_bins * sizeof(double));
  if (counts)
    for (int b = 0; b < h.n_bins; ++b) counts[b] = (int64_t)std::llround(res[(size_t)(h.nell + 1) * h.n_bins + b]);
  if (norm && !norm->use_given) {
    norm->alpha_r = dn.alpha_r;
    norm->I = dn.I;
    norm->S = dn.S;
  }
}

}  // namespace

extern "C" {

int pw_create(pw_ctx **out, int device, size_t hbm_budget_bytes, void *hip_stream) {
  if (!out) return PW_EINVAL;
  *out = nullptr;
  pw_ctx *ctx = new pw_ctx();
  try {
    int ndev = 0;
    HIPCHECK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) fail(PW_EINVAL, "device %d out of range (%d devices)", device, ndev);
    ctx->device = device;
    HIPCHECK(hipSetDevice(device));
    size_t free_b = 0, total_b = 0;
    HIPCHECK(hipMemGetInfo(&free_b, &total_b));
    ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)free_b);
    if (hip_stream) {
      ctx->stream = (hipStream_t)hip_stream;
    } else {
      HIPCHECK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
      ctx->own_stream = true;
    }
    ensure_sh(device);
    {
      int lds = 0;
      HIPCHECK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
      ctx->lds_per_block = (size_t)lds;
    }
    for (int i = 0; i <= kMaxStages; ++i) HIPCHECK(hipEventCreate(&ctx->ev[i]));
  } catch (const Fail &f) {
    delete ctx;
    return f.code;
  }
  *out = ctx;
  return PW_OK;
}

int pw_destroy(pw_ctx *ctx) {
  if (!ctx) return PW_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (auto &kv : ctx->plans) free_plan(ctx, kv.second.get());
  ctx->plans.clear();
  for (int i = 0; i < 2; ++i) dev_free(ctx, ctx->stage[i], ctx->stage_bytes[i]);
  dev_free(ctx, ctx->stage_nbar, ctx->stage_nbar_bytes);
  for (int i = 0; i <= kMaxStages; ++i)
    if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return PW_OK;
}

int pw_estimate(pw_ctx *ctx, const pw_config *cfg, const pw_catalog *gal, const pw_catalog *ran,
                pw_norm *norm, double *out, double *bin_mean, int64_t *counts) {
  if (!ctx) return PW_EINVAL;
  try {
    if (!cfg) fail(PW_EINVAL, "cfg is NULL");
    run_estimate(ctx, cfg, gal, ran, norm, out, bin_mean, counts);
  } catch (const Fail &f) {
    ctx->err = f.msg;
    return f.code;
  } catch (const std::exception &e) {
    ctx->err = e.what();
    return PW_EINVAL;
  }
  ctx->err.clear();
  return PW_OK;
}

const char *pw_last_error(const pw_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int pw_footprint(const pw_config *cfg, int64_t n_gal, int64_t n_ran, size_t *bytes) {
  if (!cfg || !bytes) return PW_EINVAL;
  try {
    validate_config(*cfg);
    *bytes = footprint_bytes(*cfg, n_gal, n_ran);
  } catch (const Fail &f) {
    return f.code;
  } catch (const std::exception &) {
    return PW_EINVAL;
  }
  return PW_OK;
}

int pw_coupling_table(int kind, int ell_max, int order, int alpha, double *rows, int64_t max_rows,
                      int64_t *n_rows) {
  if (!n_rows || ell_max < 0 || ell_max > 8 || (ell_max & 1) || order < 0 || order > 8) return PW_EINVAL;
  std::vector<double> r;
  try {
    if (kind == 0) {
      for (const Term &t : bisector_terms(ell_max, order / 2)) {
        double v[7] = {(double)t.l, (double)t.nu, (double)t.J1, (double)t.mu1, (double)t.J2, (double)t.mu2, t.c};
        r.insert(r.end(), v, v + 7);
      }
    } else if (kind == 1) {
      if (alpha < 0 || (alpha & 1)) return PW_EINVAL;
      for (const Term &t : midpoint_terms(ell_max, alpha)) {
        double v[7] = {(double)t.l, (double)t.nu, (double)t.J1, (double)t.mu1, (double)t.J2, (double)t.mu2, t.c};
        r.insert(r.end(), v, v + 7);
      }
    } else if (kind == 2) {
      for (int l = 0; l <= ell_max; l += 2)
        for (int J = 0; J <= l + alpha; J += 2) {
          double F = legendre_F(alpha, l, J);
          if (F == 0.0) continue;
          double v[7] = {(double)l, 0.0, (double)J, 0.0, 0.0, 0.0, F};
          r.insert(r.end(), v, v + 7);
        }
    } else {
      return PW_EINVAL;
    }
  } catch (const std::exception &) {
    return PW_EINVAL;
  }
  int64_t n = (int64_t)(r.size() / 7);
  *n_rows = n;
  if (rows) std::memcpy(rows, r.data(), (size_t)std::min(n, max_rows) * 7 * sizeof(double));
  return PW_OK;
}

int pw_set_timing(pw_ctx *ctx, int on) {
  if (!ctx) return PW_EINVAL;
  ctx->timing = on != 0;
  return PW_OK;
}

int pw_stage_info(pw_ctx *ctx, int stage, const char **name, double *ms, double *bytes) {
  if (!ctx || stage < 0 || stage >= ctx->n_stages) return PW_EINVAL;
  if (name) *name = ctx->st_name[stage];
  if (ms) *ms = ctx->st_ms[stage];
  if (bytes) *bytes = ctx->st_bytes[stage];
  return PW_OK;
}

int pw_inspect(pw_ctx *ctx, int what, void *dst, size_t dst_bytes, size_t *needed) {
  if (!ctx || !needed) return PW_EINVAL;
  try {
    DevPlan *dp = ctx->last;
    if (!dp) fail(PW_EINVAL, "pw_inspect: no estimate has run on this context");
    const HostPlan &h = *dp->host;
    size_t rsz = h.prec == PW_FP32 ? 4 : 8;
    const void *src = nullptr;
    size_t bytes = 0;
    if (what == 0) { src = dp->mesh; bytes = (size_t)h.N * h.N * h.N * rsz; }
    else if (what == 1) { src = dp->bufA; bytes = (size_t)h.nfields * h.fwd.nmodes * 2 * rsz; }
    else if (what == 2) {
      if (h.fwd.modecoord.empty()) fail(PW_EINVAL, "pw_inspect: this path keeps full spectra (no mode list)");
      src = dp->fwd.modecoord;
      bytes = (size_t)h.fwd.nmodes * 4;
    }
    else fail(PW_EINVAL, "pw_inspect: unknown buffer %d", what);
    *needed = bytes;
    if (dst) {
      if (dst_bytes < bytes) fail(PW_EINVAL, "pw_inspect: destination too small");
      HIPCHECK(hipSetDevice(ctx->device));
      HIPCHECK(hipStreamSynchronize(ctx->stream));
      HIPCHECK(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
    }
  } catch (const Fail &f) {
    ctx->err = f.msg;
    return f.code;
  }
  return PW_OK;
}

int pw_submit(pw_ctx *ctx, const pw_config *, const pw_catalog *, const pw_catalog *, pw_norm *,
              double *, double *, int64_t *, uint64_t *) {
  if (ctx) ctx->err = "pw_submit: not available in this build";
  return PW_EINVAL;
}
int pw_poll(pw_ctx *, uint64_t) { return PW_EINVAL; }
int pw_wait(pw_ctx *, uint64_t) { return PW_EINVAL; }
int pw_cancel(pw_ctx *, uint64_t) { return PW_EINVAL; }

}  // extern "C"

namespace pw {
[[noreturn]] void plan_fail(int code, const char *msg) { fail(code, "%s", msg); }
}  // namespace pw
