// C ABI of libpw: context, planner, the estimate pipeline and the serving loop.
//
// A context owns lanes.  Each lane has its own HIP stream, plan cache (tables and work
// buffers per configuration), catalog staging and pinned result buffers.  Lane 0 runs the
// synchronous pw_estimate on the caller's (or the context's) stream; lanes 1..n serve
// pw_submit requests: a worker thread admits pending requests as a lane and enough of the HBM
// budget free up (evicting the plans of idle lanes, least recently used first), enqueues their
// whole pipeline on the lane's stream, and finishes them when the lane's completion event
// fires, so requests of different sizes and meshes overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cfloat>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
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

constexpr int kMaxStages = 24;
constexpr int kMaxLanes = 8;

struct Lane {
  int id = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::map<PlanKey, std::unique_ptr<DevPlan>> plans;
  std::map<PlanKey, uint64_t> plan_stamp;  // last use (LRU eviction)
  void *stage[2] = {nullptr, nullptr};
  size_t stage_bytes[2] = {0, 0};
  void *stage_nbar = nullptr;
  size_t stage_nbar_bytes = 0;
  void *records = nullptr;  // tile-sorted particle records
  size_t records_bytes = 0;
  void *work = nullptr;  // the workspace all plans of the lane run in (see WorkLayout)
  size_t work_bytes = 0;
  uint64_t used_stamp = 0;  // last estimate launched on the lane (LRU eviction of `work`)
  double *host_res = nullptr;  // pinned: [(res_rows + 2) * nbins] results + DevNorm
  int res_rows = 0;            // multipole rows of the result in flight (n_ell, or per order)
  size_t host_res_bytes = 0;
  hipEvent_t done = nullptr;
  hipEvent_t tev[2] = {nullptr, nullptr};  // autotuning: around one candidate launch
  DevPlan *last = nullptr;
  // stage timing (lane 0 on request; every lane while the context traces)
  bool timing = false;
  hipEvent_t ev[kMaxStages + 1] = {};
  int n_stages = 0;
  const char *st_name[kMaxStages] = {};
  double st_ms[kMaxStages] = {};
  double st_bytes[kMaxStages] = {};
  struct Req *cur = nullptr;  // serving lanes: the request in flight
  int occ_rows = 0, occ_planes = 0;  // occupancy of the most recent estimate (lane 0)
  std::vector<double> noalloc_res;   // lane 0: pageable results of pw_estimate_noalloc
  // batched launches (bisector P_l, one configuration): the plans of catalogs 1 .. n-1 (catalog
  // 0 runs in the lane's own plan and workspace) and their workspaces, one after another
  std::map<PlanKey, std::vector<std::unique_ptr<DevPlan>>> bplans;
  void *bwork = nullptr;
  size_t bwork_bytes = 0;
  std::vector<struct Req *> batch;  // serving lanes: every request of the launch in flight
  size_t res_slice = 0;             // bytes of one catalog's results in host_res
};

struct Req {
  uint64_t ticket = 0;
  pw_config cfg;
  pw_catalog gal, ran;
  pw_norm norm_in;
  pw_norm *norm_out = nullptr;
  double *out = nullptr, *bin_mean = nullptr;
  int64_t *counts = nullptr;
  size_t need_tables = 0, need_work = 0;  // device bytes of cfg's plan tables and workspace
  size_t reserved = 0;  // bytes promised to this request's launch (pw_ctx::reserved)
  int status = PW_EAGAIN;
  std::string err;
  DevPlan *dp = nullptr;
  void *pin = nullptr;  // context-owned pinned copy of the host catalogs (pw_submit), or NULL
  size_t pin_bytes = 0;
  double t_submit = 0.0, t_start = 0.0;  // ms since the context's creation (tracing)
};

}  // namespace

struct pw_ctx {
  int device = 0;
  size_t budget = 0;
  size_t used = 0;
  std::mutex mem_mu;  // guards `used`
  mutable std::mutex err_mu;  // guards `err` (written by the caller's and the worker's threads)
  std::string err;
  size_t lds_per_block = 65536;
  std::atomic<uint64_t> stamp{0};
  std::unique_ptr<Lane> main;                 // lane 0: pw_estimate
  std::vector<std::unique_ptr<Lane>> lanes;   // serving lanes
  int n_lanes = 2;
  // serving state (guarded by mu)
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req *> pending;
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  uint64_t next_ticket = 1;
  // host plans by configuration, shared by the lanes' device plans (guarded by hp_mu); beyond
  // kHostPlans entries, the least recently used one that no device plan holds is dropped
  std::mutex hp_mu;
  std::map<PlanKey, std::pair<std::shared_ptr<const HostPlan>, uint64_t>> hplans;
  uint64_t hp_stamp = 0;
  std::thread worker;
  bool worker_started = false;
  bool stop = false;
  // lane 0 in use by a pw_estimate / pw_inspect call: the admission of served requests may
  // evict lane 0's cached plans only while this is false
  bool main_busy = false;
  // launch shapes of the column passes: 1 = autotuned, 0 = defaults, 2 + i = candidate i
  int tune_mode = 1;
  // device bytes promised to launches that allocate outside `mu` (lane 0's, or a serving
  // lane's just admitted), so that two launches do not count the same free bytes
  size_t reserved = 0;
  // pw_submit refuses a request (PW_EBUSY) while this many are pending or running
  size_t queue_limit = 1024;
  // serving launches made and the requests they carried (batched launches carry several)
  uint64_t served_launches = 0, served_requests = 0;
  // pinned host buffers holding copies of pageable host catalogs of submitted requests
  // (guarded by pin_mu): the free ones, and the bytes held in all (free and in use)
  std::mutex pin_mu;
  std::vector<std::pair<void *, size_t>> pin_free;
  size_t pin_held = 0;
  size_t pin_cap = (size_t)8 << 30;
  // PW_TRACE=<file> at pw_create: one JSON line per completed estimate (guarded by trace_mu)
  std::FILE *trace = nullptr;
  std::mutex trace_mu;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
};

// ------------------------------------------------------------------------------ static scratch
// pw_estimate_noalloc runs in this fixed device array: one estimate's plan tables, workspace
// (mesh, spectrum buffers, paint tiles) and particle records, carved in that order.  Each
// device the library runs on holds its own copy until the process ends.  Host code reaches it
// only through the address hipGetSymbolAddress gives for that device (scratch_of), never
// through the array's name.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, char *> g_scratch_at;         // device -> address of that device's `scratch`
std::map<int, std::string> g_scratch_err;  // device -> why its address could not be resolved

// Once per device, with the device current (pw_create): resolve and keep its scratch address.
// A failure is kept for pw_estimate_noalloc to report; the other entry points do not need it.
void resolve_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_at.count(device)) return;
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess && p) {
    g_scratch_at[device] = (char *)p;
    return;
  }
  (void)hipGetLastError();
  g_scratch_err[device] = std::string("hipGetSymbolAddress(scratch) failed: ") +
                          (e == hipSuccess ? "null address" : hipGetErrorString(e));
}

char *scratch_of(int device, std::string *why) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_at.find(device);
  if (it != g_scratch_at.end()) return it->second;
  auto er = g_scratch_err.find(device);
  *why = er == g_scratch_err.end() ? std::string("not resolved") : er->second;
  return nullptr;
}
}  // namespace

// A promise of device bytes to one launch (pw_ctx::reserved), kept until its allocations are
// made or it fails.
struct Reservation {
  pw_ctx *ctx;
  size_t bytes = 0;
  explicit Reservation(pw_ctx *c) : ctx(c) {}
  Reservation(const Reservation &) = delete;
  Reservation &operator=(const Reservation &) = delete;
  ~Reservation() { release(); }
  void release() {
    if (!bytes) return;
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->reserved -= bytes;
      bytes = 0;
    }
    ctx->cv.notify_all();
  }
};

// Marks lane 0 busy for the scope (guarded by ctx->mu); wakes the serving worker when done.
struct MainBusy {
  pw_ctx *ctx;
  explicit MainBusy(pw_ctx *c) : ctx(c) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->main_busy = true;
  }
  ~MainBusy() {
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->main_busy = false;
    }
    ctx->cv.notify_all();
  }
};

namespace {

void set_err(pw_ctx *ctx, const std::string &msg) {
  std::lock_guard<std::mutex> lk(ctx->err_mu);
  ctx->err = msg;
}

// Pinned staging of pageable host catalogs (pw_submit): a buffer of at least `bytes` from the
// context's pool, or NULL when holding it would exceed the pool's cap (the request then reads
// the caller's memory at launch, as pw_estimate does).
void *pin_acquire(pw_ctx *ctx, size_t bytes, size_t *got) {
  std::lock_guard<std::mutex> lk(ctx->pin_mu);
  size_t best = ctx->pin_free.size();
  for (size_t i = 0; i < ctx->pin_free.size(); ++i)
    if (ctx->pin_free[i].second >= bytes && (best == ctx->pin_free.size() ||
                                             ctx->pin_free[i].second < ctx->pin_free[best].second))
      best = i;
  if (best < ctx->pin_free.size()) {
    void *p = ctx->pin_free[best].first;
    *got = ctx->pin_free[best].second;
    ctx->pin_free.erase(ctx->pin_free.begin() + (long)best);
    return p;
  }
  // drop free buffers that are too small while the cap is in the way
  while (ctx->pin_held + bytes > ctx->pin_cap && !ctx->pin_free.empty()) {
    (void)hipHostFree(ctx->pin_free.back().first);
    ctx->pin_held -= ctx->pin_free.back().second;
    ctx->pin_free.pop_back();
  }
  if (ctx->pin_held + bytes > ctx->pin_cap) return nullptr;
  void *p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  ctx->pin_held += bytes;
  *got = bytes;
  return p;
}

void pin_release(pw_ctx *ctx, Req *r) {
  if (!r->pin) return;
  std::lock_guard<std::mutex> lk(ctx->pin_mu);
  ctx->pin_free.push_back({r->pin, r->pin_bytes});
  r->pin = nullptr;
  r->pin_bytes = 0;
}

// True when `p` is host memory the device can read directly (pinned or registered).
bool host_pinned(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // pageable memory the runtime does not know: not an error here
    return false;
  }
  return a.type == hipMemoryTypeHost;
}

void *dev_alloc(pw_ctx *ctx, size_t bytes) {
  if (bytes == 0) return nullptr;
  {
    std::lock_guard<std::mutex> lk(ctx->mem_mu);
    if (ctx->used + bytes > ctx->budget)
      fail(PW_ENOMEM, "device memory budget exceeded: need %zu more bytes, %zu of %zu in use", bytes,
           ctx->used, ctx->budget);
    ctx->used += bytes;
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    std::lock_guard<std::mutex> lk(ctx->mem_mu);
    ctx->used -= bytes;
    fail(PW_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  return p;
}

void dev_free(pw_ctx *ctx, void *p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  std::lock_guard<std::mutex> lk(ctx->mem_mu);
  ctx->used -= std::min(ctx->used, bytes);
}

size_t mem_used(pw_ctx *ctx) {
  std::lock_guard<std::mutex> lk(ctx->mem_mu);
  return ctx->used;
}

void ensure_buffer(pw_ctx *ctx, void **p, size_t *have, size_t need) {
  if (*have >= need) return;
  dev_free(ctx, *p, *have);
  *p = nullptr;
  *have = 0;
  *p = dev_alloc(ctx, need);
  *have = need;
}

// Where a plan's device memory comes from: the context's allocations (counted against its
// budget, freed with the plan), or consecutive 256-byte-aligned pieces of a fixed region that
// nothing allocates (pw_estimate_noalloc's static scratch).
struct PlanMem {
  pw_ctx *ctx;
  DevPlan *dp;
  char *region = nullptr;  // fixed region, or NULL for allocations
  size_t cap = 0, off = 0;
  void *get(size_t bytes) {
    if (bytes == 0) return nullptr;
    if (region) {
      const size_t o = (off + 255) & ~(size_t)255;
      if (o > cap || bytes > cap - o)
        fail(PW_ENOMEM, "the static scratch (%zu bytes) is too small for this estimate", cap);
      off = o + bytes;
      return region + o;
    }
    void *p = dev_alloc(ctx, bytes);
    dp->allocs.push_back({p, bytes});
    return p;
  }
};

template <typename T>
T *upload(PlanMem &m, const std::vector<T> &v) {
  if (v.empty()) return nullptr;
  size_t bytes = v.size() * sizeof(T);
  T *p = (T *)m.get(bytes);
  HIPCHECK(hipMemcpy(p, v.data(), bytes, hipMemcpyHostToDevice));
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

constexpr size_t kHostPlans = 16;

// The host plan of cfg: from the context's cache, else built (outside every lock: building
// takes from milliseconds to a second) and cached.
std::shared_ptr<const HostPlan> host_plan(pw_ctx *ctx, const pw_config &cfg) {
  const PlanKey key = make_key(cfg);
  {
    std::lock_guard<std::mutex> lk(ctx->hp_mu);
    auto it = ctx->hplans.find(key);
    if (it != ctx->hplans.end()) {
      it->second.second = ++ctx->hp_stamp;
      return it->second.first;
    }
  }
  std::shared_ptr<const HostPlan> built = std::make_shared<const HostPlan>(build_host_plan(cfg));
  std::lock_guard<std::mutex> lk(ctx->hp_mu);
  auto ins = ctx->hplans.emplace(key, std::make_pair(built, (uint64_t)0)).first;  // or another thread's
  ins->second.second = ++ctx->hp_stamp;
  std::shared_ptr<const HostPlan> hp = ins->second.first;
  while (ctx->hplans.size() > kHostPlans) {
    auto victim = ctx->hplans.end();
    for (auto e = ctx->hplans.begin(); e != ctx->hplans.end(); ++e)
      if (e != ins && e->second.first.use_count() == 1 &&
          (victim == ctx->hplans.end() || e->second.second < victim->second.second))
        victim = e;
    if (victim == ctx->hplans.end()) break;
    ctx->hplans.erase(victim);
  }
  return hp;
}

// A device plan of cfg: its tables uploaded, its workspace layout computed (bind_work points it
// into a workspace).  With `region`, every table is carved from that fixed region (and *used
// receives the bytes taken) instead of being allocated.
std::unique_ptr<DevPlan> build_dev_plan(pw_ctx *ctx, const pw_config *cfg, char *region = nullptr,
                                        size_t cap = 0, size_t *used = nullptr) {
  std::unique_ptr<DevPlan> dp(new DevPlan());
  PlanMem M{ctx, dp.get(), region, cap, 0};
  dp->host = host_plan(ctx, *cfg);
  const HostPlan &h = *dp->host;
  dp->work = work_layout(h);
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
      dp->tw = upload(M, twf);
    } else {
      dp->tw = upload(M, tw);
    }
    dp->jobs = upload(M, h.jobs);
    dp->ijobs = upload(M, h.ijobs);
    dp->ajobs = upload(M, h.ajobs);
    auto up_prune = [&](const Prune &p, DevPrune &d) {
      d.ycnt = upload(M, p.ycnt);
      d.yoff = upload(M, p.yoff);
      d.pinfo = upload(M, p.pinfo);
      d.moff = upload(M, p.moff);
      d.modecoord = upload(M, p.modecoord);
      d.goff = upload(M, p.goff);
      d.gsize = upload(M, p.gsize);
    };
    up_prune(h.fwd, dp->fwd);
    up_prune(h.sph, dp->sph);
    dp->bin_of_s2 = upload(M, h.bin_of_s2);
    dp->ells = upload(M, h.ells);
    dp->zrank = upload(M, h.zrank);
    dp->zidx = upload(M, h.zidx);
    dp->yidx = upload(M, h.yidx);
    dp->iycnt = upload(M, h.iycnt);
    dp->iyoff = upload(M, h.iyoff);
    auto up_real = [&](const std::vector<double> &v) -> void * {
      if (h.prec == PW_FP32) {
        std::vector<float> f(v.begin(), v.end());
        return upload(M, f);
      }
      return upload(M, v);
    };
    dp->winv = up_real(h.winv);
    dp->icoef = up_real(h.icoef);
    dp->t_start = upload(M, h.t_start);
    dp->t_sh = upload(M, h.t_sh);
    dp->t_ell = upload(M, h.t_ell);
    dp->t_p1 = upload(M, h.t_p1);
    dp->t_p2 = upload(M, h.t_p2);
    dp->t_coef = up_real(h.t_coef);
    // the mesh, spectrum buffers and paint tiles live in the lane's workspace (bind_work);
    // memory-lean: A holds the k-sphere of every field, B and C one group's x / y passes
    if (h.lean) {
      dp->lean_jobs = upload(M, h.lean_jobs);
      dp->lean_fmap = upload(M, h.lean_fmap);
    }
    // result rows: n_ell, or n_ell per series order for the one-pass per-order contraction
    const size_t rows = (size_t)std::max(h.nell, h.n_orders_native * h.nell) + 2;
    dp->acc = (double *)M.get(rows * h.n_bins * sizeof(double));
    dp->out = (double *)M.get(rows * h.n_bins * sizeof(double));
    dp->ells_orders = upload(M, h.ells_orders);
    dp->part_g = (double *)M.get(kScalarBlocks * kScalarCols * sizeof(double));
    dp->part_r = (double *)M.get(kScalarBlocks * kScalarCols * sizeof(double));
    dp->norm = (DevNorm *)M.get(sizeof(DevNorm));
    {
      const int ts = tile_size(h.N), nt = h.N / ts;
      dp->ntiles = nt * nt * nt;
      dp->tile_counts = (int *)M.get((size_t)dp->ntiles * sizeof(int));
      dp->tile_offsets = (int *)M.get((size_t)(dp->ntiles + 1) * sizeof(int));
      dp->tile_slot = (int *)M.get((size_t)(dp->ntiles + 1) * sizeof(int));
      dp->rowmask = (int *)M.get((size_t)h.N * h.N * sizeof(int));
      dp->rowlist = (int *)M.get((size_t)h.N * h.N * sizeof(int));
      dp->planemask = (int *)M.get((size_t)h.N * sizeof(int));
      dp->zlist = (int *)M.get((size_t)h.N * sizeof(int));
      dp->occ_blockcnt = (int *)M.get((size_t)occupancy_blocks(h.N) * sizeof(int));
      // the sort kernels hold one counter per tile (and the count kernel its FP64 reduction rows)
      if ((size_t)dp->ntiles * sizeof(int) + kSortLdsExtra > ctx->lds_per_block)
        fail(PW_EINVAL, "n_mesh too large for the tile sort on this device (%zu bytes of LDS per block)",
             ctx->lds_per_block);
    }
  } catch (...) {
    free_plan(ctx, dp.get());
    throw;
  }
  if (used) *used = M.off;
  return dp;
}

DevPlan *get_plan(pw_ctx *ctx, Lane &ln, const pw_config *cfg) {
  PlanKey key = make_key(*cfg);
  auto it = ln.plans.find(key);
  if (it == ln.plans.end()) {
    it = ln.plans.emplace(key, build_dev_plan(ctx, cfg)).first;
  }
  ln.plan_stamp[key] = ln.used_stamp = ++ctx->stamp;
  return it->second.get();
}

// Points the plan's work buffers into the lane's workspace, growing the workspace first when
// the plan needs more.  The lane has nothing in flight (one estimate at a time per lane).
void bind_work(pw_ctx *ctx, Lane &ln, DevPlan *dp) {
  if (ln.work_bytes < dp->work.total) {
    ln.last = nullptr;  // its buffers go with the old workspace
    ensure_buffer(ctx, &ln.work, &ln.work_bytes, dp->work.total);
  }
  char *w = (char *)ln.work;
  dp->mesh = w + dp->work.mesh;
  dp->bufA = w + dp->work.bufA;
  dp->bufB = w + dp->work.bufB;
  dp->bufC = dp->host->lean ? w + dp->work.bufC : nullptr;
  dp->tile_blocks = w + dp->work.tiles;
}

void evict_work(pw_ctx *ctx, Lane &ln) {
  ln.last = nullptr;
  dev_free(ctx, ln.work, ln.work_bytes);
  ln.work = nullptr;
  ln.work_bytes = 0;
  dev_free(ctx, ln.bwork, ln.bwork_bytes);
  ln.bwork = nullptr;
  ln.bwork_bytes = 0;
}

void evict_plan(pw_ctx *ctx, Lane &ln, const PlanKey &key) {
  auto bt = ln.bplans.find(key);
  if (bt != ln.bplans.end()) {
    for (auto &p : bt->second) free_plan(ctx, p.get());
    ln.bplans.erase(bt);
  }
  auto it = ln.plans.find(key);
  if (it == ln.plans.end()) return;
  if (ln.last == it->second.get()) ln.last = nullptr;
  free_plan(ctx, it->second.get());
  ln.plans.erase(it);
  ln.plan_stamp.erase(key);
}

const void *stage_catalog(pw_ctx *ctx, Lane &ln, const pw_catalog *c, int slot, const void **nbar_out) {
  size_t rs = c->dtype == PW_FP32 ? 4 : 8;
  *nbar_out = nullptr;
  if (c->on_device) {
    *nbar_out = c->nbar;
    return c->xyzw;
  }
  size_t bytes = (size_t)c->n * 4 * rs;
  ensure_buffer(ctx, &ln.stage[slot], &ln.stage_bytes[slot], bytes);
  if (bytes) HIPCHECK(hipMemcpyAsync(ln.stage[slot], c->xyzw, bytes, hipMemcpyHostToDevice, ln.stream));
  if (c->nbar && slot == 1) {
    size_t nb = (size_t)c->n * rs;
    ensure_buffer(ctx, &ln.stage_nbar, &ln.stage_nbar_bytes, nb);
    HIPCHECK(hipMemcpyAsync(ln.stage_nbar, c->nbar, nb, hipMemcpyHostToDevice, ln.stream));
    *nbar_out = ln.stage_nbar;
  }
  return ln.stage[slot];
}

void check_catalog(const pw_catalog *c, const char *name) {
  if (!c) fail(PW_EINVAL, "%s catalog is NULL", name);
  if (c->n < 0) fail(PW_EINVAL, "%s catalog has n < 0", name);
  if (c->n > 0 && !c->xyzw) fail(PW_EINVAL, "%s catalog has no xyzw array", name);
  if (c->dtype != PW_FP32 && c->dtype != PW_FP64) fail(PW_EINVAL, "%s catalog dtype must be PW_FP32 or PW_FP64", name);
}

void check_request(const pw_config *cfg, const pw_catalog *gal, const pw_catalog *ran, const pw_norm *norm,
                   const double *out) {
  if (!cfg) fail(PW_EINVAL, "cfg is NULL");
  validate_config(*cfg);
  check_catalog(gal, "galaxy");
  check_catalog(ran, "random");
  if (!out) fail(PW_EINVAL, "out is NULL");
  if (!(norm && norm->use_given) && !ran->nbar)
    fail(PW_EINVAL, "random catalog needs nbar when the normalisation is not given");
}

// ------------------------------------------------------------------------------ autotuner
// Launch shapes (ColTune) of the x pass, the column passes, the tile paint and gather and the
// bisector contraction are picked per shape key, once per process: on the first launch of a
// key, every candidate runs twice on the lane's stream, on the estimate's own data, timed with
// events, the fastest is kept and run once more unless it ran last.  Each candidate reads one
// buffer and writes another (the contraction clears its sums first), so a repeat recomputes the
// same output and the estimate goes on from there.  Candidate 0 is the default shape.  PW_TUNE=0 in the environment turns the timing off (the
// defaults are used); PW_TUNE_CACHE names a file of "key choice" lines read at first use and
// appended to with each new choice.
struct TuneEntry {
  std::string key;
  int choice;
  double ms_best, ms_default;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;          // in the order the keys were settled
std::map<std::string, size_t> g_tune_at;  // key -> index into g_tune
bool g_tune_loaded = false;

bool tune_env_on() {
  const char *e = std::getenv("PW_TUNE");
  return !(e && e[0] == '0' && e[1] == 0);
}

// Called with g_tune_mu held.
void tune_load_cache() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char *path = std::getenv("PW_TUNE_CACHE");
  if (!path || !*path) return;
  std::ifstream f(path);
  std::string key;
  int choice;
  while (f >> key >> choice) {
    if (choice < 0 || g_tune_at.count(key)) continue;
    g_tune_at[key] = g_tune.size();
    g_tune.push_back(TuneEntry{key, choice, -1.0, -1.0});
  }
}

int tune_lookup(const std::string &key) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_cache();
  auto it = g_tune_at.find(key);
  return it == g_tune_at.end() ? -1 : g_tune[it->second].choice;
}

void tune_store(const std::string &key, int choice, double ms_best, double ms_default) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tune_at.count(key)) return;  // another lane settled it first
  g_tune_at[key] = g_tune.size();
  g_tune.push_back(TuneEntry{key, choice, ms_best, ms_default});
  const char *path = std::getenv("PW_TUNE_CACHE");
  if (path && *path) {
    std::ofstream f(path, std::ios::app);
    f << key << " " << choice << "\n";
  }
}

template <typename Run>
void tuned_launch(pw_ctx *ctx, Lane &ln, const std::string &key, const std::vector<ColTune> &cands, Run run) {
  const int mode = ctx->tune_mode;
  if (mode == 0 || cands.size() < 2) return run(cands[0]);
  if (mode >= 2) return run(cands[(size_t)(mode - 2) < cands.size() ? (size_t)(mode - 2) : 0]);
  const int known = tune_lookup(key);
  if (known >= 0) return run(cands[known < (int)cands.size() ? (size_t)known : 0]);  // (a stale file: default)
  if (!tune_env_on()) return run(cands[0]);
  std::vector<float> ms(cands.size(), FLT_MAX);
  for (int rep = 0; rep < 2; ++rep)
    for (size_t i = 0; i < cands.size(); ++i) {
      HIPCHECK(hipEventRecord(ln.tev[0], ln.stream));
      run(cands[i]);
      HIPCHECK(hipEventRecord(ln.tev[1], ln.stream));
      HIPCHECK(hipEventSynchronize(ln.tev[1]));
      float t = 0.0f;
      HIPCHECK(hipEventElapsedTime(&t, ln.tev[0], ln.tev[1]));
      ms[i] = std::min(ms[i], t);
    }
  const size_t best = (size_t)(std::min_element(ms.begin(), ms.end()) - ms.begin());
  // the estimate goes on from the chosen shape's output, as every later launch of the key will
  // (shapes that sum in another order, like the contraction's workgroup count, round otherwise)
  if (best + 1 != cands.size()) run(cands[best]);
  tune_store(key, (int)best, ms[best], ms[0]);
}

// Launch shape of a pass as the autotuner settled it (no timing here: a key not yet
// settled uses the default shape).
ColTune tuned_choice(pw_ctx *ctx, const std::string &key, const std::vector<ColTune> &cands) {
  const int mode = ctx->tune_mode;
  if (mode == 0) return cands[0];
  if (mode >= 2) return cands[(size_t)(mode - 2) < cands.size() ? (size_t)(mode - 2) : 0];
  const int k = tune_lookup(key);
  return (k >= 0 && k < (int)cands.size()) ? cands[(size_t)k] : cands[0];
}

std::string tune_key(const char *pass, const HostPlan &h, int nfields, int64_t a, int64_t b) {
  char buf[160];
  std::snprintf(buf, sizeof(buf), "%s:p%d:N%d:f%d:a%lld:b%lld", pass, h.prec, h.N, nfields, (long long)a,
                (long long)b);
  return buf;
}

// Candidates: the default, then other field groupings (and half-segment columns for the y pass
// in FP32).
std::vector<ColTune> fy_candidates(int prec, int nfields) {
  std::vector<ColTune> c(1);
  for (int f : {1, 2, 4, 7}) {
    if (f >= nfields) continue;
    ColTune t;
    t.fpb = f;
    c.push_back(t);
  }
  if (prec == PW_FP32) {
    ColTune t;
    t.cols = 8;
    c.push_back(t);
  }
  return c;
}

std::vector<ColTune> fz_candidates(int nfields) {
  std::vector<ColTune> c(1);
  for (int f : {nfields, (nfields + 1) / 2, (nfields + 3) / 4}) {
    if (f < 1 || (c.size() > 1 && c.back().fpb == f)) continue;
    ColTune t;
    t.fpb = f;
    c.push_back(t);
  }
  return c;
}

// x pass: rows (wavefronts) per workgroup where a row is one wavefront (FP32 at N = 512)
std::vector<ColTune> fx_candidates(int prec, int N) {
  std::vector<ColTune> c(1);
  if (prec == PW_FP32 && N == 512) {
    for (int r : {1, 2, 8}) {
      ColTune t;
      t.rows = r;
      c.push_back(t);
    }
  }
  return c;
}

// tile paint: threads per workgroup
std::vector<ColTune> paint_candidates() {
  std::vector<ColTune> c(1);
  for (int n : {128, 512}) {
    ColTune t;
    t.threads = n;
    c.push_back(t);
  }
  return c;
}

// gather: one tile per workgroup as well as the default two (FP32 with two tiles or more a side)
std::vector<ColTune> gather_candidates(int prec, int N) {
  std::vector<ColTune> c(1);
  if (prec == PW_FP32 && N / tile_size(N) >= 2) {
    ColTune t;
    t.gx = 1;
    c.push_back(t);
  }
  return c;
}

// bisector contraction: a quarter, half and twice the default workgroup count (one per 256
// modes, at most 4096)
std::vector<ColTune> contract_candidates(int64_t nmodes) {
  std::vector<ColTune> c(1);
  const int64_t d = std::max<int64_t>(1, std::min<int64_t>((nmodes + 255) / 256, 4096));
  for (int64_t b : {d / 4, d / 2, 2 * d}) {
    if (b < 1 || b == d || b == c.back().blocks) continue;
    ColTune t;
    t.blocks = (int)b;
    c.push_back(t);
  }
  return c;
}

// a1 + a2 for one catalog on stream s: FP64 scalars and the tile sort (two passes over the
// particles), paint, gather and occupancy into dp's mesh, masks and norm.  gx / rx / rnb: the
// catalogs' device arrays; records: the sort's buffer (records_bytes + the chunk histograms).
// The paint and gather shapes are autotuned on ln's stream, or (ln null) taken as settled.
void enqueue_paint(pw_ctx *ctx, Lane *ln, hipStream_t s, const DevPlan *dp, const pw_config *cfg,
                   const pw_catalog *gal, const void *gx, const pw_catalog *ran, const void *rx, const void *rnb,
                   const pw_norm *norm, void *records) {
  const HostPlan &h = *dp->host;
  const SortLayout SL = sort_layout(h.N, gal->n, ran->n);
  int *chunk_hist = (int *)((char *)records + records_bytes(h.prec, gal->n, ran->n));
  launch_fill(s, dp->tile_counts, (size_t)dp->ntiles, 0);
  launch_fill(s, dp->rowmask, (size_t)h.N * h.N, 0);
  launch_sort_count(s, SL, gx, gal->dtype, rx, ran->dtype, rnb, gal->n, ran->n, h.N, cfg->box_origin, h.H,
                    cfg->assign, chunk_hist, dp->tile_counts, dp->part_g, dp->part_r);
  const bool use_given = norm && norm->use_given;
  launch_finalize_norm(s, dp->part_g, SL.nblk_g, dp->part_r, SL.nblk_r, dp->norm, cfg->box_origin, cfg->box_len,
                       h.check_extent, use_given ? 1 : 0, use_given ? norm->alpha_r : 0.0,
                       use_given ? norm->I : 0.0, use_given ? norm->S : 0.0);
  launch_tile_scan(s, dp->tile_counts, dp->ntiles, dp->tile_offsets, dp->tile_slot);
  launch_sort_scatter(s, SL, gx, gal->dtype, rx, ran->dtype, gal->n, ran->n, h.prec, h.N, cfg->box_origin, h.H,
                      cfg->assign, dp->norm, chunk_hist, dp->tile_offsets, records);
  auto paint = [&](ColTune t) {
    launch_tile_paint(s, h.prec, h.N, cfg->assign, dp->tile_offsets, dp->tile_slot, records, dp->norm,
                      dp->tile_blocks, t);
  };
  auto gather = [&](ColTune t) {
    launch_tile_gather(s, h.prec, h.N, dp->tile_slot, dp->tile_blocks, dp->mesh, dp->rowmask, t);
  };
  const std::string pkey = tune_key("paint", h, cfg->assign, dp->ntiles, 0);
  const std::string gkey = tune_key("gather", h, 0, dp->ntiles, 0);
  if (ln) {
    tuned_launch(ctx, *ln, pkey, paint_candidates(), paint);
    tuned_launch(ctx, *ln, gkey, gather_candidates(h.prec, h.N), gather);
  } else {
    paint(tuned_choice(ctx, pkey, paint_candidates()));
    gather(tuned_choice(ctx, gkey, gather_candidates(h.prec, h.N)));
  }
  launch_occupancy(s, h.N, dp->rowmask, dp->rowlist, dp->planemask, dp->zlist, dp->occ_blockcnt, dp->norm);
}

// An estimate whose device memory is all in place (pw_estimate_noalloc): the plan with its
// tables and workspace, the particle records, and a host buffer for the results.
struct Placed {
  DevPlan *dp;
  void *records;
  double *host_res;  // (rows + 2) * n_bins doubles + DevNorm, pageable
};

// Enqueue the whole estimate on the lane's stream, ending with the copy of the results into
// the lane's pinned buffer (or `placed`'s) and the lane's completion event.  Returns the plan
// used.
DevPlan *launch_estimate(pw_ctx *ctx, Lane &ln, const pw_config *cfg, const pw_catalog *gal,
                         const pw_catalog *ran, const pw_norm *norm, bool orders = false,
                         const Placed *placed = nullptr) {
  HIPCHECK(hipSetDevice(ctx->device));
  ensure_sh(ctx->device);
  DevPlan *dp = placed ? placed->dp : get_plan(ctx, ln, cfg);
  if (!placed) bind_work(ctx, ln, dp);
  const HostPlan &h = *dp->host;
  hipStream_t s = ln.stream;
  ln.last = placed ? nullptr : dp;
  const void *gnb = nullptr, *rnb = nullptr;
  const void *gx = stage_catalog(ctx, ln, gal, 0, &gnb);
  const void *rx = stage_catalog(ctx, ln, ran, 1, &rnb);
  const bool timing = ln.timing || ctx->trace != nullptr;
  int ns = 0;
  auto mark = [&](const char *name, double bytes) {
    if (ns > kMaxStages) fail(PW_EINVAL, "internal: too many stages");
    if (timing) HIPCHECK(hipEventRecord(ln.ev[ns], s));
    if (name && ns < kMaxStages) { ln.st_name[ns] = name; ln.st_bytes[ns] = bytes; }
    ++ns;
  };
  const double rsz = h.prec == PW_FP32 ? 4.0 : 8.0, csz = 2.0 * rsz;
  const double isz_g = gal->dtype == PW_FP32 ? 4.0 : 8.0, isz_r = ran->dtype == PW_FP32 ? 4.0 : 8.0;
  const double ncell = (double)h.N * h.N * h.N;
  // a1 + a2: FP64 scalars and the tile sort (two passes over the particles), paint, gather and
  // occupancy; algorithmic bytes: particles (and the randoms' nbar) read once, mesh written once
  mark("paint", 4.0 * isz_g * gal->n + 5.0 * isz_r * ran->n + ncell * rsz);
  if (!placed)
    ensure_buffer(ctx, &ln.records, &ln.records_bytes,
                  records_bytes(h.prec, gal->n, ran->n) + sort_layout(h.N, gal->n, ran->n).hist_bytes);
  enqueue_paint(ctx, &ln, s, dp, cfg, gal, gx, ran, rx, rnb, norm, placed ? placed->records : ln.records);
  // a3 + a4: weighted fields and the forward transforms
  const int N = h.N;
  const Prune &F = h.fwd;
  // algorithmic bytes (retained values only, no padding)
  const double modes_real = F.full ? (double)N * F.npen_real : (double)F.nretained;
  const double x1 = (double)h.nfields * N * N * F.nkx * csz;
  const double x2 = (double)h.nfields * N * F.npen_real * csz;
  const double x3 = (double)h.nfields * modes_real * csz;
  char *A = (char *)dp->bufA, *B = (char *)dp->bufB;
  const bool mid = h.path == PATH_MID_PK || h.path == PATH_MID_XI;
  const int fx_kind = mid ? FX_RADIAL : FX_HARMONIC;  // midpoint fields carry (u/2r)^alpha
  if (h.lean) {
    // groups of fields through the x, y and z passes; the z pass writes each field's k-sphere
    // into A at its own index (fmap), so the contraction below sees the usual layout
    mark("forward", ncell * rsz + 2.0 * x1 + 2.0 * x2 + x3);
    const int ng = F.npen > 0 ? (int)h.lean_jstart.size() - 1 : 0;
    for (int g = 0; g < ng; ++g) {
      const int j0 = h.lean_jstart[g], nj = h.lean_jstart[g + 1] - j0;
      const int f0 = h.lean_fstart[g], nf = h.lean_fstart[g + 1] - f0;
      tuned_launch(ctx, ln, tune_key("fx", h, nj, fx_kind, F.nkx), fx_candidates(h.prec, N), [&](ColTune t) {
        launch_fx(s, h.prec, N, fx_kind, dp->mesh, B, dp->lean_jobs + j0, nj, F.nkx, F.rs, cfg->box_origin, h.H,
                  h.unit, dp->tw, dp->rowlist, dp->norm, nullptr, t);
      });
      launch_fy(s, h.prec, N, 0, B, dp->bufC, nf, N, F.nkx, F.rs, dp->fwd.ycnt, dp->fwd.yoff, F.npen, dp->tw,
                dp->rowmask, dp->zlist, dp->norm);
      launch_fz(s, h.prec, N, dp->bufC, A, nf, F.npen, dp->fwd.pinfo, dp->fwd.moff, dp->fwd.goff, dp->fwd.gsize,
                F.mstride, dp->tw, dp->planemask, dp->lean_fmap + f0);
    }
  } else {
    mark("fx", ncell * rsz + x1);
    tuned_launch(ctx, ln, tune_key("fx", h, (int)h.jobs.size(), fx_kind, F.nkx), fx_candidates(h.prec, N),
                 [&](ColTune t) {
                   launch_fx(s, h.prec, N, fx_kind, dp->mesh, A, dp->jobs, (int)h.jobs.size(), F.nkx, F.rs,
                             cfg->box_origin, h.H, h.unit, dp->tw, dp->rowlist, dp->norm, nullptr, t);
                 });
    mark("fy", x1 + x2);
    if (F.npen > 0)
      tuned_launch(ctx, ln, tune_key("fy", h, h.nfields, F.nkx, F.npen), fy_candidates(h.prec, h.nfields),
                   [&](ColTune t) {
                     launch_fy(s, h.prec, N, 0, A, B, h.nfields, N, F.nkx, F.rs, dp->fwd.ycnt, dp->fwd.yoff,
                               F.npen, dp->tw, dp->rowmask, dp->zlist, dp->norm, t);
                   });
    // (midpoint: the z pass is fused with the product and the inverse z pass below)
    if (!mid) {
      mark("fz", x2 + x3);
      if (F.npen > 0)
        tuned_launch(ctx, ln, tune_key("fz", h, h.nfields, F.npen, F.goff.empty() ? 0 : 1),
                     fz_candidates(h.nfields), [&](ColTune t) {
                       launch_fz(s, h.prec, N, B, A, h.nfields, F.npen, dp->fwd.pinfo, dp->fwd.moff, dp->fwd.goff,
                                 dp->fwd.gsize, F.mstride, dp->tw, dp->planemask, nullptr, t);
                     });
    }
  }
  const int64_t n_s2 = (int64_t)h.bin_of_s2.size();
  if (orders && (h.path != PATH_BIS_PK || h.n_orders_native == 0))
    fail(PW_EINVAL, "internal: no one-pass per-order contraction for this configuration");
  ln.res_rows = orders ? h.n_orders_native * h.nell : h.nell;
  const size_t nacc = (size_t)(ln.res_rows + 2) * h.n_bins;
  if (h.path == PATH_BIS_PK) {
    // a7: contraction and FP64 binning
    mark("contract", x3 + 4.0 * F.nretained);
    // (the shell sums accumulate: every autotuning run clears them first)
    const std::string ckey = tune_key(orders ? "contract_orders" : "contract", h, h.nfields, F.nmodes, 0);
    if (orders) {
      // every order's terms into accumulators of their own (one pass over the spectra)
      tuned_launch(ctx, ln, ckey, contract_candidates(F.nmodes), [&](ColTune t) {
        launch_fill(s, dp->acc, nacc, 1);
        launch_contract_bis_generated(s, h.prec, h.ell_max, h.order / 2, A, F.nmodes, F.mstride, dp->fwd.modecoord,
                                      N, dp->bin_of_s2, n_s2, h.n_bins, h.kf, dp->winv, dp->acc, 1, nullptr, t);
      });
      mark("finalize", 0.0);
      launch_finalize_pk(s, dp->acc, ln.res_rows, h.n_bins, dp->ells_orders, dp->norm, dp->out);
    } else {
      TermTable tab;
      tab.tstart = dp->t_start; tab.tsh = dp->t_sh; tab.tell = dp->t_ell;
      tab.p1 = dp->t_p1; tab.p2 = dp->t_p2; tab.coef = dp->t_coef;
      tab.ntargets = (int)h.t_sh.size();
      tuned_launch(ctx, ln, ckey, contract_candidates(F.nmodes), [&](ColTune t) {
        launch_fill(s, dp->acc, nacc, 1);
        launch_contract_bis(s, h.prec, h.ell_max, h.order / 2, A, h.nfields, F.nmodes, F.mstride,
                            dp->fwd.modecoord, N, dp->bin_of_s2, n_s2, h.n_bins, h.nell, tab, h.kf, dp->winv,
                            dp->acc, t);
      });
      mark("finalize", 0.0);
      launch_finalize_pk(s, dp->acc, h.nell, h.n_bins, dp->ells, dp->norm, dp->out);
    }
  } else {
    // Full sets: pencil q = ky * rs + kx, N values each (bisector xi: the z-pass spectra in A,
    // pencil-major [p][q * N + kz]; midpoint: the y-pass output in B, [p][z][q]).
    const double sfull = (double)N * N * F.nkx * csz;  // one full half spectrum (algorithmic)
    const size_t sfull_b = (size_t)N * F.npen * (size_t)csz;  // one full pencil-major spectrum
    const double inv_n3 = 1.0 / ncell;
    const int npl = h.nz;  // retained z planes (= y rows) of the inverse outputs
    const double zpart = (double)h.n_inv * npl * F.npen_real * csz;
    const double ypart = (double)h.n_inv * npl * h.ny * F.nkx * csz;
    const bool xi = h.path != PATH_MID_PK;
    if (xi) launch_fill(s, dp->acc, nacc, 1);
    void *zout;
    const double sqrt4pi = std::sqrt(4.0 * 3.14159265358979323846);
    if (h.path == PATH_BIS_XI) {
      // a8 (bisector): T_{l nu}(k) = sum S Re(conj R_p1 R_p2) / W^2 on every mode, then the
      // inverse z pass of the real targets
      mark("targets", x3 + (double)h.n_targets * modes_real * rsz);
      launch_targets(s, h.prec, N, h.ell_max, h.order / 2, A, F.nmodes, F.mstride, F.rs, dp->winv, B);
      zout = A;
      mark("iz", (double)h.n_targets * modes_real * rsz + zpart);
      launch_iz(s, h.prec, N, B, zout, h.n_targets, 0, 1, F.npen, F.nkx, F.rs, nullptr, sqrt4pi, nullptr,
                dp->zrank, npl, dp->tw);
    } else {
      // a4 z pass + a5: conj(D) Q / W^2 (D = sqrt(4 pi) Q_{0,0,0}) + inverse z pass, one kernel
      // from the y-pass output (B): the alpha = 0 products of P_l stay in k-space at the front
      // of A, the retained z planes of the others follow them
      zout = A + (size_t)h.n_inplace * sfull_b;
      // the fused kernel addresses one field with 32-bit byte offsets below 2^31 (its masked
      // lanes use offset 2^31); with N <= 512 a field is at most 1.2 GB
      if ((double)N * F.npen * csz >= 2147483648.0) fail(PW_EINVAL, "field too large for the fused z pass");
      mark("fziz", x2 + (double)h.n_inplace * sfull + zpart);
      tuned_launch(ctx, ln, tune_key("fziz", h, h.nfields, h.n_inplace, npl), fz_candidates(h.nfields),
                   [&](ColTune t) {
                     launch_fziz(s, h.prec, N, B, A, zout, h.nfields, h.n_inplace, F.npen, F.rs, sqrt4pi, dp->winv,
                                 dp->zrank, npl, dp->tw, dp->planemask, t);
                   });
    }
    // inverse y pass of the retained z planes into B
    void *yout = B;
    mark("iy", (double)h.n_inv * npl * N * F.nkx * csz + ypart);
    tuned_launch(ctx, ln, tune_key("iy", h, h.n_inv, npl, h.ny), fy_candidates(h.prec, h.n_inv), [&](ColTune t) {
      launch_fy(s, h.prec, N, 1, zout, yout, h.n_inv, npl, F.nkx, F.rs, dp->iycnt, dp->iyoff,
                (int64_t)h.ny * F.rs, dp->tw, nullptr, nullptr, nullptr, t);
    });
    if (xi) {
      // a8: c2r along x fused with the |D|^alpha y(D^) weighting and FP64 r-binning
      mark("ix_bin", ypart);
      launch_ix(s, h.prec, N, 1, yout, nullptr, F.rs, dp->ijobs, (int)h.ijobs.size(), dp->icoef, h.nell, h.nz, h.ny,
                dp->zidx, dp->yidx, h.H, h.unit, inv_n3, dp->bin_of_s2, n_s2, h.n_bins, dp->acc, dp->tw);
      mark("finalize", 0.0);
      launch_finalize_xi(s, dp->acc, h.nell, h.n_bins, h.H * h.H * h.H, dp->norm, dp->out);
    } else {
      void *Aoff = A + (size_t)h.n_inplace * sfull_b;  // behind the alpha = 0 products
      if (h.n_inv > 0) {
        // g fields in real space (Aoff), then a6: A_{l nu} = sum Phi' y(D^) |D|^alpha g (into B)
        mark("ix", ypart + (double)h.n_inv * ncell * rsz);
        launch_ix(s, h.prec, N, 0, yout, Aoff, F.rs, dp->ijobs, (int)h.ijobs.size(), nullptr, h.nell, h.nz, h.ny,
                  dp->zidx, dp->yidx, h.H, h.unit, inv_n3, nullptr, 0, 0, nullptr, dp->tw);
        mark("reweight", (double)(h.n_inv + h.n_a) * ncell * rsz);
        launch_reweight(s, h.prec, N, h.ell_max, h.order, h.all_parity, Aoff, B, h.H / h.unit);
        // forward transforms of A, pruned to the k-sphere of the bins (ending in Aoff)
        const Prune &P = h.sph;
        const double a1 = (double)h.n_a * N * N * P.nkx * csz, a2 = (double)h.n_a * N * P.npen * csz,
                     a3 = (double)h.n_a * P.nretained * csz;
        mark("afx", (double)h.n_a * ncell * rsz + a1);
        tuned_launch(ctx, ln, tune_key("fx", h, (int)h.ajobs.size(), FX_PLAIN, P.nkx), fx_candidates(h.prec, N),
                     [&](ColTune t) {
                       launch_fx(s, h.prec, N, FX_PLAIN, B, Aoff, dp->ajobs, (int)h.ajobs.size(), P.nkx, P.rs,
                                 cfg->box_origin, h.H, h.unit, dp->tw, nullptr, nullptr, nullptr, t);
                     });
        mark("afy", a1 + a2);
        if (P.npen > 0)
          launch_fy(s, h.prec, N, 0, Aoff, B, h.n_a, N, P.nkx, P.rs, dp->sph.ycnt, dp->sph.yoff, P.npen, dp->tw,
                    nullptr, nullptr, nullptr);
        mark("afz", a2 + a3);
        if (P.npen > 0)
          launch_fz(s, h.prec, N, B, Aoff, h.n_a, P.npen, dp->sph.pinfo, dp->sph.moff, dp->sph.goff, dp->sph.gsize,
                    P.mstride, dp->tw, nullptr);
      }
      // a7 (midpoint): sum_nu y_l^nu(k^) Re[G_{l nu} + A_{l nu}] and FP64 k-binning
      mark("contract", (double)(h.n0 + h.n_a) * h.sph.nretained * csz + 4.0 * h.sph.nretained);
      launch_fill(s, dp->acc, nacc, 1);
      launch_contract_mid(s, h.prec, h.ell_max, A, F.rs, h.n_a > 0 ? Aoff : nullptr, h.sph.nmodes, h.sph.mstride,
                          dp->sph.modecoord, N, dp->bin_of_s2, n_s2, h.n_bins, h.kf, dp->acc);
      mark("finalize", 0.0);
      launch_finalize_pk(s, dp->acc, h.nell, h.n_bins, dp->ells, dp->norm, dp->out);
    }
  }
  mark(nullptr, 0.0);
  ln.n_stages = ns - 1;
  HIPCHECK(hipGetLastError());
  const size_t nres = (size_t)(ln.res_rows + 2) * h.n_bins;
  const size_t need = nres * sizeof(double) + sizeof(DevNorm);
  if (!placed && ln.host_res_bytes < need) {
    if (ln.host_res) (void)hipHostFree(ln.host_res);
    ln.host_res = nullptr;
    ln.host_res_bytes = 0;
    HIPCHECK(hipHostMalloc((void **)&ln.host_res, need, hipHostMallocDefault));
    ln.host_res_bytes = need;
  }
  double *res_host = placed ? placed->host_res : ln.host_res;
  HIPCHECK(hipMemcpyAsync(res_host, dp->out, nres * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync((char *)res_host + nres * sizeof(double), dp->norm, sizeof(DevNorm),
                          hipMemcpyDeviceToHost, s));
  ln.res_slice = need;
  HIPCHECK(hipEventRecord(ln.done, s));
  return dp;
}

// Whether a configuration has the batched path: the bisector P_l with a generated contraction,
// default plan (several catalogs of one configuration in each forward pass and contraction).
bool batchable(const pw_config &c) {
  return c.stat == PW_PK && c.los == PW_BISECTOR && !c.memory_lean && bis_contract_generated(c.ell_max, c.order / 2);
}

// Enqueue the estimates of n catalogs of one batchable configuration on the lane's stream:
// each catalog is painted into its own plan buffers and workspace, then the x, y and z passes
// and the contraction each run once over all n catalogs (grid z = catalog).  Catalog 0 uses
// the lane's plan and workspace; catalogs 1 .. n-1 the lane's batch plans and batch workspace.
// Results go to slices of res_slice bytes of the lane's pinned buffer.  Returns catalog 0's plan.
DevPlan *launch_batch(pw_ctx *ctx, Lane &ln, const pw_config *cfg, int n, const pw_catalog *const *gals,
                      const pw_catalog *const *rans, const pw_norm *const *norms) {
  if (n < 1 || n > kMaxBatch || !batchable(*cfg)) fail(PW_EINVAL, "internal: not a batchable launch");
  HIPCHECK(hipSetDevice(ctx->device));
  ensure_sh(ctx->device);
  DevPlan *dp0 = get_plan(ctx, ln, cfg);
  bind_work(ctx, ln, dp0);
  const HostPlan &h = *dp0->host;
  auto &extra = ln.bplans[make_key(*cfg)];
  while ((int)extra.size() < n - 1) extra.push_back(build_dev_plan(ctx, cfg));
  const size_t per = (dp0->work.total + 255) & ~(size_t)255;
  if (n > 1) ensure_buffer(ctx, &ln.bwork, &ln.bwork_bytes, per * (size_t)(n - 1));
  std::vector<DevPlan *> plans((size_t)n);
  plans[0] = dp0;
  for (int i = 1; i < n; ++i) {
    DevPlan *p = extra[(size_t)i - 1].get();
    char *w = (char *)ln.bwork + (size_t)(i - 1) * per;
    p->mesh = w + p->work.mesh;
    p->bufA = w + p->work.bufA;
    p->bufB = w + p->work.bufB;
    p->bufC = nullptr;
    p->tile_blocks = w + p->work.tiles;
    plans[(size_t)i] = p;
  }
  ln.last = dp0;
  ln.n_stages = 0;  // no stage timing for batched launches
  hipStream_t s = ln.stream;
  // a1 + a2 per catalog, one after another through the lane's staging and sort buffers
  size_t rec = 0;
  for (int i = 0; i < n; ++i)
    rec = std::max(rec, records_bytes(h.prec, gals[i]->n, rans[i]->n) +
                            sort_layout(h.N, gals[i]->n, rans[i]->n).hist_bytes);
  ensure_buffer(ctx, &ln.records, &ln.records_bytes, rec);
  for (int i = 0; i < n; ++i) {
    const void *gnb = nullptr, *rnb = nullptr;
    const void *gx = stage_catalog(ctx, ln, gals[i], 0, &gnb);
    const void *rx = stage_catalog(ctx, ln, rans[i], 1, &rnb);
    enqueue_paint(ctx, nullptr, s, plans[(size_t)i], cfg, gals[i], gx, rans[i], rx, rnb, norms[i], ln.records);
  }
  // a3 + a4 + a7: one launch per pass over every catalog
  Batch ba;
  std::memset(&ba, 0, sizeof(ba));
  ba.n = n;
  for (int i = 0; i < n; ++i) {
    const DevPlan *p = plans[(size_t)i];
    ba.s[i] = BatchSlot{p->mesh, p->bufA, p->bufB, p->rowlist, p->rowmask, p->zlist, p->planemask, p->norm, p->acc};
  }
  const int N = h.N;
  const Prune &F = h.fwd;
  launch_fx(s, h.prec, N, FX_HARMONIC, dp0->mesh, dp0->bufA, dp0->jobs, (int)h.jobs.size(), F.nkx, F.rs,
            cfg->box_origin, h.H, h.unit, dp0->tw, dp0->rowlist, dp0->norm, &ba,
            tuned_choice(ctx, tune_key("fx", h, (int)h.jobs.size(), FX_HARMONIC, F.nkx), fx_candidates(h.prec, N)));
  if (F.npen > 0) {
    launch_fy(s, h.prec, N, 0, dp0->bufA, dp0->bufB, h.nfields, N, F.nkx, F.rs, dp0->fwd.ycnt, dp0->fwd.yoff,
              F.npen, dp0->tw, dp0->rowmask, dp0->zlist, dp0->norm,
              tuned_choice(ctx, tune_key("fy", h, h.nfields, F.nkx, F.npen), fy_candidates(h.prec, h.nfields)), &ba);
    launch_fz(s, h.prec, N, dp0->bufB, dp0->bufA, h.nfields, F.npen, dp0->fwd.pinfo, dp0->fwd.moff, dp0->fwd.goff,
              dp0->fwd.gsize, F.mstride, dp0->tw, dp0->planemask, nullptr,
              tuned_choice(ctx, tune_key("fz", h, h.nfields, F.npen, F.goff.empty() ? 0 : 1),
                           fz_candidates(h.nfields)),
              &ba);
  }
  ln.res_rows = h.nell;
  const size_t nacc = (size_t)(h.nell + 2) * h.n_bins;
  for (int i = 0; i < n; ++i) launch_fill(s, plans[(size_t)i]->acc, nacc, 1);
  if (!launch_contract_bis_generated(s, h.prec, h.ell_max, h.order / 2, dp0->bufA, F.nmodes, F.mstride,
                                     dp0->fwd.modecoord, N, dp0->bin_of_s2, (int64_t)h.bin_of_s2.size(), h.n_bins,
                                     h.kf, dp0->winv, dp0->acc, 0, &ba))
    fail(PW_EINVAL, "internal: no generated contraction for a batched launch");
  for (int i = 0; i < n; ++i)
    launch_finalize_pk(s, plans[(size_t)i]->acc, h.nell, h.n_bins, dp0->ells, plans[(size_t)i]->norm,
                       plans[(size_t)i]->out);
  HIPCHECK(hipGetLastError());
  const size_t nres = (size_t)(h.nell + 2) * h.n_bins;
  const size_t slice = (nres * sizeof(double) + sizeof(DevNorm) + 255) & ~(size_t)255;
  if (ln.host_res_bytes < slice * (size_t)n) {
    if (ln.host_res) (void)hipHostFree(ln.host_res);
    ln.host_res = nullptr;
    ln.host_res_bytes = 0;
    HIPCHECK(hipHostMalloc((void **)&ln.host_res, slice * (size_t)n, hipHostMallocDefault));
    ln.host_res_bytes = slice * (size_t)n;
  }
  for (int i = 0; i < n; ++i) {
    char *dst = (char *)ln.host_res + (size_t)i * slice;
    HIPCHECK(hipMemcpyAsync(dst, plans[(size_t)i]->out, nres * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(dst + nres * sizeof(double), plans[(size_t)i]->norm, sizeof(DevNorm),
                            hipMemcpyDeviceToHost, s));
  }
  ln.res_slice = slice;
  HIPCHECK(hipEventRecord(ln.done, s));
  return dp0;
}

// Results of catalog i of the launch in flight on the lane (host copy).
const double *lane_result(const Lane &ln, int i) {
  return (const double *)((const char *)ln.host_res + (size_t)i * ln.res_slice);
}

// The error flags an estimate raised on the device (PW_ERANGE, PW_EINVAL), as a failure.
void check_flags(const DevNorm &dn) {
  if (dn.flags & 1) fail(PW_ERANGE, "a particle lies outside [box_origin, box_origin + box_len)");
  if (dn.flags & 2)
    fail(PW_EINVAL, "midpoint P_l with order > 0 needs the catalog extent <= box_len / 2 on every axis");
}

// After the lane's completion event: check the flags and write the caller's outputs from the
// copied results `res`.
void finish_estimate(Lane &ln, const DevPlan *dp, const double *res, pw_norm *norm, double *out,
                     double *bin_mean, int64_t *counts) {
  const HostPlan &h = *dp->host;
  const int rows = ln.res_rows;
  const size_t nres = (size_t)(rows + 2) * h.n_bins;
  DevNorm dn;
  std::memcpy(&dn, (const char *)res + nres * sizeof(double), sizeof(DevNorm));
  check_flags(dn);
  std::memcpy(out, res, (size_t)rows * h.n_bins * sizeof(double));
  if (bin_mean) std::memcpy(bin_mean, res + (size_t)rows * h.n_bins, h.n_bins * sizeof(double));
  if (counts)
    for (int b = 0; b < h.n_bins; ++b) counts[b] = (int64_t)std::llround(res[(size_t)(rows + 1) * h.n_bins + b]);
  if (norm && !norm->use_given) {
    norm->alpha_r = dn.alpha_r;
    norm->I = dn.I;
    norm->S = dn.S;
  }
}

// Make room on lane 0 for cfg's plan tables, workspace and catalogs by evicting idle serving
// lanes' workspaces, then cached plans (lane 0's other ones, idle serving lanes'), least
// recently used first.
// (n catalogs gal[0 .. n), ran[0 .. n) of one configuration: a batched launch also needs the
// lane's batch plans and batch workspace)
void make_room_main(pw_ctx *ctx, const pw_config *cfg, const pw_catalog *gal, const pw_catalog *ran,
                    Reservation &res, int nb = 1) {
  Lane &ln = *ctx->main;
  const PlanKey key = make_key(*cfg);
  std::shared_ptr<const HostPlan> hp = host_plan(ctx, *cfg);
  const size_t tables = table_bytes(*hp), work = work_layout(*hp).total;
  const size_t per = (work + 255) & ~(size_t)255;
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto need = [&]() -> size_t {
    size_t n = ln.plans.count(key) ? 0 : tables;
    n += work > ln.work_bytes ? work - ln.work_bytes : 0;
    if (nb > 1) {
      auto it = ln.bplans.find(key);
      const size_t have = it == ln.bplans.end() ? 0 : it->second.size();
      n += have < (size_t)(nb - 1) ? ((size_t)(nb - 1) - have) * tables : 0;
      const size_t bw = per * (size_t)(nb - 1);
      n += bw > ln.bwork_bytes ? bw - ln.bwork_bytes : 0;
    }
    return n;
  };
  if (need() == 0) return;
  size_t cat = 0;  // catalogs are staged and sorted one at a time: the largest one's buffers
  for (int i = 0; i < nb; ++i) cat = std::max(cat, catalog_bytes(*cfg, gal[i], ran[i]));
  while (mem_used(ctx) + ctx->reserved + need() + cat > ctx->budget) {
    Lane *wl = nullptr;
    uint64_t oldest = (uint64_t)-1;
    for (auto &lp : ctx->lanes)
      if (!lp->cur && lp->work && lp->used_stamp < oldest) { oldest = lp->used_stamp; wl = lp.get(); }
    if (wl) {
      evict_work(ctx, *wl);
      continue;
    }
    Lane *vl = nullptr;
    PlanKey vk;
    for (auto &kv : ln.plan_stamp)
      if (kv.first != key && kv.second < oldest) { oldest = kv.second; vl = &ln; vk = kv.first; }
    for (auto &lp : ctx->lanes) {
      if (lp->cur) continue;
      for (auto &kv : lp->plan_stamp)
        if (kv.second < oldest) { oldest = kv.second; vl = lp.get(); vk = kv.first; }
    }
    if (!vl) break;
    evict_plan(ctx, *vl, vk);
  }
  res.bytes = need() + cat;  // (if it does not fit, the allocation fails with PW_ENOMEM)
  ctx->reserved += res.bytes;
}

void complete_main(Lane &ln, const DevPlan *dp, const double *res_host, pw_norm *norm, double *out,
                   double *bin_mean, int64_t *counts);

// ------------------------------------------------------------------------------ tracing
double ms_since_create(const pw_ctx *ctx) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ctx->t0).count();
}

// One JSON line per completed estimate into the PW_TRACE file: when it ended (ms since
// pw_create), what ran (kind, ticket, lane, configuration, catalog sizes, catalogs in its
// launch), how long it waited for admission and ran on the host's clock, and the stage times
// from the lane's events (launches of one catalog only; a batched launch has none).
void trace_write(pw_ctx *ctx, const Lane &ln, const char *kind, uint64_t ticket, const pw_config &c, int64_t n_gal,
                 int64_t n_ran, size_t batch, double t_submit, double t_start, int status) {
  if (!ctx->trace) return;
  std::lock_guard<std::mutex> lk(ctx->trace_mu);  // (lines in the order of their end times)
  const double t_end = ms_since_create(ctx);
  std::string stages;
  if (batch == 1 && status == PW_OK) {
    for (int i = 0; i < ln.n_stages; ++i) {
      float ms = -1.0f;
      if (hipEventElapsedTime(&ms, ln.ev[i], ln.ev[i + 1]) != hipSuccess) ms = -1.0f;
      char b[96];
      std::snprintf(b, sizeof(b), "%s\"%s\": %.4f", i ? ", " : "", ln.st_name[i] ? ln.st_name[i] : "?", (double)ms);
      stages += b;
    }
  }
  char line[768];
  std::snprintf(line, sizeof(line),
                "{\"t_ms\": %.3f, \"kind\": \"%s\", \"ticket\": %llu, \"lane\": %d, \"status\": %d, "
                "\"stat\": \"%s\", \"los\": \"%s\", \"n_mesh\": %d, \"prec\": \"%s\", \"n_gal\": %lld, "
                "\"n_ran\": %lld, \"batch\": %zu, \"queued_ms\": %.3f, \"run_ms\": %.3f, \"stages_ms\": {",
                t_end, kind, (unsigned long long)ticket, ln.id, status, c.stat == PW_PK ? "pk" : "xi",
                c.los == PW_BISECTOR ? "bisector" : "midpoint", c.n_mesh, c.prec == PW_FP32 ? "fp32" : "fp64",
                (long long)n_gal, (long long)n_ran, batch, t_start - t_submit, t_end - t_start);
  std::fputs(line, ctx->trace);
  std::fputs(stages.c_str(), ctx->trace);
  std::fputs("}}\n", ctx->trace);
  std::fflush(ctx->trace);
}

void run_estimate(pw_ctx *ctx, const pw_config *cfg, const pw_catalog *gal, const pw_catalog *ran,
                  pw_norm *norm, double *out, double *bin_mean, int64_t *counts, bool orders = false) {
  check_request(cfg, gal, ran, norm, out);
  const double t_start = ms_since_create(ctx);
  MainBusy busy(ctx);
  Reservation res(ctx);
  make_room_main(ctx, cfg, gal, ran, res);
  Lane &ln = *ctx->main;
  DevPlan *dp = launch_estimate(ctx, ln, cfg, gal, ran, norm, orders);
  res.release();
  complete_main(ln, dp, ln.host_res, norm, out, bin_mean, counts);
  trace_write(ctx, ln, orders ? "orders" : "estimate", 0, *cfg, gal->n, ran->n, 1, t_start, t_start, PW_OK);
}

// pw_estimate_batch: n catalogs of one configuration (arrays gal[n], ran[n], norm[n] or NULL;
// outputs [n][...]), in batched launches when the configuration has them, else one estimate
// after another.
void run_estimate_batch(pw_ctx *ctx, const pw_config *cfg, int n, const pw_catalog *gal, const pw_catalog *ran,
                        pw_norm *norm, double *out, double *bin_mean, int64_t *counts) {
  if (!cfg || !gal || !ran || !out) fail(PW_EINVAL, "null configuration, catalogs or output");
  if (n < 1 || n > kMaxBatch) fail(PW_EINVAL, "pw_estimate_batch: n must be in 1..%d", kMaxBatch);
  validate_config(*cfg);
  const size_t nb = (size_t)cfg->n_bins, so = (size_t)(cfg->ell_max / 2 + 1) * nb;
  for (int i = 0; i < n; ++i) check_request(cfg, &gal[i], &ran[i], norm ? &norm[i] : nullptr, out + i * so);
  if (!batchable(*cfg) || n == 1) {
    for (int i = 0; i < n; ++i)
      run_estimate(ctx, cfg, &gal[i], &ran[i], norm ? &norm[i] : nullptr, out + i * so,
                   bin_mean ? bin_mean + i * nb : nullptr, counts ? counts + i * nb : nullptr);
    return;
  }
  const double t_start = ms_since_create(ctx);
  MainBusy busy(ctx);
  Reservation res(ctx);
  make_room_main(ctx, cfg, gal, ran, res, n);
  Lane &ln = *ctx->main;
  std::vector<const pw_catalog *> gp((size_t)n), rp((size_t)n);
  std::vector<const pw_norm *> np((size_t)n);
  for (int i = 0; i < n; ++i) {
    gp[(size_t)i] = &gal[i];
    rp[(size_t)i] = &ran[i];
    np[(size_t)i] = norm ? &norm[i] : nullptr;
  }
  DevPlan *dp = launch_batch(ctx, ln, cfg, n, gp.data(), rp.data(), np.data());
  res.release();
  HIPCHECK(hipEventSynchronize(ln.done));
  const size_t nres = (size_t)(ln.res_rows + 2) * nb;
  for (int i = 0; i < n; ++i) {  // every catalog's flags before any output is written
    DevNorm dn;
    std::memcpy(&dn, (const char *)lane_result(ln, i) + nres * sizeof(double), sizeof(DevNorm));
    check_flags(dn);
  }
  for (int i = 0; i < n; ++i) {
    finish_estimate(ln, dp, lane_result(ln, i), norm ? &norm[i] : nullptr, out + i * so,
                    bin_mean ? bin_mean + i * nb : nullptr, counts ? counts + i * nb : nullptr);
    trace_write(ctx, ln, "batch", 0, *cfg, gal[i].n, ran[i].n, (size_t)n, t_start, t_start, PW_OK);
  }
}

// Lane 0 after launch_estimate: wait, read the stage times, scale the forward passes'
// algorithmic bytes by the measured occupancy, and write the outputs.
void complete_main(Lane &ln, const DevPlan *dp, const double *res_host, pw_norm *norm, double *out,
                   double *bin_mean, int64_t *counts) {
  HIPCHECK(hipEventSynchronize(ln.done));
  for (int i = 0; i < ln.n_stages; ++i) {
    float ms = -1.0f;
    if (ln.timing) HIPCHECK(hipEventElapsedTime(&ms, ln.ev[i], ln.ev[i + 1]));
    ln.st_ms[i] = ln.timing ? (double)ms : -1.0;
  }
  {
    // forward passes touch only the occupied rows / planes: scale their algorithmic bytes
    const HostPlan &h = *dp->host;
    const size_t nres = (size_t)(ln.res_rows + 2) * h.n_bins;
    DevNorm dn;
    std::memcpy(&dn, (const char *)res_host + nres * sizeof(double), sizeof(DevNorm));
    const double N = h.N, rsz = h.prec == PW_FP32 ? 4.0 : 8.0, csz = 2 * rsz;
    const double fr = dn.nrows_occ / (N * N), fp = dn.nplanes_occ / N;
    const double modes_real = h.fwd.full ? N * (double)h.fwd.npen_real : (double)h.fwd.nretained;
    const double x1 = (double)h.nfields * N * N * h.fwd.nkx * csz;
    const double x2 = (double)h.nfields * N * h.fwd.npen_real * csz;
    const double x3 = (double)h.nfields * modes_real * csz;
    for (int i = 0; i < ln.n_stages; ++i) {
      const std::string nm = ln.st_name[i] ? ln.st_name[i] : "";
      if (nm == "fx") ln.st_bytes[i] = fr * (N * N * N * rsz + x1);
      else if (nm == "fy") ln.st_bytes[i] = fr * x1 + fp * x2;
      else if (nm == "fz") ln.st_bytes[i] = fp * x2 + x3;
      else if (nm == "fziz") ln.st_bytes[i] -= (1.0 - fp) * x2;  // reads the occupied planes only
      else if (nm == "forward") ln.st_bytes[i] = fr * (N * N * N * rsz + 2 * x1) + 2 * fp * x2 + x3;
    }
    ln.occ_rows = dn.nrows_occ;
    ln.occ_planes = dn.nplanes_occ;
  }
  finish_estimate(ln, dp, res_host, norm, out, bin_mean, counts);
}

// pw_submit: copy the request's pageable host catalogs (and the randoms' nbar) into one pinned
// buffer of the context's pool, on the caller's thread, so that the lane's copies to the device
// run asynchronously beside other lanes' kernels.  Host memory that is already pinned is read
// in place.  Without room in the pool the request keeps the caller's pointers.
void stage_pinned(pw_ctx *ctx, Req *r) {
  struct Piece {
    const void **ptr;
    size_t bytes;
  };
  std::vector<Piece> pieces;
  auto add = [&](pw_catalog &c, bool with_nbar) {
    if (c.on_device || c.n <= 0) return;
    const size_t isz = c.dtype == PW_FP32 ? 4 : 8;
    if (!host_pinned(c.xyzw)) pieces.push_back({&c.xyzw, (size_t)c.n * 4 * isz});
    if (with_nbar && c.nbar && !host_pinned(c.nbar)) pieces.push_back({&c.nbar, (size_t)c.n * isz});
  };
  add(r->gal, false);
  add(r->ran, true);
  if (pieces.empty()) return;
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  size_t need = 0;
  for (auto &p : pieces) need += up(p.bytes);
  size_t got = 0;
  void *buf = pin_acquire(ctx, need, &got);
  if (!buf) return;
  r->pin = buf;
  r->pin_bytes = got;
  char *dst = (char *)buf;
  for (auto &p : pieces) {
    std::memcpy(dst, *p.ptr, p.bytes);
    *p.ptr = dst;
    dst += up(p.bytes);
  }
}

// pw_estimate_noalloc: pw_estimate with every device buffer in the static scratch (nothing is
// allocated on the device or pinned on the host); device-resident catalogs only.
void run_estimate_noalloc(pw_ctx *ctx, const pw_config *cfg, const pw_catalog *gal, const pw_catalog *ran,
                          pw_norm *norm, double *out, double *bin_mean, int64_t *counts) {
  check_request(cfg, gal, ran, norm, out);
  if ((gal->n > 0 && !gal->on_device) || (ran->n > 0 && !ran->on_device))
    fail(PW_EINVAL, "pw_estimate_noalloc reads device-resident catalogs only (on_device = 1)");
  std::string why;
  char *region = scratch_of(ctx->device, &why);
  if (!region) fail(PW_EDEVICE, "the static scratch of device %d: %s", ctx->device, why.c_str());
  std::shared_ptr<const HostPlan> hp = host_plan(ctx, *cfg);
  const size_t rec = records_bytes(hp->prec, gal->n, ran->n) + sort_layout(hp->N, gal->n, ran->n).hist_bytes;
  const size_t need = table_bytes(*hp) + work_layout(*hp).total + rec + 2 * 256;
  if (need > kScratchBytes)
    fail(PW_ENOMEM,
         "pw_estimate_noalloc: this estimate needs about %zu bytes of device scratch, the static scratch holds "
         "%zu (%zu MiB); use pw_estimate",
         need, kScratchBytes, kScratchBytes >> 20);
  MainBusy busy(ctx);
  Lane &ln = *ctx->main;
  size_t used = 0;
  std::unique_ptr<DevPlan> dp = build_dev_plan(ctx, cfg, region, kScratchBytes, &used);
  PlanMem M{ctx, dp.get(), region, kScratchBytes, used};
  char *w = (char *)M.get(dp->work.total);
  dp->mesh = w + dp->work.mesh;
  dp->bufA = w + dp->work.bufA;
  dp->bufB = w + dp->work.bufB;
  dp->bufC = hp->lean ? w + dp->work.bufC : nullptr;
  dp->tile_blocks = w + dp->work.tiles;
  void *records = M.get(rec);
  const size_t words = (size_t)(hp->nell + 2) * hp->n_bins + (sizeof(DevNorm) + 7) / 8;
  if (ln.noalloc_res.size() < words) ln.noalloc_res.resize(words);
  Placed pl{dp.get(), records, ln.noalloc_res.data()};
  const double t_start = ms_since_create(ctx);
  launch_estimate(ctx, ln, cfg, gal, ran, norm, false, &pl);
  complete_main(ln, dp.get(), pl.host_res, norm, out, bin_mean, counts);
  trace_write(ctx, ln, "noalloc", 0, *cfg, gal->n, ran->n, 1, t_start, t_start, PW_OK);
}

Lane *make_lane(int id, hipStream_t user_stream, bool stage_events) {
  std::unique_ptr<Lane> ln(new Lane());
  ln->id = id;
  if (user_stream) {
    ln->stream = user_stream;
  } else {
    HIPCHECK(hipStreamCreateWithFlags(&ln->stream, hipStreamNonBlocking));  // default priority
    ln->own_stream = true;
  }
  HIPCHECK(hipEventCreateWithFlags(&ln->done, hipEventDisableTiming));
  for (int i = 0; i < 2; ++i) HIPCHECK(hipEventCreate(&ln->tev[i]));
  if (id == 0 || stage_events)
    for (int i = 0; i <= kMaxStages; ++i) HIPCHECK(hipEventCreate(&ln->ev[i]));
  ln->timing = id != 0 && stage_events;  // lane 0: pw_set_timing, or tracing (launch_estimate)
  return ln.release();
}

void destroy_lane(pw_ctx *ctx, Lane *ln) {
  if (!ln) return;
  if (ln->stream) (void)hipStreamSynchronize(ln->stream);
  for (auto &kv : ln->plans) free_plan(ctx, kv.second.get());
  ln->plans.clear();
  for (auto &kv : ln->bplans)
    for (auto &p : kv.second) free_plan(ctx, p.get());
  ln->bplans.clear();
  for (int i = 0; i < 2; ++i) dev_free(ctx, ln->stage[i], ln->stage_bytes[i]);
  dev_free(ctx, ln->stage_nbar, ln->stage_nbar_bytes);
  dev_free(ctx, ln->records, ln->records_bytes);
  evict_work(ctx, *ln);
  if (ln->host_res) (void)hipHostFree(ln->host_res);
  for (int i = 0; i <= kMaxStages; ++i)
    if (ln->ev[i]) (void)hipEventDestroy(ln->ev[i]);
  if (ln->done) (void)hipEventDestroy(ln->done);
  for (int i = 0; i < 2; ++i)
    if (ln->tev[i]) (void)hipEventDestroy(ln->tev[i]);
  if (ln->own_stream && ln->stream) (void)hipStreamDestroy(ln->stream);
}

// ------------------------------------------------------------------------------ serving
// Bytes a lane still has to allocate to run `r` (0 when its plan and buffers are resident).
size_t lane_extra_bytes(const Lane &ln, const Req &r) {
  size_t extra = 0;
  if (ln.plans.find(make_key(r.cfg)) == ln.plans.end()) extra += r.need_tables;
  if (ln.work_bytes < r.need_work) extra += r.need_work - ln.work_bytes;
  const size_t rec = records_bytes(r.cfg.prec, r.gal.n, r.ran.n) +
                    sort_layout(r.cfg.n_mesh, r.gal.n, r.ran.n).hist_bytes;
  if (ln.records_bytes < rec) extra += rec;
  auto stg = [&](const pw_catalog &c, size_t have) -> size_t {
    if (c.on_device) return 0;
    size_t b = (size_t)c.n * 4 * (c.dtype == PW_FP32 ? 4 : 8);
    return have >= b ? 0 : b;
  };
  extra += stg(r.gal, ln.stage_bytes[0]) + stg(r.ran, ln.stage_bytes[1]);
  if (!r.ran.on_device && r.ran.nbar) {
    const size_t nb = (size_t)r.ran.n * (r.ran.dtype == PW_FP32 ? 4 : 8);
    if (ln.stage_nbar_bytes < nb) extra += nb;
  }
  return extra;
}

// Meshes up to this size batch pending requests of one configuration into one launch (at 512^3
// one catalog already fills the device).
constexpr int kBatchMaxMesh = 256;

// Batching in the serving loop: after `lead` is admitted on `ln`, later pending requests of the
// same batchable configuration join its launch (up to kMaxBatch catalogs) while the memory they
// add fits the budget: a batch plan's tables when the lane holds too few, a workspace slot,
// their sort buffers and staging.  A lane's batch workspace stays within 1/16 of the budget, so
// batching never crowds out other lanes' workspaces.  Called with ctx->mu held.
void add_followers(pw_ctx *ctx, Lane &ln, Req *lead) {
  if (!batchable(lead->cfg) || lead->cfg.n_mesh > kBatchMaxMesh) return;
  const PlanKey key = make_key(lead->cfg);
  auto bt = ln.bplans.find(key);
  const size_t have = bt == ln.bplans.end() ? 0 : bt->second.size();
  const size_t per = (lead->need_work + 255) & ~(size_t)255;
  const size_t max_slots = per > 0 ? (ctx->budget / 16) / per : 0;  // catalogs beyond the lead
  for (auto jt = ctx->pending.begin();
       jt != ctx->pending.end() && (int)ln.batch.size() < kMaxBatch && ln.batch.size() <= max_slots;) {
    Req *q = *jt;
    if (make_key(q->cfg) != key) {
      ++jt;
      continue;
    }
    const size_t slot = ln.batch.size();  // catalog index of q in the launch (>= 1)
    size_t add = (slot - 1 < have) ? 0 : q->need_tables;
    if (per * slot > ln.bwork_bytes) add += per;
    add += catalog_bytes(q->cfg, q->gal, q->ran);
    if (mem_used(ctx) + ctx->reserved + add > ctx->budget) break;
    q->reserved = add;
    ctx->reserved += add;
    ln.batch.push_back(q);
    jt = ctx->pending.erase(jt);
  }
}

// Try to admit the oldest pending request that can run now.  Called with ctx->mu held.
// Returns the (request, lane) to launch, or (nullptr, nullptr).
std::pair<Req *, Lane *> pick_admission(pw_ctx *ctx) {
  for (auto it = ctx->pending.begin(); it != ctx->pending.end(); ++it) {
    Req *r = *it;
    // free lanes, preferring one whose plan for this configuration is resident
    Lane *best = nullptr;
    size_t best_extra = (size_t)-1;
    for (auto &lp : ctx->lanes) {
      if (lp->cur) continue;
      size_t e = lane_extra_bytes(*lp, *r);
      if (e < best_extra) { best = lp.get(); best_extra = e; }
    }
    if (!best) return {nullptr, nullptr};  // every lane busy
    // make room: evict the workspaces of idle lanes other than `best` (lane 0's too while no
    // pw_estimate runs), then idle lanes' cached plans, least recently used first
    const bool main_idle = !ctx->main_busy;
    while (mem_used(ctx) + ctx->reserved + best_extra > ctx->budget) {
      Lane *wl = nullptr;
      uint64_t oldest = (uint64_t)-1;
      for (auto &lp : ctx->lanes)
        if (!lp->cur && lp.get() != best && lp->work && lp->used_stamp < oldest) {
          oldest = lp->used_stamp;
          wl = lp.get();
        }
      if (main_idle && ctx->main->work && ctx->main->used_stamp < oldest) wl = ctx->main.get();
      if (wl) {
        evict_work(ctx, *wl);
        best_extra = lane_extra_bytes(*best, *r);
        continue;
      }
      Lane *vl = nullptr;
      const PlanKey *vk = nullptr;
      for (auto &lp : ctx->lanes) {
        if (lp->cur) continue;
        for (auto &kv : lp->plan_stamp) {
          if (lp.get() == best && kv.first == make_key(r->cfg)) continue;
          if (kv.second < oldest) { oldest = kv.second; vl = lp.get(); vk = &kv.first; }
        }
      }
      if (main_idle)
        for (auto &kv : ctx->main->plan_stamp)
          if (kv.second < oldest) { oldest = kv.second; vl = ctx->main.get(); vk = &kv.first; }
      if (!vl) break;
      PlanKey k = *vk;
      evict_plan(ctx, *vl, k);
      best_extra = lane_extra_bytes(*best, *r);
    }
    if (mem_used(ctx) + ctx->reserved + best_extra <= ctx->budget) {
      ctx->pending.erase(it);
      r->reserved = best_extra;  // released once the launch has made its allocations
      ctx->reserved += best_extra;
      best->batch.assign(1, r);
      add_followers(ctx, *best, r);
      return {r, best};
    }
    bool running = ctx->main_busy;  // lane 0 may still release memory
    for (auto &lp : ctx->lanes) running = running || lp->cur != nullptr;
    if (!running) {
      // can never fit: fail it and look at the next one
      r->status = PW_ENOMEM;
      r->err = "request does not fit the context's HBM budget";
      pin_release(ctx, r);
      ctx->pending.erase(it);
      ctx->cv.notify_all();
      return pick_admission(ctx);
    }
    // wait for memory: keep arrival order for requests that need more memory
    return {nullptr, nullptr};
  }
  return {nullptr, nullptr};
}

void worker_loop(pw_ctx *ctx) {
  (void)hipSetDevice(ctx->device);
  std::unique_lock<std::mutex> lk(ctx->mu);
  for (;;) {
    bool any_running = false;
    // completions
    for (auto &lp : ctx->lanes) {
      Lane &ln = *lp;
      if (!ln.cur) continue;
      hipError_t q = hipEventQuery(ln.done);
      if (q == hipErrorNotReady) { any_running = true; continue; }
      for (size_t i = 0; i < ln.batch.size(); ++i) {
        Req *r = ln.batch[i];
        if (q != hipSuccess) {
          r->status = PW_EDEVICE;
          r->err = std::string("device error: ") + hipGetErrorString(q);
        } else {
          try {
            finish_estimate(ln, r->dp, lane_result(ln, (int)i), r->norm_out, r->out, r->bin_mean, r->counts);
            r->status = PW_OK;
          } catch (const Fail &f) {
            r->status = f.code;
            r->err = f.msg;
          }
        }
        trace_write(ctx, ln, "served", r->ticket, r->cfg, r->gal.n, r->ran.n, ln.batch.size(), r->t_submit,
                    r->t_start, r->status);
        pin_release(ctx, r);  // the lane's copies out of it are complete
      }
      ln.batch.clear();
      ln.cur = nullptr;
      ctx->cv.notify_all();
    }
    // admissions
    for (;;) {
      std::pair<Req *, Lane *> a = pick_admission(ctx);
      if (!a.first) break;
      Req *r = a.first;
      Lane &ln = *a.second;
      ln.cur = r;
      const std::vector<Req *> batch = ln.batch;  // r first (pick_admission)
      const double t_adm = ms_since_create(ctx);
      for (Req *q : batch) q->t_start = t_adm;
      ctx->served_launches += 1;
      ctx->served_requests += batch.size();
      lk.unlock();
      int code = PW_OK;
      std::string msg;
      try {
        if (batch.size() > 1) {
          std::vector<const pw_catalog *> gp, rp;
          std::vector<const pw_norm *> np;
          for (Req *q : batch) {
            gp.push_back(&q->gal);
            rp.push_back(&q->ran);
            np.push_back(&q->norm_in);
          }
          DevPlan *dp = launch_batch(ctx, ln, &r->cfg, (int)batch.size(), gp.data(), rp.data(), np.data());
          for (Req *q : batch) q->dp = dp;
        } else {
          r->dp = launch_estimate(ctx, ln, &r->cfg, &r->gal, &r->ran, &r->norm_in);
        }
      } catch (const Fail &f) {
        code = f.code;
        msg = f.msg;
      } catch (const std::exception &e) {
        code = PW_EINVAL;
        msg = e.what();
      }
      if (code != PW_OK) {
        bool pinned = false;
        for (Req *q : batch) pinned = pinned || q->pin;
        if (pinned) (void)hipStreamSynchronize(ln.stream);  // staging copies enqueued before the failure
        for (Req *q : batch) pin_release(ctx, q);
      }
      lk.lock();
      for (Req *q : batch) {
        ctx->reserved -= q->reserved;
        q->reserved = 0;
      }
      if (code != PW_OK) {
        for (Req *q : batch) {
          q->status = code;
          q->err = msg;
        }
        ln.batch.clear();
        ln.cur = nullptr;
        ctx->cv.notify_all();
      } else {
        any_running = true;
      }
    }
    if (ctx->stop && ctx->pending.empty() && !any_running) break;
    if (any_running || (ctx->main_busy && !ctx->pending.empty())) {
      ctx->cv.wait_for(lk, std::chrono::microseconds(100));
    } else {
      ctx->cv.wait(lk, [&] { return ctx->stop || !ctx->pending.empty(); });
    }
  }
}

void start_worker(pw_ctx *ctx) {
  if (ctx->worker_started) return;
  for (int i = 0; i < ctx->n_lanes; ++i) ctx->lanes.emplace_back(make_lane(i + 1, nullptr, ctx->trace != nullptr));
  ctx->worker = std::thread(worker_loop, ctx);
  ctx->worker_started = true;
}

int req_final(pw_ctx *ctx, uint64_t ticket, bool erase) {
  auto it = ctx->reqs.find(ticket);
  if (it == ctx->reqs.end()) return PW_EINVAL;
  int st = it->second->status;
  if (st != PW_EAGAIN) {
    set_err(ctx, it->second->err);
    if (erase) ctx->reqs.erase(it);
  }
  return st;
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
    ensure_sh(device);
    resolve_scratch(device);
    {
      int lds = 0;
      HIPCHECK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
      ctx->lds_per_block = (size_t)lds;
    }
    ctx->main.reset(make_lane(0, (hipStream_t)hip_stream, false));
    const char *tp = std::getenv("PW_TRACE");
    if (tp && *tp) {
      ctx->trace = std::fopen(tp, "a");
      if (!ctx->trace) fail(PW_EINVAL, "PW_TRACE: cannot open %s for appending", tp);
    }
  } catch (const Fail &f) {
    if (ctx->main) destroy_lane(ctx, ctx->main.release());
    delete ctx;
    return f.code;
  }
  *out = ctx;
  return PW_OK;
}

int pw_destroy(pw_ctx *ctx) {
  if (!ctx) return PW_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->worker_started) {
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      for (Req *r : ctx->pending) {
        r->status = PW_ECANCELED;
        r->err = "context destroyed";
        pin_release(ctx, r);
      }
      ctx->pending.clear();
      ctx->stop = true;
    }
    ctx->cv.notify_all();
    ctx->worker.join();
  }
  for (auto &lp : ctx->lanes) {
    destroy_lane(ctx, lp.get());
  }
  ctx->lanes.clear();
  if (ctx->main) destroy_lane(ctx, ctx->main.get());
  ctx->main.reset();
  for (auto &b : ctx->pin_free) (void)hipHostFree(b.first);
  ctx->pin_free.clear();
  if (ctx->trace) std::fclose(ctx->trace);
  delete ctx;
  return PW_OK;
}

int pw_estimate(pw_ctx *ctx, const pw_config *cfg, const pw_catalog *gal, const pw_catalog *ran,
                pw_norm *norm, double *out, double *bin_mean, int64_t *counts) {
  if (!ctx) return PW_EINVAL;
  try {
    run_estimate(ctx, cfg, gal, ran, norm, out, bin_mean, counts);
  } catch (const Fail &f) {
    set_err(ctx, f.msg);
    return f.code;
  } catch (const std::exception &e) {
    set_err(ctx, e.what());
    return PW_EINVAL;
  }
  set_err(ctx, std::string());
  return PW_OK;
}

int pw_estimate_batch(pw_ctx *ctx, const pw_config *cfg, int n, const pw_catalog *gal, const pw_catalog *ran,
                      pw_norm *norm, double *out, double *bin_mean, int64_t *counts) {
  if (!ctx) return PW_EINVAL;
  try {
    run_estimate_batch(ctx, cfg, n, gal, ran, norm, out, bin_mean, counts);
  } catch (const Fail &f) {
    set_err(ctx, f.msg);
    return f.code;
  } catch (const std::exception &e) {
    set_err(ctx, e.what());
    return PW_EINVAL;
  }
  set_err(ctx, std::string());
  return PW_OK;
}

int pw_serving_stats(pw_ctx *ctx, uint64_t *launches, uint64_t *requests) {
  if (!ctx) return PW_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (launches) *launches = ctx->served_launches;
  if (requests) *requests = ctx->served_requests;
  return PW_OK;
}

int pw_estimate_noalloc(pw_ctx *ctx, const pw_config *cfg, const pw_catalog *gal, const pw_catalog *ran,
                        pw_norm *norm, double *out, double *bin_mean, int64_t *counts) {
  if (!ctx) return PW_EINVAL;
  try {
    run_estimate_noalloc(ctx, cfg, gal, ran, norm, out, bin_mean, counts);
  } catch (const Fail &f) {
    set_err(ctx, f.msg);
    return f.code;
  } catch (const std::exception &e) {
    set_err(ctx, e.what());
    return PW_EINVAL;
  }
  set_err(ctx, std::string());
  return PW_OK;
}

int pw_estimate_orders(pw_ctx *ctx, const pw_config *cfg, const pw_catalog *gal, const pw_catalog *ran,
                       pw_norm *norm, double *out, double *bin_mean, int64_t *counts) {
  if (!ctx) return PW_EINVAL;
  try {
    if (!cfg || !out) fail(PW_EINVAL, "null configuration or output");
    validate_config(*cfg);
    // orders theta^(step * o): every alpha for the all-parity midpoint, even ones otherwise
    const int step = (cfg->los == PW_MIDPOINT && cfg->midpoint_parity == PW_PARITY_ALL) ? 1 : 2;
    const int nell = cfg->ell_max / 2 + 1, no = cfg->order / step + 1;
    const size_t slice = (size_t)nell * cfg->n_bins;
    if (one_pass_orders(*cfg)) {
      run_estimate(ctx, cfg, gal, ran, norm, out, bin_mean, counts, true);
    } else {
      // each series order's terms as the difference of successive truncations K = 0, step, ..
      std::vector<double> prev(slice, 0.0), cur(slice);
      pw_norm nm = norm ? *norm : pw_norm{0.0, 0.0, 0.0, 0};
      std::vector<double> res((size_t)no * slice), bm0;
      std::vector<int64_t> ct0;
      pw_norm n0 = nm;
      for (int o = 0; o < no; ++o) {
        pw_config c = *cfg;
        c.order = step * o;
        pw_norm n1 = nm;
        std::vector<double> bm(cfg->n_bins);
        std::vector<int64_t> ct(cfg->n_bins);
        run_estimate(ctx, &c, gal, ran, &n1, cur.data(), bm.data(), ct.data());
        for (size_t i = 0; i < slice; ++i) res[(size_t)o * slice + i] = cur[i] - prev[i];
        prev.swap(cur);
        if (o == 0) {
          n0 = n1;
          bm0.swap(bm);
          ct0.swap(ct);
        }
      }
      std::memcpy(out, res.data(), res.size() * sizeof(double));
      if (bin_mean) std::memcpy(bin_mean, bm0.data(), bm0.size() * sizeof(double));
      if (counts) std::memcpy(counts, ct0.data(), ct0.size() * sizeof(int64_t));
      if (norm && !norm->use_given) *norm = n0;
    }
  } catch (const Fail &f) {
    set_err(ctx, f.msg);
    return f.code;
  } catch (const std::exception &e) {
    set_err(ctx, e.what());
    return PW_EINVAL;
  }
  set_err(ctx, std::string());
  return PW_OK;
}

// Solve the n x n system A x = b in place by Gaussian elimination with partial pivoting
// (n <= 5: the multipoles of one r-bin).
static void solve_small(int n, double *A, double *b) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > std::fabs(A[piv * n + k])) piv = i;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[piv * n + j]);
      std::swap(b[k], b[piv]);
    }
    if (A[k * n + k] == 0.0) fail(PW_EINVAL, "window matrix is singular in a bin");
    for (int i = k + 1; i < n; ++i) {
      const double f = A[i * n + k] / A[k * n + k];
      for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
    for (int j = k + 1; j < n; ++j) s -= A[k * n + j] * b[j];
    b[k] = s / A[k * n + k];
  }
}

int pw_estimate_xi_normalized(pw_ctx *ctx, const pw_config *cfg, const pw_catalog *gal, const pw_catalog *ran,
                              pw_norm *norm, double *xi_rr, double *xi_edge, double *window, int *n_window,
                              double *bin_mean, int64_t *counts) {
  if (!ctx) return PW_EINVAL;
  try {
    if (!cfg || !xi_rr || !gal) fail(PW_EINVAL, "null configuration, catalog or output");
    if (cfg->stat != PW_XI) fail(PW_EINVAL, "pw_estimate_xi_normalized needs stat = PW_XI");
    validate_config(*cfg);
    const int nell = cfg->ell_max / 2 + 1, nb = cfg->n_bins;
    std::vector<double> data((size_t)nell * nb), bm(nb);
    std::vector<int64_t> ct(nb);
    pw_norm nm = norm ? *norm : pw_norm{0.0, 0.0, 0.0, 0};
    run_estimate(ctx, cfg, gal, ran, &nm, data.data(), bm.data(), ct.data());
    // the randoms alone, alpha_r w n_r, with the data's normalisation
    pw_config wc = *cfg;
    wc.ell_max = std::min(2 * cfg->ell_max, cfg->los == PW_BISECTOR ? 6 : 8);
    const int nL = wc.ell_max / 2 + 1;
    pw_catalog none = *gal;
    none.n = 0;
    pw_norm given = nm;
    given.use_given = 1;
    std::vector<double> win((size_t)nL * nb);
    run_estimate(ctx, &wc, &none, ran, &given, win.data(), nullptr, nullptr);
    std::vector<double> rr((size_t)nell * nb, 0.0), edge((size_t)nell * nb, 0.0), f((size_t)nL * nb, 0.0);
    for (int a = 0; a < nb; ++a) {
      const double R0 = win[a];
      if (R0 == 0.0) continue;
      for (int i = 0; i < nL; ++i) f[(size_t)i * nb + a] = win[(size_t)i * nb + a] / R0;
      double M[25], x[5];
      for (int i = 0; i < nell; ++i) {
        const int l = 2 * i;
        rr[(size_t)i * nb + a] = x[i] = data[(size_t)i * nb + a] / R0;
        for (int j = 0; j < nell; ++j) {
          const int lp = 2 * j;
          double t = 0.0;
          for (int k = 0; k < nL; ++k) {
            const double w = wigner3j(l, 2 * k, lp, 0, 0, 0);
            t += w * w * f[(size_t)k * nb + a];
          }
          M[i * nell + j] = (2 * l + 1) * t;
        }
      }
      solve_small(nell, M, x);
      for (int i = 0; i < nell; ++i) edge[(size_t)i * nb + a] = x[i];
    }
    std::memcpy(xi_rr, rr.data(), rr.size() * sizeof(double));
    if (xi_edge) std::memcpy(xi_edge, edge.data(), edge.size() * sizeof(double));
    if (window) std::memcpy(window, f.data(), f.size() * sizeof(double));
    if (n_window) *n_window = nL;
    if (bin_mean) std::memcpy(bin_mean, bm.data(), bm.size() * sizeof(double));
    if (counts) std::memcpy(counts, ct.data(), ct.size() * sizeof(int64_t));
    if (norm && !norm->use_given) *norm = nm;
  } catch (const Fail &e) {
    set_err(ctx, e.msg);
    return e.code;
  } catch (const std::exception &e) {
    set_err(ctx, e.what());
    return PW_EINVAL;
  }
  set_err(ctx, std::string());
  return PW_OK;
}

int pw_set_lanes(pw_ctx *ctx, int n_lanes) {
  if (!ctx) return PW_EINVAL;
  if (n_lanes < 1 || n_lanes > kMaxLanes) {
    set_err(ctx, "n_lanes must be in 1..8");
    return PW_EINVAL;
  }
  if (ctx->worker_started) {
    set_err(ctx, "pw_set_lanes: the serving loop has already started");
    return PW_EBUSY;
  }
  ctx->n_lanes = n_lanes;
  return PW_OK;
}

int pw_submit(pw_ctx *ctx, const pw_config *cfg, const pw_catalog *gal, const pw_catalog *ran, pw_norm *norm,
              double *out, double *bin_mean, int64_t *counts, uint64_t *ticket) {
  if (!ctx || !ticket) return PW_EINVAL;
  std::unique_ptr<Req> r(new Req());
  try {
    check_request(cfg, gal, ran, norm, out);
    r->cfg = *cfg;
    r->gal = *gal;
    r->ran = *ran;
    if (norm) r->norm_in = *norm;
    else std::memset(&r->norm_in, 0, sizeof(pw_norm));
    r->norm_out = norm;
    r->out = out;
    r->bin_mean = bin_mean;
    r->counts = counts;
    {
      std::shared_ptr<const HostPlan> hp = host_plan(ctx, *cfg);
      r->need_tables = table_bytes(*hp);
      r->need_work = work_layout(*hp).total;
    }
    size_t whole = r->need_tables + r->need_work + catalog_bytes(*cfg, *gal, *ran);
    if (whole > ctx->budget) fail(PW_ENOMEM, "request needs %zu bytes, budget is %zu", whole, ctx->budget);
    auto in_flight = [&]() {
      size_t n = ctx->pending.size();
      for (auto &lp : ctx->lanes) n += lp->cur ? 1 : 0;
      return n;
    };
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      if (in_flight() >= ctx->queue_limit)
        fail(PW_EBUSY, "the submission queue is full: %zu requests pending or running (limit %zu)", in_flight(),
             ctx->queue_limit);
    }
    // (one submitting thread: the count can only fall until the request is queued below)
    stage_pinned(ctx, r.get());
    std::lock_guard<std::mutex> lk(ctx->mu);
    start_worker(ctx);
    r->ticket = ctx->next_ticket++;
    r->t_submit = ms_since_create(ctx);
    *ticket = r->ticket;
    ctx->pending.push_back(r.get());
    ctx->reqs[r->ticket] = std::move(r);
  } catch (const Fail &f) {
    pin_release(ctx, r.get());
    set_err(ctx, f.msg);
    return f.code;
  } catch (const std::exception &e) {
    pin_release(ctx, r.get());
    set_err(ctx, e.what());
    return PW_EINVAL;
  }
  ctx->cv.notify_all();
  return PW_OK;
}

int pw_set_queue_limit(pw_ctx *ctx, int64_t max_in_flight) {
  if (!ctx) return PW_EINVAL;
  if (max_in_flight < 1 || max_in_flight > ((int64_t)1 << 30)) {
    set_err(ctx, "pw_set_queue_limit: max_in_flight must be in 1..2^30");
    return PW_EINVAL;
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->queue_limit = (size_t)max_in_flight;
  return PW_OK;
}

int pw_poll(pw_ctx *ctx, uint64_t ticket) {
  if (!ctx) return PW_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  return req_final(ctx, ticket, true);
}

int pw_wait(pw_ctx *ctx, uint64_t ticket) {
  if (!ctx) return PW_EINVAL;
  std::unique_lock<std::mutex> lk(ctx->mu);
  auto it = ctx->reqs.find(ticket);
  if (it == ctx->reqs.end()) return PW_EINVAL;
  Req *r = it->second.get();
  ctx->cv.wait(lk, [&] { return r->status != PW_EAGAIN; });
  return req_final(ctx, ticket, true);
}

int pw_cancel(pw_ctx *ctx, uint64_t ticket) {
  if (!ctx) return PW_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->reqs.find(ticket);
  if (it == ctx->reqs.end()) return PW_EINVAL;
  Req *r = it->second.get();
  auto pit = std::find(ctx->pending.begin(), ctx->pending.end(), r);
  if (pit == ctx->pending.end()) {
    if (r->status == PW_EAGAIN) {
      set_err(ctx, "pw_cancel: the request is already running");
      return PW_EBUSY;
    }
    return PW_OK;  // already finished; the ticket keeps its status
  }
  ctx->pending.erase(pit);
  r->status = PW_ECANCELED;
  r->err = "cancelled";
  pin_release(ctx, r);
  ctx->cv.notify_all();
  return PW_OK;
}

const char *pw_last_error(const pw_ctx *ctx) {
  if (!ctx) return "null context";
  thread_local std::string copy;  // stays valid until this thread's next pw_last_error
  std::lock_guard<std::mutex> lk(ctx->err_mu);
  copy = ctx->err;
  return copy.c_str();
}
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
    } else if (kind == 2 || kind == 4) {
      if (alpha < 0) return PW_EINVAL;
      for (int l = 0; l <= ell_max; l += 2)
        for (int J = 0; J <= l + alpha; ++J) {
          double F = kind == 2 ? legendre_F(alpha, l, J) : legendre_f(alpha, l, J);
          if (F == 0.0) continue;
          double v[7] = {(double)l, 0.0, (double)J, 0.0, 0.0, 0.0, F};
          r.insert(r.end(), v, v + 7);
        }
    } else if (kind == 3) {
      if (alpha < 0) return PW_EINVAL;
      for (const Term &t : midpoint_terms_all(ell_max, alpha)) {
        double v[7] = {(double)t.l, (double)t.nu, (double)t.J1, (double)t.mu1, (double)t.J2, (double)t.mu2, t.c};
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
  ctx->main->timing = on != 0;
  return PW_OK;
}

int pw_set_tuning(pw_ctx *ctx, int mode) {
  if (!ctx || mode < 0) return PW_EINVAL;
  ctx->tune_mode = mode;
  return PW_OK;
}

int pw_tune_entry(int index, char *key, size_t key_len, int *choice, double *ms_best, double *ms_default) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_cache();
  if (index < 0 || (size_t)index >= g_tune.size()) return PW_EINVAL;
  const TuneEntry &e = g_tune[(size_t)index];
  if (key && key_len > 0) {
    const size_t n = std::min(key_len - 1, e.key.size());
    std::memcpy(key, e.key.data(), n);
    key[n] = 0;
  }
  if (choice) *choice = e.choice;
  if (ms_best) *ms_best = e.ms_best;
  if (ms_default) *ms_default = e.ms_default;
  return PW_OK;
}

int pw_stage_info(pw_ctx *ctx, int stage, const char **name, double *ms, double *bytes) {
  if (!ctx || stage < 0 || stage >= ctx->main->n_stages) return PW_EINVAL;
  if (name) *name = ctx->main->st_name[stage];
  if (ms) *ms = ctx->main->st_ms[stage];
  if (bytes) *bytes = ctx->main->st_bytes[stage];
  return PW_OK;
}

int pw_inspect(pw_ctx *ctx, int what, void *dst, size_t dst_bytes, size_t *needed) {
  if (!ctx || !needed) return PW_EINVAL;
  try {
    MainBusy busy(ctx);  // keeps the serving admission from evicting lane 0's last plan
    DevPlan *dp = ctx->main->last;
    if (!dp) fail(PW_EINVAL, "pw_inspect: no estimate has run on this context");
    const HostPlan &h = *dp->host;
    size_t rsz = h.prec == PW_FP32 ? 4 : 8;
    const void *src = nullptr;
    size_t bytes = 0;
    if (what == 0) { src = dp->mesh; bytes = (size_t)h.N * h.N * h.N * rsz; }
    else if (what == 1) { src = dp->bufA; bytes = (size_t)h.nfields * h.fwd.nmodes * 2 * rsz; }  // compact copy
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
      HIPCHECK(hipStreamSynchronize(ctx->main->stream));
      if (what == 1) {
        // fields are stored with the padded stride mstride: copy them out compactly
        const size_t w = (size_t)h.fwd.nmodes * 2 * rsz;
        HIPCHECK(hipMemcpy2D(dst, w, src, (size_t)h.fwd.mstride * 2 * rsz, w, (size_t)h.nfields,
                             hipMemcpyDeviceToHost));
      } else {
        HIPCHECK(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
      }
      if (what == 0) {
        // rows outside the occupied-row mask hold no value: the gather leaves them unwritten
        std::vector<int> mask((size_t)h.N * h.N);
        HIPCHECK(hipMemcpy(mask.data(), dp->rowmask, mask.size() * sizeof(int), hipMemcpyDeviceToHost));
        for (size_t r = 0; r < mask.size(); ++r)
          if (!mask[r]) std::memset((char *)dst + r * h.N * rsz, 0, (size_t)h.N * rsz);
      }
    }
  } catch (const Fail &f) {
    set_err(ctx, f.msg);
    return f.code;
  }
  return PW_OK;
}

}  // extern "C"

namespace pw {
[[noreturn]] void plan_fail(int code, const char *msg) { fail(code, "%s", msg); }
}  // namespace pw
