// Planner: validates a configuration and derives everything the kernels need — the real
// fields of each series order, the pair jobs of the fused x pass, the pruned index sets of the
// y and z passes, the per-mode coordinates, the FP64 bin decisions and the coupling tables.
#pragma once
#include <cstdint>
#include <memory>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/pw.h"
#include "kernels.h"

namespace pw {

[[noreturn]] void plan_fail(int code, const char *msg);

typedef std::tuple<int, int, int, int, int, double, double, double, double, int, int, int, double,
                   double, int>
    PlanKey;

PlanKey make_key(const pw_config &c);
void validate_config(const pw_config &c);

struct HostPlan {
  int stat, los, prec, N, ell_max, order, n_bins, nell;
  double L, H, kf;
  int check_extent;
  std::vector<int> ells;
  // fields / jobs
  int nfields;
  std::vector<FieldJob> jobs;
  // pruned spectra
  int64_t K2;            // largest retained |n|^2
  int nkx;
  std::vector<int> ycnt;
  std::vector<int64_t> yoff;
  int64_t npen;
  std::vector<PencilInfo> pinfo;
  std::vector<int64_t> moff;
  int64_t nmodes;
  std::vector<uint32_t> modecoord;
  // FP64 bin decision per integer |n|^2
  std::vector<int> bin_of_s2;
  // 1 / sinc(pi s / N)^p per axis index (empty when compensation is off)
  std::vector<double> winv;
  // coupling terms grouped by target
  std::vector<int> t_start, t_sh, t_ell, t_p1, t_p2;
  std::vector<double> t_coef;
};

HostPlan build_host_plan(const pw_config &c);
size_t footprint_bytes(const pw_config &c, int64_t n_gal, int64_t n_ran);

struct DevPlan {
  std::unique_ptr<HostPlan> host;
  std::vector<std::pair<void *, size_t>> allocs;
  void *tw = nullptr;
  FieldJob *jobs = nullptr;
  int *ycnt = nullptr;
  int64_t *yoff = nullptr;
  PencilInfo *pinfo = nullptr;
  int64_t *moff = nullptr;
  uint32_t *modecoord = nullptr;
  int *bin_of_s2 = nullptr;
  int *ells = nullptr;
  void *winv = nullptr;
  int *t_start = nullptr, *t_sh = nullptr, *t_ell = nullptr, *t_p1 = nullptr, *t_p2 = nullptr;
  void *t_coef = nullptr;
  void *mesh = nullptr, *bufA = nullptr, *bufB = nullptr;
  double *acc = nullptr, *out = nullptr, *part_g = nullptr, *part_r = nullptr;
  DevNorm *norm = nullptr;
  int *tile_counts = nullptr, *tile_offsets = nullptr, *tile_cursor = nullptr, *tile_slot = nullptr;
  void *tile_blocks = nullptr;
  int ntiles = 0;
};

}  // namespace pw
