// Planner: validates a configuration and derives everything the kernels need — the real
// fields of each series order, the pair jobs of the fused x pass, the pruned index sets of the
// y and z passes, the per-mode coordinates, the FP64 bin decisions and the coupling tables.
//
// Four paths share the forward passes:
//   bisector P_l   forward transforms pruned to the k-sphere of the bins, contraction.
//   midpoint P_l   full forward transforms; conj(D) Q / W^2 fused into an inverse z pass;
//                  alpha = 0 products stay in k-space; alpha > 0 ones go back to real space,
//                  are re-weighted into A_{l nu}, and A is transformed forward (pruned).
//   midpoint xi_l  full forward transforms; product + inverse transforms output-pruned to the
//                  separations of the r-bins; weighting and binning fused into the x pass.
//   bisector xi_l  full forward transforms; per-mode targets T_{l nu}; inverse transforms
//                  output-pruned as above; y_l^nu(D^) weighting and binning fused.
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
                   double, int, int, int>
    PlanKey;

PlanKey make_key(const pw_config &c);
void validate_config(const pw_config &c);

enum Path { PATH_BIS_PK = 0, PATH_MID_PK = 1, PATH_MID_XI = 2, PATH_BIS_XI = 3 };

// Retained modes of a forward transform: |n|^2 <= K2 (all modes when `full`).  Every row and
// field start is padded to 128 bytes (Q = 16 FP32 / 8 FP64 complex values) so that the column
// passes move whole cache lines: x-pass rows have stride rs; each ky row of a y-pass plane
// starts at a multiple of Q (padding pencils have kzcnt = 0, or for full retention are
// ordinary all-zero pencils q = ky * rs + kx, kx >= nkx); z-pass fields have stride mstride.
struct Prune {
  bool full = false;
  int nkx = 0;
  int rs = 0;                       // padded row stride of the x-pass output (complex values)
  std::vector<int> ycnt;
  std::vector<int64_t> yoff;
  int64_t npen = 0;                 // pencils per y-pass plane, padding included
  int64_t npen_real = 0;            // retained pencils (sum of ycnt)
  std::vector<PencilInfo> pinfo;    // [npen]
  std::vector<int64_t> moff;        // [npen] (full sets: pencil q holds modes [moff[q], +N))
  // z-pass output.  Full sets: pencil-major, kz fastest.  Sphere-pruned sets: groups of `grp`
  // adjacent pencils, each stored as [kz slot][pencil of the group]: slot j of group g holds
  // kz = j for j <= h_g and kz = N - (gsize[g] - j) above (all N kz when gsize[g] == N), with
  // h_g = (gsize[g] - 1) / 2 the largest half-count of the group's pencils.  Slots outside a
  // pencil's own sphere (and padding pencils) carry the coordinate kModeNone.
  int grp = 0;
  std::vector<int64_t> goff;        // [ngroups + 1] first slot of each group
  std::vector<int> gsize;           // [ngroups] kz slots of each group
  int64_t nmodes = 0;               // slots per field (full: N per pencil, padding pencils included)
  int64_t nretained = 0;            // retained modes per field (slots with a coordinate)
  int64_t mstride = 0;              // field stride of the z-pass output
  std::vector<uint32_t> modecoord;  // kx | ky << 11 | kz << 22 per slot (pruned sets only)
};

// coordinate of a slot that holds no retained mode: decodes to |n|^2 > 2047^2, beyond any bin
constexpr uint32_t kModeNone = 0xFFFFFFFFu;

struct HostPlan {
  int path;
  int stat, los, prec, N, ell_max, order, n_bins, nell;
  double L, H, kf;
  double unit;               // length unit of the radial weights (about twice the box-centre distance)
  int check_extent;
  int all_parity;            // midpoint: 1 = all-parity series (every alpha), 0 = parity-even
  std::vector<int> ells;
  // forward fields and the pair jobs of the x pass
  int nfields;
  std::vector<FieldJob> jobs;
  int n0;                    // midpoint: number of alpha = 0 fields (stored first)
  Prune fwd;                 // forward retention
  Prune sph;                 // midpoint P: the k-sphere of the bins (A fields, contraction)
  int64_t K2;                // largest |n|^2 in a k-bin (P) ; largest |s|^2 in an r-bin (xi)
  std::vector<int> bin_of_s2;  // FP64 bin decision per integer |n|^2 (k for P, r for xi)
  std::vector<double> winv;    // 1 / sinc(pi s / N)^p per axis index (empty: no compensation)
  // bisector P: coupling terms grouped by target (table-driven contraction)
  std::vector<int> t_start, t_sh, t_ell, t_p1, t_p2;
  std::vector<double> t_coef;
  // inverse transforms (midpoint, xi)
  int n_inv;                 // fields of the inverse stack
  int n_inplace;             // fields kept in k-space by the inverse z pass (midpoint P)
  int nz, ny;                // retained z planes / y rows of the inverse outputs
  std::vector<int> zrank, zidx, yidx;   // index -> rank (-1: dropped) ; rank -> index
  std::vector<int> iycnt;    // per y index: nkx if retained else 0
  std::vector<int64_t> iyoff;  // per y index: rank * rs
  std::vector<FieldJob> ijobs;   // pair jobs of the inverse x pass (indices into the stack)
  std::vector<double> icoef;     // xi: [ijob][2][nell] per-field multipole coefficients
  int n_targets;             // bisector xi: T_{l nu} spectra
  // midpoint P: A_{l nu} fields (l >= 2) and their forward pair jobs
  int n_a;
  std::vector<FieldJob> ajobs;
  // bisector P: series orders of the one-pass per-order contraction (0: not available) and
  // the multipole of each of its result rows (beta * nell + l/2; -1 beyond zeroth order,
  // where no shot noise is subtracted)
  int n_orders_native = 0;
  std::vector<int> ells_orders;
  // bisector P, memory-lean: the sorted jobs in groups of about kLeanFields fields; group g has
  // jobs [lean_jstart[g], lean_jstart[g+1]) of lean_jobs (field slots local to the group) and
  // fields [lean_fstart[g], lean_fstart[g+1]) of lean_fmap (local slot -> field index)
  int lean = 0;
  int lean_maxf = 0;
  std::vector<FieldJob> lean_jobs;
  std::vector<int> lean_jstart, lean_fstart, lean_fmap;
};

constexpr int kLeanFields = 8;

// Whether pw_estimate_orders has a one-pass path for cfg (bisector P_l with a generated
// coupling whose per-order accumulators fit the contraction kernel's LDS).
bool one_pass_orders(const pw_config &c);

HostPlan build_host_plan(const pw_config &c);
size_t footprint_bytes(const pw_config &c, int64_t n_gal, int64_t n_ran);
size_t plan_bytes(const pw_config &c);       // device bytes of one plan (tables + work buffers)

// The work buffers of one estimate (the mesh, the spectrum buffers, the paint tiles) as byte
// offsets into one workspace.  A lane runs one estimate at a time, so all plans cached on a
// lane share one workspace of the largest size any of them needs.
struct WorkLayout {
  size_t mesh = 0, bufA = 0, bufB = 0, bufC = 0, tiles = 0;  // offsets (bufC: memory-lean only)
  size_t total = 0;
};
WorkLayout work_layout(const HostPlan &h);
// device bytes of a plan's own tables (everything but the workspace), an upper bound
size_t table_bytes(const HostPlan &h);
// device bytes of an estimate's particle buffers: the tile-sorted records (mesh precision) and
// the staging of host catalogs (their own dtype) with the randoms' nbar; the count form assumes
// host catalogs of the mesh precision with nbar (pw_footprint)
size_t catalog_bytes(const pw_config &c, int64_t n_gal, int64_t n_ran);
size_t catalog_bytes(const pw_config &c, const pw_catalog &gal, const pw_catalog &ran);
// tile-sorted particle records in the mesh precision, padded to 256 bytes (the sort's chunk
// histograms follow them in the same buffer)
size_t records_bytes(int prec, int64_t n_gal, int64_t n_ran);
// bytes of each of the two spectrum buffers (memory-lean: of the k-sphere buffer)
size_t spectrum_buffer_bytes(const HostPlan &h);
// memory-lean bisector: x-pass and y-pass work buffers of one field group
size_t lean_x_bytes(const HostPlan &h);
size_t lean_y_bytes(const HostPlan &h);

struct DevPrune {
  int *ycnt = nullptr;
  int64_t *yoff = nullptr;
  PencilInfo *pinfo = nullptr;
  int64_t *moff = nullptr;
  uint32_t *modecoord = nullptr;
  int64_t *goff = nullptr;   // sphere-pruned sets only
  int *gsize = nullptr;
};

struct DevPlan {
  std::shared_ptr<const HostPlan> host;  // shared with the context's host-plan cache
  WorkLayout work;
  std::vector<std::pair<void *, size_t>> allocs;
  void *tw = nullptr;
  FieldJob *jobs = nullptr, *ijobs = nullptr, *ajobs = nullptr, *lean_jobs = nullptr;
  int *lean_fmap = nullptr;
  void *bufC = nullptr;  // memory-lean: y-pass output of one field group
  DevPrune fwd, sph;
  int *bin_of_s2 = nullptr;
  int *ells = nullptr, *ells_orders = nullptr;
  void *winv = nullptr;
  int *t_start = nullptr, *t_sh = nullptr, *t_ell = nullptr, *t_p1 = nullptr, *t_p2 = nullptr;
  void *t_coef = nullptr;
  int *zrank = nullptr, *zidx = nullptr, *yidx = nullptr, *iycnt = nullptr;
  int64_t *iyoff = nullptr;
  void *icoef = nullptr;
  void *mesh = nullptr, *bufA = nullptr, *bufB = nullptr;
  double *acc = nullptr, *out = nullptr, *part_g = nullptr, *part_r = nullptr;
  DevNorm *norm = nullptr;
  int *tile_counts = nullptr, *tile_offsets = nullptr, *tile_slot = nullptr;
  void *tile_blocks = nullptr;
  int ntiles = 0;
  int *rowmask = nullptr, *rowlist = nullptr, *planemask = nullptr, *zlist = nullptr;  // survey occupancy
  int *occ_blockcnt = nullptr;
};

}  // namespace pw
