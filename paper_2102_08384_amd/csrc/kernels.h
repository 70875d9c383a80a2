// Launch wrappers of the HIP kernels (host-callable).  All launches are asynchronous on the
// given stream; shapes are validated by the caller (the planner) before any launch.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace pw {

struct ShConst;

// Per-catalog FP64 partial sums written by the scalars kernel (one row per block):
// [0] sum w, [1] sum w^2, [2] sum w^2 nbar, [3..5] min x,y,z, [6..8] max x,y,z, [9] count,
// [10] sum |w|
constexpr int kScalarCols = 11;
constexpr int kScalarBlocks = 4096;  // at most this many partial rows (sort chunks) per catalog

// Device-resident normalisation, filled by the finalize kernel.
struct DevNorm {
  double alpha_r, I, S;
  double sum_wg, sum_wr;
  double fix_scale;  // 2^e: painting accumulates round(contribution * fix_scale) in int64
  int flags;         // bit 0: particle outside the box, bit 1: extent > L/2 (midpoint P)
  int nrows_occ;     // x-rows (z, y) of the mesh with a non-zero node
  int nplanes_occ;   // z-planes of the mesh with a non-zero node
  int pad;
};

// A pair job of the fused weighting + x-FFT pass: two real fields generated together as the
// real and imaginary parts of one complex transform.
// kind 0: fields (J, +m) and (J, -m), m > 0, of weight (2r)^-alpha;  pa / pb their indices.
// kind 1: fields (Ja, 0) of weight (2r)^-alpha and (Jb, 0) of weight (2r)^-alpha_b
//         (Jb < 0: single field, pb < 0).
// kind 2: no weighting: real input fields Ja and Jb (Jb < 0: none) of a field stack.
// Jobs must be sorted by m, then by J (the x pass carries its recurrences across jobs).
// The inverse x pass reads the same records with |D|^alpha y(D^) in place of (2r)^-alpha y(x^).
struct FieldJob {
  int alpha, kind, Ja, m, Jb, pa, pb, alpha_b;
};

struct PencilInfo {   // a retained (kx, ky) pencil of the z pass
  int kx, ky, kzcnt, pad;
};

// Catalogs of one batched launch of the bisector P_l passes (same configuration, so the
// plan's tables are shared): each catalog's own buffers.  Kernels take the table by value and
// work on catalog blockIdx.z; n = 0 (the default) means no batch, and the kernels use their
// pointer arguments.
constexpr int kMaxBatch = 8;
struct BatchSlot {
  const void *mesh;
  void *A, *B;  // spectrum buffers: x- and z-pass output (A), y-pass output (B)
  const int *rowlist, *rowmask, *zlist, *planemask;
  const DevNorm *norm;
  double *acc;
};
struct Batch {
  int n;
  BatchSlot s[kMaxBatch];
};

void upload_sh_const(const ShConst &c);
void upload_sh_const_inverse(const ShConst &c);
void upload_sh_const_generated(const ShConst &c);

// alpha_r, I, S, the range / extent flags and the painting scale from the partial rows of the
// two catalogs (nblk_g, nblk_r rows of kScalarCols written by launch_sort_count).
void launch_finalize_norm(hipStream_t s, const double *pg, int nblk_g, const double *pr, int nblk_r,
                          DevNorm *norm, const double *b0, double L, int check_extent, int use_given,
                          double ga, double gI, double gS);
// Zero n_elems values: prec 0 float, 1 double, 2 int.
void launch_fill(hipStream_t s, void *p, size_t n_elems, int prec);

// Tile-binned painting: particles are counting-sorted by the tile of their anchor node
// (nearest for TSC, lower for CIC); each occupied tile (+ one-node halo) is accumulated in
// LDS and stored as a block; a gather pass sums the blocks covering every node.  Tiles are
// TS^3 nodes, TS = min(16, N).  Records are (l + d) per axis (l the node index inside the
// tile, d the offset in cells) and the signed weight, in the mesh precision.  The sort
// kernels keep one LDS counter per tile (ntiles * 4 bytes per workgroup).
constexpr int kTile = 16;
inline int tile_size(int N) { return N < kTile ? N : kTile; }
// Launch shape of a pass, as picked by the autotuner (0 everywhere: the defaults).  Every shape
// computes the same values; only the speed differs.
struct ColTune {
  int fpb = 0;      // column passes: fields per workgroup (0: about 4096 workgroups per launch)
  int cols = 0;     // y pass: adjacent columns (0: one 128-byte row segment; 8: half of one, FP32)
  int rows = 0;     // x pass, FP32 at N = 512: rows (wavefronts) per workgroup (0: 4; 1, 2 or 8)
  int threads = 0;  // tile paint: threads per workgroup (0: 256; 128 or 512)
  int gx = 0;       // gather: tiles per workgroup along x (0: two in FP32 where N allows; 1: one)
  int blocks = 0;   // bisector contraction: workgroups per catalog (0: one per 256 modes, at most
                    // 4096 in all)
};

// The sort reads the particles twice.  Both catalogs are cut into chunks of `chunk` particles,
// one workgroup each (galaxy chunks first), a layout fixed by the mesh and the catalog sizes.
constexpr int kSortNominalCUs = 256;
constexpr size_t kSortLdsExtra = 16 * 11 * sizeof(double);  // k_sort_count: per-wave reduction rows
struct SortLayout {
  int64_t chunk = 0;
  int nblk_g = 0, nblk_r = 0, ntiles = 0;
  size_t hist_bytes = 0;  // chunk_hist: one row of ntiles counts per chunk
};
SortLayout sort_layout(int N, int64_t n_gal, int64_t n_ran);
// Pass 1: FP64 scalar partial rows (part_g / part_r), each chunk's tile histogram into
// chunk_hist and the tile totals added to counts (zeroed by the caller).  rnbar: the randoms'
// nbar (or NULL).
void launch_sort_count(hipStream_t s, const SortLayout &L, const void *gx, int gdtype, const void *rx, int rdtype,
                       const void *rnbar, int64_t ng, int64_t nr, int N, const double *b0, double H, int assign,
                       int *chunk_hist, int *counts, double *part_g, double *part_r);
void launch_tile_scan(hipStream_t s, const int *counts, int ntiles, int *offsets, int *slot);
// Pass 2: tile-sorted records in the mesh precision (prec), randoms weighted by -alpha_r.
// chunk_hist's counts become run bases in place (offsets: the tile offsets of the scan).
void launch_sort_scatter(hipStream_t s, const SortLayout &L, const void *gx, int gdtype, const void *rx,
                         int rdtype, int64_t ng, int64_t nr, int prec, int N, const double *b0, double H,
                         int assign, const DevNorm *norm, int *chunk_hist, const int *offsets, void *records);
// blocks: scratch of ntiles * (TS+2)^3 values of the mesh precision, one block per occupied tile
// (slot: [ntiles + 1] from the scan).
void launch_tile_paint(hipStream_t s, int prec, int N, int assign, const int *offsets, const int *slot,
                       const void *records, const DevNorm *norm, void *blocks, ColTune tune = ColTune());
// Every mesh node = the sum of the blocks covering it.  rowmask (N*N ints, zeroed by the
// caller; may be null) receives 1 for every x-row (z, y) holding a non-zero node.
void launch_tile_gather(hipStream_t s, int prec, int N, const int *slot, const void *blocks, void *mesh,
                        int *rowmask, ColTune tune = ColTune());
// Survey occupancy: rowlist = the non-empty rows in increasing order, planemask[z] = 1 for
// z-planes with a non-empty row, zlist = those planes in increasing order; counts into
// norm->nrows_occ / nplanes_occ.  Every field of the forward transforms is the mesh times a
// weight, so it vanishes exactly on empty rows.
// blockcnt: occupancy_blocks(N) ints of scratch.
int occupancy_blocks(int N);
void launch_occupancy(hipStream_t s, int N, const int *rowmask, int *rowlist, int *planemask, int *zlist,
                      int *blockcnt, DevNorm *norm);

// Row strides: every row of a half spectrum (kx = 0 .. nkx-1) starts at a multiple of `rs`
// complex values, rs >= nkx rounded up to 128 bytes, so that column-pencil passes read whole
// cache lines.
inline int row_stride(int nkx, int prec) {
  const int q = prec == 0 ? 16 : 8;
  return (nkx + q - 1) / q * q;
}

// Fused weighting + r2c along x: out[p][z][y * rs + kx], kx < nkx.  Radial weights are taken in the
// length unit `unit`: (unit / 2r)^alpha (the inverse passes use (|D| / unit)^alpha, so every
// product (2r)^-alpha |D|^alpha is unchanged while fields of every alpha stay O(1)).
// rowlist (may be null: every row) restricts the pass to the non-empty rows; the output rows of
// empty ones are not written (the y pass reads them as zeros).
// kind FX_PLAIN: every job is kind 2 (pairs of real input fields, no weighting); else kinds 0 and 1.
// x-pass inputs: FX_HARMONIC generates y_J^mu(x^) F (bisector), FX_RADIAL also (u/2r)^alpha
// (midpoint), FX_PLAIN transforms real input fields of a stack (midpoint A fields)
enum { FX_HARMONIC = 0, FX_RADIAL = 1, FX_PLAIN = 2 };
void launch_fx(hipStream_t s, int prec, int N, int kind, const void *mesh, void *out, const FieldJob *jobs,
               int njobs, int nkx, int rs, const double *b0, double H, double unit, const void *tw,
               const int *rowlist, const DevNorm *norm, const Batch *batch = nullptr,
               ColTune tune = ColTune());
// c2c along y (forward, or inverse when inv), on nplanes planes per field:
// in[p][plane][y * rs + kx] -> out[p][plane][yoff[y'] + kx] for kx < ycnt[y'] (y' the output
// index, npen values per output plane).
// rowmask / zlist (forward pass only; may be null): only the planes zlist[0 .. norm->nplanes_occ)
// are transformed (the others are not written; the z pass reads them as zeros) and empty
// input rows are read as zeros.
void launch_fy(hipStream_t s, int prec, int N, int inv, const void *in, void *out, int nfields,
               int nplanes, int nkx, int rs, const int *ycnt, const int64_t *yoff, int64_t npen,
               const void *tw, const int *rowmask, const int *zlist, const DevNorm *norm,
               ColTune tune = ColTune(), const Batch *batch = nullptr);
// c2c along z.  Full sets (goff null): out[p][moff[q] + kz], all N kz of every pencil.
// Sphere-pruned sets: out[p][goff[g] + slot * C + c] for pencil q = g C + c, slot as in Prune
// (C = 128 bytes / complex size, the pencils per workgroup).  Field stride mstride.
// planemask (may be null): empty z-planes of the input are read as zeros.
// fmap (may be null): the output field index of each input field p (sphere-pruned sets only)
void launch_fz(hipStream_t s, int prec, int N, const void *in, void *out, int nfields,
               int64_t npen, const PencilInfo *pinfo, const int64_t *moff, const int64_t *goff,
               const int *gsize, int64_t mstride, const void *tw, const int *planemask,
               const int *fmap = nullptr, ColTune tune = ColTune(), const Batch *batch = nullptr);

// Bisector contraction + FP64 k-binning.
struct TermTable {
  const int *tstart;     // [ntargets + 1] term ranges per target
  const int *tsh;        // [ntargets] real-SH index l*l+l+nu of each target
  const int *tell;       // [ntargets] slot of l in the output
  const int *p1, *p2;    // field indices
  const void *coef;      // float or double
  int ntargets;
};
// Threads per block of the table-driven bisector contraction: every field value of a block's
// modes is staged in LDS (nfields * threads complex values) beside the FP64 bins, within 64 KiB;
// 0 when not even the smallest block fits.
inline int contract_bis_threads(int prec, int nfields, int nell, int nbins) {
  const size_t csz = prec == 0 ? 8 : 16, bins = (size_t)(nell + 2) * nbins * 8;
  for (int nth = prec == 0 ? 128 : 64; nth >= 16; nth /= 2)
    if ((size_t)nfields * nth * csz + bins <= 65536) return nth;
  return 0;
}
void launch_contract_bis(hipStream_t s, int prec, int lmax, int bmax, const void *spec, int nfields,
                         int64_t nmodes, int64_t mstride, const uint32_t *modecoord, int N, const int *bin_of_s2,
                         int64_t n_s2, int nbins, int nell, TermTable tab, double kf,
                         const void *winv, double *acc, ColTune tune = ColTune());
void launch_finalize_pk(hipStream_t s, const double *acc, int nell, int nbins, const int *ells,
                        const DevNorm *norm, double *out);

// Register-resident bisector contraction when its coupling is generated; false otherwise.
// orders != 0: one accumulator row per (beta, l), rows beta * nell + l/2, then the mode count
// and the |k| sum ((bmax + 1) * nell + 2 rows of nbins).
bool launch_contract_bis_generated(hipStream_t s, int prec, int lmax, int bmax, const void *spec, int64_t nmodes,
                                   int64_t mstride, const uint32_t *modecoord, int N, const int *bin_of_s2, int64_t n_s2,
                                   int nbins, double kf, const void *winv, double *acc, int orders, const Batch *batch = nullptr,
                                   ColTune tune = ColTune());
// Which (ell_max, beta_max) / (ell_max, order) have build-time generated couplings.
bool bis_contract_generated(int lmax, int bmax);
bool mid_reweight_generated(int lmax, int order, int all_parity);
// Number of g fields the generated re-weighting reads (-1: not generated).
int mid_reweight_nfields(int lmax, int order, int all_parity);

// ---- inverse path (inverse.hip) ----
// Inverse z pass over full pencil-major spectra in[p][q * N + kz] (q = ky * nkx + kx):
//   D != null: Z = conj(d_scale * D) * in / W(k)^2 (D is read before anything is written);
//   fields p < n_inplace get Z written back in place and are not transformed;
//   real_in: the input holds real values (imaginary part zero).
// Other fields: inverse FFT along z, out[p - n_inplace][zrank[z]][ky * rs + kx] for retained z
// (N * rs values per output plane).
void launch_iz(hipStream_t s, int prec, int N, void *in, void *out, int nfields, int n_inplace,
               int real_in, int64_t npen, int nkx, int rs, const void *D, double d_scale,
               const void *winv, const int *zrank, int nz, const void *tw);
// Midpoint g fields: forward z pass of the y-pass output in[p][z][q] (full sets), the product
// conj(D) Q / W^2 with D = d_scale * (field 0's transform), then either the product stays
// pencil-major in prod[p][q * N + kz] (p < n_inplace) or the inverse z pass writes the
// retained planes out[p - n_inplace][zrank[z]][q].  planemask: z planes with data (others zero).
void launch_fziz(hipStream_t s, int prec, int N, const void *in, void *prod, void *out, int nfields, int n_inplace,
                 int64_t npen, int rs, double d_scale, const void *winv, const int *zrank, int nz, const void *tw,
                 const int *planemask, ColTune tune = ColTune());
// Inverse x pass (complex-to-real) of pair jobs on the rows (zr, yr) of in[p][zr][yr * rs + kx],
// kx <= N/2, scaled by `scale`.
//   mode 0: out[p][z][y][x] real fields (nz = ny = N).
//   mode 1: X_l += coef[j][side][l] (|D| / unit)^alpha y_J^mu(D^) h, then FP64 r-binning of
//           X_l into acc[l][b], acc[nell][b] (count), acc[nell + 1][b] (sum |D|).
void launch_ix(hipStream_t s, int prec, int N, int mode, const void *in, void *out, int rs,
               const FieldJob *jobs, int njobs, const void *coef, int nell, int nz, int ny,
               const int *zidx, const int *yidx, double H, double unit, double scale, const int *bin_of_s2,
               int64_t n_s2, int nbins, double *acc, const void *tw);
// Midpoint real-space re-weighting: A_{l nu}(D) from the alpha > 0 g fields (generated),
// with |D| in the length unit of the forward weights (Hu = H / unit).
void launch_reweight(hipStream_t s, int prec, int N, int lmax, int order, int all_parity, const void *g, void *A,
                     double Hu);
// Bisector xi targets: T[t][i] = sum S Re(conj(R_p1) R_p2) / W(k)^2 over the full
// pencil-major spectra (i = q * N + kz, q = ky * rs + kx), written as real values (generated).
// Field p of spec starts at p * mstride; target t of T at t * nmodes.
void launch_targets(hipStream_t s, int prec, int N, int lmax, int bmax, const void *spec, int64_t nmodes,
                    int64_t mstride, int rs, const void *winv, void *T);
// Midpoint P contraction: E_l = sum_nu y_l^nu(k^) Re[G_{l nu}(k) + A_{l nu}(k)] on the k-sphere
// modes; G: full pencil-major products (alpha = 0 fields, index even_index(l, nu)); A: pruned
// spectra of the A fields (l >= 2, index even_index(l, nu) - 1; null when absent).
void launch_contract_mid(hipStream_t s, int prec, int lmax, const void *G, int rs_full, const void *A,
                         int64_t nmodes, int64_t mstride, const uint32_t *modecoord, int N, const int *bin_of_s2,
                         int64_t n_s2, int nbins, double kf, double *acc);
void launch_finalize_xi(hipStream_t s, const double *acc, int nell, int nbins, double cell_volume,
                        const DevNorm *norm, double *out);

}  // namespace pw
