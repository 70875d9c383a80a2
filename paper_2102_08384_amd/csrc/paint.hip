// Catalog reductions, normalisation and mass assignment (gfx950).
//
//   sort_count    first pass over the particles (galaxies and randoms in one launch): FP64
//                 reductions per workgroup (sum w, sum w^2, sum w^2 nbar, sum |w|, bounding
//                 box, count) and the workgroup's LDS histogram of anchor tiles, stored per
//                 chunk and added to the tile totals
//   norm          alpha_r = sum w_g / sum w_r, I = alpha_r sum_r w_r^2 nbar_r,
//                 S = sum_g w_g^2 + alpha_r^2 sum_r w_r^2 (Section 2.1), range / extent flags
//   tile_scan     exclusive scan of the tile counts, compact slots of the occupied tiles
//   chunk_bases   each chunk's run base in every tile (the tile offset plus the earlier
//                 chunks' counts), in place of the stored histograms
//   sort_scatter  second (last) pass over the particles: each chunk writes tile-sorted records
//                 (node offset inside the tile, signed weight) into its runs
//   tile_paint    CIC / TSC taps of one tile's particles accumulated in LDS (tile + halo),
//                 written as a block to the tile's scratch slot
//   tile_gather   every mesh node = sum of the (at most eight) blocks that cover it
// No global atomics touch the mesh: each node is written once with a plain store.
#include "kernels.h"

namespace pw {


constexpr int kNormThreads = 256;
__device__ __forceinline__ double combine(int c, double a, double b) {
  return (c >= 3 && c < 6) ? fmin(a, b) : (c >= 6 && c < 9) ? fmax(a, b) : a + b;
}

__global__ void __launch_bounds__(kNormThreads)
k_finalize_norm(const double *pg, int nblk_g, const double *pr, int nblk_r, DevNorm *norm, double b0x, double b0y,
                double b0z, double L, int check_extent, int use_given, double ga, double gI, double gS) {
  // fixed-order (deterministic) reduction of the per-workgroup partial rows: thread t folds rows
  // t, t + 256, ..., then a tree in LDS
  __shared__ double red[2 * kScalarCols][kNormThreads];
  for (int k = 0; k < 2; ++k) {
    const double *p = k ? pr : pg;
    const int nb = k ? nblk_r : nblk_g;
    for (int c = 0; c < kScalarCols; ++c) {
      double v = (c >= 3 && c < 6) ? 1e300 : (c >= 6 && c < 9) ? -1e300 : 0.0;
      for (int b = threadIdx.x; b < nb; b += kNormThreads) v = combine(c, v, p[b * kScalarCols + c]);
      red[k * kScalarCols + c][threadIdx.x] = v;
    }
  }
  __syncthreads();
  for (int off = kNormThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int q = 0; q < 2 * kScalarCols; ++q)
        red[q][threadIdx.x] = combine(q % kScalarCols, red[q][threadIdx.x], red[q][threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double g[kScalarCols], r[kScalarCols];
  for (int c = 0; c < kScalarCols; ++c) {
    g[c] = red[c][0];
    r[c] = red[kScalarCols + c][0];
  }
  DevNorm n;
  n.sum_wg = g[0];
  n.sum_wr = r[0];
  if (use_given) {
    n.alpha_r = ga; n.I = gI; n.S = gS;
  } else {
    n.alpha_r = g[0] / r[0];
    n.I = n.alpha_r * r[2];
    n.S = g[1] + n.alpha_r * n.alpha_r * r[1];
  }
  int flags = 0;
  const double b0[3] = {b0x, b0y, b0z};
  for (int a = 0; a < 3; ++a) {
    const double *cats[2] = {g, r};
    for (int k = 0; k < 2; ++k) {
      const double *c = cats[k];
      if (c[9] > 0 && (c[3 + a] - b0[a] < 0.0 || c[6 + a] - b0[a] >= L)) flags |= 1;
    }
    if (check_extent) {
      double lo = fmin(g[9] > 0 ? g[3 + a] : 1e300, r[9] > 0 ? r[3 + a] : 1e300);
      double hi = fmax(g[9] > 0 ? g[6 + a] : -1e300, r[9] > 0 ? r[6 + a] : -1e300);
      if (hi - lo > 0.5 * L) flags |= 2;
    }
  }
  // fixed-point scale for painting: every node sum is bounded by sum |w_g| + |alpha_r| sum |w_r|,
  // which must stay below 2^62 after scaling (int64 accumulators with headroom).
  const double wabs = g[10] + fabs(n.alpha_r) * r[10];
  int e = 40;
  if (wabs > 0.0) {
    int ex;
    frexp(wabs, &ex);          // wabs < 2^ex
    e = 61 - ex;
  }
  e = e > 1000 ? 1000 : (e < -1000 ? -1000 : e);
  n.fix_scale = ldexp(1.0, e);
  n.flags = flags;
  n.nrows_occ = 0;
  n.nplanes_occ = 0;
  n.pad = 0;
  *norm = n;
}

void launch_finalize_norm(hipStream_t s, const double *pg, int nblk_g, const double *pr, int nblk_r,
                          DevNorm *norm, const double *b0, double L, int check_extent, int use_given,
                          double ga, double gI, double gS) {
  hipLaunchKernelGGL(k_finalize_norm, dim3(1), dim3(kNormThreads), 0, s, pg, nblk_g, pr, nblk_r, norm, b0[0],
                     b0[1], b0[2], L, check_extent, use_given, ga, gI, gS);
}

// ------------------------------------------------------------------------------ fill
template <typename T>
__global__ void k_fill(T *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = (T)0;
}

void launch_fill(hipStream_t s, void *p, size_t n, int prec) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks == 0) return;
  if (prec == 0) hipLaunchKernelGGL(k_fill<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float *)p, n);
  else if (prec == 2) hipLaunchKernelGGL(k_fill<int>, dim3((unsigned)blocks), dim3(256), 0, s, (int *)p, n);
  else hipLaunchKernelGGL(k_fill<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double *)p, n);
}

// ------------------------------------------------------------------------------ tiled paint
// Anchor node of a particle (decided in FP64): CIC i0 = floor(u) with taps i0, i0+1;
// TSC i0 = floor(u + 1/2) with taps i0-1, i0, i0+1; d = u - i0; u = (x - b0) / H.
// Particles outside [0, N) on some axis are skipped (the norm kernel flags them).
__device__ __forceinline__ bool anchor3(const double u[3], int assign, int N, int i0[3], double d[3]) {
  if (!(u[0] >= 0.0 && u[0] < N && u[1] >= 0.0 && u[1] < N && u[2] >= 0.0 && u[2] < N)) return false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double f = (assign == 2) ? floor(u[a]) : floor(u[a] + 0.5);
    i0[a] = ((int)f) & (N - 1);
    d[a] = u[a] - f;
  }
  return true;
}

template <typename R> struct Rec4;
template <> struct Rec4<float> { typedef float4 T; };
template <> struct Rec4<double> { typedef double4 T; };

constexpr int kAggThreads = 1024;  // the sort kernels: one workgroup per chunk of particles

// One catalog record (x, y, z, w) in FP64; `vec`: the array is 16-byte aligned, so a record is
// one 16-byte load (FP32) or two (FP64).
template <typename RI>
__device__ __forceinline__ void load_record(const RI *__restrict__ p, int64_t i, bool vec, double v[4]) {
  if constexpr (sizeof(RI) == 4) {
    if (vec) {
      const float4 q = reinterpret_cast<const float4 *>(p)[i];
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
      return;
    }
  } else {
    if (vec) {
      const double2 a = reinterpret_cast<const double2 *>(p)[2 * i];
      const double2 b = reinterpret_cast<const double2 *>(p)[2 * i + 1];
      v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
      return;
    }
  }
  v[0] = (double)p[4 * i]; v[1] = (double)p[4 * i + 1]; v[2] = (double)p[4 * i + 2]; v[3] = (double)p[4 * i + 3];
}

// Anchor node, offsets and tile of a particle at (x, y, z); false outside the box.
__device__ __forceinline__ bool particle_tile(const double v[4], int N, double b0x, double b0y, double b0z,
                                              double H, int assign, int ts, int i0[3], double d[3], int *tile) {
  const double u[3] = {(v[0] - b0x) / H, (v[1] - b0y) / H, (v[2] - b0z) / H};
  if (!anchor3(u, assign, N, i0, d)) return false;
  const int nt = N / ts;
  *tile = ((i0[2] / ts) * nt + i0[1] / ts) * nt + i0[0] / ts;
  return true;
}

constexpr int kSortWaves = kAggThreads / 64;
constexpr int kSortUnroll = 4;  // particles per thread whose loads are issued together

__device__ __forceinline__ double wave_combine(int c, double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = combine(c, v, __shfl_xor(v, off));
  return v;
}

// First pass.  Workgroup b < nblk_g takes galaxy chunk b, the others random chunk
// b - nblk_g (chunks of `chunk` particles).  It folds the FP64 scalars of its particles into
// one partial row (part_g / part_r, a fixed-order reduction: wavefront butterflies, then the
// waves in order) and histograms the anchor tiles in LDS; the histogram is stored as row b of
// chunk_hist and added to the tile totals (one global atomic per occupied tile).
template <typename RG, typename RR>
__global__ void __launch_bounds__(kAggThreads)
k_sort_count(const RG *__restrict__ gx, const RR *__restrict__ rx, const RR *__restrict__ rnbar, int64_t ng,
             int64_t nr, int64_t chunk, int nblk_g, int vec_g, int vec_r, int N, double b0x, double b0y,
             double b0z, double H, int assign, int ts, int ntiles, int *__restrict__ chunk_hist,
             int *__restrict__ counts, double *__restrict__ part_g, double *__restrict__ part_r) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *red = reinterpret_cast<double *>(smem_raw);  // [kSortWaves][kScalarCols]
  int *hist = reinterpret_cast<int *>(red + kSortWaves * kScalarCols);
  for (int t = threadIdx.x; t < ntiles; t += blockDim.x) hist[t] = 0;
  __syncthreads();
  const bool ran = (int)blockIdx.x >= nblk_g;
  const int b = ran ? (int)blockIdx.x - nblk_g : (int)blockIdx.x;
  const int64_t n = ran ? nr : ng;
  const int64_t c0 = (int64_t)b * chunk;
  const int64_t c1 = c0 + chunk < n ? c0 + chunk : n;
  double sw = 0, sw2 = 0, swn = 0, swa = 0, cnt = 0;
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  // kSortUnroll records per thread in flight (thread order of the particles unchanged)
  for (int64_t ib = c0 + threadIdx.x; ib < c1; ib += kSortUnroll * (int64_t)blockDim.x) {
    double v[kSortUnroll][4], nb[kSortUnroll];
#pragma unroll
    for (int k = 0; k < kSortUnroll; ++k) {
      const int64_t i = ib + k * (int64_t)blockDim.x;
      nb[k] = 0.0;
      if (i < c1) {
        if (ran) load_record(rx, i, vec_r != 0, v[k]);
        else load_record(gx, i, vec_g != 0, v[k]);
        if (ran && rnbar) nb[k] = (double)rnbar[i];
      }
    }
#pragma unroll
    for (int k = 0; k < kSortUnroll; ++k) {
      if (ib + k * (int64_t)blockDim.x >= c1) break;
      const double w = v[k][3];
      sw += w;
      sw2 += w * w;
      swa += fabs(w);
      if (ran && rnbar) swn += w * w * nb[k];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        mn[a] = fmin(mn[a], v[k][a]);
        mx[a] = fmax(mx[a], v[k][a]);
      }
      cnt += 1;
      int i0[3], tile;
      double d[3];
      if (particle_tile(v[k], N, b0x, b0y, b0z, H, assign, ts, i0, d, &tile)) atomicAdd(&hist[tile], 1);
    }
  }
  double vals[kScalarCols] = {sw, sw2, swn, mn[0], mn[1], mn[2], mx[0], mx[1], mx[2], cnt, swa};
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < kScalarCols; ++c) {
    const double r = wave_combine(c, vals[c]);
    if (lane == 0) red[wv * kScalarCols + c] = r;
  }
  __syncthreads();
  if ((int)threadIdx.x < kScalarCols) {
    const int c = threadIdx.x;
    double acc = red[c];
    for (int w = 1; w < kSortWaves; ++w) acc = combine(c, acc, red[w * kScalarCols + c]);
    (ran ? part_r : part_g)[(size_t)b * kScalarCols + c] = acc;
  }
  int *row = chunk_hist + (size_t)blockIdx.x * ntiles;
  for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
    const int c = hist[t];
    row[t] = c;
    if (c) atomicAdd(&counts[t], c);
  }
}

// offsets = exclusive scan of counts (offsets[ntiles] = total),
// slot[t] = rank of tile t among the occupied tiles (-1 if empty), slots[ntiles] = count.
// Thread i owns the run [i * per, (i + 1) * per); when ntiles is a multiple of 4 * 1024 (and
// per <= 64) the runs are read and written as 16-byte vectors.
__global__ void __launch_bounds__(1024) k_tile_scan(const int *__restrict__ counts, int ntiles,
                                                    int *__restrict__ offsets,
                                                    int *__restrict__ slot) {
  __shared__ int part[1024];
  __shared__ int occ[1024];
  const int per = (ntiles + 1023) / 1024;
  const int b = threadIdx.x * per, e = min(ntiles, b + per);
  const bool vec = (ntiles % 4096) == 0 && per <= 64;
  int c[64];
  int s = 0, o = 0;
  if (vec) {
#pragma unroll
    for (int k = 0; k < 64; k += 4) {
      if (k < per) {
        const int4 q = *reinterpret_cast<const int4 *>(counts + b + k);
        c[k] = q.x; c[k + 1] = q.y; c[k + 2] = q.z; c[k + 3] = q.w;
      }
    }
#pragma unroll
    for (int k = 0; k < 64; ++k)
      if (k < per) { s += c[k]; o += c[k] > 0; }
  } else {
    for (int i = b; i < e; ++i) {
      s += counts[i];
      o += counts[i] > 0;
    }
  }
  part[threadIdx.x] = s;
  occ[threadIdx.x] = o;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scans
    int v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    int w = (int)threadIdx.x >= off ? occ[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    occ[threadIdx.x] += w;
    __syncthreads();
  }
  int run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
  int orun = threadIdx.x > 0 ? occ[threadIdx.x - 1] : 0;
  if (vec) {
#pragma unroll
    for (int k = 0; k < 64; k += 4) {
      if (k < per) {
        int4 of, sl;
        of.x = run; run += c[k]; sl.x = c[k] > 0 ? orun++ : -1;
        of.y = run; run += c[k + 1]; sl.y = c[k + 1] > 0 ? orun++ : -1;
        of.z = run; run += c[k + 2]; sl.z = c[k + 2] > 0 ? orun++ : -1;
        of.w = run; run += c[k + 3]; sl.w = c[k + 3] > 0 ? orun++ : -1;
        *reinterpret_cast<int4 *>(offsets + b + k) = of;
        *reinterpret_cast<int4 *>(slot + b + k) = sl;
      }
    }
  } else {
    for (int i = b; i < e; ++i) {
      offsets[i] = run;
      run += counts[i];
      slot[i] = counts[i] > 0 ? orun++ : -1;
    }
  }
  if (threadIdx.x == 1023) {
    offsets[ntiles] = part[1023];
    slot[ntiles] = occ[1023];
  }
}

// Run bases of the sort: chunk b's records of tile t start at offsets[t] plus the counts of tile
// t in the chunks before b.  One thread per tile turns its column of the per-chunk histograms
// into those bases in place (kBaseUnroll loads in flight), so the scatter reserves its runs
// without atomics and a tile's runs follow the chunk order.
constexpr int kBaseUnroll = 32;
__global__ void __launch_bounds__(256) k_chunk_bases(const int *__restrict__ offsets, int ntiles, int nchunks,
                                                     int *__restrict__ hist) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  int base = offsets[t];
  for (int b0 = 0; b0 < nchunks; b0 += kBaseUnroll) {
    int v[kBaseUnroll];
#pragma unroll
    for (int k = 0; k < kBaseUnroll; ++k)
      v[k] = b0 + k < nchunks ? hist[(size_t)(b0 + k) * ntiles + t] : 0;
#pragma unroll
    for (int k = 0; k < kBaseUnroll; ++k) {
      if (b0 + k < nchunks) {
        hist[(size_t)(b0 + k) * ntiles + t] = base;
        base += v[k];
      }
    }
  }
}

// Second pass, same chunks as k_sort_count: the chunk's run bases (its row of chunk_hist, turned
// into bases by k_chunk_bases) go to LDS, then the chunk's particles are ranked inside their
// runs with LDS atomics and their records written (randoms carry -alpha_r w).
template <typename RG, typename RR, typename RM>
__global__ void __launch_bounds__(kAggThreads)
k_sort_scatter(const RG *__restrict__ gx, const RR *__restrict__ rx, int64_t ng, int64_t nr, int64_t chunk,
               int nblk_g, int vec_g, int vec_r, int N, double b0x, double b0y, double b0z, double H, int assign,
               int ts, int ntiles, const DevNorm *__restrict__ norm, const int *__restrict__ chunk_base,
               typename Rec4<RM>::T *__restrict__ rec) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int *hist = reinterpret_cast<int *>(smem_raw);
  const int *row = chunk_base + (size_t)blockIdx.x * ntiles;
  // base of this chunk's run in every tile, eight loads per thread in flight
  for (int t0 = threadIdx.x; t0 < ntiles; t0 += 8 * (int)blockDim.x) {
    int v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int t = t0 + k * (int)blockDim.x;
      v[k] = t < ntiles ? row[t] : 0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int t = t0 + k * (int)blockDim.x;
      if (t < ntiles) hist[t] = v[k];
    }
  }
  __syncthreads();
  const bool ran = (int)blockIdx.x >= nblk_g;
  const int b = ran ? (int)blockIdx.x - nblk_g : (int)blockIdx.x;
  const int64_t n = ran ? nr : ng;
  const int64_t c0 = (int64_t)b * chunk;
  const int64_t c1 = c0 + chunk < n ? c0 + chunk : n;
  const double wmul = ran ? -norm->alpha_r : 1.0;
  for (int64_t ib = c0 + threadIdx.x; ib < c1; ib += kSortUnroll * (int64_t)blockDim.x) {
    double v[kSortUnroll][4];
#pragma unroll
    for (int k = 0; k < kSortUnroll; ++k) {
      const int64_t i = ib + k * (int64_t)blockDim.x;
      if (i < c1) {
        if (ran) load_record(rx, i, vec_r != 0, v[k]);
        else load_record(gx, i, vec_g != 0, v[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < kSortUnroll; ++k) {
      if (ib + k * (int64_t)blockDim.x >= c1) break;
      int i0[3], tile;
      double d[3];
      if (!particle_tile(v[k], N, b0x, b0y, b0z, H, assign, ts, i0, d, &tile)) continue;
      const int pos = atomicAdd(&hist[tile], 1);
      typename Rec4<RM>::T r;
      r.x = (RM)((double)(i0[0] % ts) + d[0]);
      r.y = (RM)((double)(i0[1] % ts) + d[1]);
      r.z = (RM)((double)(i0[2] % ts) + d[2]);
      r.w = (RM)(v[k][3] * wmul);
      rec[pos] = r;
    }
  }
}

// One workgroup per tile: the tile's nodes plus a one-node halo (local index -1 .. ts on each
// axis, E = ts + 2) accumulated in LDS, then stored as block `slot[tile]` of the scratch in the
// mesh precision.  Contributions are accumulated as 64-bit fixed point, round(c * scale) with
// scale a power of two (integer LDS atomics run at full rate where floating-point LDS atomics
// are serialised per lane); integer sums are exact, so a block does not depend on the order of
// its particles.  FP64 meshes use scale = fix_scale (node sums below 2^62).  FP32 meshes use
// scale = fix_scale / 2^11, so every contribution is below 2^50 in magnitude and converts to
// int64 by adding 1.5 * 2^52 in double (the sum lands in [2^52, 2^53), where the ulp is 1 and
// the bit pattern minus that of 1.5 * 2^52 is the rounded integer in two's complement): three
// operations in place of the dozen of a general float-to-int64 conversion.  The quantum, 2^-50
// of the catalog's total |weight|, stays far below FP32 resolution.
template <typename RM, int ASSIGN>
__global__ void __launch_bounds__(512) k_tile_paint(int ts, const int *__restrict__ offsets,
                                                    const int *__restrict__ slot,
                                                    const typename Rec4<RM>::T *__restrict__ rec,
                                                    const DevNorm *__restrict__ norm,
                                                    RM *__restrict__ blocks) {
  const int tile = blockIdx.x;
  const int beg = offsets[tile], end = offsets[tile + 1];
  if (beg == end) return;  // uniform for the block
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem_raw);
  const int E = ts + 2, E3 = E * E * E;
  for (int c = threadIdx.x; c < E3; c += blockDim.x) acc[c] = 0ull;
  constexpr bool MAGIC = sizeof(RM) == 4;
  const double qscale = MAGIC ? norm->fix_scale * (1.0 / 2048.0) : norm->fix_scale;
  const RM scale = (RM)qscale;
  __syncthreads();
  constexpr int NTAP = (ASSIGN == 2) ? 2 : 3;
  constexpr int O0 = (ASSIGN == 2) ? 1 : 0;   // LDS index of tap a on an axis: l + a + O0
  // each thread's records in turn, the next one loaded while the current one is deposited
  typename Rec4<RM>::T nxt;
  if (beg + (int)threadIdx.x < end) nxt = rec[beg + threadIdx.x];
  for (int p = beg + threadIdx.x; p < end; p += blockDim.x) {
    const typename Rec4<RM>::T r = nxt;
    if (p + (int)blockDim.x < end) nxt = rec[p + blockDim.x];
    const RM v[3] = {r.x, r.y, r.z};
    int l[3];
    RM wt[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      int li = (ASSIGN == 2) ? (int)floor(v[a]) : (int)floor(v[a] + (RM)0.5);
      li = li < 0 ? 0 : (li > ts - 1 ? ts - 1 : li);
      const RM d = v[a] - (RM)li;
      l[a] = li;
      if (ASSIGN == 2) {
        wt[a][0] = (RM)1 - d;
        wt[a][1] = d;
      } else {
        wt[a][0] = (RM)0.5 * ((RM)0.5 - d) * ((RM)0.5 - d);
        wt[a][1] = (RM)0.75 - d * d;
        wt[a][2] = (RM)0.5 * ((RM)0.5 + d) * ((RM)0.5 + d);
      }
    }
#pragma unroll
    for (int a = 0; a < NTAP; ++a) {
      const RM wz = wt[2][a] * r.w * scale;
      const int zz = l[2] + a + O0;
#pragma unroll
      for (int b = 0; b < NTAP; ++b) {
        const RM wyz = wt[1][b] * wz;
        const int base = (zz * E + l[1] + b + O0) * E + l[0] + O0;
#pragma unroll
        for (int c = 0; c < NTAP; ++c) {
          long long q;
          if constexpr (MAGIC)
            q = __double_as_longlong((double)(wt[0][c] * wyz) + 6755399441055744.0) - 0x4338000000000000LL;
          else
            q = (long long)rint(wt[0][c] * wyz);
          atomicAdd(&acc[base + c], (unsigned long long)q);
        }
      }
    }
  }
  __syncthreads();
  const double inv = 1.0 / qscale;
  RM *dst = blocks + (size_t)slot[tile] * E3;
  for (int c = threadIdx.x; c < E3; c += blockDim.x) dst[c] = (RM)((double)(long long)acc[c] * inv);
}

// Node (x, y, z) of tile T at local (lx, ly, lz) is covered by the block of tile T + d for
// d in {-1, 0, 1}^3 where d_a = -1 needs l_a = 0 and d_a = +1 needs l_a = ts - 1; inside that
// block it sits at local l - d ts, block index l - d ts + 1.  Empty tiles have no block.
// One workgroup per group of GX tiles along x (GX = 2 for FP32 with at least two tiles per
// axis, so mesh rows are written as whole 128-byte lines); the slots of the group's
// neighbourhood are read into LDS once.  Every thread first loads all the block values it
// will need (its nodes' own values and its share of the neighbours' halo values), so a
// workgroup waits on memory about twice; the values are then summed in LDS: each node takes
// its own block's value, then the halo values in a fixed order of classes (x faces, y faces,
// z faces, xy / xz / yz edges, corners).  Within one class a node receives at most one value
// (ts > 1), so the mesh is the same on every run.  N and ts are powers of two, ts = 16 (or N).
// A workgroup whose whole row of tiles (every tx at its ty, tz) has no occupied tile within
// one tile in y and z writes nothing: every x-row it covers is zero, stays out of rowmask, and
// no kernel reads mesh rows outside the occupied-row list.
template <typename RM>
__global__ void __launch_bounds__(256) k_tile_gather(int lgN, int lgts, int lggx, const int *__restrict__ slot,
                                                     const RM *__restrict__ blocks, RM *__restrict__ mesh,
                                                     int *__restrict__ rowmask) {
  constexpr int kNodes = 32768 / (int)sizeof(RM);  // GX * ts^3 nodes: 8192 FP32 (GX 2), 4096 FP64
  constexpr int kOwn = kNodes / 256;               // nodes per thread, at most
  const int N = 1 << lgN, ts = 1 << lgts, nt = N >> lgts, E = ts + 2, GX = 1 << lggx;
  const size_t E3 = (size_t)E * E * E;
  __shared__ int sl[3][3][4];  // [dz + 1][dy + 1][tile offset along x + 1], offsets -1 .. GX
  __shared__ RM acc[kNodes];   // node lxg + W (ly + ts lz) of the group, W = GX ts
  const int ngx = nt >> lggx;
  const int gx = (int)blockIdx.x % ngx, ty = ((int)blockIdx.x / ngx) % nt, tz = (int)blockIdx.x / (ngx * nt);
  const int tx0 = gx << lggx;
  const int tid = threadIdx.x;
  // occupancy of the tile row's neighbourhood (9 nt <= 288 slots) and the group's slots
  int occ = 0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int i = tid + 256 * k;
    if (i < 9 * nt) {
      const int tx = i % nt, dy = (i / nt) % 3 - 1, dz = i / (3 * nt) - 1;
      occ |= slot[(((tz + dz + nt) & (nt - 1)) * nt + ((ty + dy + nt) & (nt - 1))) * nt + tx] >= 0;
    }
  }
  if (tid < 9 * (GX + 2)) {
    const int dxi = tid % (GX + 2), dy = (tid / (GX + 2)) % 3 - 1, dz = tid / (3 * (GX + 2)) - 1;
    const int tx = (tx0 + dxi - 1 + nt) & (nt - 1), tyy = (ty + dy + nt) & (nt - 1), tzz = (tz + dz + nt) & (nt - 1);
    sl[dz + 1][dy + 1][dxi] = slot[(tzz * nt + tyy) * nt + tx];
  }
  if (!__syncthreads_or(occ)) return;  // uniform for the workgroup
  const int lgW = lggx + lgts;  // nodes per row of the group: W = GX * ts
  const int W = 1 << lgW;
  const int nown = 1 << (lgW + 2 * lgts - 8);  // nodes per thread (the group has a multiple of 256)
  const int hi = ts - 1;
  // the value of neighbour d at node (lxg, ly, lz) and the node's index (-1: no block)
  auto fetch = [&](int dx, int dy, int dz, int lxg, int ly, int lz, int &node) -> RM {
    const int s = sl[dz + 1][dy + 1][(lxg >> lgts) + dx + 1];
    node = s < 0 ? -1 : lxg + ((ly + (lz << lgts)) << lgW);
    if (s < 0) return (RM)0;
    const int ex = (lxg & hi) - dx * ts + 1, ey = ly - dy * ts + 1, ez = lz - dz * ts + 1;
    return blocks[(size_t)s * E3 + (size_t)((ez * E + ey) * E + ex)];
  };
  // own values: node tid + 256 k, block index l + 1
  RM own[kOwn];
#pragma unroll
  for (int k = 0; k < kOwn; ++k) {
    if (k < nown) {
      const int n = tid + (k << 8);
      const int lxg = n & (W - 1), ly = (n >> lgW) & hi, lz = n >> (lgW + lgts);
      const int s = sl[1][1][(lxg >> lgts) + 1];
      own[k] = s < 0 ? (RM)0 : blocks[(size_t)s * E3 + (size_t)(((lz + 1) * E + ly + 1) * E + (lxg & hi) + 1)];
    }
  }
  // faces: item i = 2 r + f, f the face (0: low, 1: high); x: r -> (tile, ly, lz);
  // y: r -> (lxg, lz); z: r -> (lxg, ly).  At most 4 items of each per thread.
  RM fv[3][4];
  int fn[3][4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = tid + (k << 8), f = i & 1, r = i >> 1;
    fn[0][k] = fn[1][k] = fn[2][k] = -1;
    if (i < 2 * GX * ts * ts)
      fv[0][k] = fetch(f ? 1 : -1, 0, 0, ((r & (GX - 1)) << lgts) + (f ? hi : 0), (r >> lggx) & hi,
                       r >> (lggx + lgts), fn[0][k]);
    if (i < 2 * W * ts) {
      fv[1][k] = fetch(0, f ? 1 : -1, 0, r & (W - 1), f ? hi : 0, r >> lgW, fn[1][k]);
      fv[2][k] = fetch(0, 0, f ? 1 : -1, r & (W - 1), r >> lgW, f ? hi : 0, fn[2][k]);
    }
  }
  // edges: item i = 4 r + f, f the two signs; xy: r -> (tile, lz); xz: r -> (tile, ly);
  // yz: r -> lxg.  Corners: item i = 8 tile + f, f the three signs.
  RM ev[3], cv = (RM)0;
  int en[3] = {-1, -1, -1}, cn = -1;
  {
    const int f = tid & 3, r = tid >> 2;
    const int sa = (f & 1) ? 1 : -1, sb = (f & 2) ? 1 : -1;
    if (tid < 4 * GX * ts) {
      const int lx = ((r & (GX - 1)) << lgts) + (sa > 0 ? hi : 0);
      ev[0] = fetch(sa, sb, 0, lx, sb > 0 ? hi : 0, r >> lggx, en[0]);
      ev[1] = fetch(sa, 0, sb, lx, r >> lggx, sb > 0 ? hi : 0, en[1]);
    }
    if (tid < 4 * W) ev[2] = fetch(0, sa, sb, r, sa > 0 ? hi : 0, sb > 0 ? hi : 0, en[2]);
    if (tid < 8 * GX) {
      const int c = tid & 7, dx = (c & 1) ? 1 : -1, dy = (c & 2) ? 1 : -1, dz = (c & 4) ? 1 : -1;
      cv = fetch(dx, dy, dz, ((tid >> 3) << lgts) + (dx > 0 ? hi : 0), dy > 0 ? hi : 0, dz > 0 ? hi : 0, cn);
    }
  }
  // sums in LDS, class by class
#pragma unroll
  for (int k = 0; k < kOwn; ++k)
    if (k < nown) acc[tid + (k << 8)] = own[k];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (fn[c][k] >= 0) acc[fn[c][k]] += fv[c][k];
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (en[c] >= 0) acc[en[c]] += ev[c];
    __syncthreads();
  }
  if (cn >= 0) acc[cn] += cv;
  __syncthreads();
  // store: each row segment is W adjacent lanes (W divides 64); its first lane marks the row
  const int lane = tid & 63;
  const unsigned long long seg = (1ull << W) - 1;  // W <= 32
#pragma unroll 8
  for (int k = 0; k < kOwn; ++k) {
    if (k < nown) {  // uniform: whole waves
      const int n = tid + (k << 8);
      const int lxg = n & (W - 1), ly = (n >> lgW) & hi, lz = n >> (lgW + lgts);
      const RM v = acc[n];
      const int x = (tx0 << lgts) + lxg, y = (ty << lgts) + ly, z = (tz << lgts) + lz;
      const size_t g = ((size_t)z * N + y) * N + x;
      mesh[g] = v;
      const unsigned long long nz = __ballot(v != (RM)0);
      if (rowmask && (lane & (W - 1)) == 0 && ((nz >> lane) & seg)) rowmask[g >> lgN] = 1;
    }
  }
}

// Occupancy in two passes over blocks of 1024 rows: (1) per-block counts and the plane flags,
// (2) each block's offset (sum of the earlier blocks' counts), an in-block scan by wavefront
// ballots, and the writes of the row list; block 0 also compacts the plane list and stores the
// counts.
constexpr int kOccThreads = 1024;
__global__ void __launch_bounds__(kOccThreads) k_occ_count(int N, const int *__restrict__ rowmask,
                                                           int *__restrict__ blockcnt, int *__restrict__ planemask) {
  __shared__ int wsum[kOccThreads / 64];
  const int nrows = N * N;
  const int i = blockIdx.x * kOccThreads + threadIdx.x;
  const bool f = i < nrows && rowmask[i] != 0;
  if (f) planemask[i / N] = 1;  // every writer stores the same value
  const unsigned long long bal = __ballot(f);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0;
    for (int w = 0; w < kOccThreads / 64; ++w) c += wsum[w];
    blockcnt[blockIdx.x] = c;
  }
}

__global__ void __launch_bounds__(kOccThreads) k_occ_write(int N, int nblocks, const int *__restrict__ rowmask,
                                                           const int *__restrict__ blockcnt,
                                                           const int *__restrict__ planemask,
                                                           int *__restrict__ rowlist, int *__restrict__ zlist,
                                                           DevNorm *__restrict__ norm) {
  __shared__ int wsum[kOccThreads / 64];
  __shared__ int part[kOccThreads];
  const int nrows = N * N;
  // offset of this block: sum of blockcnt[0 .. blockIdx.x)
  int acc = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += kOccThreads) acc += blockcnt[b];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kOccThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  const int base = part[0];
  const int i = blockIdx.x * kOccThreads + threadIdx.x;
  const bool f = i < nrows && rowmask[i] != 0;
  const unsigned long long bal = __ballot(f);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) wsum[w] = __popcll(bal);
  __syncthreads();
  int wo = 0;
  for (int k = 0; k < w; ++k) wo += wsum[k];
  const unsigned long long below = lane ? (bal & ((1ull << lane) - 1ull)) : 0ull;
  if (f) rowlist[base + wo + __popcll(below)] = i;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int tot = 0;
    for (int b = 0; b < nblocks; ++b) tot += blockcnt[b];
    int k = 0;
    for (int z = 0; z < N; ++z)
      if (planemask[z]) zlist[k++] = z;
    norm->nrows_occ = tot;
    norm->nplanes_occ = k;
  }
}

int occupancy_blocks(int N) { return (N * N + kOccThreads - 1) / kOccThreads; }

void launch_occupancy(hipStream_t s, int N, const int *rowmask, int *rowlist, int *planemask, int *zlist,
                      int *blockcnt, DevNorm *norm) {
  const int nb = occupancy_blocks(N);
  launch_fill(s, planemask, (size_t)N, 2);
  hipLaunchKernelGGL(k_occ_count, dim3(nb), dim3(kOccThreads), 0, s, N, rowmask, blockcnt, planemask);
  hipLaunchKernelGGL(k_occ_write, dim3(nb), dim3(kOccThreads), 0, s, N, nb, rowmask, blockcnt, planemask, rowlist,
                     zlist, norm);
}

SortLayout sort_layout(int N, int64_t n_gal, int64_t n_ran) {
  SortLayout L;
  const int64_t n = n_gal + n_ran;
  // one chunk size for both catalogs: about one workgroup per CU of a 256-CU device for up to
  // 2^25 particles, chunks of 2^17 beyond, and never more than kScalarBlocks chunks per catalog
  int64_t c = (n + kSortNominalCUs - 1) / kSortNominalCUs;
  if (c > 131072) c = 131072;
  const int64_t cmin = (n + kScalarBlocks - 1) / kScalarBlocks;
  if (c < cmin) c = cmin;
  c = (c + kAggThreads - 1) / kAggThreads * kAggThreads;
  if (c < 4096) c = 4096;
  L.chunk = c;
  L.nblk_g = (int)((n_gal + c - 1) / c);
  L.nblk_r = (int)((n_ran + c - 1) / c);
  const int ts = tile_size(N), nt = N / ts;
  L.ntiles = nt * nt * nt;
  L.hist_bytes = (size_t)(L.nblk_g + L.nblk_r) * L.ntiles * sizeof(int);
  return L;
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

void launch_sort_count(hipStream_t s, const SortLayout &L, const void *gx, int gdtype, const void *rx, int rdtype,
                       const void *rnbar, int64_t ng, int64_t nr, int N, const double *b0, double H, int assign,
                       int *chunk_hist, int *counts, double *part_g, double *part_r) {
  const unsigned nblk = (unsigned)(L.nblk_g + L.nblk_r);
  if (nblk == 0) return;
  static_assert(kSortLdsExtra == (size_t)kSortWaves * kScalarCols * sizeof(double), "LDS rows");
  const size_t lds = kSortLdsExtra + (size_t)L.ntiles * sizeof(int);
  const int ts = tile_size(N);
  const int vg = aligned16(gx), vr = aligned16(rx);
#define PW_SC(RG, RR)                                                                                         \
  hipLaunchKernelGGL((k_sort_count<RG, RR>), dim3(nblk), dim3(kAggThreads), lds, s, (const RG *)gx, (const RR *)rx, \
                     (const RR *)rnbar, ng, nr, L.chunk, L.nblk_g, vg, vr, N, b0[0], b0[1], b0[2], H, assign, ts,    \
                     L.ntiles, chunk_hist, counts, part_g, part_r)
  if (gdtype == 0 && rdtype == 0) PW_SC(float, float);
  else if (gdtype == 0) PW_SC(float, double);
  else if (rdtype == 0) PW_SC(double, float);
  else PW_SC(double, double);
#undef PW_SC
}

void launch_sort_scatter(hipStream_t s, const SortLayout &L, const void *gx, int gdtype, const void *rx,
                         int rdtype, int64_t ng, int64_t nr, int prec, int N, const double *b0, double H,
                         int assign, const DevNorm *norm, int *chunk_hist, const int *offsets, void *records) {
  const unsigned nblk = (unsigned)(L.nblk_g + L.nblk_r);
  if (nblk == 0) return;
  hipLaunchKernelGGL(k_chunk_bases, dim3((unsigned)((L.ntiles + 255) / 256)), dim3(256), 0, s, offsets, L.ntiles,
                     (int)nblk, chunk_hist);
  const size_t lds = (size_t)L.ntiles * sizeof(int);
  const int ts = tile_size(N);
  const int vg = aligned16(gx), vr = aligned16(rx);
#define PW_SS(RG, RR, RM)                                                                                   \
  hipLaunchKernelGGL((k_sort_scatter<RG, RR, RM>), dim3(nblk), dim3(kAggThreads), lds, s, (const RG *)gx,     \
                     (const RR *)rx, ng, nr, L.chunk, L.nblk_g, vg, vr, N, b0[0], b0[1], b0[2], H, assign, ts, \
                     L.ntiles, norm, chunk_hist, (typename Rec4<RM>::T *)records)
#define PW_SS_M(RG, RR) \
  if (prec == 0) PW_SS(RG, RR, float); else PW_SS(RG, RR, double);
  if (gdtype == 0 && rdtype == 0) { PW_SS_M(float, float) }
  else if (gdtype == 0) { PW_SS_M(float, double) }
  else if (rdtype == 0) { PW_SS_M(double, float) }
  else { PW_SS_M(double, double) }
#undef PW_SS_M
#undef PW_SS
}

void launch_tile_scan(hipStream_t s, const int *counts, int ntiles, int *offsets, int *slot) {
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, s, counts, ntiles, offsets, slot);
}

static int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}

void launch_tile_paint(hipStream_t s, int prec, int N, int assign, const int *offsets, const int *slot,
                       const void *records, const DevNorm *norm, void *blocks, ColTune tune) {
  const int ts = tile_size(N);
  const int nt = N / ts;
  const unsigned ntiles = (unsigned)(nt * nt * nt);
  const size_t E3 = (size_t)(ts + 2) * (ts + 2) * (ts + 2);
  const int threads = (tune.threads == 128 || tune.threads == 512) ? tune.threads : 256;
#define PW_TP(RM, A)                                                                              \
  hipLaunchKernelGGL((k_tile_paint<RM, A>), dim3(ntiles), dim3(threads), E3 * sizeof(unsigned long long), s, \
                     ts, offsets, slot, (const typename Rec4<RM>::T *)records, norm, (RM *)blocks)
  if (prec == 0) { if (assign == 2) PW_TP(float, 2); else PW_TP(float, 3); }
  else { if (assign == 2) PW_TP(double, 2); else PW_TP(double, 3); }
#undef PW_TP
}

void launch_tile_gather(hipStream_t s, int prec, int N, const int *slot, const void *blocks, void *mesh,
                        int *rowmask, ColTune tune) {
  const int ts = tile_size(N);
  const int nt = N / ts;
  const unsigned ntiles = (unsigned)(nt * nt * nt);
  // FP32: two tiles per workgroup along x (128-byte rows) unless tuned to one
  const int lggx_f = (nt >= 2 && tune.gx != 1) ? 1 : 0;
  if (prec == 0)
    hipLaunchKernelGGL(k_tile_gather<float>, dim3(ntiles >> lggx_f), dim3(256), 0, s, ilog2(N), ilog2(ts), lggx_f,
                       slot, (const float *)blocks, (float *)mesh, rowmask);
  else
    hipLaunchKernelGGL(k_tile_gather<double>, dim3(ntiles), dim3(256), 0, s, ilog2(N), ilog2(ts), 0, slot,
                       (const double *)blocks, (double *)mesh, rowmask);
}

}  // namespace pw
