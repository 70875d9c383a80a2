// HIP kernels of the estimator hot path (gfx950, wave64).
//
//   scalars      FP64 reductions over a catalog (sum w, sum w^2, sum w^2 nbar, bounding box)
//   norm         alpha_r = sum w_g / sum w_r, I = alpha_r sum_r w_r^2 nbar_r,
//                S = sum_g w_g^2 + alpha_r^2 sum_r w_r^2 (Section 2.1), range / extent flags
//   paint        CIC / TSC mass assignment with FP32 (or FP64) atomics
//   fx           fused field generation F (2r)^-alpha y_J^mu(x^) + real-to-complex FFT along x,
//                two real fields per complex transform, output pruned to kx < nkx
//   fy, fz       complex FFTs along y and z, output pruned to the retained k-sphere
//   contract     bisector contraction sum_nu y_l^nu(k^) sum S Re(conj(R_1) R_2) (Section 5.2
//                boxed estimator in the real-harmonic basis) with FP64 shell sums
//   finalize_pk  P_l = (4 pi / I) <..>_shell - d_l0 S / I
#include "kernels.h"

#include "dev_core.h"

namespace pw {

__constant__ ShConst c_sh;

void upload_sh_const(const ShConst &c) {
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_sh), &c, sizeof(ShConst));
}

// ------------------------------------------------------------------------------ scalars
template <typename R>
__global__ void __launch_bounds__(256) k_scalars(const R *__restrict__ xyzw, const R *__restrict__ nbar,
                                                 int64_t n, double *__restrict__ partial) {
  double sw = 0, sw2 = 0, swn = 0;
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  double cnt = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double x = xyzw[4 * i], y = xyzw[4 * i + 1], z = xyzw[4 * i + 2], w = xyzw[4 * i + 3];
    sw += w;
    sw2 += w * w;
    if (nbar) swn += w * w * (double)nbar[i];
    mn[0] = fmin(mn[0], x); mn[1] = fmin(mn[1], y); mn[2] = fmin(mn[2], z);
    mx[0] = fmax(mx[0], x); mx[1] = fmax(mx[1], y); mx[2] = fmax(mx[2], z);
    cnt += 1;
  }
  __shared__ double red[256];
  double vals[kScalarCols] = {sw, sw2, swn, mn[0], mn[1], mn[2], mx[0], mx[1], mx[2], cnt};
  for (int c = 0; c < kScalarCols; ++c) {
    red[threadIdx.x] = vals[c];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) {
        double a = red[threadIdx.x], b = red[threadIdx.x + off];
        red[threadIdx.x] = (c >= 3 && c < 6) ? fmin(a, b) : (c >= 6 && c < 9) ? fmax(a, b) : a + b;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x * kScalarCols + c] = red[0];
    __syncthreads();
  }
}

void launch_scalars(hipStream_t s, const void *xyzw, const void *nbar, int64_t n, int dtype,
                    double *partial) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_scalars<float>, dim3(kScalarBlocks), dim3(256), 0, s,
                       (const float *)xyzw, (const float *)nbar, n, partial);
  else
    hipLaunchKernelGGL(k_scalars<double>, dim3(kScalarBlocks), dim3(256), 0, s,
                       (const double *)xyzw, (const double *)nbar, n, partial);
}

__device__ void reduce_partials(const double *p, double out[kScalarCols]) {
  // thread-0-only helper: deterministic sequential reduction over the block rows
  for (int c = 0; c < kScalarCols; ++c) out[c] = (c >= 3 && c < 6) ? 1e300 : (c >= 6 && c < 9) ? -1e300 : 0.0;
  for (int b = 0; b < kScalarBlocks; ++b)
    for (int c = 0; c < kScalarCols; ++c) {
      double v = p[b * kScalarCols + c];
      if (c >= 3 && c < 6) out[c] = fmin(out[c], v);
      else if (c >= 6 && c < 9) out[c] = fmax(out[c], v);
      else out[c] += v;
    }
}

__global__ void k_finalize_norm(const double *pg, const double *pr, DevNorm *norm, double b0x,
                                double b0y, double b0z, double L, int check_extent, int use_given,
                                double ga, double gI, double gS) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double g[kScalarCols], r[kScalarCols];
  reduce_partials(pg, g);
  reduce_partials(pr, r);
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
  n.flags = flags;
  n.pad = 0;
  *norm = n;
}

void launch_finalize_norm(hipStream_t s, const double *pg, const double *pr, DevNorm *norm,
                          const double *b0, double L, int check_extent, int use_given,
                          double ga, double gI, double gS) {
  hipLaunchKernelGGL(k_finalize_norm, dim3(1), dim3(64), 0, s, pg, pr, norm, b0[0], b0[1], b0[2],
                     L, check_extent, use_given, ga, gI, gS);
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
  else hipLaunchKernelGGL(k_fill<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double *)p, n);
}

// ------------------------------------------------------------------------------ paint
// Node masses m_n += w W(u - n), u = (x - b0) / H, periodic indices (N is a power of two).
// CIC: i0 = floor(u), weights (1-d, d).  TSC: i0 = floor(u + 1/2), d = u - i0,
// weights (1/2 (1/2-d)^2, 3/4 - d^2, 1/2 (1/2+d)^2) at i0-1, i0, i0+1.  Positions are turned
// into u in FP64 so that the cell decision does not depend on the storage precision.
template <typename RI, typename RM, int ASSIGN>
__global__ void __launch_bounds__(256) k_paint(const RI *__restrict__ xyzw, int64_t n, RM *__restrict__ mesh,
                                               int N, double b0x, double b0y, double b0z, double H,
                                               const DevNorm *__restrict__ norm, int is_random) {
  const double wmul = is_random ? -norm->alpha_r : 1.0;
  const int mask = N - 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double u[3];
    u[0] = ((double)xyzw[4 * i] - b0x) / H;
    u[1] = ((double)xyzw[4 * i + 1] - b0y) / H;
    u[2] = ((double)xyzw[4 * i + 2] - b0z) / H;
    const double w = (double)xyzw[4 * i + 3] * wmul;
    if (!(u[0] >= 0.0 && u[0] < N && u[1] >= 0.0 && u[1] < N && u[2] >= 0.0 && u[2] < N)) continue;
    int i0[3];
    RM wt[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (ASSIGN == 2) {
        double f = floor(u[a]);
        double d = u[a] - f;
        i0[a] = (int)f;
        wt[a][0] = (RM)(1.0 - d);
        wt[a][1] = (RM)d;
      } else {
        double f = floor(u[a] + 0.5);
        double d = u[a] - f;
        i0[a] = (int)f - 1;
        wt[a][0] = (RM)(0.5 * (0.5 - d) * (0.5 - d));
        wt[a][1] = (RM)(0.75 - d * d);
        wt[a][2] = (RM)(0.5 * (0.5 + d) * (0.5 + d));
      }
    }
    constexpr int NT = (ASSIGN == 2) ? 2 : 3;
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const int iz = (i0[2] + a + N) & mask;
      const RM wz = wt[2][a] * (RM)w;
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        const int iy = (i0[1] + b + N) & mask;
        const RM wyz = wt[1][b] * wz;
        const size_t rowb = ((size_t)iz * N + iy) * N;
#pragma unroll
        for (int c = 0; c < NT; ++c) {
          const int ix = (i0[0] + c + N) & mask;
          atomicAdd(&mesh[rowb + ix], wt[0][c] * wyz);
        }
      }
    }
  }
}

void launch_paint(hipStream_t s, const void *xyzw, int64_t n, int dtype, int prec, void *mesh,
                  int N, const double *b0, double H, int assign, const DevNorm *norm, int is_random) {
  if (n <= 0) return;
  int64_t blocks64 = (n + 255) / 256;
  unsigned blocks = (unsigned)(blocks64 > 65536 ? 65536 : blocks64);
#define PW_PAINT(RI, RM, A)                                                                        \
  hipLaunchKernelGGL((k_paint<RI, RM, A>), dim3(blocks), dim3(256), 0, s, (const RI *)xyzw, n,     \
                     (RM *)mesh, N, b0[0], b0[1], b0[2], H, norm, is_random)
  if (dtype == 0 && prec == 0) { if (assign == 2) PW_PAINT(float, float, 2); else PW_PAINT(float, float, 3); }
  else if (dtype == 0 && prec == 1) { if (assign == 2) PW_PAINT(float, double, 2); else PW_PAINT(float, double, 3); }
  else if (dtype == 1 && prec == 0) { if (assign == 2) PW_PAINT(double, float, 2); else PW_PAINT(double, float, 3); }
  else { if (assign == 2) PW_PAINT(double, double, 2); else PW_PAINT(double, double, 3); }
#undef PW_PAINT
}

// ------------------------------------------------------------------------------ fx
template <int N> struct FxShape {
  static constexpr int T = N / 8;                          // lanes per pencil
  static constexpr int ROWS = (T >= 64) ? (256 / T > 0 ? 256 / T : 1) : 64 / T * 2;
  static constexpr int THREADS = ROWS * T;
};

template <typename R, int N>
__global__ void __launch_bounds__(FxShape<N>::THREADS)
k_fx(const R *__restrict__ mesh, cplx<R> *__restrict__ out, const FieldJob *__restrict__ jobs,
     int njobs, int nkx, R b0x, R b0y, R b0z, R H, const cplx<R> *__restrict__ tw) {
  constexpr int T = FxShape<N>::T, ROWS = FxShape<N>::ROWS;
  constexpr int LN = N + N / 8;
  __shared__ cplx<R> lds[ROWS * LN];
  const int rl = threadIdx.x / T, t = threadIdx.x % T;
  const int row = blockIdx.x * ROWS + rl;  // row = z * N + y (grid covers N*N exactly)
  const int y = row & (N - 1), z = row / N;
  cplx<R> *my = lds + rl * LN;
  auto at = [my](int i) -> cplx<R> & { return my[i + (i >> 3)]; };
  auto sync = []() { __syncthreads(); };

  R f[8], ux[8], uy[8], uz[8], inv2r[8];
  const R py = b0y + (R)y * H, pz = b0z + (R)z * H;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int x = t + s * T;
    f[s] = mesh[(size_t)row * N + x];
    const R px = b0x + (R)x * H;
    const R r = sqrt(px * px + py * py + pz * pz);
    if (r > (R)0) {
      const R ir = (R)1 / r;
      ux[s] = px * ir; uy[s] = py * ir; uz[s] = pz * ir;
      inv2r[s] = (R)0.5 * ir;
    } else {
      ux[s] = 0; uy[s] = 0; uz[s] = 1;
      inv2r[s] = 0;
    }
  }
  const size_t fstride = (size_t)N * N * nkx;
  for (int jb = 0; jb < njobs; ++jb) {
    const FieldJob J = jobs[jb];
    cplx<R> v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      R w = f[s];
      for (int a = 0; a < J.alpha; ++a) w *= inv2r[s];
      R ya, yb;
      if (J.kind == 0) {
        real_sh_pair<R>(c_sh, J.Ja, J.m, ux[s], uy[s], uz[s], &ya, &yb);
      } else {
        R dummy;
        real_sh_pair<R>(c_sh, J.Ja, 0, ux[s], uy[s], uz[s], &ya, &dummy);
        yb = 0;
        if (J.Jb >= 0) real_sh_pair<R>(c_sh, J.Jb, 0, ux[s], uy[s], uz[s], &yb, &dummy);
      }
      v[s] = mk<R>(w * ya, w * yb);
    }
    fft_pencil<R, N, false>(v, t, tw, at, sync);
#pragma unroll
    for (int s = 0; s < 8; ++s) at(t + s * T) = v[s];
    __syncthreads();
    cplx<R> *oa = out + (size_t)J.pa * fstride + (size_t)row * nkx;
    cplx<R> *ob = out + (size_t)(J.pb < 0 ? 0 : J.pb) * fstride + (size_t)row * nkx;
    for (int kx = t; kx < nkx; kx += T) {
      const cplx<R> a = at(kx), b = at((N - kx) & (N - 1));
      // A = (Z(k) + conj Z(N-k)) / 2,  B = (Z(k) - conj Z(N-k)) / (2i)
      oa[kx] = mk<R>((R)0.5 * (a.x + b.x), (R)0.5 * (a.y - b.y));
      if (J.pb >= 0) ob[kx] = mk<R>((R)0.5 * (a.y + b.y), (R)0.5 * (b.x - a.x));
    }
    __syncthreads();
  }
}

template <typename R, int N>
static void fx_launch(hipStream_t s, const void *mesh, void *out, const FieldJob *jobs, int njobs,
                      int nkx, const double *b0, double H, const void *tw) {
  constexpr int ROWS = FxShape<N>::ROWS;
  unsigned blocks = (unsigned)((size_t)N * N / ROWS);
  hipLaunchKernelGGL((k_fx<R, N>), dim3(blocks), dim3(FxShape<N>::THREADS), 0, s, (const R *)mesh,
                     (cplx<R> *)out, jobs, njobs, nkx, (R)b0[0], (R)b0[1], (R)b0[2], (R)H,
                     (const cplx<R> *)tw);
}

#define PW_DISPATCH_N(FN, R, ...)                                                                  \
  switch (N) {                                                                                     \
    case 16: FN<R, 16>(__VA_ARGS__); break;                                                        \
    case 32: FN<R, 32>(__VA_ARGS__); break;                                                        \
    case 64: FN<R, 64>(__VA_ARGS__); break;                                                        \
    case 128: FN<R, 128>(__VA_ARGS__); break;                                                      \
    case 256: FN<R, 256>(__VA_ARGS__); break;                                                      \
    case 512: FN<R, 512>(__VA_ARGS__); break;                                                      \
    default: break;                                                                                \
  }

void launch_fx(hipStream_t s, int prec, int N, const void *mesh, void *out, const FieldJob *jobs,
               int njobs, int nkx, const double *b0, double H, const void *tw) {
  if (prec == 0) { PW_DISPATCH_N(fx_launch, float, s, mesh, out, jobs, njobs, nkx, b0, H, tw) }
  else { PW_DISPATCH_N(fx_launch, double, s, mesh, out, jobs, njobs, nkx, b0, H, tw) }
}

// ------------------------------------------------------------------------------ fy / fz
// Column-mode pencils: C pencils adjacent in memory, lane (t, c) with c fastest so that every
// global access of a wavefront covers C consecutive complex values.
template <typename R, int N> struct ColShape {
  static constexpr int T = N / 8;
  static constexpr int C0 = (sizeof(R) == 4) ? 16 : 8;
  static constexpr int C = (C0 * T > 1024) ? 1024 / T : C0;
  static constexpr int THREADS = C * T;
};

template <typename R, int N>
__global__ void __launch_bounds__((ColShape<R, N>::THREADS))
k_fy(const cplx<R> *__restrict__ in, cplx<R> *__restrict__ out, int nkx, const int *__restrict__ ycnt,
     const int64_t *__restrict__ yoff, int64_t npen, const cplx<R> *__restrict__ tw) {
  constexpr int T = ColShape<R, N>::T, C = ColShape<R, N>::C;
  __shared__ cplx<R> lds[N * (C + 1)];
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int kx = blockIdx.x * C + c;
  const int z = blockIdx.y, p = blockIdx.z;
  const cplx<R> *src = in + ((size_t)p * N + z) * N * nkx;
  cplx<R> v[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) v[s] = (kx < nkx) ? src[(size_t)(t + s * T) * nkx + kx] : mk<R>(0, 0);
  auto at = [c](int i) -> cplx<R> & { return lds[i * (C + 1) + c]; };
  auto sync = []() { __syncthreads(); };
  fft_pencil<R, N, false>(v, t, tw, at, sync);
  cplx<R> *dst = out + ((size_t)p * N + z) * npen;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int ky = t + s * T;
    if (kx < ycnt[ky]) dst[yoff[ky] + kx] = v[s];
  }
}

template <typename R, int N>
static void fy_launch(hipStream_t s, const void *in, void *out, int nfields, int nkx, const int *ycnt,
                      const int64_t *yoff, int64_t npen, const void *tw) {
  constexpr int C = ColShape<R, N>::C;
  dim3 grid((nkx + C - 1) / C, N, nfields);
  hipLaunchKernelGGL((k_fy<R, N>), grid, dim3(ColShape<R, N>::THREADS), 0, s, (const cplx<R> *)in,
                     (cplx<R> *)out, nkx, ycnt, yoff, npen, (const cplx<R> *)tw);
}

void launch_fy(hipStream_t s, int prec, int N, const void *in, void *out, int nfields, int nkx,
               const int *ycnt, const int64_t *yoff, int64_t npen, const void *tw) {
  if (prec == 0) { PW_DISPATCH_N(fy_launch, float, s, in, out, nfields, nkx, ycnt, yoff, npen, tw) }
  else { PW_DISPATCH_N(fy_launch, double, s, in, out, nfields, nkx, ycnt, yoff, npen, tw) }
}

template <typename R, int N>
__global__ void __launch_bounds__((ColShape<R, N>::THREADS))
k_fz(const cplx<R> *__restrict__ in, cplx<R> *__restrict__ out, int64_t npen,
     const PencilInfo *__restrict__ pinfo, const int64_t *__restrict__ moff, int64_t nmodes,
     const cplx<R> *__restrict__ tw) {
  constexpr int T = ColShape<R, N>::T, C = ColShape<R, N>::C, NT = ColShape<R, N>::THREADS;
  __shared__ cplx<R> lds[N * (C + 1)];
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int64_t q0 = (int64_t)blockIdx.x * C;
  const int64_t q = q0 + c;
  const int p = blockIdx.y;
  const cplx<R> *src = in + (size_t)p * N * npen;
  cplx<R> v[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) v[s] = (q < npen) ? src[(size_t)(t + s * T) * npen + q] : mk<R>(0, 0);
  auto at = [c](int i) -> cplx<R> & { return lds[i * (C + 1) + c]; };
  auto sync = []() { __syncthreads(); };
  fft_pencil<R, N, false>(v, t, tw, at, sync);
#pragma unroll
  for (int s = 0; s < 8; ++s) at(t + s * T) = v[s];
  __syncthreads();
  cplx<R> *dst = out + (size_t)p * nmodes;
  for (int cc = 0; cc < C; ++cc) {
    const int64_t qq = q0 + cc;
    if (qq >= npen) break;
    const int cnt = pinfo[qq].kzcnt;
    const int half = (cnt - 1) / 2;
    const int64_t base = moff[qq];
    for (int j = threadIdx.x; j < cnt; j += NT) {
      const int kz = (cnt == N) ? j : (j <= half ? j : N - (cnt - j));
      dst[base + j] = lds[kz * (C + 1) + cc];
    }
  }
}

template <typename R, int N>
static void fz_launch(hipStream_t s, const void *in, void *out, int nfields, int64_t npen,
                      const PencilInfo *pinfo, const int64_t *moff, int64_t nmodes, const void *tw) {
  constexpr int C = ColShape<R, N>::C;
  dim3 grid((unsigned)((npen + C - 1) / C), nfields);
  hipLaunchKernelGGL((k_fz<R, N>), grid, dim3(ColShape<R, N>::THREADS), 0, s, (const cplx<R> *)in,
                     (cplx<R> *)out, npen, pinfo, moff, nmodes, (const cplx<R> *)tw);
}

void launch_fz(hipStream_t s, int prec, int N, const void *in, void *out, int nfields, int64_t npen,
               const PencilInfo *pinfo, const int64_t *moff, int64_t nmodes, const void *tw) {
  if (prec == 0) { PW_DISPATCH_N(fz_launch, float, s, in, out, nfields, npen, pinfo, moff, nmodes, tw) }
  else { PW_DISPATCH_N(fz_launch, double, s, in, out, nfields, npen, pinfo, moff, nmodes, tw) }
}

// ------------------------------------------------------------------------------ contraction
// One thread per retained mode of the half spectrum (kx in [0, N/2]).  Modes with
// 0 < kx < N/2 stand for themselves and their mirror -k (whose values are the complex
// conjugates, so Re(conj(a) b) is the same); the mirror's direction is that of the signed
// index (-n) mod N, which is -k except on Nyquist planes.
constexpr int kMaxVals = 4096;

template <typename R, int LMAX, int NTH>
__global__ void __launch_bounds__(NTH)
k_contract_bis(const cplx<R> *__restrict__ spec, int nfields, int64_t nmodes,
               const uint32_t *__restrict__ modecoord, int N, const int *__restrict__ bin_of_s2,
               int64_t n_s2, int nbins, int nell, TermTable tab, double kf,
               const R *__restrict__ winv, double *__restrict__ acc) {
  extern __shared__ unsigned char smem_raw[];
  cplx<R> *vals = reinterpret_cast<cplx<R> *>(smem_raw);          // [nfields][NTH]
  double *bacc = reinterpret_cast<double *>(vals + (size_t)nfields * NTH);  // [(nell + 2) * nbins]
  const int nacc = (nell + 2) * nbins;
  for (int i = threadIdx.x; i < nacc; i += NTH) bacc[i] = 0.0;
  __syncthreads();
  const R *coef = reinterpret_cast<const R *>(tab.coef);
  constexpr int NSH = (LMAX + 1) * (LMAX + 1);
  const int half = N / 2;
  for (int64_t base = (int64_t)blockIdx.x * NTH; base < nmodes; base += (int64_t)gridDim.x * NTH) {
    const int64_t mode = base + threadIdx.x;
    const bool live = mode < nmodes;
    __syncthreads();
    for (int p = 0; p < nfields; ++p)
      vals[p * NTH + threadIdx.x] = live ? spec[(size_t)p * nmodes + mode] : mk<R>(0, 0);
    __syncthreads();
    if (!live) continue;
    const uint32_t mc = modecoord[mode];
    const int kx = mc & 0x7ff, ky = (mc >> 11) & 0x7ff, kz = (mc >> 22) & 0x3ff;
    const int sx = (kx == half) ? -half : kx;
    const int sy = (ky < half) ? ky : ky - N;
    const int sz = (kz < half) ? kz : kz - N;
    const int64_t s2 = (int64_t)sx * sx + (int64_t)sy * sy + (int64_t)sz * sz;
    const int b = (s2 < n_s2) ? bin_of_s2[s2] : -1;
    if (b < 0) continue;
    const bool pair = (kx != 0 && kx != half);
    R wdir[NSH];
    {
      R ux = 0, uy = 0, uz = 1;
      if (s2 > 0) {
        const R ir = (R)1 / sqrt((R)s2);
        ux = (R)sx * ir; uy = (R)sy * ir; uz = (R)sz * ir;
      }
      real_sh_even<R, LMAX>(c_sh, ux, uy, uz, wdir);
      if (pair) {
        // mirror: signed index of (-n) mod N on each axis
        const int mx = -sx;
        const int my = (ky == half) ? sy : -sy;
        const int mz = (kz == half) ? sz : -sz;
        R wm[NSH];
        const R ir = (R)1 / sqrt((R)s2);
        real_sh_even<R, LMAX>(c_sh, (R)mx * ir, (R)my * ir, (R)mz * ir, wm);
#pragma unroll
        for (int i = 0; i < NSH; ++i) wdir[i] += wm[i];
      }
    }
    R E[LMAX / 2 + 1];
#pragma unroll
    for (int i = 0; i <= LMAX / 2; ++i) E[i] = 0;
    for (int tg = 0; tg < tab.ntargets; ++tg) {
      R a = 0;
      const int e = tab.tstart[tg + 1];
      for (int q = tab.tstart[tg]; q < e; ++q) {
        const cplx<R> u = vals[tab.p1[q] * NTH + threadIdx.x];
        const cplx<R> w = vals[tab.p2[q] * NTH + threadIdx.x];
        a += coef[q] * (u.x * w.x + u.y * w.y);
      }
      R wd = 0;
      const int sh = tab.tsh[tg];
#pragma unroll
      for (int i = 0; i < NSH; ++i) if (i == sh) wd = wdir[i];
      const int li = tab.tell[tg];
#pragma unroll
      for (int i = 0; i <= LMAX / 2; ++i) if (i == li) E[i] += wd * a;
    }
    if (winv) {
      // assignment-window compensation: every spectrum value is divided by W(k)
      const R iw = winv[kx] * winv[ky] * winv[kz];
      const R iw2 = iw * iw;
#pragma unroll
      for (int i = 0; i <= LMAX / 2; ++i) E[i] *= iw2;
    }
    const double mult = pair ? 2.0 : 1.0;
    for (int i = 0; i < nell; ++i) atomicAdd(&bacc[i * nbins + b], (double)E[i]);
    atomicAdd(&bacc[nell * nbins + b], mult);
    atomicAdd(&bacc[(nell + 1) * nbins + b], mult * kf * sqrt((double)s2));
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nacc; i += NTH)
    if (bacc[i] != 0.0) atomicAdd(&acc[i], bacc[i]);
}

void launch_contract_bis(hipStream_t s, int prec, int lmax, const void *spec, int nfields,
                         int64_t nmodes, const uint32_t *modecoord, int N, const int *bin_of_s2,
                         int64_t n_s2, int nbins, int nell, TermTable tab, double kf,
                         const void *winv, double *acc) {
  int64_t want = (nmodes + 127) / 128;
  unsigned blocks = (unsigned)(want < 2048 ? (want > 0 ? want : 1) : 2048);
#define PW_CONTRACT(R, L, NTH)                                                                     \
  {                                                                                                \
    size_t sh = (size_t)nfields * NTH * sizeof(cplx<R>) + (size_t)(nell + 2) * nbins * sizeof(double); \
    hipLaunchKernelGGL((k_contract_bis<R, L, NTH>), dim3(blocks), dim3(NTH), sh, s,                \
                       (const cplx<R> *)spec, nfields, nmodes, modecoord, N, bin_of_s2, n_s2,      \
                       nbins, nell, tab, kf, (const R *)winv, acc);                                \
  }
  if (prec == 0) {
    switch (lmax) {
      case 0: PW_CONTRACT(float, 0, 128) break;
      case 2: PW_CONTRACT(float, 2, 128) break;
      case 4: PW_CONTRACT(float, 4, 128) break;
      case 6: PW_CONTRACT(float, 6, 128) break;
      default: PW_CONTRACT(float, 8, 128) break;
    }
  } else {
    switch (lmax) {
      case 0: PW_CONTRACT(double, 0, 64) break;
      case 2: PW_CONTRACT(double, 2, 64) break;
      case 4: PW_CONTRACT(double, 4, 64) break;
      case 6: PW_CONTRACT(double, 6, 64) break;
      default: PW_CONTRACT(double, 8, 64) break;
    }
  }
#undef PW_CONTRACT
}

// ------------------------------------------------------------------------------ finalize
__global__ void k_finalize_pk(const double *acc, int nell, int nbins, const int *ells,
                              const DevNorm *norm, double *out) {
  const double fourpi = 12.566370614359172953850573533118;
  const double I = norm->I, S = norm->S;
  for (int i = threadIdx.x; i < (nell + 1) * nbins; i += blockDim.x) {
    const int l = i / nbins, b = i % nbins;
    const double cnt = acc[nell * nbins + b];
    if (l < nell) {
      double v = (cnt > 0) ? fourpi / I * acc[l * nbins + b] / cnt : 0.0;
      if (ells[l] == 0 && cnt > 0) v -= S / I;
      out[l * nbins + b] = v;
    } else {
      out[nell * nbins + b] = (cnt > 0) ? acc[(nell + 1) * nbins + b] / cnt : 0.0;  // mean |k|
      out[(nell + 1) * nbins + b] = cnt;
    }
  }
}

void launch_finalize_pk(hipStream_t s, const double *acc, int nell, int nbins, const int *ells,
                        const DevNorm *norm, double *out) {
  hipLaunchKernelGGL(k_finalize_pk, dim3(1), dim3(256), 0, s, acc, nell, nbins, ells, norm, out);
}

}  // namespace pw
