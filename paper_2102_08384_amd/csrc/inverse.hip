// HIP kernels of the inverse-transform paths (gfx950, wave64).
//
//   iz             inverse FFT along z of full pencil-major spectra (bisector xi_l targets);
//                  output pruned to the retained z planes
//   fziz           midpoint g fields: forward FFT along z, the product conj(D) Q / W^2
//                  (Section 3.2) and the inverse FFT along z in one pass over each pencil
//   ix             complex-to-real inverse FFT along x of field pairs; either stores the real
//                  fields or, for xi_l, weights them by |D|^alpha y_J^mu(D^) times the per-field
//                  multipole coefficient and bins the sums into r-shells in FP64
//                  (Section 4.3 midpoint estimator, Section 6 bisector estimator)
//   contract_mid   midpoint P_l contraction sum_nu y_l^nu(k^) Re[G + A] (Section 3.3 boxed
//                  estimator in the real-harmonic basis) with FP64 shell sums
//   finalize_xi    xi_l = (4 pi / I) sum / (N_a H^3)
#include "kernels.h"

#include <type_traits>

#include "dev_core.h"

namespace pw {

__constant__ ShConst c_sh_inv;

void upload_sh_const_inverse(const ShConst &c) {
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_sh_inv), &c, sizeof(ShConst));
}

// ------------------------------------------------------------------------------ iz
template <typename R, int N, bool REAL_IN>

__global__ void __launch_bounds__((ColShape<R, N>::THREADS))
k_iz(cplx<R> *in, const R *in_real, cplx<R> *__restrict__ out, int nfields, int n_inplace, int64_t npen,
     int nkx, int rs, const cplx<R> *D, R d_scale, const R *__restrict__ winv, const int *__restrict__ zrank, int nz,
     const cplx<R> *__restrict__ tw) {
  constexpr int T = ColShape<R, N>::T, C = ColShape<R, N>::C, NT = ColShape<R, N>::THREADS;
  constexpr int LOGN = log2i(N);
  __shared__ cplx<R> lds[N * (C + 1)];
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int64_t q0 = (int64_t)blockIdx.x * C;
  const int64_t q = q0 + c;
  const int64_t left = npen - q0;
  const int nval = (int)((left < C ? left : C) * N);  // valid values of this block's chunk
  auto at = [c](int i) -> cplx<R> & { return lds[i * (C + 1) + c]; };
  auto sync = []() { __syncthreads(); };
  FftTw<R, N> twr;
  twr.load(t, tw);
  wait_vmem();
  const size_t fstride = (size_t)npen * N;
  // the chunk of pencils q0 .. q0 + C - 1 is contiguous: element e = cc * N + kz
  auto load_chunk = [&](const cplx<R> *src) {
    for (int e = threadIdx.x; e < C * N; e += NT) {
      const int cc = e >> LOGN, kz = e & (N - 1);
      lds[kz * (C + 1) + cc] = (e < nval) ? src[(size_t)q0 * N + e] : mk<R>(0, 0);
    }
  };
  // full retention: pencil q = ky * rs + kx (kx >= nkx: all-zero padding pencils)
  const int qky = (int)(q / rs), qkx = (int)(q - (int64_t)qky * rs);
  const int64_t qo = q;
  const int64_t plane_o = npen;
  cplx<R> dv[8];
  if (!REAL_IN && D) {
    load_chunk(D);
    sync();
    R iwxy = (R)1;
    if (winv && q < npen) iwxy = winv[qkx] * winv[qky];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int kz = t + s * T;
      R f = d_scale;
      if (winv) {
        const R iw = iwxy * winv[kz];
        f *= iw * iw;
      }
      const cplx<R> d = at(kz);
      dv[s] = mk<R>(d.x * f, -d.y * f);
    }
    sync();
  }
  // each field's chunk: PER values per thread, loaded together into registers, then placed in
  // LDS; real inputs (held as reals: half the registers) load the next field's chunk while the
  // current one is transformed
  constexpr int PER = C * N / NT;
  typedef typename std::conditional<REAL_IN, R, cplx<R>>::type In;
  auto fetch = [&](int p, In *x) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = threadIdx.x + k * NT;
      if constexpr (REAL_IN) {
        const R *src = in_real + (size_t)p * fstride;
        x[k] = (e < nval) ? src[(size_t)q0 * N + e] : (R)0;
      } else {
        const cplx<R> *src = in + (size_t)p * fstride;
        x[k] = (e < nval) ? src[(size_t)q0 * N + e] : mk<R>(0, 0);
      }
    }
  };
  // output plane of every kz (-1: not kept), read once into LDS
  __shared__ int zsh[N];
  for (int i = threadIdx.x; i < N; i += NT) zsh[i] = zrank[i];
  In xb[PER];
  if constexpr (REAL_IN) {
    if (nfields > 0) fetch(0, xb);
  }
  for (int p = 0; p < nfields; ++p) {
    if constexpr (!REAL_IN) fetch(p, xb);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = threadIdx.x + k * NT;
      if constexpr (REAL_IN) lds[(e & (N - 1)) * (C + 1) + (e >> LOGN)] = mk<R>(xb[k], (R)0);
      else lds[(e & (N - 1)) * (C + 1) + (e >> LOGN)] = xb[k];
    }
    sync();
    cplx<R> v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = at(t + s * T);
    if (!REAL_IN && D) {
#pragma unroll
      for (int s = 0; s < 8; ++s) v[s] = cmul(dv[s], v[s]);
    }
    sync();
    if constexpr (REAL_IN) {
      if (p + 1 < nfields) fetch(p + 1, xb);
    }
    if (p < n_inplace) {
      // the product stays in k-space: store it back in place, coalesced through LDS
#pragma unroll
      for (int s = 0; s < 8; ++s) at(t + s * T) = v[s];
      sync();
      cplx<R> *dst = in + (size_t)p * fstride;
      for (int e = threadIdx.x; e < nval; e += NT) {
        const int cc = e >> LOGN, kz = e & (N - 1);
        dst[(size_t)q0 * N + e] = lds[kz * (C + 1) + cc];
      }
      sync();
      continue;
    }
    fft_pencil<R, N, true>(v, t, twr, at, sync);
    if (q < npen) {
      cplx<R> *dst = out + (size_t)(p - n_inplace) * nz * plane_o;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int zr = zsh[t + s * T];
        if (zr >= 0) dst[(size_t)zr * plane_o + qo] = v[s];
      }
    }
  }
}

template <typename R, int N>
static void iz_launch(hipStream_t s, void *in, void *out, int nfields, int n_inplace, int real_in, int64_t npen,
                      int nkx, int rs, const void *D, double d_scale, const void *winv, const int *zrank, int nz,
                      const void *tw) {
  constexpr int C = ColShape<R, N>::C;
  dim3 grid((unsigned)((npen + C - 1) / C));
  if (real_in)
    hipLaunchKernelGGL((k_iz<R, N, true>), grid, dim3(ColShape<R, N>::THREADS), 0, s, (cplx<R> *)nullptr,
                       (const R *)in, (cplx<R> *)out, nfields, n_inplace, npen, nkx, rs, (const cplx<R> *)D,
                       (R)d_scale, (const R *)winv, zrank, nz, (const cplx<R> *)tw);
  else
    hipLaunchKernelGGL((k_iz<R, N, false>), grid, dim3(ColShape<R, N>::THREADS), 0, s, (cplx<R> *)in,
                       (const R *)nullptr, (cplx<R> *)out, nfields, n_inplace, npen, nkx, rs, (const cplx<R> *)D,
                       (R)d_scale, (const R *)winv, zrank, nz, (const cplx<R> *)tw);
}

void launch_iz(hipStream_t s, int prec, int N, void *in, void *out, int nfields, int n_inplace, int real_in,
               int64_t npen, int nkx, int rs, const void *D, double d_scale, const void *winv, const int *zrank,
               int nz, const void *tw) {
  if (nfields <= 0 || npen <= 0) return;
  if (prec == 0) {
    PW_DISPATCH_N(iz_launch, float, s, in, out, nfields, n_inplace, real_in, npen, nkx, rs, D, d_scale, winv,
                  zrank, nz, tw)
  } else {
    PW_DISPATCH_N(iz_launch, double, s, in, out, nfields, n_inplace, real_in, npen, nkx, rs, D, d_scale, winv,
                  zrank, nz, tw)
  }
}

// ------------------------------------------------------------------------------ fziz
// Midpoint g fields (Section 3.2): the forward z pass, the product conj(D) Q / W^2 and the
// inverse z pass all act along one pencil (kx, ky), so one kernel does the three and the full
// spectra never go through HBM.  Input: the y-pass output of full sets, [field][z][pencil q]
// (q = ky * rs + kx, every pencil N long; pencils kx >= nkx are zero padding).  Field 0 is
// Q_{0,0,0}; D = d_scale * its transform.  Fields p < n_inplace keep the product in k-space,
// pencil-major at prod[p][q * N + kz]; the others go back to z and leave the retained planes
// at out[p - n_inplace][zrank[z]][q].  A block owns C adjacent pencils and one group of fields
// [p0, p1); it transforms field 0 first (every group does) and prefetches the next field's
// loads across each transform.  conj(D) / W^2 waits in LDS (each lane its own 8 values), which
// keeps the N = 512 FP32 form within 128 VGPRs.  Loads and the z-side stores are raw buffer
// accesses whose per-lane offsets (empty planes, padding pencils and planes outside the
// r-bins masked out) are fixed for the whole kernel, so the per-field work is the transforms.
template <typename R, int N>
__global__ void __launch_bounds__((ColShape<R, N>::THREADS))
k_fziz(const cplx<R> *__restrict__ in, cplx<R> *__restrict__ prod, cplx<R> *__restrict__ out, int nfields,
       int n_inplace, int fpb, int64_t npen, int rs, R d_scale, const R *__restrict__ winv,
       const int *__restrict__ zrank, int nz, const cplx<R> *__restrict__ tw, const int *__restrict__ planemask) {
  constexpr int T = ColShape<R, N>::T, C = ColShape<R, N>::C, NT = ColShape<R, N>::THREADS;
  constexpr int LOGN = log2i(N);
  constexpr int64_t E = sizeof(cplx<R>);
  __shared__ cplx<R> lds[N * (C + 1)];
  __shared__ cplx<R> dls[8 * NT];
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int64_t q0 = (int64_t)blockIdx.x * C;
  const int64_t q = q0 + c;
  const int p0 = blockIdx.y * fpb;
  const int p1 = min(nfields, p0 + fpb);
  if (p0 >= p1) return;  // uniform
  FftTw<R, N> twr;
  twr.load(t, tw);
  const bool has = q < npen;
  // byte offsets: input plane z = t + s T of pencil q sits at lo[s] + s * sT in its field, and
  // the output row of a retained plane z at zo[s] in its output field
  const uint32_t sT = (uint32_t)(T * npen * E);
  const uint32_t lane_in = (uint32_t)((t * npen + q) * E);
  // wave-uniform bit s of wload / wstore: some lane of the wave loads / stores plane t + s T (a
  // wave spans 4 adjacent planes, so empty planes and planes outside the r-bins skip whole
  // instructions, not only lanes)
  uint32_t lo[8], zo[8], wload = 0, wstore = 0;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int z = t + s * T;
    lo[s] = (has && (!planemask || planemask[z])) ? lane_in : kOob;
    const int zr = zrank ? zrank[z] : -1;
    zo[s] = (has && zr >= 0) ? (uint32_t)((zr * npen + q) * E) : kOob;
    if (__builtin_amdgcn_ballot_w64(lo[s] != kOob)) wload |= 1u << s;
    if (__builtin_amdgcn_ballot_w64(zo[s] != kOob)) wstore |= 1u << s;
  }
  const uint32_t in_bytes = (uint32_t)(N * npen * E);
  const uint32_t out_bytes = (uint32_t)(nz * npen * E);
  R iwxy = (R)1;
  if (winv && has) {
    const int qky = (int)(q / rs), qkx = (int)(q - (int64_t)qky * rs);
    iwxy = winv[qkx] * winv[qky];
  }
  wait_vmem();
  auto load = [&](int p, cplx<R> *v) {
    const __amdgpu_buffer_rsrc_t r = buf_rsrc(in + (size_t)p * N * npen, in_bytes);
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = (wload >> s & 1) ? buf_load<R>(r, lo[s], (uint32_t)s * sT) : mk<R>(0, 0);
  };
  auto at = [c](int i) -> cplx<R> & { return lds[i * (C + 1) + c]; };
  auto sync = []() { __syncthreads(); };
  cplx<R> nxt[8];
  const int pf = p0 > 0 ? p0 : 1;  // first field after D's own
  // field p's product (in v, kz = t + s T): stored in k-space, or transformed back to z
  auto finish = [&](int p, cplx<R> *v) {
    if (p < n_inplace) {
      // stays in k-space: pencil-major, coalesced through LDS
#pragma unroll
      for (int s = 0; s < 8; ++s) at(t + s * T) = v[s];
      __syncthreads();
      cplx<R> *dst = prod + (size_t)p * npen * N + (size_t)q0 * N;
      const int nval = (int)(((npen - q0) < C ? (npen - q0) : C) * N);
      for (int e = threadIdx.x; e < nval; e += NT) {
        const int cc = e >> LOGN, kz = e & (N - 1);
        dst[e] = lds[kz * (C + 1) + cc];
      }
      __syncthreads();
    } else {
      fft_pencil<R, N, true>(v, t, twr, at, sync);
      const __amdgpu_buffer_rsrc_t r = buf_rsrc(out + (size_t)(p - n_inplace) * nz * npen, out_bytes);
#pragma unroll
      for (int s = 0; s < 8; ++s)
        if (wstore >> s & 1) buf_store<R>(v[s], r, zo[s], 0);
    }
  };
  // conj(D) / W^2 on every mode, D = d_scale Q_000~; field 0's own product is then
  // d_scale |Q_000~|^2 / W^2
  {
    cplx<R> d[8], v[8];
    load(0, d);
    if (pf < p1) load(pf, nxt);
    fft_pencil<R, N, false>(d, t, twr, at, sync);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const R iw = iwxy * (winv ? winv[t + s * T] : (R)1);
      const R f = d_scale * iw * iw;
      v[s] = mk<R>(f * (d[s].x * d[s].x + d[s].y * d[s].y), (R)0);
      dls[s * NT + threadIdx.x] = mk<R>(d[s].x * f, -d[s].y * f);
    }
    if (p0 == 0) finish(0, v);
  }
  for (int p = pf; p < p1; ++p) {
    cplx<R> v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = nxt[s];
    if (p + 1 < p1) load(p + 1, nxt);
    fft_pencil<R, N, false>(v, t, twr, at, sync);
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = cmul(dls[s * NT + threadIdx.x], v[s]);
    finish(p, v);
  }
}

template <typename R, int N>
static void fziz_launch(hipStream_t s, const void *in, void *prod, void *out, int nfields, int n_inplace,
                        int64_t npen, int rs, double d_scale, const void *winv, const int *zrank, int nz,
                        const void *tw, const int *planemask, ColTune tune) {
  constexpr int C = ColShape<R, N>::C;
  const unsigned ng = (unsigned)((npen + C - 1) / C);
  int fpb = tune.fpb;
  if (fpb <= 0) {
    // field groups fill the chip on small meshes; each group transforms D again, so keep >= 8
    // fields per group
    int G = field_groups(nfields, (int)std::min<int64_t>(ng, 1 << 20));
    G = std::max(1, std::min(G, nfields / 8));
    fpb = (nfields + G - 1) / G;
  }
  fpb = std::min(fpb, nfields);
  dim3 grid(ng, (nfields + fpb - 1) / fpb);
  hipLaunchKernelGGL((k_fziz<R, N>), grid, dim3(ColShape<R, N>::THREADS), 0, s, (const cplx<R> *)in,
                     (cplx<R> *)prod, (cplx<R> *)out, nfields, n_inplace, fpb, npen, rs, (R)d_scale,
                     (const R *)winv, zrank, nz, (const cplx<R> *)tw, planemask);
}

void launch_fziz(hipStream_t s, int prec, int N, const void *in, void *prod, void *out, int nfields, int n_inplace,
                 int64_t npen, int rs, double d_scale, const void *winv, const int *zrank, int nz, const void *tw,
                 const int *planemask, ColTune tune) {
  if (nfields <= 0 || npen <= 0) return;
  if (prec == 0) {
    PW_DISPATCH_N(fziz_launch, float, s, in, prod, out, nfields, n_inplace, npen, rs, d_scale, winv, zrank, nz,
                  tw, planemask, tune)
  } else {
    PW_DISPATCH_N(fziz_launch, double, s, in, prod, out, nfields, n_inplace, npen, rs, d_scale, winv, zrank, nz,
                  tw, planemask, tune)
  }
}

// ------------------------------------------------------------------------------ ix
constexpr int kMaxEll = 5;  // multipoles 0, 2, .., 8

template <typename R, int N, int MODE>
__global__ void __launch_bounds__(FxShape<N>::THREADS)
k_ix(const cplx<R> *__restrict__ in, R *__restrict__ out, int rs, const FieldJob *__restrict__ jobs, int njobs,
     const R *__restrict__ coef, int nell, int nz, int ny, const int *__restrict__ zidx,
     const int *__restrict__ yidx, R Hu, double Hd, R scale, const int *__restrict__ bin_of_s2, int64_t n_s2,
     int nbins, double *__restrict__ acc, const cplx<R> *__restrict__ tw) {
  constexpr int T = FxShape<N>::T, ROWS = FxShape<N>::ROWS, NKX = N / 2 + 1;
  constexpr int LN = N + N / 8;
  __shared__ cplx<R> lds[ROWS * LN];
  extern __shared__ double bacc[];  // mode 1: (nell + 2) * nbins
  const int rl = threadIdx.x / T, t = threadIdx.x % T;
  const int64_t nrows = (int64_t)nz * ny;
  const int64_t row = (int64_t)blockIdx.x * ROWS + rl;
  const bool live = row < nrows;
  const int zr = live ? (int)(row / ny) : 0, yr = live ? (int)(row - (int64_t)zr * ny) : 0;
  const int z = zidx[zr], y = yidx[yr];
  cplx<R> *my = lds + rl * LN;
  auto at = [my](int i) -> cplx<R> & { return my[i + (i >> 3)]; };
  auto sync = []() { __syncthreads(); };
  const int sy = y < N / 2 ? y : y - N, sz = z < N / 2 ? z : z - N;


  // mode 1 geometry of the eight cells this lane holds
  R ux[8], uy[8], uz[8], dm[8];
  int bin[8];
  R X[kMaxEll][8];
  if constexpr (MODE == 1) {
    const int nacc = (nell + 2) * nbins;
    for (int i = threadIdx.x; i < nacc; i += blockDim.x) bacc[i] = 0.0;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int x = t + s * T;
      const int sx = x < N / 2 ? x : x - N;
      const int64_t s2 = (int64_t)sx * sx + (int64_t)sy * sy + (int64_t)sz * sz;
      bin[s] = (live && s2 < n_s2) ? bin_of_s2[s2] : -1;
      dm[s] = Hu * sqrt((R)s2);  // |D| / unit
      if (s2 > 0) {
        const R ir = (R)1 / sqrt((R)s2);
        ux[s] = (R)sx * ir; uy[s] = (R)sy * ir; uz[s] = (R)sz * ir;
      } else {
        ux[s] = 0; uy[s] = 0; uz[s] = 1;
      }
#pragma unroll
      for (int l = 0; l < kMaxEll; ++l) X[l][s] = 0;
    }
  }
  ShRec8<R> rec;
  rec.init();
  const size_t fstride = (size_t)nrows * rs;  // rows padded to rs
  for (int jb = 0; jb < njobs; ++jb) {
    const FieldJob J = jobs[jb];
    const cplx<R> *ha = in + (size_t)J.pa * fstride + (size_t)row * rs;
    const cplx<R> *hb = in + (size_t)(J.pb < 0 ? 0 : J.pb) * fstride + (size_t)row * rs;
    // Z = Ha + i Hb on the full x range from the half spectra (Ha(-k) = conj Ha(k) after the
    // y and z inverse passes of a real field); the self-conjugate kx = 0, N/2 keep real parts.
    for (int kx = t; kx < NKX; kx += T) {
      const cplx<R> a = live ? ha[kx] : mk<R>(0, 0);
      const cplx<R> b = (live && J.pb >= 0) ? hb[kx] : mk<R>(0, 0);
      if (kx == 0 || kx == N / 2) {
        at(kx) = mk<R>(a.x, b.x);
      } else {
        at(kx) = mk<R>(a.x - b.y, a.y + b.x);
        at(N - kx) = mk<R>(a.x + b.y, b.x - a.y);
      }
    }
    sync();
    cplx<R> v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = at(t + s * T);
    sync();
    fft_pencil<R, N, true>(v, t, tw, at, sync);
    if constexpr (MODE == 0) {
      if (live) {
        R *oa = out + (size_t)J.pa * N * N * N + ((size_t)z * N + y) * N;
        R *ob = out + (size_t)(J.pb < 0 ? 0 : J.pb) * N * N * N + ((size_t)z * N + y) * N;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          oa[t + s * T] = v[s].x * scale;
          if (J.pb >= 0) ob[t + s * T] = v[s].y * scale;
        }
      }
    } else {
      R ya[8], yb[8];
      if (J.kind == 0) {
        rec.set_m(J.m, ux, uy);
        rec.advance(c_sh_inv, J.Ja, uz);
        const R n = sh_n<R>(c_sh_inv, J.Ja, J.m);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          R w = n * rec.q0[s];
          for (int a = 0; a < J.alpha; ++a) w *= dm[s];
          ya[s] = w * rec.cr[s];
          yb[s] = w * rec.ci[s];
        }
      } else {
        rec.set_m(0, ux, uy);
        rec.advance(c_sh_inv, J.Ja, uz);
        const R na = sh_n<R>(c_sh_inv, J.Ja, 0);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          R w = na * rec.q0[s];
          for (int a = 0; a < J.alpha; ++a) w *= dm[s];
          ya[s] = w;
          yb[s] = 0;
        }
        if (J.Jb >= 0) {
          rec.advance(c_sh_inv, J.Jb, uz);
          const R nb = sh_n<R>(c_sh_inv, J.Jb, 0);
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            R w = nb * rec.q0[s];
            for (int a = 0; a < J.alpha_b; ++a) w *= dm[s];
            yb[s] = w;
          }
        }
      }
      const R *ca = coef + (size_t)jb * 2 * nell, *cb = ca + nell;
#pragma unroll
      for (int l = 0; l < kMaxEll; ++l) {
        if (l < nell) {
          const R fa = ca[l], fb = cb[l];
#pragma unroll
          for (int s = 0; s < 8; ++s) X[l][s] += fa * ya[s] * v[s].x + fb * yb[s] * v[s].y;
        }
      }
    }
  }
  if constexpr (MODE == 1) {
    sync();  // bacc cleared by every thread before any accumulation
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int b = bin[s];
      if (b < 0) continue;
      const int x = t + s * T;
      const int sx = x < N / 2 ? x : x - N;
      const double s2 = (double)sx * sx + (double)sy * sy + (double)sz * sz;
#pragma unroll
      for (int l = 0; l < kMaxEll; ++l)
        if (l < nell) atomicAdd(&bacc[l * nbins + b], (double)(X[l][s] * scale));
      atomicAdd(&bacc[nell * nbins + b], 1.0);
      atomicAdd(&bacc[(nell + 1) * nbins + b], Hd * sqrt(s2));
    }
    sync();
    const int nacc = (nell + 2) * nbins;
    for (int i = threadIdx.x; i < nacc; i += blockDim.x)
      if (bacc[i] != 0.0) atomicAdd(&acc[i], bacc[i]);
  }
}

template <typename R, int N>
static void ix_launch(hipStream_t s, int mode, const void *in, void *out, int rs, const FieldJob *jobs, int njobs,
                      const void *coef, int nell, int nz, int ny, const int *zidx, const int *yidx, double H,
                      double unit, double scale, const int *bin_of_s2, int64_t n_s2, int nbins, double *acc,
                      const void *tw) {
  constexpr int ROWS = FxShape<N>::ROWS;
  const int64_t nrows = (int64_t)nz * ny;
  dim3 grid((unsigned)((nrows + ROWS - 1) / ROWS));
  if (mode == 0) {
    hipLaunchKernelGGL((k_ix<R, N, 0>), grid, dim3(FxShape<N>::THREADS), 0, s, (const cplx<R> *)in, (R *)out,
                       rs, jobs, njobs, (const R *)coef, nell, nz, ny, zidx, yidx, (R)(H / unit), H, (R)scale, bin_of_s2,
                       n_s2, nbins, acc, (const cplx<R> *)tw);
  } else {
    size_t sh = (size_t)(nell + 2) * nbins * sizeof(double);
    hipLaunchKernelGGL((k_ix<R, N, 1>), grid, dim3(FxShape<N>::THREADS), sh, s, (const cplx<R> *)in, (R *)out,
                       rs, jobs, njobs, (const R *)coef, nell, nz, ny, zidx, yidx, (R)(H / unit), H, (R)scale, bin_of_s2,
                       n_s2, nbins, acc, (const cplx<R> *)tw);
  }
}

void launch_ix(hipStream_t s, int prec, int N, int mode, const void *in, void *out, int rs, const FieldJob *jobs,
               int njobs, const void *coef, int nell, int nz, int ny, const int *zidx, const int *yidx, double H,
               double unit, double scale, const int *bin_of_s2, int64_t n_s2, int nbins, double *acc,
               const void *tw) {
  if (njobs <= 0 || nz <= 0 || ny <= 0 || nell > kMaxEll) return;
  if (prec == 0) {
    PW_DISPATCH_N(ix_launch, float, s, mode, in, out, rs, jobs, njobs, coef, nell, nz, ny, zidx, yidx, H, unit, scale,
                  bin_of_s2, n_s2, nbins, acc, tw)
  } else {
    PW_DISPATCH_N(ix_launch, double, s, mode, in, out, rs, jobs, njobs, coef, nell, nz, ny, zidx, yidx, H, unit, scale,
                  bin_of_s2, n_s2, nbins, acc, tw)
  }
}

// ------------------------------------------------------------------------------ contract_mid
// One thread per retained mode of the half spectrum; a mode with 0 < kx < N/2 also stands for
// its mirror (conjugate values, same real parts) whose direction is that of (-n) mod N.
template <typename R, int LMAX>
__global__ void __launch_bounds__(256)
k_contract_mid(const cplx<R> *__restrict__ G, int rs_full, const cplx<R> *__restrict__ A, int64_t nmodes,
               int64_t mstride,
               const uint32_t *__restrict__ modecoord, int N, const int *__restrict__ bin_of_s2, int64_t n_s2,
               int nbins, double kf, double *__restrict__ acc) {
  constexpr int NSH = (LMAX + 1) * (LMAX + 1);
  constexpr int NE = LMAX / 2 + 1;
  extern __shared__ double bacc[];
  const int nacc = (NE + 2) * nbins;
  for (int i = threadIdx.x; i < nacc; i += blockDim.x) bacc[i] = 0.0;
  __syncthreads();
  const int half = N / 2;
  const size_t gstride = (size_t)N * rs_full * N;
  for (int64_t mode = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; mode < nmodes;
       mode += (int64_t)gridDim.x * blockDim.x) {
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
#pragma unroll
    for (int i = 0; i < NSH; ++i) wdir[i] = 0;
    {
      R ux = 0, uy = 0, uz = 1;
      const R ir = s2 > 0 ? (R)1 / sqrt((R)s2) : (R)0;
      if (s2 > 0) { ux = (R)sx * ir; uy = (R)sy * ir; uz = (R)sz * ir; }
      real_sh_even<R, LMAX>(c_sh_inv, ux, uy, uz, wdir);
      if (pair) {
        const int my = (ky == half) ? sy : -sy;
        const int mz = (kz == half) ? sz : -sz;
        R wm[NSH];
#pragma unroll
        for (int i = 0; i < NSH; ++i) wm[i] = 0;
        real_sh_even<R, LMAX>(c_sh_inv, (R)(-sx) * ir, (R)my * ir, (R)mz * ir, wm);
#pragma unroll
        for (int i = 0; i < NSH; ++i) wdir[i] += wm[i];
      }
    }
    const size_t gi = ((size_t)ky * rs_full + kx) * N + kz;
    R E[NE];
#pragma unroll
    for (int l = 0, o = 0; l <= LMAX; l += 2) {
      R e = 0;
#pragma unroll
      for (int nu = -l; nu <= l; ++nu, ++o) {
        R v = G[(size_t)o * gstride + gi].x;
        if (l >= 2 && A) v += A[(size_t)(o - 1) * mstride + mode].x;
        e += wdir[l * l + l + nu] * v;
      }
      E[l / 2] = e;
    }
    const double mult = pair ? 2.0 : 1.0;
#pragma unroll
    for (int i = 0; i < NE; ++i) atomicAdd(&bacc[i * nbins + b], (double)E[i]);
    atomicAdd(&bacc[NE * nbins + b], mult);
    atomicAdd(&bacc[(NE + 1) * nbins + b], mult * kf * sqrt((double)s2));
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nacc; i += blockDim.x)
    if (bacc[i] != 0.0) atomicAdd(&acc[i], bacc[i]);
}

void launch_contract_mid(hipStream_t s, int prec, int lmax, const void *G, int rs_full, const void *A,
                         int64_t nmodes, int64_t mstride, const uint32_t *modecoord, int N, const int *bin_of_s2, int64_t n_s2,
                         int nbins, double kf, double *acc) {
  if (nmodes <= 0) return;
  int64_t want = (nmodes + 255) / 256;
  unsigned blocks = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
  size_t sh = (size_t)(lmax / 2 + 3) * nbins * sizeof(double);
#define PW_CM(R, L)                                                                                \
  hipLaunchKernelGGL((k_contract_mid<R, L>), dim3(blocks), dim3(256), sh, s, (const cplx<R> *)G, rs_full, \
                     (const cplx<R> *)A, nmodes, mstride, modecoord, N, bin_of_s2, n_s2, nbins, kf, acc);
  if (prec == 0) {
    switch (lmax) {
      case 0: PW_CM(float, 0) break;
      case 2: PW_CM(float, 2) break;
      case 4: PW_CM(float, 4) break;
      case 6: PW_CM(float, 6) break;
      default: PW_CM(float, 8) break;
    }
  } else {
    switch (lmax) {
      case 0: PW_CM(double, 0) break;
      case 2: PW_CM(double, 2) break;
      case 4: PW_CM(double, 4) break;
      case 6: PW_CM(double, 6) break;
      default: PW_CM(double, 8) break;
    }
  }
#undef PW_CM
}

// ------------------------------------------------------------------------------ finalize_xi
__global__ void k_finalize_xi(const double *acc, int nell, int nbins, double cell_volume, const DevNorm *norm,
                              double *out) {
  const double fourpi = 12.566370614359172953850573533118;
  const double I = norm->I;
  for (int i = threadIdx.x; i < (nell + 1) * nbins; i += blockDim.x) {
    const int l = i / nbins, b = i % nbins;
    const double cnt = acc[nell * nbins + b];
    if (l < nell) {
      out[l * nbins + b] = (cnt > 0) ? fourpi / I * acc[l * nbins + b] / (cnt * cell_volume) : 0.0;
    } else {
      out[nell * nbins + b] = (cnt > 0) ? acc[(nell + 1) * nbins + b] / cnt : 0.0;  // mean |D|
      out[(nell + 1) * nbins + b] = cnt;
    }
  }
}

void launch_finalize_xi(hipStream_t s, const double *acc, int nell, int nbins, double cell_volume,
                        const DevNorm *norm, double *out) {
  hipLaunchKernelGGL(k_finalize_xi, dim3(1), dim3(256), 0, s, acc, nell, nbins, cell_volume, norm, out);
}

}  // namespace pw
