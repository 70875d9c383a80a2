// HIP kernels whose couplings are straight-line code generated at build time from the FP64
// host coefficient generator (contract_gen.inc):
//   contract_bis_reg  bisector P_l contraction with every field value of a mode in VGPRs
//                     (Section 5.2 boxed estimator, real-harmonic basis)
//   targets           bisector xi_l per-mode targets T_{l nu} (Section 6 boxed estimator)
//   reweight          midpoint A_{l nu}(D) = sum Phi' y(D^) |D|^alpha g (Section 3.3, Appendix D)
#include "kernels.h"

#include "dev_core.h"

namespace pw {

__constant__ ShConst c_sh_gen;

void upload_sh_const_generated(const ShConst &c) {
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_sh_gen), &c, sizeof(ShConst));
}

template <int L, int B, typename R> struct BisContract {
  static constexpr bool kGenerated = false;
};
template <int L, int K, typename R> struct MidReweight {
  static constexpr bool kGenerated = false;
};
template <int L, int K, typename R> struct MidReweightAll {
  static constexpr bool kGenerated = false;
};
#include "contract_gen.inc"

// Register-resident variant: the coupling for (LMAX, BMAX) is straight-line code generated at
// build time (BisContract<L, B, R>::run), so all field values of a mode stay in VGPRs.  With
// ORD the terms of each order beta go to accumulators of their own (run_orders): rows
// beta * (LMAX/2 + 1) + l/2, then the mode count and the |k| sum.

template <typename R, int LMAX, int BMAX, bool ORD>
__global__ void __launch_bounds__(256)
k_contract_bis_reg(const cplx<R> *__restrict__ spec, int64_t nmodes, int64_t mstride,
                   const uint32_t *__restrict__ modecoord,
                   int N, const int *__restrict__ bin_of_s2, int64_t n_s2, int nbins, double kf,
                   const R *__restrict__ winv, double *__restrict__ acc, const Batch ba) {
  using CT = BisContract<LMAX, BMAX, R>;
  if (ba.n) {  // catalog blockIdx.z of a batch
    const BatchSlot &bs = ba.s[blockIdx.z];
    spec = (const cplx<R> *)bs.A;
    acc = bs.acc;
  }
  constexpr int NF = CT::NF;
  constexpr int NSH = (LMAX + 1) * (LMAX + 1);
  constexpr int NE = ORD ? CT::NO * (LMAX / 2 + 1) : LMAX / 2 + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *bacc = reinterpret_cast<double *>(smem_raw);
  const int nacc = (NE + 2) * nbins;
  for (int i = threadIdx.x; i < nacc; i += blockDim.x) bacc[i] = 0.0;
  __syncthreads();
  const int half = N / 2;
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
    cplx<R> a[NF];
#pragma unroll
    for (int p = 0; p < NF; ++p) a[p] = spec[(size_t)p * mstride + mode];
    const bool pair = (kx != 0 && kx != half);
    R wdir[NSH];
#pragma unroll
    for (int i = 0; i < NSH; ++i) wdir[i] = 0;
    {
      R ux = 0, uy = 0, uz = 1;
      const R ir = s2 > 0 ? (R)1 / sqrt((R)s2) : (R)0;
      if (s2 > 0) { ux = (R)sx * ir; uy = (R)sy * ir; uz = (R)sz * ir; }
      real_sh_even<R, LMAX>(c_sh_gen, ux, uy, uz, wdir);
      if (pair) {
        const int my = (ky == half) ? sy : -sy;
        const int mz = (kz == half) ? sz : -sz;
        R wm[NSH];
#pragma unroll
        for (int i = 0; i < NSH; ++i) wm[i] = 0;
        real_sh_even<R, LMAX>(c_sh_gen, (R)(-sx) * ir, (R)my * ir, (R)mz * ir, wm);
#pragma unroll
        for (int i = 0; i < NSH; ++i) wdir[i] += wm[i];
      }
    }
    R E[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) E[i] = 0;
    if constexpr (ORD) CT::run_orders(a, wdir, E);
    else CT::run(a, wdir, E);
    if (winv) {
      const R iw = winv[kx] * winv[ky] * winv[kz];
      const R iw2 = iw * iw;
#pragma unroll
      for (int i = 0; i < NE; ++i) E[i] *= iw2;
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

template <typename R, int L, int B>
static bool contract_reg_launch(hipStream_t s, const void *spec, int64_t nmodes, int64_t mstride,
                                const uint32_t *modecoord,
                                int N, const int *bin_of_s2, int64_t n_s2, int nbins, double kf,
                                const void *winv, double *acc, int orders, const Batch *batch, ColTune tune) {
  if constexpr (BisContract<L, B, R>::kGenerated) {
    Batch ba;
    ba.n = 0;
    if (batch) ba = *batch;
    const int nb = ba.n ? ba.n : 1;
    int64_t want = (nmodes + 255) / 256;
    // workgroups per catalog: the tuned count, else up to 4096 over all catalogs
    const int64_t cap = tune.blocks > 0 ? tune.blocks : (4096 / nb > 0 ? 4096 / nb : 1);
    unsigned blocks = (unsigned)(want < cap ? (want > 0 ? want : 1) : cap);
    const int ne = (orders ? B + 1 : 1) * (L / 2 + 1);
    size_t sh = (size_t)(ne + 2) * nbins * sizeof(double);
    if (orders)
      hipLaunchKernelGGL((k_contract_bis_reg<R, L, B, true>), dim3(blocks, 1, nb), dim3(256), sh, s,
                         (const cplx<R> *)spec, nmodes, mstride, modecoord, N, bin_of_s2, n_s2, nbins, kf,
                         (const R *)winv, acc, ba);
    else
      hipLaunchKernelGGL((k_contract_bis_reg<R, L, B, false>), dim3(blocks, 1, nb), dim3(256), sh, s,
                         (const cplx<R> *)spec, nmodes, mstride, modecoord, N, bin_of_s2, n_s2, nbins, kf,
                         (const R *)winv, acc, ba);
    return true;
  } else {
    return false;
  }
}

template <typename R>
static bool contract_reg_dispatch(int lmax, int bmax, hipStream_t s, const void *spec, int64_t nmodes,
                                  int64_t mstride,
                                  const uint32_t *modecoord, int N, const int *bin_of_s2, int64_t n_s2,
                                  int nbins, double kf, const void *winv, double *acc, int orders,
                                  const Batch *batch, ColTune tune) {
#define PW_CR(L, B)                                                                                \
  if (lmax == L && bmax == B)                                                                      \
    return contract_reg_launch<R, L, B>(s, spec, nmodes, mstride, modecoord, N, bin_of_s2, n_s2, nbins, kf, winv, \
                                        acc, orders, batch, tune);
  PW_CR(0, 0) PW_CR(0, 1) PW_CR(0, 2) PW_CR(2, 0) PW_CR(2, 1) PW_CR(2, 2)
  PW_CR(4, 0) PW_CR(4, 1) PW_CR(4, 2) PW_CR(6, 0) PW_CR(6, 1) PW_CR(6, 2)
#undef PW_CR
  return false;
}

bool launch_contract_bis_generated(hipStream_t s, int prec, int lmax, int bmax, const void *spec, int64_t nmodes,
                                   int64_t mstride, const uint32_t *modecoord, int N, const int *bin_of_s2, int64_t n_s2,
                                   int nbins, double kf, const void *winv, double *acc, int orders,
                                   const Batch *batch, ColTune tune) {
  return prec == 0 ? contract_reg_dispatch<float>(lmax, bmax, s, spec, nmodes, mstride, modecoord, N, bin_of_s2,
                                                  n_s2, nbins, kf, winv, acc, orders, batch, tune)
                   : contract_reg_dispatch<double>(lmax, bmax, s, spec, nmodes, mstride, modecoord, N, bin_of_s2,
                                                   n_s2, nbins, kf, winv, acc, orders, batch, tune);
}

// ------------------------------------------------------------------------------ generated
bool bis_contract_generated(int lmax, int bmax) {
#define PW_BG(L, B) if (lmax == L && bmax == B) return BisContract<L, B, float>::kGenerated;
  PW_BG(0, 0) PW_BG(0, 1) PW_BG(0, 2) PW_BG(2, 0) PW_BG(2, 1) PW_BG(2, 2)
  PW_BG(4, 0) PW_BG(4, 1) PW_BG(4, 2) PW_BG(6, 0) PW_BG(6, 1) PW_BG(6, 2)
#undef PW_BG
  return false;
}

int mid_reweight_nfields(int lmax, int order, int all_parity) {
#define PW_MN(L, K) if (!all_parity && lmax == L && order == K) return MidReweight<L, K, float>::kGenerated ? MidReweight<L, K, float>::NG : -1;
  PW_MN(2, 2) PW_MN(2, 4) PW_MN(2, 6) PW_MN(4, 2) PW_MN(4, 4) PW_MN(4, 6) PW_MN(6, 2) PW_MN(6, 4)
#undef PW_MN
#define PW_MNA(L, K) if (all_parity && lmax == L && order == K) return MidReweightAll<L, K, float>::kGenerated ? MidReweightAll<L, K, float>::NG : -1;
  PW_MNA(2, 1) PW_MNA(2, 2) PW_MNA(2, 3) PW_MNA(2, 4) PW_MNA(4, 1) PW_MNA(4, 2) PW_MNA(4, 3) PW_MNA(4, 4)
#undef PW_MNA
  return -1;
}

bool mid_reweight_generated(int lmax, int order, int all_parity) {
  return mid_reweight_nfields(lmax, order, all_parity) >= 0;
}

// Bisector xi targets over the full pencil-major spectra: one thread per mode.
template <typename R, int LMAX, int BMAX>
__global__ void __launch_bounds__(256)
k_targets(const cplx<R> *__restrict__ spec, int64_t nmodes, int64_t mstride, int N, int rs,
          const R *__restrict__ winv, R *__restrict__ T) {
  using CT = BisContract<LMAX, BMAX, R>;
  constexpr int NF = CT::NF;
  constexpr int NT = (LMAX + 1) * (LMAX + 2) / 2;   // targets of even l <= LMAX
  constexpr int NSH = (LMAX + 1) * (LMAX + 1);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nmodes;
       i += (int64_t)gridDim.x * blockDim.x) {
    cplx<R> a[NF];
#pragma unroll
    for (int p = 0; p < NF; ++p) a[p] = spec[(size_t)p * mstride + i];
    R full[NSH];
    CT::targets(a, full);
    R iw2 = (R)1;
    if (winv) {
      const int64_t q = i / N;
      const int kz = (int)(i - q * N), ky = (int)(q / rs), kx = (int)(q - (int64_t)ky * rs);
      const R iw = winv[kx] * winv[ky] * winv[kz];
      iw2 = iw * iw;
    }
#pragma unroll
    for (int l = 0, o = 0; l <= LMAX; l += 2)
#pragma unroll
      for (int nu = -l; nu <= l; ++nu, ++o) T[(size_t)o * nmodes + i] = full[l * l + l + nu] * iw2;
    (void)NT;
  }
}

template <typename R, int L, int B>
static bool targets_launch(hipStream_t s, const void *spec, int64_t nmodes, int64_t mstride, int N, int rs,
                           const void *winv, void *T) {
  if constexpr (BisContract<L, B, R>::kGenerated) {
    int64_t want = (nmodes + 255) / 256;
    unsigned blocks = (unsigned)(want < 65536 ? (want > 0 ? want : 1) : 65536);
    hipLaunchKernelGGL((k_targets<R, L, B>), dim3(blocks), dim3(256), 0, s, (const cplx<R> *)spec, nmodes, mstride, N,
                       rs, (const R *)winv, (R *)T);
    return true;
  } else {
    return false;
  }
}

void launch_targets(hipStream_t s, int prec, int N, int lmax, int bmax, const void *spec, int64_t nmodes,
                    int64_t mstride, int rs, const void *winv, void *T) {
#define PW_TG(L, B)                                                                               \
  if (lmax == L && bmax == B) {                                                                   \
    if (prec == 0) targets_launch<float, L, B>(s, spec, nmodes, mstride, N, rs, winv, T);         \
    else targets_launch<double, L, B>(s, spec, nmodes, mstride, N, rs, winv, T);                  \
    return;                                                                                       \
  }
  PW_TG(0, 0) PW_TG(0, 1) PW_TG(0, 2) PW_TG(2, 0) PW_TG(2, 1) PW_TG(2, 2)
  PW_TG(4, 0) PW_TG(4, 1) PW_TG(4, 2) PW_TG(6, 0) PW_TG(6, 1) PW_TG(6, 2)
#undef PW_TG
}

// Midpoint real-space re-weighting: one thread per cell of the separation grid
// (D = H * signed index, minimum image), g[i][cell] -> A[j][cell].  Parity-even (ALLP false):
// even alpha and J1, Dp[i] = |D|^(2i); all-parity: every alpha and J1, Dp[i] = |D|^i.
template <typename R, int L, int K, bool ALLP>
__global__ void __launch_bounds__(256)
k_reweight(const R *__restrict__ g, R *__restrict__ A, int N, R Hu) {
  using MR = typename std::conditional<ALLP, MidReweightAll<L, K, R>, MidReweight<L, K, R>>::type;
  constexpr int NSH = (K + 1) * (K + 1);
  constexpr int NDP = ALLP ? K + 1 : K / 2 + 1;
  const size_t ncell = (size_t)N * N * N;
  // one cell per thread, no grid-stride loop: the fields' base addresses are then formed next
  // to their loads instead of being kept live across a loop (up to 130 fields: more scalar
  // registers than there are, spilled into vector lanes)
  {
    const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int x = (int)(c % N), y = (int)((c / N) % N), z = (int)(c / ((size_t)N * N));
    const int sx = x < N / 2 ? x : x - N, sy = y < N / 2 ? y : y - N, sz = z < N / 2 ? z : z - N;
    const R dx = (R)sx * Hu, dy = (R)sy * Hu, dz = (R)sz * Hu;  // D / unit
    const R d2 = dx * dx + dy * dy + dz * dz;
    R yD[NSH];
#pragma unroll
    for (int i = 0; i < NSH; ++i) yD[i] = 0;
    R Dp[NDP];
    Dp[0] = 1;
    const R dstep = ALLP ? sqrt(d2) : d2;
#pragma unroll
    for (int i = 1; i < NDP; ++i) Dp[i] = Dp[i - 1] * dstep;
    if (d2 > (R)0) {
      const R ir = (R)1 / sqrt(d2);
      real_sh_even<R, K, ALLP>(c_sh_gen, dx * ir, dy * ir, dz * ir, yD);
    } else {
      // D = 0: |D|^alpha = 0 for every alpha > 0, so the direction is immaterial
      real_sh_even<R, K, ALLP>(c_sh_gen, (R)0, (R)0, (R)1, yD);
    }
    R gv[MR::NG];
#pragma unroll
    for (int i = 0; i < MR::NG; ++i) gv[i] = g[(size_t)i * ncell + c];
    R av[MR::NA];
    MR::run(gv, yD, Dp, av);
#pragma unroll
    for (int i = 0; i < MR::NA; ++i) A[(size_t)i * ncell + c] = av[i];
  }
}

template <typename R, int L, int K, bool ALLP>
static void reweight_launch(hipStream_t s, int N, const void *g, void *A, double Hu) {
  using MR = typename std::conditional<ALLP, MidReweightAll<L, K, R>, MidReweight<L, K, R>>::type;
  if constexpr (MR::kGenerated) {
    const size_t ncell = (size_t)N * N * N;
    const unsigned blocks = (unsigned)((ncell + 255) / 256);  // at most 2^19 (N <= 512)
    hipLaunchKernelGGL((k_reweight<R, L, K, ALLP>), dim3(blocks), dim3(256), 0, s, (const R *)g, (R *)A, N,
                       (R)Hu);
  }
}

void launch_reweight(hipStream_t s, int prec, int N, int lmax, int order, int all_parity, const void *g, void *A,
                     double Hu) {
#define PW_RW(L, K, AP)                                                                           \
  if (lmax == L && order == K && all_parity == AP) {                                              \
    if (prec == 0) reweight_launch<float, L, K, AP>(s, N, g, A, Hu);                               \
    else reweight_launch<double, L, K, AP>(s, N, g, A, Hu);                                        \
    return;                                                                                       \
  }
  PW_RW(2, 2, 0) PW_RW(2, 4, 0) PW_RW(2, 6, 0) PW_RW(4, 2, 0) PW_RW(4, 4, 0) PW_RW(4, 6, 0) PW_RW(6, 2, 0)
  PW_RW(6, 4, 0)
  PW_RW(2, 1, 1) PW_RW(2, 2, 1) PW_RW(2, 3, 1) PW_RW(2, 4, 1) PW_RW(4, 1, 1) PW_RW(4, 2, 1) PW_RW(4, 3, 1)
  PW_RW(4, 4, 1)
#undef PW_RW
}

}  // namespace pw
