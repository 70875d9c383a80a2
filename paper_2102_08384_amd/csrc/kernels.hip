// HIP kernels of the estimator hot path (gfx950, wave64).
//
//   (catalog reductions and painting live in paint.hip)
//   fx           fused field generation F (2r)^-alpha y_J^mu(x^) + real-to-complex FFT along x,
//                two real fields per complex transform, output pruned to kx < nkx
//   fy, fz       complex FFTs along y and z, output pruned to the retained k-sphere
//   contract     bisector contraction sum_nu y_l^nu(k^) sum S Re(conj(R_1) R_2) (Section 5.2
//                boxed estimator in the real-harmonic basis) with FP64 shell sums
//   finalize_pk  P_l = (4 pi / I) <..>_shell - d_l0 S / I
#include "kernels.h"

#include <algorithm>

#include "dev_core.h"

namespace pw {

__constant__ ShConst c_sh;

void upload_sh_const(const ShConst &c) {
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_sh), &c, sizeof(ShConst));
  upload_sh_const_inverse(c);
  upload_sh_const_generated(c);
}

// ------------------------------------------------------------------------------ fx
// Legendre part of the real harmonics for the 8 values of a lane, stepped in J at fixed m
// (the Cartesian recurrence of ShRec8) with the last two orders in qa / qb: a step overwrites the
// older one in place and flips `b_cur`, so no register copies happen; callers read the current
// order through `with_cur`, which hands the right array to a generic lambda (both versions are
// compiled, the uniform flag picks one).
template <typename R>
struct ShPair8 {
  R cr[8], ci[8], qa[8], qb[8];
  int m_cur, J_cur;
  bool b_cur;  // qb holds order J_cur (qa the one before), else the reverse
  __device__ __forceinline__ void restart_q() {
#pragma unroll
    for (int s = 0; s < 8; ++s) { qa[s] = 1; qb[s] = 0; }
    b_cur = false;
    J_cur = m_cur;
  }
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int s = 0; s < 8; ++s) { cr[s] = 1; ci[s] = 0; }
    m_cur = 0;
    restart_q();
  }
  __device__ __forceinline__ void set_m(int m, const R *ux, const R *uy) {
    if (m == m_cur) return;
    if (m != m_cur + 1) {
#pragma unroll
      for (int s = 0; s < 8; ++s) { cr[s] = 1; ci[s] = 0; }
      m_cur = 0;
    }
    for (; m_cur < m; ++m_cur) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const R tr = cr[s] * ux[s] - ci[s] * uy[s];
        ci[s] = cr[s] * uy[s] + ci[s] * ux[s];
        cr[s] = tr;
      }
    }
    restart_q();
  }
  // Q_{J+1} = a z Q_J - b Q_{J-1}, from Q_m = 1 and Q_{m-1} = 0 (the first step is then
  // (2m+1) z Q_m with the general coefficients)
  // z / r = pz * ir (ir = 1/r, 0 at the origin, whose direction is taken as +z)
  __device__ __forceinline__ void advance(const ShConst &c, int Jt, R pz, const R *ir) {
    if (Jt < J_cur) restart_q();
    while (J_cur < Jt) {
      ++J_cur;
      const R a = sh_a<R>(c, J_cur, m_cur), b = sh_b<R>(c, J_cur, m_cur);
      if (b_cur) {
#pragma unroll
        for (int s = 0; s < 8; ++s) qa[s] = a * (ir[s] > (R)0 ? pz * ir[s] : (R)1) * qb[s] - b * qa[s];
      } else {
#pragma unroll
        for (int s = 0; s < 8; ++s) qb[s] = a * (ir[s] > (R)0 ? pz * ir[s] : (R)1) * qa[s] - b * qb[s];
      }
      b_cur = !b_cur;
    }
  }
  // the same with z / r of each value given (uz; +z at the origin)
  __device__ __forceinline__ void advance_uz(const ShConst &c, int Jt, const R *uz) {
    if (Jt < J_cur) restart_q();
    while (J_cur < Jt) {
      ++J_cur;
      const R a = sh_a<R>(c, J_cur, m_cur), b = sh_b<R>(c, J_cur, m_cur);
      if (b_cur) {
#pragma unroll
        for (int s = 0; s < 8; ++s) qa[s] = a * uz[s] * qb[s] - b * qa[s];
      } else {
#pragma unroll
        for (int s = 0; s < 8; ++s) qb[s] = a * uz[s] * qa[s] - b * qb[s];
      }
      b_cur = !b_cur;
    }
  }
  template <typename Fn>
  __device__ __forceinline__ void with_cur(Fn &&fn) const {
    if (b_cur) fn(qb); else fn(qa);
  }
};

// LDS ordering between the lanes of one wavefront (LDS executes a wavefront's instructions in
// order; this keeps the compiler from moving accesses across the exchange point).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// value of lane `src` (0..63) of this wavefront
template <typename R>
__device__ __forceinline__ cplx<R> lane_fetch(int src, cplx<R> v) {
  const int addr = src << 2;
  if constexpr (sizeof(R) == 4) {
    return mk<R>(__int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v.x))),
                 __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v.y))));
  } else {
    const long long xb = __double_as_longlong(v.x), yb = __double_as_longlong(v.y);
    const int xl = __builtin_amdgcn_ds_bpermute(addr, (int)(xb & 0xffffffffLL));
    const int xh = __builtin_amdgcn_ds_bpermute(addr, (int)(xb >> 32));
    const int yl = __builtin_amdgcn_ds_bpermute(addr, (int)(yb & 0xffffffffLL));
    const int yh = __builtin_amdgcn_ds_bpermute(addr, (int)(yb >> 32));
    return mk<R>(__longlong_as_double(((long long)xh << 32) | (unsigned)xl),
                 __longlong_as_double(((long long)yh << 32) | (unsigned)yl));
  }
}

// One block = ROWS rows (z, y) of N cells; lane t of a row holds cells x = t + s*T.  For every
// job, two real fields (F (u/2r)^alpha y_J^mu, or two plain input fields when PLAIN) go through
// one complex FFT Z = FFT(a + i b) and are separated as A(k) = (Z(k) + conj Z(N-k)) / 2,
// B(k) = (Z(k) - conj Z(N-k)) / 2i for kx < nkx.  When a row is one wavefront (T = 64) the FFT's
// exchanges need only wavefront ordering and Z(N-k) comes from the partner lane by a cross-lane
// permute; otherwise the rows of the block share barriers and the separation reads LDS.
// FP32 at N = 512 fits three wavefronts per SIMD without spills (FP64 would spill).
// RADIAL: jobs may carry radial weights (u/2r)^alpha (midpoint fields), so each value keeps
// 1/r; otherwise (bisector fields) it keeps z/r, the only radial quantity the harmonics need,
// and 1/r is recomputed when the recurrence changes m.  Both fields of a job enter the
// transform scaled by 1/2 (exactly), which is the factor of the two-real-field separation.
template <typename R, int N, bool PLAIN, bool RADIAL, int ROWS = FxShape<N>::ROWS>
__global__ void __launch_bounds__(ROWS * FxShape<N>::T)
__attribute__((amdgpu_waves_per_eu((sizeof(R) == 4 && N == 512) ? 3 : 1, 8)))
k_fx(const R *__restrict__ mesh, cplx<R> *__restrict__ out, const FieldJob *__restrict__ jobs,
     int njobs, int nkx, int rs, R b0x, R b0y, R b0z, R H, R uhalf, const cplx<R> *__restrict__ tw,
     const int *__restrict__ rowlist, const DevNorm *__restrict__ norm, const Batch ba) {
  constexpr int T = FxShape<N>::T;
  if (ba.n) {  // catalog blockIdx.z of a batch
    const BatchSlot &bs = ba.s[blockIdx.z];
    mesh = (const R *)bs.mesh;
    out = (cplx<R> *)bs.A;
    rowlist = bs.rowlist;
    norm = bs.norm;
  }
  constexpr bool WAVE = (T == 64);
  constexpr int LN = N + N / 8;
  __shared__ cplx<R> lds[ROWS * LN];
  const int rl = threadIdx.x / T, t = threadIdx.x % T;
  // row = z * N + y: every row (grid covers N*N exactly), or the non-empty rows in order
  int row = blockIdx.x * ROWS + rl;
  bool live = true;
  if (rowlist) {
    const int nr = norm->nrows_occ;
    if ((int)blockIdx.x * ROWS >= nr) return;  // uniform for the block: before any barrier
    live = row < nr;
    row = live ? rowlist[row] : 0;
  }
  if constexpr (WAVE) {
    if (!live) return;  // a whole wavefront, and no block-wide barrier follows
  }
  const int y = row & (N - 1), z = row / N;
  cplx<R> *my = lds + rl * LN;
  auto at = [my](int i) -> cplx<R> & { return my[i + (i >> 3)]; };
  auto sync = []() {
    if constexpr (WAVE) wave_lds_sync(); else __syncthreads();
  };

  // per value: density and 1/r (RADIAL) or z/r (the direction is rebuilt from the position
  // where needed)
  R f[8], g[8];
  const R py = b0y + (R)y * H, pz = b0z + (R)z * H;
  auto inv_r = [&](int s) -> R {
    const R px = b0x + (R)(t + s * T) * H;
    const R r = sqrt(px * px + py * py + pz * pz);
    return (r > (R)0) ? (R)1 / r : (R)0;
  };
  if constexpr (!PLAIN) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      f[s] = live ? mesh[(size_t)row * N + t + s * T] : (R)0;
      const R ir = inv_r(s);
      g[s] = RADIAL ? ir : (ir > (R)0 ? pz * ir : (R)1);
    }
  }
  const size_t fstride = (size_t)N * N * rs;  // rows padded to rs (128-byte aligned)
  ShPair8<R> rec;
  if constexpr (!PLAIN) rec.init();
  for (int jb = 0; jb < njobs; ++jb) {
    const FieldJob J = jobs[jb];
    cplx<R> v[8];
    if constexpr (PLAIN) {
      // two real input fields of the stack at `mesh` (the second may be absent)
      const R *fa = mesh + (size_t)J.Ja * N * N * N + (size_t)row * N;
      const R *fb = mesh + (size_t)(J.Jb < 0 ? 0 : J.Jb) * N * N * N + (size_t)row * N;
#pragma unroll
      for (int s = 0; s < 8; ++s)
        v[s] = mk<R>((R)0.5 * fa[t + s * T], J.Jb >= 0 ? (R)0.5 * fb[t + s * T] : (R)0);
    } else {
      // kind 0: (J, +m) and (J, -m) at one alpha: norm Q_J^m {Re, Im}(x + iy)^m;
      // kind 1: (Ja, 0) and (Jb, 0) (Jb < 0: none), each at its own alpha.
      // Written as one branch-free form: the second field uses ci + 1 = 1 when m = 0.
      const bool k0 = (J.kind == 0);
      const int Jb = (k0 || J.Jb < 0) ? J.Ja : J.Jb;
      const R na = (R)0.5 * sh_n<R>(c_sh, J.Ja, J.m);
      const R nb = k0 ? na : (J.Jb >= 0 ? (R)0.5 * sh_n<R>(c_sh, Jb, 0) : (R)0);
      const R dci = k0 ? (R)0 : (R)1;
      R wa[8];
#pragma unroll
      for (int s = 0; s < 8; ++s) wa[s] = f[s] * na;
      if constexpr (RADIAL) {
        for (int a = 0; a < J.alpha; ++a) {
#pragma unroll
          for (int s = 0; s < 8; ++s) wa[s] *= uhalf * g[s];  // u / (2r): lengths in the unit u
        }
      }
      if (J.m != rec.m_cur) {
        R ux[8], uy[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const R ir = RADIAL ? g[s] : inv_r(s);
          ux[s] = (b0x + (R)(t + s * T) * H) * ir;
          uy[s] = py * ir;
        }
        rec.set_m(J.m, ux, uy);
      }
      if constexpr (!RADIAL) {
        rec.advance_uz(c_sh, J.Ja, g);
        if (k0) {
          // (J, +m) and (J, -m): one Legendre factor, the real and imaginary parts of (x + iy)^m
          rec.with_cur([&](const R *q) {
#pragma unroll
            for (int s = 0; s < 8; ++s) {
              const R tq = wa[s] * q[s];
              v[s].x = tq * rec.cr[s];
              v[s].y = tq * rec.ci[s];
            }
          });
        } else {
          // (Ja, 0) and (Jb, 0): m = 0, so (x + iy)^0 = 1
          rec.with_cur([&](const R *q) {
#pragma unroll
            for (int s = 0; s < 8; ++s) v[s].x = wa[s] * q[s];
          });
          if (J.Jb >= 0) {
            rec.advance_uz(c_sh, J.Jb, g);
            rec.with_cur([&](const R *q) {
#pragma unroll
              for (int s = 0; s < 8; ++s) v[s].y = f[s] * nb * q[s];
            });
          } else {
#pragma unroll
            for (int s = 0; s < 8; ++s) v[s].y = (R)0;
          }
        }
      } else {
        rec.advance(c_sh, J.Ja, pz, g);
        rec.with_cur([&](const R *q) {
#pragma unroll
          for (int s = 0; s < 8; ++s) v[s].x = wa[s] * q[s] * rec.cr[s];
        });
        rec.advance(c_sh, Jb, pz, g);
        if (J.alpha_b == J.alpha) {
          const R rb = nb / na;  // na > 0 always
          rec.with_cur([&](const R *q) {
#pragma unroll
            for (int s = 0; s < 8; ++s) v[s].y = wa[s] * rb * q[s] * (rec.ci[s] + dci);
          });
        } else {
          R wb[8];
#pragma unroll
          for (int s = 0; s < 8; ++s) wb[s] = f[s] * nb;
          if constexpr (RADIAL) {
            for (int a = 0; a < J.alpha_b; ++a) {
#pragma unroll
              for (int s = 0; s < 8; ++s) wb[s] *= uhalf * g[s];
            }
          }
          rec.with_cur([&](const R *q) {
#pragma unroll
            for (int s = 0; s < 8; ++s) v[s].y = wb[s] * q[s] * (rec.ci[s] + dci);
          });
        }
      }
    }
    fft_pencil<R, N, false>(v, t, tw, at, sync);
    cplx<R> *oa = out + (size_t)J.pa * fstride + (size_t)row * rs;
    cplx<R> *ob = out + (size_t)(J.pb < 0 ? 0 : J.pb) * fstride + (size_t)row * rs;
    const bool hb = J.pb >= 0;
    if constexpr (WAVE) {
      // lane t holds Z(t + 64 s).  Z(N - k) for k = t + 64 s, s < 4: lane (64 - t) & 63, its
      // v[7 - s] (t > 0) or v[(8 - s) & 7] (lane 0); every lane publishes the value its
      // partner needs.  k = 256 (s = 4) is lane 0's own v[4]; 256 < k < rs is padding.
      // (the inputs carry the separation's factor 1/2)
      const int partner = (64 - t) & 63;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (64 * s >= rs) break;  // uniform: no lane stores at or beyond the padded row
        const cplx<R> pub = (t == 0) ? v[(8 - s) & 7] : v[7 - s];
        const cplx<R> b = lane_fetch<R>(partner, pub);
        const cplx<R> a = v[s];
        const int kx = t + 64 * s;
        if (kx < rs) {
          const bool keep = kx < nkx;
          oa[kx] = keep ? mk<R>(a.x + b.x, a.y - b.y) : mk<R>(0, 0);
          if (hb) ob[kx] = keep ? mk<R>(a.y + b.y, b.x - a.x) : mk<R>(0, 0);
        }
      }
      const int kx = 256 + t;
      if (256 < rs && kx < rs) {
        const bool keep = (t == 0) && kx < nkx;  // Z(256) pairs with itself
        const cplx<R> a = v[4];
        oa[kx] = keep ? mk<R>(a.x + a.x, (R)0) : mk<R>(0, 0);
        if (hb) ob[kx] = keep ? mk<R>(a.y + a.y, (R)0) : mk<R>(0, 0);
      }
    } else {
#pragma unroll
      for (int s = 0; s < 8; ++s) at(t + s * T) = v[s];
      __syncthreads();
      for (int kx = t; live && kx < rs; kx += T) {
        if (kx >= nkx) {  // padding to the 128-byte row stride: whole-line writes
          oa[kx] = mk<R>(0, 0);
          if (hb) ob[kx] = mk<R>(0, 0);
          continue;
        }
        const cplx<R> a = at(kx), b = at((N - kx) & (N - 1));
        oa[kx] = mk<R>(a.x + b.x, a.y - b.y);
        if (hb) ob[kx] = mk<R>(a.y + b.y, b.x - a.x);
      }
      __syncthreads();
    }
  }
}

template <typename R, int N>
static void fx_launch(hipStream_t s, int kind, const void *mesh, void *out, const FieldJob *jobs, int njobs,
                      int nkx, int rs, const double *b0, double H, double unit, const void *tw,
                      const int *rowlist, const DevNorm *norm, const Batch *batch, ColTune tune) {
  Batch ba;
  ba.n = 0;
  if (batch) ba = *batch;
  const unsigned nb = ba.n ? ba.n : 1;
#define PW_FX(PL, RAD, RW)                                                                                       \
  hipLaunchKernelGGL((k_fx<R, N, PL, RAD, RW>), dim3((unsigned)((size_t)N * N / (RW)), 1, nb),                  \
                     dim3((RW) * FxShape<N>::T), 0, s, (const R *)mesh, (cplx<R> *)out, jobs, njobs, nkx, rs,    \
                     (R)b0[0], (R)b0[1], (R)b0[2], (R)H, (R)(0.5 * unit), (const cplx<R> *)tw, rowlist, norm, ba)
#define PW_FX_KIND(RW)                                                                                           \
  do {                                                                                                           \
    if (kind == FX_PLAIN) PW_FX(true, false, RW);                                                                \
    else if (kind == FX_RADIAL) PW_FX(false, true, RW);                                                          \
    else PW_FX(false, false, RW);                                                                                \
  } while (0)
  // other row counts per workgroup where a row is one wavefront (FP32 at N = 512)
  if constexpr (sizeof(R) == 4 && FxShape<N>::T == 64) {
    if (tune.rows == 1) { PW_FX_KIND(1); return; }
    if (tune.rows == 2) { PW_FX_KIND(2); return; }
    if (tune.rows == 8) { PW_FX_KIND(8); return; }
  }
  PW_FX_KIND(FxShape<N>::ROWS);
#undef PW_FX_KIND
#undef PW_FX
}

void launch_fx(hipStream_t s, int prec, int N, int kind, const void *mesh, void *out, const FieldJob *jobs,
               int njobs, int nkx, int rs, const double *b0, double H, double unit, const void *tw,
               const int *rowlist, const DevNorm *norm, const Batch *batch, ColTune tune) {
  if (prec == 0) { PW_DISPATCH_N(fx_launch, float, s, kind, mesh, out, jobs, njobs, nkx, rs, b0, H, unit, tw, rowlist, norm, batch, tune) }
  else { PW_DISPATCH_N(fx_launch, double, s, kind, mesh, out, jobs, njobs, nkx, rs, b0, H, unit, tw, rowlist, norm, batch, tune) }
}

// ------------------------------------------------------------------------------ fy / fz
// Column-pencil passes are software-pipelined: a block owns one plane (y pass) or one group of
// C pencils (z pass) and loops over a group of fields, issuing the global loads of the next
// field before transforming the current one (barriers do not wait for global loads), so memory
// latency hides behind the FFT.  Occupancy masks live in LDS, loaded once per block.

// y pass: CC adjacent kx columns per block (CC * N/8 threads)
template <typename R, int N, bool INV, int CC>
__global__ void __launch_bounds__(CC * (N / 8))
k_fy(const cplx<R> *__restrict__ in, cplx<R> *__restrict__ out, int nfields, int fpb, int nplanes, int nkx, int rs,
     const int *__restrict__ ycnt, const int64_t *__restrict__ yoff, int64_t npen, const cplx<R> *__restrict__ tw,
     const int *__restrict__ rowmask, const int *__restrict__ zlist, const DevNorm *__restrict__ norm,
     const Batch ba) {
  constexpr int T = N / 8, C = CC, NT = CC * T;
  if (ba.n) {  // catalog blockIdx.z of a batch
    const BatchSlot &bs = ba.s[blockIdx.z];
    in = (const cplx<R> *)bs.A;
    out = (cplx<R> *)bs.B;
    rowmask = bs.rowmask;
    zlist = bs.zlist;
    norm = bs.norm;
  }
  constexpr int Q = 128 / (int)sizeof(cplx<R>);
  constexpr int LB = N * (C + 1);  // one exchange buffer; two alternate (one barrier per exchange)
  __shared__ cplx<R> lds[2 * LB];
  __shared__ int msk[N];
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  int z = blockIdx.x;
  if (zlist) {
    if ((int)blockIdx.x >= norm->nplanes_occ) return;  // uniform: before any barrier
    z = zlist[blockIdx.x];
  }
  FftTw<R, N> twr;
  twr.load(t, tw);
  // output rows of this lane (ky = t + s*T) and their padded lengths, fixed for the block
  // (offsets within one output plane: below 2^31 for every supported mesh)
  int yo[8], yl[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    yo[s] = (int)yoff[t + s * T];
    yl[s] = (ycnt[t + s * T] + Q - 1) / Q * Q;
  }
  for (int i = threadIdx.x; i < N; i += NT) msk[i] = rowmask ? rowmask[z * N + i] : 1;
  wait_vmem();
  __syncthreads();
  // Raw buffer accesses with byte offsets fixed for the block: input row y = t + s*T of this
  // lane's column sits at lo[s] + s * sT from the column group's base (kOob where the row is
  // empty), output row ky = t + s*T at so[s] from the output group's base.  Bit s of wlive is
  // set when some lane of the wave loads row t + s*T (a wave spans 4 adjacent rows, so empty
  // rows skip whole load instructions).
  constexpr uint32_t E = sizeof(cplx<R>);
  const uint32_t sT = (uint32_t)(T * rs) * E;
  uint32_t lo[8], so[8], wlive = 0;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const bool live = msk[t + s * T] != 0;
    lo[s] = live ? (uint32_t)(t * rs + c) * E : kOob;
    so[s] = (uint32_t)(yo[s] + c) * E;
    if (__builtin_amdgcn_ballot_w64(live)) wlive |= 1u << s;
  }
  const int ncb = (nkx + C - 1) / C;
  const int p0 = blockIdx.y * fpb;
  const int p1 = min(nfields, p0 + fpb);
  const int nitems = (p1 - p0) * ncb;
  if (nitems <= 0) return;
  const size_t plane = (size_t)N * rs;  // one input plane of one field
  const uint32_t in_bytes = (uint32_t)(plane * E), out_bytes = (uint32_t)(npen * E);
  auto load = [&](int p, int cb, cplx<R> *v) {
    const bool colok = cb * C + c < nkx;
    const __amdgpu_buffer_rsrc_t r = buf_rsrc(in + ((size_t)p * nplanes + z) * plane + cb * C, in_bytes);
#pragma unroll
    for (int s = 0; s < 8; ++s)
      v[s] = ((wlive >> s) & 1u) ? buf_load<R>(r, colok ? lo[s] : kOob, (uint32_t)s * sT) : mk<R>(0, 0);
  };
  int lb = 0;
  auto at = [c, &lb](int i) -> cplx<R> & { return lds[lb * LB + i * (C + 1) + c]; };
  auto sync = []() { __syncthreads(); };
  auto flip = [&lb]() { lb ^= 1; };
  // items (field p, column group cb) in order, stepped without division
  int p = p0, cb = 0;
  cplx<R> nxt[8];
  load(p, cb, nxt);
  for (int it = 0; it < nitems; ++it) {
    cplx<R> v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = nxt[s];
    const int pc = p, cbc = cb, kx = cb * C + c;
    if (++cb == ncb) {
      cb = 0;
      ++p;
    }
    if (it + 1 < nitems) load(p, cb, nxt);
    fft_pencil_db<R, N, INV>(v, t, twr, at, sync, flip);
    const __amdgpu_buffer_rsrc_t w = buf_rsrc(out + ((size_t)pc * nplanes + z) * npen + cbc * C, out_bytes);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      // whole 128-byte lines: the row's padding slots are written too (never read as modes)
      const bool keep = kx < yl[s];
      if (__builtin_amdgcn_ballot_w64(keep)) buf_store<R>(v[s], w, keep ? so[s] : kOob, 0);
    }
  }
}

template <typename R, int N>
static void fy_launch(hipStream_t s, int inv, const void *in, void *out, int nfields, int nplanes, int nkx,
                      int rs, const int *ycnt, const int64_t *yoff, int64_t npen, const void *tw,
                      const int *rowmask, const int *zlist, const DevNorm *norm, ColTune tune,
                      const Batch *batch) {
  constexpr int CY = ColShape<R, N>::C;  // 128-byte row segments
  Batch ba;
  ba.n = 0;
  if (batch) ba = *batch;
  const int nb = ba.n ? ba.n : 1;
  int fpb = tune.fpb;
  if (fpb <= 0) {
    const int G = field_groups(nfields, nplanes * nb);
    fpb = (nfields + G - 1) / G;
  }
  fpb = std::min(fpb, nfields);
  dim3 grid(nplanes, (nfields + fpb - 1) / fpb, nb);
#define PW_FY(CC)                                                                                  \
  do {                                                                                             \
    if (inv)                                                                                       \
      hipLaunchKernelGGL((k_fy<R, N, true, CC>), grid, dim3((CC) * (N / 8)), 0, s, (const cplx<R> *)in, \
                         (cplx<R> *)out, nfields, fpb, nplanes, nkx, rs, ycnt, yoff, npen,          \
                         (const cplx<R> *)tw, rowmask, zlist, norm, ba);                            \
    else                                                                                           \
      hipLaunchKernelGGL((k_fy<R, N, false, CC>), grid, dim3((CC) * (N / 8)), 0, s, (const cplx<R> *)in, \
                         (cplx<R> *)out, nfields, fpb, nplanes, nkx, rs, ycnt, yoff, npen,          \
                         (const cplx<R> *)tw, rowmask, zlist, norm, ba);                            \
  } while (0)
  // half-segment columns (8 per workgroup) only where a full segment holds 16 (FP32)
  if constexpr (CY == 16) {
    if (tune.cols == 8) {
      PW_FY(8);
      return;
    }
  }
  PW_FY(CY);
#undef PW_FY
}

void launch_fy(hipStream_t s, int prec, int N, int inv, const void *in, void *out, int nfields, int nplanes,
               int nkx, int rs, const int *ycnt, const int64_t *yoff, int64_t npen, const void *tw,
               const int *rowmask, const int *zlist, const DevNorm *norm, ColTune tune, const Batch *batch) {
  if (nfields <= 0 || nplanes <= 0) return;
  if (prec == 0) {
    PW_DISPATCH_N(fy_launch, float, s, inv, in, out, nfields, nplanes, nkx, rs, ycnt, yoff, npen, tw, rowmask,
                  zlist, norm, tune, batch)
  } else {
    PW_DISPATCH_N(fy_launch, double, s, inv, in, out, nfields, nplanes, nkx, rs, ycnt, yoff, npen, tw, rowmask,
                  zlist, norm, tune, batch)
  }
}

// Output layouts (see Prune): full sets pencil-major, written through an LDS transpose so that
// each pencil's run leaves as whole wavefront stores; sphere-pruned sets (goff != null) grouped
// as [kz slot][pencil], so the C lanes of one kz write one 128-byte line straight from registers.
template <typename R, int N, bool GROUPED>
__global__ void __launch_bounds__((ColShape<R, N>::THREADS))
k_fz(const cplx<R> *__restrict__ in, cplx<R> *__restrict__ out, int nfields, int fpb, int64_t npen,
     const PencilInfo *__restrict__ pinfo, const int64_t *__restrict__ moff, const int64_t *__restrict__ goff,
     const int *__restrict__ gsize, int64_t mstride, const cplx<R> *__restrict__ tw,
     const int *__restrict__ planemask, const int *__restrict__ fmap, const Batch ba) {
  constexpr int T = ColShape<R, N>::T, C = ColShape<R, N>::C, NT = ColShape<R, N>::THREADS;
  if (ba.n) {  // catalog blockIdx.z of a batch
    const BatchSlot &bs = ba.s[blockIdx.z];
    in = (const cplx<R> *)bs.B;
    out = (cplx<R> *)bs.A;
    planemask = bs.planemask;
  }
  constexpr int LB = N * (C + 1);  // one exchange buffer; grouped: two alternate
  __shared__ cplx<R> lds[GROUPED ? 2 * LB : LB];
  __shared__ int st[C + 1];                      // full sets: first output mode of each pencil
  __shared__ int msk[N];
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int64_t q0 = (int64_t)blockIdx.x * C;
  const int64_t q = q0 + c;
  const int p0 = blockIdx.y * fpb;
  const int p1 = min(nfields, p0 + fpb);
  if (p0 >= p1) return;  // uniform
  FftTw<R, N> twr;
  twr.load(t, tw);
  for (int i = threadIdx.x; i < N; i += NT) msk[i] = planemask ? planemask[i] : 1;
  int64_t m0;
  int S = 0;
  if constexpr (GROUPED) {
    m0 = goff[blockIdx.x];
    S = gsize[blockIdx.x];
  } else {
    m0 = moff[q0];
    if (threadIdx.x <= C) {
      const int64_t qq = q0 + threadIdx.x;
      const int64_t e = (qq < npen) ? moff[qq] : moff[npen - 1] + pinfo[npen - 1].kzcnt;
      st[threadIdx.x] = (int)(e - m0);
    }
  }
  const bool has = q < npen && pinfo[q].kzcnt > 0;  // padding pencils hold no modes
  wait_vmem();
  __syncthreads();
  if constexpr (GROUPED) {
    if (S == 0) return;  // no pencil of the group holds a mode (uniform, after the last barrier)
  }
  auto load = [&](int p, cplx<R> *v) {
    const cplx<R> *src = in + (size_t)p * N * npen;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int z = t + s * T;
      v[s] = (has && msk[z]) ? src[(size_t)z * npen + q] : mk<R>(0, 0);
    }
  };
  int lb = 0;
  auto at = [c, &lb](int i) -> cplx<R> & { return lds[lb * LB + i * (C + 1) + c]; };
  auto sync = []() { __syncthreads(); };
  auto flip = [&lb]() { lb ^= 1; };
  // grouped: slot of kz = t + s T, or -1 outside the group's kz extent
  const int h = (S - 1) / 2;
  int slot[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int kz = t + s * T;
    slot[s] = (S == N || kz <= h) ? kz : (kz >= N - h ? kz - N + S : -1);
  }
  // full: pencil oc goes out through its own T lanes (a whole wavefront when T = 64)
  const int oc = threadIdx.x / T, oj = threadIdx.x % T;
  const int obase = GROUPED ? 0 : st[oc], ocnt = GROUPED ? 0 : st[oc + 1] - obase;
  cplx<R> nxt[8];
  load(p0, nxt);
  for (int p = p0; p < p1; ++p) {
    cplx<R> v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = nxt[s];
    if (p + 1 < p1) load(p + 1, nxt);
    if constexpr (GROUPED) fft_pencil_db<R, N, false>(v, t, twr, at, sync, flip);
    else fft_pencil<R, N, false>(v, t, twr, at, sync);
    if constexpr (GROUPED) {
      // fmap: output field of input field p (a group of fields transformed at a time)
      cplx<R> *dst = out + (size_t)(fmap ? fmap[p] : p) * mstride + m0 + c;
#pragma unroll
      for (int s = 0; s < 8; ++s)
        if (slot[s] >= 0) dst[(size_t)slot[s] * C] = v[s];
    } else {
#pragma unroll
      for (int s = 0; s < 8; ++s) at(t + s * T) = v[s];
      __syncthreads();
      // the block's pencils own one contiguous run of modes starting at m0, all N kz each
      cplx<R> *dst = out + (size_t)p * mstride + m0 + obase;
      for (int j = oj; j < ocnt; j += T) dst[j] = lds[j * (C + 1) + oc];
      __syncthreads();  // LDS reads done before the next transform writes
    }
  }
}

template <typename R, int N>
static void fz_launch(hipStream_t s, const void *in, void *out, int nfields, int64_t npen,
                      const PencilInfo *pinfo, const int64_t *moff, const int64_t *goff, const int *gsize,
                      int64_t mstride, const void *tw, const int *planemask, const int *fmap,
                      ColTune tune, const Batch *batch) {
  constexpr int C = ColShape<R, N>::C;
  static_assert(C == 128 / (int)sizeof(cplx<R>), "z-pass groups must match 128-byte slot rows");
  const unsigned ng = (unsigned)((npen + C - 1) / C);
  Batch ba;
  ba.n = 0;
  if (batch) ba = *batch;
  const int nb = ba.n ? ba.n : 1;
  int fpb = tune.fpb;
  if (fpb <= 0) {
    const int G = field_groups(nfields, (int)std::min<int64_t>((int64_t)ng * nb, 1 << 20));
    fpb = (nfields + G - 1) / G;
  }
  fpb = std::min(fpb, nfields);
  dim3 grid(ng, (nfields + fpb - 1) / fpb, nb);
  if (goff)
    hipLaunchKernelGGL((k_fz<R, N, true>), grid, dim3(ColShape<R, N>::THREADS), 0, s, (const cplx<R> *)in,
                       (cplx<R> *)out, nfields, fpb, npen, pinfo, moff, goff, gsize, mstride, (const cplx<R> *)tw,
                       planemask, fmap, ba);
  else
    hipLaunchKernelGGL((k_fz<R, N, false>), grid, dim3(ColShape<R, N>::THREADS), 0, s, (const cplx<R> *)in,
                       (cplx<R> *)out, nfields, fpb, npen, pinfo, moff, goff, gsize, mstride, (const cplx<R> *)tw,
                       planemask, (const int *)nullptr, ba);
}

void launch_fz(hipStream_t s, int prec, int N, const void *in, void *out, int nfields, int64_t npen,
               const PencilInfo *pinfo, const int64_t *moff, const int64_t *goff, const int *gsize,
               int64_t mstride, const void *tw, const int *planemask, const int *fmap, ColTune tune,
               const Batch *batch) {
  if (nfields <= 0 || npen <= 0) return;
  if (prec == 0) {
    PW_DISPATCH_N(fz_launch, float, s, in, out, nfields, npen, pinfo, moff, goff, gsize, mstride, tw, planemask,
                  fmap, tune, batch)
  } else {
    PW_DISPATCH_N(fz_launch, double, s, in, out, nfields, npen, pinfo, moff, goff, gsize, mstride, tw, planemask,
                  fmap, tune, batch)
  }
}

// ------------------------------------------------------------------------------ contraction
// One thread per retained mode of the half spectrum (kx in [0, N/2]).  Modes with
// 0 < kx < N/2 stand for themselves and their mirror -k (whose values are the complex
// conjugates, so Re(conj(a) b) is the same); the mirror's direction is that of the signed
// index (-n) mod N, which is -k except on Nyquist planes.
constexpr int kMaxVals = 4096;

template <typename R, int LMAX, int NTH>
__global__ void __launch_bounds__(NTH)
k_contract_bis(const cplx<R> *__restrict__ spec, int nfields, int64_t nmodes, int64_t mstride,
               const uint32_t *__restrict__ modecoord, int N, const int *__restrict__ bin_of_s2,
               int64_t n_s2, int nbins, int nell, TermTable tab, double kf,
               const R *__restrict__ winv, double *__restrict__ acc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
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
      vals[p * NTH + threadIdx.x] = live ? spec[(size_t)p * mstride + mode] : mk<R>(0, 0);
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

void launch_contract_bis(hipStream_t s, int prec, int lmax, int bmax, const void *spec, int nfields,
                         int64_t nmodes, int64_t mstride, const uint32_t *modecoord, int N, const int *bin_of_s2,
                         int64_t n_s2, int nbins, int nell, TermTable tab, double kf,
                         const void *winv, double *acc, ColTune tune) {
  if (nmodes <= 0) return;
  if (launch_contract_bis_generated(s, prec, lmax, bmax, spec, nmodes, mstride, modecoord, N, bin_of_s2, n_s2, nbins,
                                    kf, winv, acc, 0, nullptr, tune))
    return;
  const int nth = contract_bis_threads(prec, nfields, nell, nbins);  // validated by the planner
  int64_t want = (nmodes + nth - 1) / nth;
  unsigned blocks = (unsigned)(want < 8192 ? (want > 0 ? want : 1) : 8192);
#define PW_CONTRACT(R, L, NTH)                                                                     \
  if (nth == NTH) {                                                                                \
    size_t sh = (size_t)nfields * NTH * sizeof(cplx<R>) + (size_t)(nell + 2) * nbins * sizeof(double); \
    hipLaunchKernelGGL((k_contract_bis<R, L, NTH>), dim3(blocks), dim3(NTH), sh, s,                \
                       (const cplx<R> *)spec, nfields, nmodes, mstride, modecoord, N, bin_of_s2, n_s2, \
                       nbins, nell, tab, kf, (const R *)winv, acc);                                \
  }
#define PW_CONTRACT_L(R, L) PW_CONTRACT(R, L, 128) PW_CONTRACT(R, L, 64) PW_CONTRACT(R, L, 32) PW_CONTRACT(R, L, 16)
  if (prec == 0) {
    switch (lmax) {
      case 0: PW_CONTRACT_L(float, 0) break;
      case 2: PW_CONTRACT_L(float, 2) break;
      case 4: PW_CONTRACT_L(float, 4) break;
      case 6: PW_CONTRACT_L(float, 6) break;
      default: PW_CONTRACT_L(float, 8) break;
    }
  } else {
    switch (lmax) {
      case 0: PW_CONTRACT_L(double, 0) break;
      case 2: PW_CONTRACT_L(double, 2) break;
      case 4: PW_CONTRACT_L(double, 4) break;
      case 6: PW_CONTRACT_L(double, 6) break;
      default: PW_CONTRACT_L(double, 8) break;
    }
  }
#undef PW_CONTRACT_L
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
