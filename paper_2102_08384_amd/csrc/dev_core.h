// Device building blocks for gfx950: complex arithmetic, the pencil FFT (radix-8/4/2
// Stockham, eight elements per lane, LDS exchanges between stages) and real spherical
// harmonics evaluated by Cartesian recurrences.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

namespace pw {

template <typename R>
using cplx = typename std::conditional<std::is_same<R, float>::value, float2, double2>::type;

template <typename R> __device__ __forceinline__ cplx<R> mk(R x, R y) { cplx<R> c; c.x = x; c.y = y; return c; }
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { a.x += b.x; a.y += b.y; return a; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  C r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
template <typename C> __device__ __forceinline__ C cconj(C a) { a.y = -a.y; return a; }
template <typename C, typename R> __device__ __forceinline__ C cscale(C a, R s) { a.x *= s; a.y *= s; return a; }

// multiply by exp(sign * i pi/2) : forward (sign -1) -> -i, inverse -> +i
template <bool INV, typename C> __device__ __forceinline__ C rot4(C a) {
  C r;
  if (INV) { r.x = -a.y; r.y = a.x; } else { r.x = a.y; r.y = -a.x; }
  return r;
}
// multiply by exp(sign * i pi/4)
template <bool INV, typename C, typename R> __device__ __forceinline__ C rot8_1(C a, R h) {
  C r;
  if (INV) { r.x = (a.x - a.y) * h; r.y = (a.x + a.y) * h; }
  else     { r.x = (a.x + a.y) * h; r.y = (a.y - a.x) * h; }
  return r;
}
// multiply by exp(sign * 3 i pi/4)
template <bool INV, typename C, typename R> __device__ __forceinline__ C rot8_3(C a, R h) {
  C r;
  if (INV) { r.x = (-a.x - a.y) * h; r.y = (a.x - a.y) * h; }
  else     { r.x = (a.y - a.x) * h; r.y = (-a.x - a.y) * h; }
  return r;
}

template <bool INV, typename C>
__device__ __forceinline__ void dft2(C &a, C &b) {
  C t = a; a = cadd(t, b); b = csub(t, b);
}

template <bool INV, typename C>
__device__ __forceinline__ void dft4(C &u0, C &u1, C &u2, C &u3) {
  C c0 = cadd(u0, u2), c1 = cadd(u1, u3), d0 = csub(u0, u2), d1 = rot4<INV>(csub(u1, u3));
  u0 = cadd(c0, c1); u2 = csub(c0, c1); u1 = cadd(d0, d1); u3 = csub(d0, d1);
}

// In-place 8-point DFT: u[r] <- sum_n u[n] exp(sign 2 pi i r n / 8)
template <bool INV, typename R>
__device__ __forceinline__ void dft8(cplx<R> u[8]) {
  const R h = (R)0.70710678118654752440;
  cplx<R> a0 = cadd(u[0], u[4]), a1 = cadd(u[1], u[5]), a2 = cadd(u[2], u[6]), a3 = cadd(u[3], u[7]);
  cplx<R> b0 = csub(u[0], u[4]);
  cplx<R> b1 = rot8_1<INV>(csub(u[1], u[5]), h);
  cplx<R> b2 = rot4<INV>(csub(u[2], u[6]));
  cplx<R> b3 = rot8_3<INV>(csub(u[3], u[7]), h);
  dft4<INV>(a0, a1, a2, a3);
  dft4<INV>(b0, b1, b2, b3);
  u[0] = a0; u[2] = a1; u[4] = a2; u[6] = a3;
  u[1] = b0; u[3] = b1; u[5] = b2; u[7] = b3;
}

// Number of radix stages and their radices for N = 2^n: radix-8 stages, then one radix-4
// or radix-2 stage for the remainder.
__host__ __device__ constexpr int log2i(int n) { return n <= 1 ? 0 : 1 + log2i(n >> 1); }
__host__ __device__ constexpr int n_stages(int N) { return log2i(N) / 3 + (log2i(N) % 3 ? 1 : 0); }
__host__ __device__ constexpr int stage_radix(int N, int s) {
  return (s < log2i(N) / 3) ? 8 : (log2i(N) % 3 == 2 ? 4 : 2);
}

// Span of stage S: product of the radices of the stages before it.
__host__ __device__ constexpr int stage_span(int N, int S) { return S == 0 ? 1 : stage_span(N, S - 1) * stage_radix(N, S - 1); }

// Twiddle sources: a table tw[e] = exp(-2 pi i e / N) in global memory, or the twiddles of one
// lane held in registers (FftTw, filled once per kernel).
template <typename R, int N> struct GlobalTw {
  const cplx<R> *__restrict__ tw;
  template <int S, int RADIX>
  __device__ __forceinline__ cplx<R> get(int c, int r, int k) const {
    return tw[(r * k * (N / (stage_span(N, S) * RADIX))) & (N - 1)];
  }
};
template <typename R, int N> struct FftTw {
  static constexpr int NSTAGE = n_stages(N);
  cplx<R> w[NSTAGE > 1 ? (NSTAGE - 1) * 7 : 1];
  // twiddles of lane t for every stage after the first
  __device__ __forceinline__ void load(int t, const cplx<R> *__restrict__ tw) { load_from<1>(t, tw); }
  template <int S>
  __device__ __forceinline__ void load_from(int t, const cplx<R> *__restrict__ tw) {
    if constexpr (S < NSTAGE) {
      constexpr int RADIX = stage_radix(N, S), NB = 8 / RADIX, NS = stage_span(N, S);
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const int k = (t + c * (N / 8)) % NS;
#pragma unroll
        for (int r = 1; r < RADIX; ++r)
          w[(S - 1) * 7 + c * (RADIX - 1) + r - 1] = tw[(r * k * (N / (NS * RADIX))) & (N - 1)];
      }
      load_from<S + 1>(t, tw);
    }
  }
  template <int S, int RADIX>
  __device__ __forceinline__ cplx<R> get(int c, int r, int) const { return w[(S - 1) * 7 + c * (RADIX - 1) + r - 1]; }
};

// One Stockham stage S (radix RADIX, current span NS) for lane t (0 <= t < N/8) holding
// v[s] = x[t + s*N/8].  The stage outputs go either back into v (LAST: natural order) or to
// LDS at their Stockham positions (j/NS)*NS*RADIX + j%NS + r*NS through the accessor `at`.
// Twiddles exp(-2 pi i e / N) come from `tw` (conjugated for the inverse).
template <typename R, int N, bool INV, int S, int RADIX, int NS, bool LAST, typename Tw, typename At>
__device__ __forceinline__ void fft_stage(cplx<R> v[8], int t, const Tw &tw, At at) {
  constexpr int NB = 8 / RADIX;        // butterflies per lane
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const int j = t + c * (N / 8);
    cplx<R> u[RADIX];
#pragma unroll
    for (int r = 0; r < RADIX; ++r) u[r] = v[c + NB * r];
    const int k = j % NS;
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < RADIX; ++r) {
        cplx<R> w = tw.template get<S, RADIX>(c, r, k);
        if (INV) w.y = -w.y;
        u[r] = cmul(u[r], w);
      }
    }
    if constexpr (RADIX == 8) {
      dft8<INV, R>(u);
    } else if constexpr (RADIX == 4) {
      dft4<INV>(u[0], u[1], u[2], u[3]);
    } else {
      dft2<INV>(u[0], u[1]);
    }
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < RADIX; ++r) v[c + NB * r] = u[r];
    } else {
      const int base = (j / NS) * NS * RADIX + k;
#pragma unroll
      for (int r = 0; r < RADIX; ++r) at(base + r * NS) = u[r];
    }
  }
}

// Each LDS exchange: write, sync(), read, post().  post() is the barrier again when one LDS
// buffer serves every exchange, or a switch to the other buffer when two alternate (the next
// exchange's barrier then orders these reads before that buffer is written again).
template <typename R, int N, bool INV, int S, int NS, typename Tw, typename At, typename Sync, typename Post>
__device__ __forceinline__ void fft_stages(cplx<R> v[8], int t, const Tw &tw, At at, Sync sync, Post post) {
  constexpr int RAD = stage_radix(N, S);
  if constexpr (S == n_stages(N) - 1) {
    fft_stage<R, N, INV, S, RAD, NS, true>(v, t, tw, at);
  } else {
    fft_stage<R, N, INV, S, RAD, NS, false>(v, t, tw, at);
    sync();
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = at(t + q * (N / 8));
    post();
    fft_stages<R, N, INV, S + 1, NS * RAD>(v, t, tw, at, sync, post);
  }
}

// Full N-point transform of one pencil.  On entry and exit lane t (0 <= t < N/8) holds
// v[s] = x[t + s*N/8] (natural order on exit).  `at(i)` returns a reference to this pencil's
// LDS element i; `sync()` is the barrier that covers every lane sharing the LDS.  Every lane
// of the block must call it (it contains barriers).
template <typename R, int N, bool INV, typename At, typename Sync>
__device__ __forceinline__ void fft_pencil(cplx<R> v[8], int t, const cplx<R> *__restrict__ tw, At at, Sync sync) {
  GlobalTw<R, N> g{tw};
  fft_stages<R, N, INV, 0, 1>(v, t, g, at, sync, sync);
}
// The same with the lane's twiddles in registers (FftTw::load once per kernel).  Kernels that
// prefetch the next pencil group's data across transforms use this form, with an explicit
// vmcnt(0) wait after FftTw::load: the compiler then never waits on the prefetched loads to
// read a twiddle.
template <typename R, int N, bool INV, typename At, typename Sync>
__device__ __forceinline__ void fft_pencil(cplx<R> v[8], int t, const FftTw<R, N> &tw, At at, Sync sync) {
  fft_stages<R, N, INV, 0, 1>(v, t, tw, at, sync, sync);
}
// Two alternating LDS buffers: `at` must address the buffer selected by the state that `flip`
// toggles; one barrier per exchange.
template <typename R, int N, bool INV, typename At, typename Sync, typename Flip>
__device__ __forceinline__ void fft_pencil_db(cplx<R> v[8], int t, const FftTw<R, N> &tw, At at, Sync sync,
                                              Flip flip) {
  fft_stages<R, N, INV, 0, 1>(v, t, tw, at, sync, flip);
}
// s_waitcnt vmcnt(0) (expcnt and lgkmcnt not waited on)
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Raw buffer access with byte offsets.  The hardware checks each lane's vector offset against
// the resource's byte count: a lane given kOob reads zeros and its stores are dropped, so masked
// lanes need no branch.  The uniform part of an address goes in the scalar offset.
constexpr uint32_t kOob = 0x80000000u;
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, uint32_t nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)nbytes, 0x00020000);
}
template <typename R>
__device__ __forceinline__ cplx<R> buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(R) == 4) {
    const f32x2 v = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    return mk<R>(v.x, v.y);
  } else {
    const f64x2 v = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    return mk<R>(v.x, v.y);
  }
}
template <typename R>
__device__ __forceinline__ void buf_store(cplx<R> x, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(R) == 4) {
    const f32x2 v = {x.x, x.y};
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
  } else {
    const f64x2 v = {x.x, x.y};
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff, soff, 0);
  }
}

// Groups of fields per block (grid.y) for column passes, so that a launch has about 4096
// blocks when the pencil dimension alone gives fewer.
inline int field_groups(int nfields, int nblocks_other) {
  int g = (8 * 512 + nblocks_other - 1) / (nblocks_other > 0 ? nblocks_other : 1);
  return g < 1 ? 1 : (g > nfields ? nfields : g);
}

// Row-mode pencils (x passes): ROWS rows of N elements per block, T = N/8 lanes per row.
template <int N> struct FxShape {
  static constexpr int T = N / 8;                          // lanes per pencil
  static constexpr int ROWS = (T >= 64) ? (256 / T > 0 ? 256 / T : 1) : 64 / T * 2;
  static constexpr int THREADS = ROWS * T;
};

// Column-mode pencils: C pencils adjacent in memory, lane (t, c) with c fastest so that every
// global access of a wavefront covers C consecutive complex values.
template <typename R, int N> struct ColShape {
  static constexpr int T = N / 8;
  static constexpr int C0 = (sizeof(R) == 4) ? 16 : 8;
  static constexpr int C = (C0 * T > 1024) ? 1024 / T : C0;
  static constexpr int THREADS = C * T;
};

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

// ---------------------------------------------------------------------------------------
// Real spherical harmonics y_J^mu(u) of a unit vector u, by the Cartesian recurrences
//   Qt_m^m = 1, Qt_{m+1}^m = (2m+1) z, Qt_l^m = a_lm z Qt_{l-1}^m - b_lm Qt_{l-2}^m,
//   y_l^{+-m} = norm_lm Qt_l^m(z) {Re, Im} (x + i y)^m,
// with a_lm = (2l-1)/(l-m), b_lm = (l+m-1)/(l-m) and norm_lm = sqrt((2l+1)/(4pi) (l-m)!/(l+m)!)
// * (2m-1)!! * (sqrt(2) if m > 0).  Tables come from the host (ShConst).
// ---------------------------------------------------------------------------------------
constexpr int kMaxJ = 16;

struct ShConst {
  float a[kMaxJ + 1][kMaxJ + 1];
  float b[kMaxJ + 1][kMaxJ + 1];
  float nrm[kMaxJ + 1][kMaxJ + 1];
  double a_d[kMaxJ + 1][kMaxJ + 1];
  double b_d[kMaxJ + 1][kMaxJ + 1];
  double nrm_d[kMaxJ + 1][kMaxJ + 1];
};

template <typename R> __device__ __forceinline__ R sh_a(const ShConst &c, int l, int m);
template <> __device__ __forceinline__ float sh_a<float>(const ShConst &c, int l, int m) { return c.a[l][m]; }
template <> __device__ __forceinline__ double sh_a<double>(const ShConst &c, int l, int m) { return c.a_d[l][m]; }
template <typename R> __device__ __forceinline__ R sh_b(const ShConst &c, int l, int m);
template <> __device__ __forceinline__ float sh_b<float>(const ShConst &c, int l, int m) { return c.b[l][m]; }
template <> __device__ __forceinline__ double sh_b<double>(const ShConst &c, int l, int m) { return c.b_d[l][m]; }
template <typename R> __device__ __forceinline__ R sh_n(const ShConst &c, int l, int m);
template <> __device__ __forceinline__ float sh_n<float>(const ShConst &c, int l, int m) { return c.nrm[l][m]; }
template <> __device__ __forceinline__ double sh_n<double>(const ShConst &c, int l, int m) { return c.nrm_d[l][m]; }

// y_J^{m} and y_J^{-m} (m >= 0; for m == 0 only *ym is meaningful) of the unit vector (x,y,z).
template <typename R>
__device__ __forceinline__ void real_sh_pair(const ShConst &c, int J, int m, R x, R y, R z, R *yp, R *ym) {
  // (x + i y)^m
  R cr = 1, ci = 0;
  for (int i = 0; i < m; ++i) {
    R t = cr * x - ci * y;
    ci = cr * y + ci * x;
    cr = t;
  }
  R q0 = 1, q1 = 0;  // Qt_{l-1}, Qt_{l-2}
  if (J > m) {
    R qa = (R)(2 * m + 1) * z;
    q1 = q0; q0 = qa;
    for (int l = m + 2; l <= J; ++l) {
      R qn = sh_a<R>(c, l, m) * z * q0 - sh_b<R>(c, l, m) * q1;
      q1 = q0; q0 = qn;
    }
  }
  R n = sh_n<R>(c, J, m) * q0;
  *yp = n * cr;
  *ym = n * ci;
}

// Recurrence state for the eight elements a lane holds, carried across a sequence of
// harmonics (J, m) visited in order of m, then J: (x + i y)^m in (cr, ci) and Qt_J^m,
// Qt_{J-1}^m in (q0, q1).  After set_m(m); advance(J) the harmonic of element s is
// sh_n(J, m) * q0[s] * {cr[s], ci[s]}.  Any order is valid; a decreasing m or J restarts.
template <typename R>
struct ShRec8 {
  R cr[8], ci[8], q0[8], q1[8];
  int m_cur, J_cur;
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int s = 0; s < 8; ++s) { cr[s] = 1; ci[s] = 0; q0[s] = 1; q1[s] = 0; }
    m_cur = 0;
    J_cur = 0;
  }
  __device__ __forceinline__ void set_m(int m, const R *ux, const R *uy) {
    if (m == m_cur + 1) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const R tr = cr[s] * ux[s] - ci[s] * uy[s];
        ci[s] = cr[s] * uy[s] + ci[s] * ux[s];
        cr[s] = tr;
      }
    } else if (m != m_cur) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        cr[s] = 1; ci[s] = 0;
        for (int i = 0; i < m; ++i) {
          const R tr = cr[s] * ux[s] - ci[s] * uy[s];
          ci[s] = cr[s] * uy[s] + ci[s] * ux[s];
          cr[s] = tr;
        }
      }
    }
    if (m != m_cur) {
#pragma unroll
      for (int s = 0; s < 8; ++s) { q0[s] = 1; q1[s] = 0; }
      m_cur = m;
      J_cur = m;
    }
  }
  __device__ __forceinline__ void advance(const ShConst &c, int Jt, const R *uz) {
    if (Jt < J_cur) {
#pragma unroll
      for (int s = 0; s < 8; ++s) { q0[s] = 1; q1[s] = 0; }
      J_cur = m_cur;
    }
    while (J_cur < Jt) {
      ++J_cur;
      if (J_cur == m_cur + 1) {
        const R c1 = (R)(2 * m_cur + 1);
#pragma unroll
        for (int s = 0; s < 8; ++s) { q1[s] = q0[s]; q0[s] = c1 * uz[s] * q0[s]; }
      } else {
        const R a = sh_a<R>(c, J_cur, m_cur), b = sh_b<R>(c, J_cur, m_cur);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const R qn = a * uz[s] * q0[s] - b * q1[s];
          q1[s] = q0[s];
          q0[s] = qn;
        }
      }
    }
  }
};

// All y_l^nu for even l <= LMAX (index sh_index(l, nu) - compact even-l layout given by
// the caller through out[l*l + l + nu] with odd l left untouched); with ODD every l <= LMAX.
template <typename R, int LMAX, bool ODD = false>
__device__ __forceinline__ void real_sh_even(const ShConst &c, R x, R y, R z, R *out) {
#pragma unroll
  for (int m = 0; m <= LMAX; ++m) {
    R cr = 1, ci = 0;
    for (int i = 0; i < m; ++i) { R t = cr * x - ci * y; ci = cr * y + ci * x; cr = t; }
    R q2 = 0, q1 = 1;  // Qt_{m-1} (=0), Qt_m (=1)
    for (int l = m; l <= LMAX; ++l) {
      R q;
      if (l == m) q = 1;
      else if (l == m + 1) q = (R)(2 * m + 1) * z;
      else q = sh_a<R>(c, l, m) * z * q1 - sh_b<R>(c, l, m) * q2;
      if (l > m) { q2 = q1; q1 = q; }
      if (ODD || (l & 1) == 0) {
        R n = sh_n<R>(c, l, m) * q;
        out[l * l + l + m] = n * cr;
        if (m > 0) out[l * l + l - m] = n * ci;
      }
    }
  }
}

}  // namespace pw
