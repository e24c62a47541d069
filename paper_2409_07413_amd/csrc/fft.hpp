// Stockham radix-2/3/4/8/16 FFT engine for one transform held across T lanes.
//
// A length-N transform (N = 2^a 3^b) is spread over T = N/E threads; thread t
// holds the E elements at positions t + T*m (m = 0..E-1) in registers, both
// before and after the transform (natural order, coalesced in global memory).
// Each Stockham pass of radix R computes butterflies j = t + k*T; the last pass
// writes back into the registers it read, every other pass exchanges through a
// caller-provided LDS region addressed as lds[pos * ES] (ES = element stride,
// so several transforms can interleave in one tile).
//
// Transform definition: X[k] = sum_n x[n] exp(DIR * 2 pi i n k / N) with
// DIR = -1 (forward) or +1 (inverse), unnormalised; callers apply 1/N per 2D
// round trip where needed.  Twiddles come from a table tw[e] = exp(-2 pi i e/N)
// computed in double on the host and rounded once to float.
#pragma once
#include <hip/hip_runtime.h>

namespace spr {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// The per-size kernels are built without automatic contraction, so that a
// kernel's results do not depend on how the compiler treats its context; the
// fused multiply-adds that matter are written out.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -__fmul_rn(a.y, b.y)), fmaf(a.x, b.y, __fmul_rn(a.y, b.x)));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by DIR * i
template <int DIR> __device__ __forceinline__ float2 mul_i(float2 a) {
  return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// ---------------------------------------------------------------------------
// Per-size plans: radices of the passes, elements per thread E (a common
// multiple of every radix), threads per transform T = N/E, columns per
// column-pass tile C and rows per row-pass workgroup RW.  Row-pass workgroups
// hold one wavefront from N = 256 up (1-2 % faster than four wavefronts at
// 384-1024, the row transforms needing no workgroup barrier) and 256 threads
// below.
// ---------------------------------------------------------------------------
template <int N> struct Plan;

#define SPR_DEFINE_PLAN(N_, E_, C_, ...)                                         \
  template <> struct Plan<N_> {                                                  \
    static constexpr int n = N_;                                                 \
    static constexpr int E = E_;                                                 \
    static constexpr int T = N_ / E_;                                            \
    static constexpr int C = C_;                                                 \
    static constexpr int RW = ((N_ >= 256 ? 64 : 256) / T) > 0 ? ((N_ >= 256 ? 64 : 256) / T) : 1; \
    __host__ __device__ static constexpr int radix(int i) {                      \
      constexpr int r[] = {__VA_ARGS__};                                         \
      return r[i];                                                               \
    }                                                                            \
    __host__ __device__ static constexpr int passes() {                          \
      constexpr int r[] = {__VA_ARGS__};                                         \
      return (int)(sizeof(r) / sizeof(int));                                     \
    }                                                                            \
  };

SPR_DEFINE_PLAN(8, 8, 8, 8)
SPR_DEFINE_PLAN(12, 12, 4, 3, 4)
SPR_DEFINE_PLAN(16, 4, 16, 4, 4)
SPR_DEFINE_PLAN(24, 24, 8, 3, 8)
SPR_DEFINE_PLAN(32, 8, 16, 4, 8)
SPR_DEFINE_PLAN(48, 12, 16, 3, 4, 4)
SPR_DEFINE_PLAN(64, 8, 16, 8, 8)
SPR_DEFINE_PLAN(96, 24, 16, 3, 4, 8)
SPR_DEFINE_PLAN(128, 8, 16, 2, 8, 8)
SPR_DEFINE_PLAN(192, 24, 16, 3, 8, 8)
// 384 and 768: twelve elements per thread with the pass holding the factor 3
// last (radix 6 = 2 x 3, radix 12 = 4 x 3, prime-factor butterflies), so that
// the strides of the earlier passes divide T (one twiddle set per pass, kept
// in registers), the first exchange is not a stride-3 pattern, and the
// transform takes four passes; 1024: the radix-16 pass last.
//
// Variant 1 of the served sizes is the alternative that a run-time tuner
// weighs against the default: the other column-tile width (256 to 768) or
// the other radix order (1024).
#ifndef SPR_VARIANT
#define SPR_VARIANT 0
#endif
#if SPR_VARIANT == 1
SPR_DEFINE_PLAN(256, 8, 8, 4, 8, 8)
SPR_DEFINE_PLAN(512, 8, 16, 8, 8, 8)
SPR_DEFINE_PLAN(384, 12, 16, 4, 4, 4, 6)
SPR_DEFINE_PLAN(768, 12, 16, 4, 4, 4, 12)
SPR_DEFINE_PLAN(1024, 16, 8, 16, 8, 8)
#else
SPR_DEFINE_PLAN(256, 8, 16, 4, 8, 8)
SPR_DEFINE_PLAN(512, 8, 8, 8, 8, 8)
SPR_DEFINE_PLAN(384, 12, 8, 4, 4, 4, 6)
SPR_DEFINE_PLAN(768, 12, 8, 4, 4, 4, 12)
SPR_DEFINE_PLAN(1024, 16, 8, 8, 8, 16)
#endif

// ---------------------------------------------------------------------------
// Small DFT butterflies, in place: a[k] <- sum_r a[r] exp(DIR 2 pi i r k / R)
// ---------------------------------------------------------------------------
template <int DIR> __device__ __forceinline__ void dft2(float2& a0, float2& a1) {
  float2 t = a0;
  a0 = cadd(t, a1);
  a1 = csub(t, a1);
}

template <int DIR> __device__ __forceinline__ void dft3(float2& a0, float2& a1, float2& a2) {
  const float h = 0.86602540378443864676f;  // sin(2 pi / 3)
  float2 s = cadd(a1, a2), d = csub(a1, a2);
  float2 m = make_float2(fmaf(-0.5f, s.x, a0.x), fmaf(-0.5f, s.y, a0.y));
  float2 r = mul_i<DIR>(cscale(d, h));
  a0 = cadd(a0, s);
  a1 = cadd(m, r);
  a2 = csub(m, r);
}

template <int DIR> __device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  float2 t2 = cadd(a1, a3), t3 = mul_i<DIR>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <int DIR> __device__ __forceinline__ void dft8(float2* a) {
  // even/odd split: X[k] = E[k] + w^k O[k], X[k+4] = E[k] - w^k O[k]
  const float c = 0.70710678118654752440f;
  float2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  float2 o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  // w = exp(DIR i pi/4): w o1 = c u1 and w^3 o3 = c u3 with u1 = (1 + DIR i) o1,
  // u3 = (-1 + DIR i) o3; the factor c goes into multiply-adds
  const float2 u1 = make_float2(o1.x - DIR * o1.y, o1.y + DIR * o1.x);
  const float2 w2o2 = mul_i<DIR>(o2);
  const float2 u3 = make_float2(-o3.x - DIR * o3.y, -o3.y + DIR * o3.x);
  a[0] = cadd(e0, o0);
  a[4] = csub(e0, o0);
  a[1] = make_float2(fmaf(c, u1.x, e1.x), fmaf(c, u1.y, e1.y));
  a[5] = make_float2(fmaf(-c, u1.x, e1.x), fmaf(-c, u1.y, e1.y));
  a[2] = cadd(e2, w2o2);
  a[6] = csub(e2, w2o2);
  a[3] = make_float2(fmaf(c, u3.x, e3.x), fmaf(c, u3.y, e3.y));
  a[7] = make_float2(fmaf(-c, u3.x, e3.x), fmaf(-c, u3.y, e3.y));
}

template <int DIR> __device__ __forceinline__ void dft16(float2* a) {
  // n = 4 n1 + n2, k = k1 + 4 k2
  float2 b[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    float2 x0 = a[n2], x1 = a[4 + n2], x2 = a[8 + n2], x3 = a[12 + n2];
    dft4<DIR>(x0, x1, x2, x3);
    b[n2][0] = x0;
    b[n2][1] = x1;
    b[n2][2] = x2;
    b[n2][3] = x3;
  }
  // twiddles exp(DIR 2 pi i m / 16), m = n2 * k1
  const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;
  const float c2 = 0.70710678118654752440f;
  const float2 w[10] = {
      make_float2(1.f, 0.f),        make_float2(c1, DIR * s1),    make_float2(c2, DIR * c2),
      make_float2(s1, DIR * c1),    make_float2(0.f, (float)DIR), make_float2(-s1, DIR * c1),
      make_float2(-c2, DIR * c2),   make_float2(-c1, DIR * s1),   make_float2(-1.f, 0.f),
      make_float2(-c1, -DIR * s1)};
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) b[n2][k1] = cmul(b[n2][k1], w[n2 * k1]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 x0 = b[0][k1], x1 = b[1][k1], x2 = b[2][k1], x3 = b[3][k1];
    dft4<DIR>(x0, x1, x2, x3);
    a[k1] = x0;
    a[k1 + 4] = x1;
    a[k1 + 8] = x2;
    a[k1 + 12] = x3;
  }
}

// Radices 6 = 2 x 3 and 12 = 4 x 3 as prime-factor (Good-Thomas) transforms:
// with coprime factors R = R1 R2, input n = (R2 n1 + R1 n2) mod R and output
// k = (R2 (R2^-1 mod R1) k1 + R1 (R1^-1 mod R2) k2) mod R turn the R-point DFT
// into R1-point DFTs over n1 and R2-point DFTs over n2 with no twiddles.
template <int DIR> __device__ __forceinline__ void dft6(float2* a) {
  // n = 3 n1 + 2 n2, k = 3 k1 + 4 k2 (mod 6)
  float2 b[2][3];
#pragma unroll
  for (int n2 = 0; n2 < 3; ++n2) {
    float2 x0 = a[(2 * n2) % 6], x1 = a[(3 + 2 * n2) % 6];
    dft2<DIR>(x0, x1);
    b[0][n2] = x0;
    b[1][n2] = x1;
  }
#pragma unroll
  for (int k1 = 0; k1 < 2; ++k1) {
    float2 y0 = b[k1][0], y1 = b[k1][1], y2 = b[k1][2];
    dft3<DIR>(y0, y1, y2);
    a[(3 * k1) % 6] = y0;
    a[(3 * k1 + 4) % 6] = y1;
    a[(3 * k1 + 8) % 6] = y2;
  }
}

template <int DIR> __device__ __forceinline__ void dft12(float2* a) {
  // n = 3 n1 + 4 n2, k = 9 k1 + 4 k2 (mod 12)
  float2 b[4][3];
#pragma unroll
  for (int n2 = 0; n2 < 3; ++n2) {
    float2 x0 = a[(4 * n2) % 12], x1 = a[(3 + 4 * n2) % 12], x2 = a[(6 + 4 * n2) % 12],
           x3 = a[(9 + 4 * n2) % 12];
    dft4<DIR>(x0, x1, x2, x3);
    b[0][n2] = x0;
    b[1][n2] = x1;
    b[2][n2] = x2;
    b[3][n2] = x3;
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 y0 = b[k1][0], y1 = b[k1][1], y2 = b[k1][2];
    dft3<DIR>(y0, y1, y2);
    a[(9 * k1) % 12] = y0;
    a[(9 * k1 + 4) % 12] = y1;
    a[(9 * k1 + 8) % 12] = y2;
  }
}

template <int R, int DIR> __device__ __forceinline__ void butterfly(float2* a) {
  if constexpr (R == 2) dft2<DIR>(a[0], a[1]);
  else if constexpr (R == 3) dft3<DIR>(a[0], a[1], a[2]);
  else if constexpr (R == 4) dft4<DIR>(a[0], a[1], a[2], a[3]);
  else if constexpr (R == 6) dft6<DIR>(a);
  else if constexpr (R == 8) dft8<DIR>(a);
  else if constexpr (R == 12) dft12<DIR>(a);
  else if constexpr (R == 16) dft16<DIR>(a);
  else static_assert(R == 2, "unsupported radix");
}

// Twiddle exp(DIR 2 pi i e / N) from the forward table.
template <int DIR> __device__ __forceinline__ float2 twiddle(const float2* __restrict__ tw, int e) {
  float2 w = tw[e];
  return DIR < 0 ? w : cconj(w);
}

#ifndef SPR_TW_MODE
#define SPR_TW_MODE 1
#endif

// Twiddles w[r] = exp(DIR 2 pi i r b / N), r = 1..R-1.  Mode 1 loads the
// power-of-two multiples (b, 2b, 4b, 8b) and forms the others as products of
// two or three table values (a few ulp), cutting the table loads from R-1 to
// log2 R for the power-of-two radices.
template <int R, int DIR>
__device__ __forceinline__ void twiddles_for(const float2* __restrict__ tw, int b, float2* w) {
  if constexpr (SPR_TW_MODE == 0 || R <= 3 || (R & (R - 1)) != 0) {
    // every value from the table (also for radices that are not powers of two)
#pragma unroll
    for (int r = 1; r < R; ++r) w[r] = twiddle<DIR>(tw, r * b);
  } else {
    w[1] = twiddle<DIR>(tw, b);
    w[2] = twiddle<DIR>(tw, 2 * b);
    w[3] = cmul(w[1], w[2]);
    if constexpr (R >= 8) {
      w[4] = twiddle<DIR>(tw, 4 * b);
      w[5] = cmul(w[1], w[4]);
      w[6] = cmul(w[2], w[4]);
      w[7] = cmul(w[3], w[4]);
    }
    if constexpr (R >= 16) {
      w[8] = twiddle<DIR>(tw, 8 * b);
#pragma unroll
      for (int r = 9; r < 16; ++r) w[r] = cmul(w[r - 8], w[8]);
    }
  }
}

// LDS addressing of one transform: element position `pos` lives at
// (pos + pos / PAD) * ES (PAD = 0: no padding).  WAVE = true when every
// transform sharing the buffer is held by a single wavefront, so exchanges
// need only wavefront-scope ordering, not a workgroup barrier.
template <int ES_, int PAD_, bool WAVE_> struct Lds {
  static constexpr int ES = ES_;
  static constexpr int PAD = PAD_;
  static constexpr bool WAVE = WAVE_;
  __device__ static __forceinline__ int at(int pos) { return (PAD ? pos + pos / PAD : pos) * ES; }
  __host__ __device__ static constexpr int span(int n) { return PAD ? n + n / PAD : n; }
};

template <bool WAVE> __device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    // LDS operations of one wavefront complete in order; the fences keep the
    // compiler from moving LDS accesses across the exchange point
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Per-thread twiddle set: the twiddles of every pass after the first, for the
// butterflies of thread t, in the forward direction.  A kernel that runs
// several transforms (inverse ones use the conjugates) loads them once.
// A pass whose stride NS (product of the earlier radices) divides T gives
// every butterfly j = t + k T of a thread the same twiddles (j mod NS =
// t mod NS): they are formed once per pass instead of once per butterfly.
template <int N> __host__ __device__ constexpr int pass_ns(int pass) {
  using P = Plan<N>;
  int ns = 1;
  for (int p = 0; p < pass; ++p) ns *= P::radix(p);
  return ns;
}
template <int N> __host__ __device__ constexpr bool tw_shared(int pass) { return Plan<N>::T % pass_ns<N>(pass) == 0; }
template <int N, int PASS> __host__ __device__ constexpr int tw_offset() {
  using P = Plan<N>;
  int off = 0;
  for (int p = 1; p < PASS && p < P::passes(); ++p)
    off += (tw_shared<N>(p) ? 1 : P::E / P::radix(p)) * (P::radix(p) - 1);
  return off;
}
template <int N> __host__ __device__ constexpr int tw_count() { return tw_offset<N, 64>(); }
// keep the set in registers only when it is small
#ifndef SPR_TWSET
#define SPR_TWSET 1
#endif
#ifndef SPR_TWSET_MAX
#define SPR_TWSET_MAX 20
#endif
template <int N> constexpr bool tw_in_regs() {
  return SPR_TWSET && tw_count<N>() > 0 && tw_count<N>() <= SPR_TWSET_MAX;
}

template <int N> struct TwSet {
  float2 w[tw_count<N>() > 0 ? tw_count<N>() : 1];
};

template <int N, int PASS, int NS>
__device__ __forceinline__ void fill_tw(TwSet<N>& s, int t, const float2* __restrict__ tw) {
  using P = Plan<N>;
  if constexpr (PASS < P::passes()) {
    constexpr int R = P::radix(PASS), NB = P::E / R, T = P::T;
    if constexpr (PASS > 0) {
      constexpr int step = N / (NS * R);
      constexpr int NK = tw_shared<N>(PASS) ? 1 : NB;
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        float2 w[R];
        twiddles_for<R, -1>(tw, ((t + k * T) % NS) * step, w);
#pragma unroll
        for (int r = 1; r < R; ++r) s.w[tw_offset<N, PASS>() + k * (R - 1) + r - 1] = w[r];
      }
    }
    fill_tw<N, PASS + 1, NS * R>(s, t, tw);
  }
}

template <int N>
__device__ __forceinline__ void load_twiddle_set(TwSet<N>& s, int t, const float2* __restrict__ tw) {
  if constexpr (tw_in_regs<N>()) fill_tw<N, 0, 1>(s, t, tw);
}

// One Stockham pass (and, recursively, the following ones).  With a twiddle
// set (PRE) the pass takes its twiddles from registers.
template <int N, int DIR, int PASS, int NS, class L, bool PRE = false>
__device__ __forceinline__ void fft_passes(float2 (&v)[Plan<N>::E], float2* lds, int t,
                                           const float2* __restrict__ tw, const TwSet<N>* ws = nullptr) {
  using P = Plan<N>;
  if constexpr (PASS < P::passes()) {
    constexpr int R = P::radix(PASS);
    constexpr int E = P::E, T = P::T;
    constexpr int NB = E / R;
    constexpr bool LAST = (PASS == P::passes() - 1);
    static_assert(E % R == 0, "plan: E must be a multiple of every radix");
    constexpr bool SHARED = tw_shared<N>(PASS);
    constexpr int step = N / (NS * R);
    // twiddles common to all butterflies of the thread (stride dividing T)
    float2 wsh[R];
    if constexpr (NS > 1 && SHARED && !PRE) twiddles_for<R, DIR>(tw, (t % NS) * step, wsh);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int j = t + k * T;
      float2 a[R];
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] = v[k + r * NB];
      if constexpr (NS > 1) {
        if constexpr (PRE) {
          constexpr int KS = SHARED ? 0 : 1;
#pragma unroll
          for (int r = 1; r < R; ++r) {
            const float2 w = ws->w[tw_offset<N, PASS>() + KS * k * (R - 1) + r - 1];
            a[r] = cmul(a[r], DIR < 0 ? w : cconj(w));
          }
        } else if constexpr (SHARED) {
#pragma unroll
          for (int r = 1; r < R; ++r) a[r] = cmul(a[r], wsh[r]);
        } else {
          float2 w[R];
          twiddles_for<R, DIR>(tw, (j % NS) * step, w);
#pragma unroll
          for (int r = 1; r < R; ++r) a[r] = cmul(a[r], w[r]);
        }
      }
      butterfly<R, DIR>(a);
      if constexpr (LAST) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[k + r * NB] = a[r];
      } else {
        const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) lds[L::at(base + r * NS)] = a[r];
      }
    }
    if constexpr (!LAST) {
      lds_sync<L::WAVE>();
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = lds[L::at(t + T * m)];
      lds_sync<L::WAVE>();
      fft_passes<N, DIR, PASS + 1, NS * R, L, PRE>(v, lds, t, tw, ws);
    }
  }
}

// Transform the E register elements of thread t (positions t + T*m).
// Every thread sharing the buffer must call this (it contains barriers).
template <int N, int DIR, class L>
__device__ __forceinline__ void fft(float2 (&v)[Plan<N>::E], float2* lds, int t,
                                    const float2* __restrict__ tw) {
  fft_passes<N, DIR, 0, 1, L>(v, lds, t, tw);
}

// Same, with the thread's twiddle set from load_twiddle_set (used when the set
// fits in registers, otherwise twiddles are formed per pass).
template <int N, int DIR, class L>
__device__ __forceinline__ void fft(float2 (&v)[Plan<N>::E], float2* lds, int t,
                                    const float2* __restrict__ tw, const TwSet<N>& ws) {
  if constexpr (tw_in_regs<N>()) fft_passes<N, DIR, 0, 1, L, true>(v, lds, t, tw, &ws);
  else fft_passes<N, DIR, 0, 1, L>(v, lds, t, tw);
}

}  // namespace spr
