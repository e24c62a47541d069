// Size-specialised kernels of the projection loop, compiled once per detector
// size N (macro SPR_N).  Every 2D transform is two passes through HBM:
//
//   row pass     one workgroup owns RW whole rows; each row is one Stockham
//                transform in LDS; the real-space work (support/phase
//                projection, ER/HIO/RAAR update, shrink-wrap masking) is fused
//                around the row transforms;
//   column pass  one workgroup owns a tile of C adjacent columns; the masked
//                modulus projection (Eq. pm_full) or the fitness residual
//                (Eq. error_calc) is fused between the forward and inverse
//                column transforms.
//
// The iterate is kept as its row transform T = rowFFT(x): a column pass turns
// T into rowFFT(P_M x) and the next row pass turns that back into the next
// iterate's row transform, so each iteration is one read-write sweep per pass.
#include <type_traits>

#include <hip/hip_ext.h>

#include "common.hpp"
#include "fft.hpp"

#ifndef SPR_N
#error "SPR_N must be defined"
#endif

namespace spr {
namespace {

constexpr int N = SPR_N;
using PL = Plan<N>;
constexpr int E = PL::E;
constexpr int T = PL::T;
#if defined(SPR_COLS)
constexpr int C = (N % SPR_COLS == 0) ? SPR_COLS : PL::C;
#else
constexpr int C = PL::C;
#endif
constexpr int RW = PL::RW;
constexpr size_t NN = (size_t)N * N;

#ifndef SPR_ROW_PAD
#define SPR_ROW_PAD 8
#endif
#ifndef SPR_ROW_WAVE
#define SPR_ROW_WAVE 1
#endif
// Row transforms: one row per T lanes; rows held within one wavefront (T
// divides 64) synchronise their LDS exchanges per wave, longer rows (T a
// multiple of 64) the workgroup.  The column tile interleaves C transforms
// across the workgroup.
constexpr bool kRowWave = SPR_ROW_WAVE != 0 && 64 % T == 0;
static_assert(kRowWave || T % 64 == 0, "a row transform must fill whole wavefronts or fit in one");
using RowL = Lds<1, SPR_ROW_PAD, kRowWave>;
#ifndef SPR_COL_PAD
#define SPR_COL_PAD 0
#endif
// column tile: position p of column c at (p + p / PAD) * C + c
using ColL = Lds<C, SPR_COL_PAD, false>;
constexpr size_t kColLdsBytes() { return (size_t)C * ColL::span(N) * sizeof(float2); }
constexpr int NR = RowL::span(N);  // LDS elements per row
static_assert(N % C == 0, "column tile must divide N");

// rows per workgroup for kernels whose workgroups must not straddle images
constexpr int rows_within_image() {
  int r = RW < N ? RW : N;
  while (N % r != 0) --r;
  return r;
}
constexpr int RWI = rows_within_image();
// When RW divides N the row grid covers the rows exactly, so no row of a
// launch is out of range and the per-element guards compile away.
constexpr bool kRowsExact = N % RW == 0;
// A launch processes whole members of N rows.  When every wavefront's rows lie
// in one member, the member index is wave-uniform, and the member's slot and
// descriptor are read with scalar loads, apart from the vector loads of the
// row data (whose completion is counted in order).
constexpr bool kWaveOneMember = kRowsExact && (T >= 64 || N % (64 / T) == 0);
__device__ __forceinline__ int row_member(int grow) {
  const int m = grow / N;
  if constexpr (kWaveOneMember) return __builtin_amdgcn_readfirstlane(m);
  return m;
}

// Pointers read from a descriptor in device memory are not known to the
// compiler to be global; these views make the loads global (vector memory
// only) instead of flat.
template <class V> using GPtr = const __attribute__((address_space(1))) V*;
template <class V> __device__ __forceinline__ GPtr<V> gview(const V* p) { return (GPtr<V>)p; }
typedef float F2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 gload(const float2* p, size_t i) {
  const F2v v = gview(reinterpret_cast<const F2v*>(p))[i];
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void gstore(float2* p, size_t i, float2 v) {
  ((__attribute__((address_space(1))) F2v*)(p))[i] = F2v{v.x, v.y};
}

// Buffer descriptors for the column tiles: a lane's E accesses t + T*m of
// one column split into one per-lane byte offset (a VGPR) and a per-element
// constant (an SGPR), so they need no vector address arithmetic.  The
// descriptor's range check (num_records bytes) makes any offset outside the
// array read 0 and drop its write.
typedef __amdgpu_buffer_rsrc_t BufRes;
__device__ __forceinline__ BufRes buf_res(const void* p, size_t bytes) {
  // gfx9 descriptor word 3: raw (untyped) 32-bit data format
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}
typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(BufRes(), 0, 0, 0)) B64;
constexpr int kColStep8 = T * N * 8;  // bytes between a lane's column elements (complex FP32)
__device__ __forceinline__ void col_load(float2 (&v)[E], BufRes r, int voff) {
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const F2v q = __builtin_bit_cast(F2v, __builtin_amdgcn_raw_buffer_load_b64(r, voff, m * kColStep8, 0));
    v[m] = make_float2(q.x, q.y);
  }
}
__device__ __forceinline__ void col_store(const float2 (&v)[E], BufRes r, int voff) {
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const F2v q = {v[m].x, v[m].y};
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(B64, q), r, voff, m * kColStep8, 0);
  }
}


// Nearest point of {|arg z| <= chi pi} (positivity: Re z >= 0 exactly).
// The real-space arithmetic below spells out every rounding (__fmul_rn,
// fmaf), so that the run-time and the specialised forms of a kernel, which
// the compiler would otherwise contract differently, give identical bits.
// The constraint form is a template argument: launches resolve it once (it is
// uniform), and the element loops are then straight-line code with selects.
template <int MODE>
__device__ __forceinline__ float2 proj_phase(float2 z, const Phase& ph) {
  if constexpr (MODE == PHASE_OFF) {
    return z;
  } else if constexpr (MODE == PHASE_POS) {
    return make_float2(fmaxf(z.x, 0.f), z.y);
  } else {
    const float aim = fabsf(z.y);
    const bool inside = __fmul_rn(aim, ph.c) <= __fmul_rn(z.x, ph.s);
    const float p = fmaxf(fmaf(z.x, ph.c, __fmul_rn(aim, ph.s)), 0.f);
    const float ps = __fmul_rn(p, ph.s);
    const float2 r = make_float2(__fmul_rn(p, ph.c), z.y < 0.f ? -ps : ps);
    return inside ? z : r;
  }
}

template <int MODE>
__device__ __forceinline__ bool inside_phase(float2 z, const Phase& ph) {
  if constexpr (MODE == PHASE_OFF) return true;
  else if constexpr (MODE == PHASE_POS) return z.x >= 0.f;
  else return __fmul_rn(fabsf(z.y), ph.c) <= __fmul_rn(z.x, ph.s);
}

__device__ __forceinline__ void issue_fence() { asm volatile("" ::: "memory"); }


// The modulus values of a column tile's elements t + T*m of column col; the
// storage form (FP32 or FP16) is uniform, so it is resolved once.
__device__ __forceinline__ void load_col_amp(float (&mv)[E], const float* amp, const __half* amp16, int t,
                                             int col) {
  if (amp16) {
    const BufRes r = buf_res(amp16, NN * 2);
    const int voff = (t * N + col) * 2;
#pragma unroll
    for (int m = 0; m < E; ++m)
      mv[m] = __half2float(__ushort_as_half(__builtin_amdgcn_raw_buffer_load_b16(r, voff, m * T * N * 2, 0)));
  } else {
    const BufRes r = buf_res(amp, NN * 4);
    const int voff = (t * N + col) * 4;
#pragma unroll
    for (int m = 0; m < E; ++m)
      mv[m] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, m * T * N * 4, 0));
  }
}
__device__ __forceinline__ void load_col_amp(float (&mv)[E], const SlotDesc& d, int t, int col) {
  load_col_amp(mv, d.amp, d.amp16, t, col);
}

template <int M> using ModeC = std::integral_constant<int, M>;
// Calls f(ModeC<mode>{}) for a phase-constraint mode known only at run time.
template <class F>
__device__ __forceinline__ void with_phase_mode(int mode, F&& f) {
  if (mode == PHASE_OFF) f(ModeC<PHASE_OFF>{});
  else if (mode == PHASE_POS) f(ModeC<PHASE_POS>{});
  else f(ModeC<PHASE_CONE>{});
}

// Support bits of a lane's row elements t + T*m, packed into one mask (bit m)
// as soon as the words arrive, so that one register holds them.
__device__ __forceinline__ uint32_t load_row_mask(const uint32_t* __restrict__ S, int row, int t) {
  static_assert(E <= 32, "one mask bit per element");
  uint32_t w[E];
#pragma unroll
  for (int m = 0; m < E; ++m) w[m] = gview(S)[(row * N + t + T * m) >> 5];
  uint32_t mask = 0;
#pragma unroll
  for (int m = 0; m < E; ++m) mask |= ((w[m] >> ((row * N + t + T * m) & 31)) & 1u) << m;
  return mask;
}
__device__ __forceinline__ bool mask_bit(uint32_t mask, int m) { return (mask >> m) & 1u; }
// Makes v materialise here (no instruction of its own).
__device__ __forceinline__ void materialise(uint32_t v) { asm volatile("" ::"v"(v)); }

// Column-tile placement.  Workgroups go to the 8 XCDs round-robin by linear
// id, and each XCD has its own L2.  A tile of C columns reads 8C bytes of every
// 128-byte line, so G = 128 / 8C neighbouring tiles share lines; they are given
// to workgroups lin, lin+8, ..., which run back to back on one XCD, so each
// line is fetched from HBM once.  Grid: (N/C tiles, images).
struct TileId {
  int tile, img;
};
__device__ __forceinline__ TileId col_tile_id() {
  constexpr int ntiles = N / C;
  constexpr int G = (8 * C >= 128) ? 1 : 128 / (8 * C);
  const int total = ntiles * (int)gridDim.y;
  if (G == 1 || ntiles % G != 0 || total % (8 * G) != 0) return {(int)blockIdx.x, (int)blockIdx.y};
  const int lin = blockIdx.x + blockIdx.y * ntiles;
  const int x = lin & 7, h = (lin >> 3) % G, q = lin / (8 * G);
  const int ltile = (8 * q + x) * G + h;
  return {ltile % ntiles, ltile / ntiles};
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// 1/sqrt(x) for x > 0 from the hardware reciprocal square root; a subnormal x
// (|X| below 1e-19, which FFT outputs of measured data do not reach) is first
// scaled into the normal range (2^24 x, result times 2^12).  The test is a
// wavefront vote, so the common case is one compare and one rsq.
__device__ __forceinline__ float rsqrt_pos(float x) {
  const bool tiny = x < 1.17549435e-38f;
  if (__builtin_expect(__builtin_amdgcn_ballot_w64(tiny) != 0, 0))
    return tiny ? __fmul_rn(__builtin_amdgcn_rsqf(__fmul_rn(x, 16777216.f)), 4096.f) : __builtin_amdgcn_rsqf(x);
  return __builtin_amdgcn_rsqf(x);
}

// Masked modulus replacement (Eq. pm_full) on the unnormalised column
// spectrum X = N * (unitary value), returning the projected unitary value
// divided by N, the input of the unnormalised inverse column transform; both
// normalisations are folded into one factor per element.  Measured pixels get
// modulus M with the current phase (phase 0 if X = 0).  An unknown pixel
// stores minus its amplitude bound (-0: none); a unitary value above the
// bound b is brought down to it with its phase (Eq. pm_bounds).  The branches
// follow the mask, which is coherent over neighbouring pixels.
__device__ __forceinline__ float2 modulus_replace(float2 X, float stored, float scale, float inv, float scale_inv) {
  const float m2 = fmaf(X.x, X.x, __fmul_rn(X.y, X.y));
  if (signbit(stored)) {
    const float b = __fmul_rn(-stored, scale);
    const float bn = __fmul_rn(b, (float)N);  // the bound on |X|
    if (b > 0.f && m2 > __fmul_rn(bn, bn)) return cscale(X, __fmul_rn(__fmul_rn(b, inv), rsqrt_pos(m2)));
    return cscale(X, __fmul_rn(inv, inv));
  }
  const float Mn = __fmul_rn(stored, scale_inv);  // scale_inv = scale / N
  if (m2 > 0.f) return cscale(X, __fmul_rn(Mn, rsqrt_pos(m2)));
  return make_float2(Mn, 0.f);
}

// ---------------------------------------------------------------------------
// Row ingest: real-space density -> (optional constraint) -> row FFT.
// ---------------------------------------------------------------------------
// Row group blk (rows blk*RW ... of the launch's members) of the ingest.
__device__ __forceinline__ void row_ingest_body(RowIngestArgs a, int blk, float2* lds) {
  const int tid = threadIdx.x;
  const int r = tid / T, t = tid % T;
  const int grow = blk * RW + r;
  const bool valid = kRowsExact || grow < a.nm * N;
  const int member = valid ? row_member(grow) : 0;
  const int row = valid ? grow % N : 0;
  const SlotDesc d = a.desc[a.slots[member]];
  const size_t off = (size_t)row * N;                         // within the member's density
  const size_t toff = (size_t)member * NN + (size_t)row * N;  // work buffer: by launch position
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = valid ? gload(d.X, off + t + T * m) : make_float2(0.f, 0.f);
  if (a.mode != INGEST_PLAIN) {
    const uint32_t smask = load_row_mask(d.S, row, t);
    const int mode = a.mode == INGEST_PC ? a.ph.mode : PHASE_OFF;
    with_phase_mode(mode, [&](auto MC) {
#pragma unroll
      for (int m = 0; m < E; ++m)
        v[m] = mask_bit(smask, m) ? proj_phase<MC.value>(v[m], a.ph) : make_float2(0.f, 0.f);
    });
  }
  fft<N, -1, RowL>(v, lds + r * NR, t, a.tw);
  float2* Tw = a.t_by_slot ? d.T + off : a.T + toff;
  if (valid) {
#pragma unroll
    for (int m = 0; m < E; ++m) gstore(Tw, t + T * m, v[m]);
  }
}

__global__ __launch_bounds__(RW* T) void k_row_ingest(RowIngestArgs a) {
  extern __shared__ float2 lds[];
  row_ingest_body(a, blockIdx.x, lds);
}

// ---------------------------------------------------------------------------
// Column projection: column FFT -> masked P_M -> column IFFT.
// ---------------------------------------------------------------------------
// One member's column tile, loaded into v (and its modulus values into mv):
// transform, project, transform back, store into dst.  TRACE also sums the
// FP64 residual Xi (|X| - M)^2 of the spectrum being projected over the tile
// (the iterate's Fourier error, before P_M) and writes it to *trace_out.
template <bool TRACE>
__device__ __forceinline__ void col_proj_tile(float2 (&v)[E], const float (&mv)[E], float amp_scale, float2* lds,
                                              int tid, int c, int t, int col, const TwSet<N>& ws,
                                              const float2* __restrict__ tw, float2* dst, double* trace_out) {
  fft<N, -1, ColL>(v, lds + c, t, tw, ws);
  const float inv = 1.0f / (float)N;
  double acc = 0.0;
  if constexpr (TRACE) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      if (!signbit(mv[m])) {
        const float m2 = fmaf(v[m].x, v[m].x, __fmul_rn(v[m].y, v[m].y));
        const double df = (double)__fmul_rn(sqrtf(m2), inv) - (double)__fmul_rn(mv[m], amp_scale);
        acc = fma(df, df, acc);
      }
    }
  }
  const float scale_inv = __fmul_rn(amp_scale, inv);
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = modulus_replace(v[m], mv[m], amp_scale, inv, scale_inv);
  fft<N, +1, ColL>(v, lds + c, t, tw, ws);
  col_store(v, buf_res(dst, NN * 8), (t * N + col) * 8);
  if constexpr (TRACE) {
    acc = wave_sum(acc);
    double* wsum = reinterpret_cast<double*>(lds);  // the transform left the tile buffer free
    if ((tid & 63) == 0) wsum[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
      for (int w = 0; w < (C * T + 63) / 64; ++w) sum += wsum[w];
      *trace_out = sum;
    }
    __syncthreads();  // the tile buffer is reused by the next transform
  }
}

// Column tile id of the projection.
template <bool TRACE>
__device__ __forceinline__ void col_proj_body(ColProjArgs a, TileId id, float2* lds) {
  const int tid = threadIdx.x;
  const int c = tid % C, t = tid / C;
  const int col = id.tile * C + c;
  float2* dst = a.Y + (size_t)id.img * NN;
  const SlotDesc d = a.desc[a.slots[id.img]];
  const float2* src = a.t_by_slot ? d.T : a.T + (size_t)id.img * NN;
  float2 v[E];
  float mv[E];
  col_load(v, buf_res(src, NN * 8), (t * N + col) * 8);
  load_col_amp(mv, d, t, col);
  issue_fence();
  TwSet<N> ws;
  load_twiddle_set<N>(ws, t, a.tw);
  col_proj_tile<TRACE>(v, mv, d.amp_scale, lds, tid, c, t, col, ws, a.tw, dst,
                       TRACE ? a.trace_partial + (size_t)id.img * (N / C) + id.tile : nullptr);
}

template <bool TRACE>
__global__ __launch_bounds__(C* T) void k_col_proj(ColProjArgs a) {
  extern __shared__ float2 lds[];
  col_proj_body<TRACE>(a, col_tile_id(), lds);
}

// ---------------------------------------------------------------------------
// Row update: row IFFTs -> ER/HIO/RAAR real-space step -> next row FFT (or the
// final real-space density).
// ---------------------------------------------------------------------------
// SPEC 0 takes the algorithm at run time (per-member parameters); 1, 2, 3 are
// ER, HIO and RAAR compiled alone, which frees the registers of the paths a
// uniform launch never takes.
// Row group blk of the row pass.
template <int SPEC>
__device__ __forceinline__ void row_update_body(RowUpdateArgs a, int blk, float2* lds) {
  const int tid = threadIdx.x;
  const int r = tid / T, t = tid % T;
  const int grow = blk * RW + r;
  const bool valid = kRowsExact || grow < a.nm * N;
  const int member = valid ? row_member(grow) : 0;
  const int row = valid ? grow % N : 0;
  const SlotDesc d = a.desc[a.slots[member]];
  const size_t off = (size_t)row * N;                         // within the member's density
  const size_t toff = (size_t)member * NN + (size_t)row * N;  // work buffers: by launch position
  float2* l = lds + r * NR;
  int alg = a.alg, out_mode = a.out_mode;
  float beta = a.beta;
  Phase ph = a.ph, ph_next = a.ph_next;
  if (SPEC == 0 && a.ip) {
    // per-member parameters (rows of one member share them; a wavefront may
    // hold rows of several members when N is small, which is safe because the
    // row transforms only synchronise within their own wavefront)
    const IterParam q = a.ip[member];
    alg = q.alg;
    out_mode = q.out_mode;
    beta = q.beta;
    ph = q.ph;
    ph_next = q.ph_next;
  }
  if constexpr (SPEC == 1) alg = ALG_ER;
  if constexpr (SPEC == 2) alg = ALG_HIO;
  if constexpr (SPEC == 3) alg = ALG_RAAR;

  const bool ia = alg != ALG_ER;
  float2* Tw = a.t_by_slot ? d.T + off : a.T + toff;
  TwSet<N> ws;
  load_twiddle_set<N>(ws, t, a.tw);  // first: the table is cache-resident
  // the support words first: their mask is formed while the row data are
  // still in flight (loads complete in issue order)
  const uint32_t smask = (ia || out_mode == OUT_T_PC) ? load_row_mask(d.S, row, t) : 0u;
  float2 y[E], x[E];
#pragma unroll
  for (int m = 0; m < E; ++m) y[m] = valid ? gload(a.Y, toff + t + T * m) : make_float2(0.f, 0.f);
  if (ia) {
#pragma unroll
    for (int m = 0; m < E; ++m) x[m] = valid ? gload(Tw, t + T * m) : make_float2(0.f, 0.f);
  }
  // keep every load of the row ahead of the first transform (compiler fence
  // only: no instruction), so that all of them are in flight together
  issue_fence();
  materialise(smask);
  fft<N, +1, RowL>(y, l, t, a.tw, ws);  // y = P_M x (real space)

  float2 xn[E];
  if (!ia) {
#pragma unroll
    for (int m = 0; m < E; ++m) xn[m] = y[m];
  } else {
    fft<N, +1, RowL>(x, l, t, a.tw, ws);
    const float inv = 1.0f / (float)N;
    with_phase_mode(ph.mode, [&](auto MC) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const float2 xv = make_float2(__fmul_rn(x[m].x, inv), __fmul_rn(x[m].y, inv));
        const float2 yv = y[m];
        const bool s = mask_bit(smask, m);
        if (alg == ALG_HIO) {
          const bool feasible = s & inside_phase<MC.value>(yv, ph);
          xn[m] = feasible ? yv : make_float2(fmaf(-beta, yv.x, xv.x), fmaf(-beta, yv.y, xv.y));
        } else {  // RAAR
          const float2 z = make_float2(fmaf(2.f, yv.x, -xv.x), fmaf(2.f, yv.y, -xv.y));
          const float2 pz = proj_phase<MC.value>(z, ph);
          const float2 pc = s ? pz : make_float2(0.f, 0.f);
          const float g = fmaf(-2.f, beta, 1.f);
          xn[m] = make_float2(fmaf(beta, pc.x, fmaf(beta, xv.x, __fmul_rn(g, yv.x))),
                              fmaf(beta, pc.y, fmaf(beta, xv.y, __fmul_rn(g, yv.y))));
        }
      }
    });
  }

  if (out_mode == OUT_REAL) {
    if (valid) {
#pragma unroll
      for (int m = 0; m < E; ++m) gstore(d.X, off + t + T * m, xn[m]);
    }
    return;
  }
  if (out_mode == OUT_T_PC) {
    with_phase_mode(ph_next.mode, [&](auto MC) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const float2 pz = proj_phase<MC.value>(xn[m], ph_next);
        xn[m] = mask_bit(smask, m) ? pz : make_float2(0.f, 0.f);
      }
    });
  }
  fft<N, -1, RowL>(xn, l, t, a.tw, ws);
  if (valid) {
#pragma unroll
    for (int m = 0; m < E; ++m) gstore(Tw, t + T * m, xn[m]);
  }
}

template <int SPEC>
__global__ __launch_bounds__(RW* T) void k_row_update(RowUpdateArgs a) {
  extern __shared__ float2 lds[];
  row_update_body<SPEC>(a, blockIdx.x, lds);
}

// ---------------------------------------------------------------------------
// Fitness column pass: column FFT of rowFFT(S x), FP64 partial sums of
// Xi (|X| - M)^2 per tile (Eq. error_calc numerator).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(C* T) void k_col_err(ColErrArgs a) {
  extern __shared__ float2 lds[];
  const int tid = threadIdx.x;
  const int c = tid % C, t = tid / C;
  const TileId id = col_tile_id();
  const int col = id.tile * C + c;
  const SlotDesc d = a.desc[a.slots[id.img]];
  const float2* src = a.t_by_slot ? d.T : a.T + (size_t)id.img * NN;
  float2 v[E];
  float mv[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = gload(src, (size_t)(t + T * m) * N + col);
  load_col_amp(mv, d, t, col);
  fft<N, -1, ColL>(v, lds + c, t, a.tw);
  const float inv = 1.0f / (float)N;
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const float stored = mv[m];
    if (!signbit(stored)) {
      const float2 X = cscale(v[m], inv);
      const double df = (double)sqrtf(fmaf(X.x, X.x, __fmul_rn(X.y, X.y))) - (double)(stored * d.amp_scale);
      acc = fma(df, df, acc);
    }
  }
  acc = wave_sum(acc);
  const int nw = (blockDim.x + 63) / 64;
  double* wsum = reinterpret_cast<double*>(lds);  // the transform left the tile buffer free
  if ((tid & 63) == 0) wsum[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += wsum[w];
    a.partial[(size_t)id.img * (N / C) + id.tile] = s;
  }
}

// ---------------------------------------------------------------------------
// Generic row / column transforms (spectra for crossover, the fft2 entry point).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RW* T) void k_row_fft(RowFftArgs a) {
  extern __shared__ float2 lds[];
  const int tid = threadIdx.x;
  const int r = tid / T, t = tid % T;
  const int grow = blockIdx.x * RW + r;
  const bool valid = kRowsExact || grow < a.nm * N;
  const int member = valid ? row_member(grow) : 0;
  const int row = valid ? grow % N : 0;
  const int si = a.slots_in ? a.slots_in[member] : member;
  const int so = a.slots_out ? a.slots_out[member] : member;
  const size_t offi = (size_t)si * NN + (size_t)row * N;
  const size_t offo = (size_t)so * NN + (size_t)row * N;
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = valid ? a.in[offi + t + T * m] : make_float2(0.f, 0.f);
  if (a.dir < 0) fft<N, -1, RowL>(v, lds + r * NR, t, a.tw);
  else fft<N, +1, RowL>(v, lds + r * NR, t, a.tw);
  if (valid) {
#pragma unroll
    for (int m = 0; m < E; ++m) a.out[offo + t + T * m] = cscale(v[m], a.scale);
  }
}

__global__ __launch_bounds__(C* T) void k_col_fft(ColFftArgs a) {
  extern __shared__ float2 lds[];
  const int tid = threadIdx.x;
  const int c = tid % C, t = tid / C;
  const TileId id = col_tile_id();
  const int col = id.tile * C + c;
  const int member = id.img;
  const int si = a.slots_in ? a.slots_in[member] : member;
  const int so = a.slots_out ? a.slots_out[member] : member;
  const float2* src = a.in + (size_t)si * NN;
  float2* dst = a.out + (size_t)so * NN;
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = gload(src, (size_t)(t + T * m) * N + col);
  if (a.dir < 0) fft<N, -1, ColL>(v, lds + c, t, a.tw);
  else fft<N, +1, ColL>(v, lds + c, t, a.tw);
#pragma unroll
  for (int m = 0; m < E; ++m) dst[(size_t)(t + T * m) * N + col] = cscale(v[m], a.scale);
}

// ---------------------------------------------------------------------------
// Reshift cross-correlations (Eq. crosscorr): column IFFT of the masked
// products Xi conj(Xq) Xp (parent as is) and Xi Xq Xp (its twin).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(C* T) void k_col_corr(ColCorrArgs a) {
  extern __shared__ float2 lds[];
  const int tid = threadIdx.x;
  const int c = tid % C, t = tid / C;
  const TileId id = col_tile_id();
  const int col = id.tile * C + c;
  const int pair = id.img;
  const int p = a.ref_idx ? *a.ref_idx : pair / 3;
  const int q = a.ref_idx ? pair : a.abc[pair];
  const float2* Xq = a.F + (size_t)q * NN;
  const float2* Xp = a.F + (size_t)p * NN;
  float2 v1[E], v2[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const size_t i = (size_t)(t + T * m) * N + col;
    const float2 xq = Xq[i], xp = Xp[i];
    const bool known = !signbit(amp_load(a.amp, a.amp16, i));
    v1[m] = known ? cmul(cconj(xq), xp) : make_float2(0.f, 0.f);
    v2[m] = known ? cmul(xq, xp) : make_float2(0.f, 0.f);
  }
  TwSet<N> ws;
  load_twiddle_set<N>(ws, t, a.tw);
  fft<N, +1, ColL>(v1, lds + c, t, a.tw, ws);
  fft<N, +1, ColL>(v2, lds + c, t, a.tw, ws);
  float2* d1 = a.C + (size_t)(2 * pair) * NN;
  float2* d2 = d1 + NN;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const size_t i = (size_t)(t + T * m) * N + col;
    d1[i] = v1[m];
    d2[i] = v2[m];
  }
}

// Row IFFT of the correlation images and per-workgroup argmax of |C|^2
// (ties to the lowest linear index).
__device__ __forceinline__ bool better(float v1, int i1, float v2, int i2) {
  return v1 > v2 || (v1 == v2 && i1 < i2);
}

__global__ __launch_bounds__(RWI* T) void k_row_argmax(RowArgmaxArgs a) {
  extern __shared__ float2 lds[];
  __shared__ ArgmaxRec red[RWI * T];
  const int tid = threadIdx.x;
  const int r = tid / T, t = tid % T;
  const int img = blockIdx.y;
  const int row = blockIdx.x * RWI + r;
  const float2* src = a.C + (size_t)img * NN + (size_t)row * N;
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = src[t + T * m];
  fft<N, +1, RowL>(v, lds + r * NR, t, a.tw);
  ArgmaxRec b;
  b.val = -1.f;
  b.idx = 0x7fffffff;
  b.re = b.im = 0.f;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const float q = fmaf(v[m].x, v[m].x, __fmul_rn(v[m].y, v[m].y));
    const int idx = row * N + t + T * m;
    if (better(q, idx, b.val, b.idx)) {
      b.val = q;
      b.idx = idx;
      b.re = v[m].x;
      b.im = v[m].y;
    }
  }
  constexpr int NT = RWI * T;
  if constexpr (NT % 64 == 0) {
    // wavefront butterfly reduction, then one record per wavefront
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const float ov = __shfl_xor(b.val, o, 64);
      const int oi = __shfl_xor(b.idx, o, 64);
      const float ore = __shfl_xor(b.re, o, 64);
      const float oim = __shfl_xor(b.im, o, 64);
      if (better(ov, oi, b.val, b.idx)) {
        b.val = ov;
        b.idx = oi;
        b.re = ore;
        b.im = oim;
      }
    }
    if ((tid & 63) == 0) red[tid >> 6] = b;
    __syncthreads();
    if (tid == 0) {
      ArgmaxRec best = red[0];
      for (int i = 1; i < NT / 64; ++i)
        if (better(red[i].val, red[i].idx, best.val, best.idx)) best = red[i];
      a.partial[(size_t)img * (N / RWI) + blockIdx.x] = best;
    }
  } else {
    red[tid] = b;
    __syncthreads();
    if (tid == 0) {
      ArgmaxRec best = red[0];
      for (int i = 1; i < NT; ++i)
        if (better(red[i].val, red[i].idx, best.val, best.idx)) best = red[i];
      a.partial[(size_t)img * (N / RWI) + blockIdx.x] = best;
    }
  }
}

// ---------------------------------------------------------------------------
// Crossover mixing in the Fourier domain, fused with the column IFFT:
// aligned parents X' = e^{i phi} e^{-2 pi i k.d/N} (X or conj X); on the
// crossover map X_a' + C_w (X_b' - X_c'), elsewhere the child's own parent.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(C* T) void k_col_mix(ColMixArgs a) {
  extern __shared__ float2 lds[];
  const int tid = threadIdx.x;
  const int c = tid % C, t = tid / C;
  const TileId id = col_tile_id();
  const int col = id.tile * C + c;
  const int p = id.img;
  const int* abc = a.abc + 3 * p;
  const int* mp = a.mapprm + 5 * p;
  const int tx = mp[0], ty = mp[1], sx = mp[2], sy = mp[3];
  int ra, rb, rh;
  rotation(mp[4], ra, rb, rh);
  const AlignRec al[3] = {a.align[3 * p], a.align[3 * p + 1], a.align[3 * p + 2]};
  const float2* Fq[3] = {a.F + (size_t)abc[0] * NN, a.F + (size_t)abc[1] * NN,
                         a.F + (size_t)abc[2] * NN};
  const float2* Fp = a.F + (size_t)p * NN;
  const int vv = col < N / 2 ? col : col - N;
  float2 v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int e = t + T * m;
    const size_t i = (size_t)e * N + col;
    const int u = e < N / 2 ? e : e - N;
    const int ur = ra * u + rb * vv;
    const int vr = -rb * u + ra * vv;
    const int qx = floor_div(ur + rh * sx, rh * tx);
    const int qy = floor_div(vr + rh * sy, rh * ty);
    const uint32_t key = ((uint32_t)(qx & 0xFFFF) << 16) | (uint32_t)(qy & 0xFFFF);
    const U4 o = philox4x32_10(key, (uint32_t)p, (uint32_t)a.gen, PURPOSE_TILE, (uint32_t)a.seed,
                               (uint32_t)(a.seed >> 32));
    float2 out;
    if ((uint64_t)o.v[0] < a.cp_thr) {
      float2 xs[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        float2 xq = Fq[k][i];
        if (al[k].twin) xq = cconj(xq);
        const int ridx = (int)(((long long)e * al[k].dr + (long long)col * al[k].dc) % N);
        const float2 w = a.tw[ridx];  // exp(-2 pi i ridx / N)
        xs[k] = cmul(make_float2(al[k].pr, al[k].pi), cmul(w, xq));
      }
      if (a.c_a > 0.f) {
        // Eq. crossavg: parent a keeps its phase, its modulus moves towards the average one
        const float A = sqrtf(fmaf(xs[0].x, xs[0].x, __fmul_rn(xs[0].y, xs[0].y)));
        const float target = fmaf(a.c_a, a.Mavg[i], __fmul_rn(1.f - a.c_a, A));
        xs[0] = A > 0.f ? cscale(xs[0], target / A) : make_float2(target, 0.f);
      }
      out = make_float2(fmaf(a.c_w, xs[1].x - xs[2].x, xs[0].x), fmaf(a.c_w, xs[1].y - xs[2].y, xs[0].y));
    } else {
      out = Fp[i];
    }
    v[m] = cscale(out, a.inv_n);
  }
  fft<N, +1, ColL>(v, lds + c, t, a.tw);
  float2* dst = a.out + (size_t)a.table[a.P + p] * NN;
#pragma unroll
  for (int m = 0; m < E; ++m) dst[(size_t)(t + T * m) * N + col] = v[m];
}

// ---------------------------------------------------------------------------
// Resident Sequence (128^2): one cooperative launch runs the ingest and the
// iterations of a Sequence.  K = N / RW workgroups work on each member: in a
// row pass workgroup k takes the member's row group k, in a column pass its
// column tile k (RW * T = C * T threads either way), so each pass is the body
// of the launch-per-pass kernels and the results are the same bits.  Between
// passes the member's K workgroups meet at a barrier in device memory.
// Measured at 128^2 with 8 members, it runs 1.8 times slower than the launch
// pairs (18.7 against 10.4 us per iteration: the device-scope release and
// acquire of each barrier cost more than a launch), so it is the size's
// alternative plan (variant 1), which the run-time tuner weighs, and the
// launch pairs stay the default.
// ---------------------------------------------------------------------------
#if SPR_N == 128 && SPR_VARIANT == 1
#define SPR_SEQ_RES 1
constexpr int kResK = N / RW;
constexpr size_t kResLds = kColLdsBytes() > (size_t)RW * NR * sizeof(float2) ? kColLdsBytes()
                                                                             : (size_t)RW * NR * sizeof(float2);

// Sense-reversing barrier of the K workgroups of one member: bar[0] counts
// arrivals, bar[1] is the sense the last arrival publishes.  Each workgroup
// reads the sense once before its first arrival (the sense changes only when
// every workgroup has arrived); the count returns to zero at every barrier, so
// the words stay valid for the next launch.  A wait ends early when it passes
// wait_ticks of the device's constant-rate clock or when bit 1 of the
// population's status word is set (by a wait that ran out elsewhere); the
// workgroup then sets that bit and leaves, and every other workgroup of the
// population follows within one poll.
__device__ __forceinline__ bool res_barrier(unsigned* bar, unsigned& sense, int* status, int* bail,
                                            long long wait_ticks) {
  __syncthreads();  // the workgroup's stores are complete
  if (threadIdx.x == 0) {
    sense ^= 1u;
    __threadfence();  // release them at device scope before arriving
    const unsigned arrived = atomicAdd(&bar[0], 1u);
    if (arrived == (unsigned)kResK - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&bar[1], sense, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const long long t0 = wall_clock64();
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != sense) {
        if (wall_clock64() - t0 > wait_ticks ||
            (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2)) {
          atomicOr(status, 2);
          *bail = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __threadfence();  // acquire the other workgroups' stores
  }
  __syncthreads();
  return *bail == 0;
}

__global__ __launch_bounds__(RW* T) void k_seq_res(SeqResArgs a) {
  extern __shared__ float2 lds[];
  __shared__ int bail;
  const int member = blockIdx.x / kResK, k = blockIdx.x % kResK;
  unsigned* bar = a.res_bar + 2 * member;
  int* status = a.desc[a.slots[member]].flags;
  unsigned sense = 0;
  if (threadIdx.x == 0) {
    // a population whose earlier resident launch ran out of a wait stays
    // stopped until the host has reset its barrier words
    bail = (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2) ? 1 : 0;
    sense = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (bail) return;
  const int blk = member * kResK + k;  // the member's row group k in launch-wide numbering
  if (a.ingest) {
    RowIngestArgs ia{a.slots, a.nm, a.desc, a.T, a.W, a.t_by_slot, a.ingest_mode, a.ingest_ph, a.tw};
    row_ingest_body(ia, blk, lds);
    if (!res_barrier(bar, sense, status, &bail, a.wait_ticks)) return;
  }
  const ColProjArgs ca{a.slots, a.nm, a.desc, a.t_by_slot, a.T, a.Y, a.tw, nullptr};
  for (int i = 0; i < a.iters; ++i) {
    col_proj_body<false>(ca, TileId{k, member}, lds);
    if (!res_barrier(bar, sense, status, &bail, a.wait_ticks)) return;
    const ResIter q = a.it[i];
    RowUpdateArgs ra;
    ra.slots = a.slots;
    ra.nm = a.nm;
    ra.desc = a.desc;
    ra.Y = a.Y;
    ra.T = a.T;
    ra.W = a.W;
    ra.t_by_slot = a.t_by_slot;
    ra.ip = nullptr;
    ra.alg = q.alg;
    ra.beta = q.beta;
    ra.ph = q.ph;
    ra.out_mode = q.out_mode;
    ra.ph_next = q.ph_next;
    ra.tw = a.tw;
    if (q.alg == ALG_ER) row_update_body<1>(ra, blk, lds);
    else row_update_body<0>(ra, blk, lds);
    if (i + 1 < a.iters && !res_barrier(bar, sense, status, &bail, a.wait_ticks)) return;
  }
}
#endif

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
constexpr size_t kColLds = kColLdsBytes();
constexpr size_t kRowLds = (size_t)RW * NR * sizeof(float2);
constexpr size_t kRowLdsI = (size_t)RWI * NR * sizeof(float2);

template <typename K>
hipError_t set_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

int row_blocks(int nm) { return (nm * N + RW - 1) / RW; }

// Launch, with the dispatch recording ev's events around the kernel when given.
template <typename K, typename A>
void launch_k(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, const LaunchEvents* ev, const A& a) {
  if (ev) hipExtLaunchKernelGGL(kernel, grid, block, lds, s, ev->start, ev->stop, 0, a);
  else hipLaunchKernelGGL(kernel, grid, block, lds, s, a);
}

hipError_t l_row_ingest(const RowIngestArgs& a, hipStream_t s, const LaunchEvents* ev) {
  launch_k(k_row_ingest, dim3(row_blocks(a.nm)), dim3(RW * T), kRowLds, s, ev, a);
  return hipGetLastError();
}
hipError_t l_col_proj(const ColProjArgs& a, hipStream_t s, const LaunchEvents* ev) {
  static const hipError_t init = set_lds(k_col_proj<false>, kColLds);
  static const hipError_t init_t = set_lds(k_col_proj<true>, kColLds);
  if (init != hipSuccess) return init;
  if (init_t != hipSuccess) return init_t;
  if (a.trace_partial) launch_k(k_col_proj<true>, dim3(N / C, a.nm), dim3(C * T), kColLds, s, ev, a);
  else launch_k(k_col_proj<false>, dim3(N / C, a.nm), dim3(C * T), kColLds, s, ev, a);
  return hipGetLastError();
}
hipError_t l_row_update(const RowUpdateArgs& a, hipStream_t s, const LaunchEvents* ev) {
  const dim3 grid(row_blocks(a.nm)), block(RW * T);
  // the HIO/RAAR-only kernels gain on power-of-two sizes up to 512 and lose on
  // the radix-3 ones and at 1024, where the run-time form keeps fewer
  // registers live (at 1024: 165 against 197, three waves per SIMD instead of
  // two)
  constexpr bool kSpecIA = (N & (N - 1)) == 0 && N < 1024;
  if (a.ip) launch_k(k_row_update<0>, grid, block, kRowLds, s, ev, a);
  else if (a.alg == ALG_ER) launch_k(k_row_update<1>, grid, block, kRowLds, s, ev, a);
  else if (!kSpecIA) launch_k(k_row_update<0>, grid, block, kRowLds, s, ev, a);
  else if (a.alg == ALG_HIO) launch_k(k_row_update<2>, grid, block, kRowLds, s, ev, a);
  else launch_k(k_row_update<3>, grid, block, kRowLds, s, ev, a);
  return hipGetLastError();
}
hipError_t l_col_err(const ColErrArgs& a, hipStream_t s) {
  static const hipError_t init = set_lds(k_col_err, kColLds);
  if (init != hipSuccess) return init;
  hipLaunchKernelGGL(k_col_err, dim3(N / C, a.nm), dim3(C * T), kColLds, s, a);
  return hipGetLastError();
}
hipError_t l_row_fft(const RowFftArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_row_fft, dim3(row_blocks(a.nm)), dim3(RW * T), kRowLds, s, a);
  return hipGetLastError();
}
hipError_t l_col_fft(const ColFftArgs& a, hipStream_t s) {
  static const hipError_t init = set_lds(k_col_fft, kColLds);
  if (init != hipSuccess) return init;
  hipLaunchKernelGGL(k_col_fft, dim3(N / C, a.nm), dim3(C * T), kColLds, s, a);
  return hipGetLastError();
}
hipError_t l_col_corr(const ColCorrArgs& a, hipStream_t s) {
  static const hipError_t init = set_lds(k_col_corr, kColLds);
  if (init != hipSuccess) return init;
  hipLaunchKernelGGL(k_col_corr, dim3(N / C, a.npairs), dim3(C * T), kColLds, s, a);
  return hipGetLastError();
}
hipError_t l_row_argmax(const RowArgmaxArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_row_argmax, dim3(N / RWI, a.nimg), dim3(RWI * T), kRowLdsI, s, a);
  return hipGetLastError();
}
hipError_t l_col_mix(const ColMixArgs& a, hipStream_t s) {
  static const hipError_t init = set_lds(k_col_mix, kColLds);
  if (init != hipSuccess) return init;
  hipLaunchKernelGGL(k_col_mix, dim3(N / C, a.P), dim3(C * T), kColLds, s, a);
  return hipGetLastError();
}

#ifdef SPR_SEQ_RES
hipError_t l_seq_res(const SeqResArgs& a, hipStream_t s) {
  static_assert(RW * T == C * T && N / RW == N / C, "row groups and column tiles must pair up");
  static const hipError_t init = set_lds(k_seq_res, kResLds);
  if (init != hipSuccess) return init;
  // members per launch: every workgroup of a cooperative launch is resident
  static int per_dev[64] = {0};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  static long long ticks_dev[64] = {0};
  if (per_dev[dev] == 0) {
    int cus = 0, per_cu = 0, khz = 0;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev)) != hipSuccess) return e;
    ticks_dev[dev] = (long long)(khz > 0 ? khz : 100000) * 50;  // 50 ms
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_seq_res, RW * T, kResLds)) != hipSuccess)
      return e;
    per_dev[dev] = cus * per_cu / kResK;
    if (per_dev[dev] < 1) return hipErrorCooperativeLaunchTooLarge;
  }
  for (int m0 = 0; m0 < a.nm; m0 += per_dev[dev]) {
    SeqResArgs c = a;
    c.wait_ticks = ticks_dev[dev];
    c.slots = a.slots + m0;
    c.nm = a.nm - m0 < per_dev[dev] ? a.nm - m0 : per_dev[dev];
    if (!a.t_by_slot) c.T = a.T + (size_t)m0 * NN;
    c.Y = a.Y + (size_t)m0 * NN;
    c.res_bar = a.res_bar + 2 * (size_t)m0;
    const int grid = c.nm * kResK;
    void* args[] = {&c};
    e = hipLaunchCooperativeKernel((const void*)k_seq_res, dim3(grid), dim3(RW * T), args, (unsigned)kResLds, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
#define SPR_SEQ_RES_FN l_seq_res
#else
#define SPR_SEQ_RES_FN nullptr
#endif

const SizeKernels kTable = {N,          E,          T,          C,           RW,         RWI,
                            kColLds,    kRowLds,    l_row_ingest, l_col_proj, l_row_update,
                            l_col_err,  l_row_fft,  l_col_fft,  l_col_corr,  l_row_argmax,
                            l_col_mix,  SPR_SEQ_RES_FN};

}  // namespace

#define SPR_CAT4_(a, b, c, d) a##b##c##d
#define SPR_CAT4(a, b, c, d) SPR_CAT4_(a, b, c, d)
const SizeKernels* SPR_CAT4(size_kernels_, SPR_N, _, SPR_VARIANT)() { return &kTable; }

}  // namespace spr
