// Size-independent kernels: fitness finalisation, shrink-wrap smoothing and
// thresholds, the exact top-k support (UpdateSupportSize), population
// statistics, RandomChoice / crossover-map parameters, Reshift decisions,
// support mixing, Select, and support packing.
#include <algorithm>

#include "common.hpp"
#include "kernels_common.hpp"

namespace spr {
namespace {

__device__ __forceinline__ bool bit_at(const uint32_t* __restrict__ S, long idx) {
  return (S[idx >> 5] >> (idx & 31)) & 1u;
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum of ints (fixed order).  All threads must call it.
__device__ int block_sum_int(int v, int* sh) {
  v = wave_sum_int(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  int s = 0;
  for (int i = 0; i < nw; ++i) s += sh[i];
  __syncthreads();
  return s;
}

// Block-wide exclusive scan of ints in thread order; returns the prefix and
// writes the block total to *total.  All threads must call it.
__device__ int block_exclusive_scan(int v, int* sh, int* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int u = __shfl_up(incl, o, 64);
    if (lane >= o) incl += u;
  }
  __syncthreads();
  if (lane == 63 || threadIdx.x == blockDim.x - 1) sh[w] = incl;
  __syncthreads();
  int before = 0, all = 0;
  for (int i = 0; i < nw; ++i) {
    if (i < w) before += sh[i];
    all += sh[i];
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

// ---------------------------------------------------------------------------
// Fitness: E = sqrt(sum partials / sum Xi M^2) per member (Eq. error_calc).
// ---------------------------------------------------------------------------
__global__ void k_err_final(ErrFinalArgs a) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= a.nm) return;
  double s = 0.0;
  for (int i = 0; i < a.ntiles; ++i) s += a.partial[(size_t)m * a.ntiles + i];
  const SlotDesc& d = a.desc[a.slots[m]];
  const double e = sqrt(s / d.den);
  *d.E = e;
  if (!isfinite(e)) atomicOr(d.flags, 1);
}

__global__ void k_trace_final(TraceFinalArgs a) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= a.nm) return;
  double s = 0.0;
  for (int i = 0; i < a.ntiles; ++i) s += a.partial[(size_t)m * a.ntiles + i];
  a.row[a.pos0 + m] = sqrt(s / a.desc[a.slots[m]].den);
}

// A fill kernel (not a memset), so that it can sit in a captured graph.
__global__ void k_fill(FillArgs a) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.count) a.dst[i] = a.value;
}

// ---------------------------------------------------------------------------
// Shrink-wrap: |x| smoothed by a circular separable Gaussian (rows, columns).
// ---------------------------------------------------------------------------

// Fused 2D smoothing: a workgroup smooths a tile of up to 64 x 64 outputs of
// one member.  |x| of the tile and a periodic halo of RC on every side is
// staged in LDS, the row taps go to a second LDS array for the tile's columns
// (halo rows included), and the column taps produce the outputs and the tile
// maximum.  Each thread slides a window of 8 outputs along its row or column,
// so every staged value is read once per window.  The 2 RC + 1 taps are the
// 2r + 1 Gaussian weights centred in zeros (RC >= r, chosen per launch): the
// products of the zero taps add nothing, so each output accumulates exactly
// the Gaussian taps, in k order, with fused multiply-adds, as the separate
// row and column passes do (a non-finite |x| within RC - r pixels beyond an
// output's window also reaches that output; such a density already has a
// non-finite fitness).
struct Smooth2dArgs {
  const int* slots;
  const SlotDesc* desc;
  int nm, n;
  float* out;        // [member][n*n]
  float* block_max;  // [member][tiles]
  float w[MAX_TAPS];  // centred: w[RC - r + k] = Gaussian tap k, zero elsewhere
};
constexpr int SM_TILE = 64;
constexpr int SM_SEG = 8;
constexpr int SM_THREADS = 512;
constexpr int SM_BATCH = 4;

__host__ __device__ inline int round8(int v) { return (v + 7) & ~7; }

template <int RC, bool FULL>
__global__ __launch_bounds__(SM_THREADS) void k_smooth2d(Smooth2dArgs a) {
  extern __shared__ float sm[];
  __shared__ float wmax[SM_THREADS / 64];
  const int n = a.n;
  // FULL: n >= SM_TILE, so the tile geometry (and every LDS offset) is known
  // at compile time
  const int tw = FULL ? SM_TILE : (n < SM_TILE ? n : SM_TILE), th = tw;
  const int twr = round8(tw), thr = round8(th);
  // odd pitches: a wavefront reading one element of 64 consecutive rows hits
  // 64 different LDS banks
  const int apitch = twr + 2 * RC + 1;  // A: (thr + 2 RC) rows x apitch
  const int bpitch = twr + 1;           // B: (thr + 2 RC) rows x bpitch
  const int arows = thr + 2 * RC;
  float* A = sm;
  float* Bt = sm;  // B (row-smoothed), written over A once A is consumed
  const int c0 = blockIdx.x * tw, i0 = blockIdx.y * th, m = blockIdx.z;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = SM_THREADS / 64;
  typedef float F2v __attribute__((ext_vector_type(2)));
  const __attribute__((address_space(1))) F2v* X = (const __attribute__((address_space(1))) F2v*)a.desc[a.slots[m]].X;
  // stage A: |x| with the periodic halo; the wrapped columns of a lane are
  // the same on every row
  constexpr int MAXC = (SM_TILE + 2 * RC + 63) / 64;
  int gcol[MAXC];
#pragma unroll
  for (int q = 0; q < MAXC; ++q) {
    int gj = (c0 - RC + lane + 64 * q) % n;
    gcol[q] = gj < 0 ? gj + n : gj;
  }
  // rows in batches of SM_BATCH per wavefront: all loads of a batch are in
  // flight before the first is used
  for (int row0 = wave; row0 < arows; row0 += NW * SM_BATCH) {
    F2v z[SM_BATCH][MAXC];
#pragma unroll
    for (int b = 0; b < SM_BATCH; ++b) {
      const int row = row0 + NW * b;
      // the row is the same for the whole wavefront: its base address is scalar
      int gi = i0 - RC + row;
      if (gi < 0 || gi >= n) {
        gi %= n;
        gi = gi < 0 ? gi + n : gi;
      }
      gi = __builtin_amdgcn_readfirstlane(gi);
      const __attribute__((address_space(1))) F2v* xr = X + (size_t)gi * n;
#pragma unroll
      for (int q = 0; q < MAXC; ++q) {
        const int col = lane + 64 * q;
        if (row < arows && col < apitch) z[b][q] = xr[gcol[q]];
      }
    }
#pragma unroll
    for (int b = 0; b < SM_BATCH; ++b) {
      const int row = row0 + NW * b;
#pragma unroll
      for (int q = 0; q < MAXC; ++q) {
        const int col = lane + 64 * q;
        if (row < arows && col < apitch) A[row * apitch + col] = sqrtf(z[b][q].x * z[b][q].x + z[b][q].y * z[b][q].y);
      }
    }
  }
  __syncthreads();
  // stage B: row taps, windows of 8 outputs along the rows, held in registers
  // until every thread has read A
  const int nseg_b = twr / SM_SEG;
  constexpr int MAXI = ((SM_TILE + 2 * RC) * (SM_TILE / SM_SEG) + SM_THREADS - 1) / SM_THREADS;
  float accb[MAXI][SM_SEG];
#pragma unroll
  for (int it = 0; it < MAXI; ++it) {
    const int item = threadIdx.x + it * SM_THREADS;
    if (item < arows * nseg_b) {
      int seg = 0, row = item;
      while (row >= arows) {  // at most SM_TILE / SM_SEG steps, no division
        row -= arows;
        ++seg;
      }
      const float* src = A + row * apitch + seg * SM_SEG;
#pragma unroll
      for (int j = 0; j < SM_SEG; ++j) accb[it][j] = 0.f;
#pragma unroll
      for (int t = 0; t < SM_SEG + 2 * RC; ++t) {
        const float v = src[t];
#pragma unroll
        for (int j = 0; j < SM_SEG; ++j) {
          const int k = t - j;
          if (k >= 0 && k <= 2 * RC) accb[it][j] += a.w[k] * v;
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MAXI; ++it) {
    const int item = threadIdx.x + it * SM_THREADS;
    if (item < arows * nseg_b) {
      int seg = 0, row = item;
      while (row >= arows) {
        row -= arows;
        ++seg;
      }
#pragma unroll
      for (int j = 0; j < SM_SEG; ++j) Bt[row * bpitch + seg * SM_SEG + j] = accb[it][j];
    }
  }
  __syncthreads();
  // stage C: column taps, windows of 8 outputs down the columns
  float mx = 0.f;
  float* out = a.out + (size_t)m * n * n;
  const int nseg_c = thr / SM_SEG;
  for (int item = threadIdx.x; item < twr * nseg_c; item += SM_THREADS) {
    int seg = 0, col = item;
    while (col >= twr) {
      col -= twr;
      ++seg;
    }
    const float* src = Bt + seg * SM_SEG * bpitch + col;
    float acc[SM_SEG];
#pragma unroll
    for (int j = 0; j < SM_SEG; ++j) acc[j] = 0.f;
#pragma unroll
    for (int t = 0; t < SM_SEG + 2 * RC; ++t) {
      const float v = src[t * bpitch];
#pragma unroll
      for (int j = 0; j < SM_SEG; ++j) {
        const int k = t - j;
        if (k >= 0 && k <= 2 * RC) acc[j] += a.w[k] * v;
      }
    }
    if (col < tw && c0 + col < n) {
#pragma unroll
      for (int j = 0; j < SM_SEG; ++j) {
        const int oi = seg * SM_SEG + j;
        if (oi < th && i0 + oi < n) {
          out[(size_t)(i0 + oi) * n + c0 + col] = acc[j];
          mx = fmaxf(mx, acc[j]);
        }
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  if (lane == 0) wmax[wave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    float v = wmax[0];
    for (int w = 1; w < NW; ++w) v = fmaxf(v, wmax[w]);
    a.block_max[(size_t)m * (gridDim.x * gridDim.y) + blockIdx.y * gridDim.x + blockIdx.x] = v;
  }
}

size_t smooth2d_lds(int n, int rc) {
  const int t = n < SM_TILE ? n : SM_TILE;
  const int tr = round8(t);
  return (size_t)(tr + 2 * rc) * (tr + 2 * rc + 1) * sizeof(float);
}

template <int RC, bool FULL>
hipError_t launch_smooth2d_tile(const Smooth2dArgs& a, dim3 grid, hipStream_t s) {
  const size_t lds = smooth2d_lds(a.n, RC);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_smooth2d<RC, FULL>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_smooth2d<RC, FULL>), grid, dim3(SM_THREADS), lds, s, a);
  return hipGetLastError();
}

template <int RC>
hipError_t launch_smooth2d_rc(Smooth2dArgs a, const float* w, int r, dim3 grid, hipStream_t s) {
  for (int k = 0; k < MAX_TAPS; ++k) a.w[k] = 0.f;
  for (int k = 0; k <= 2 * r; ++k) a.w[RC - r + k] = w[k];
  if (a.n >= SM_TILE) return launch_smooth2d_tile<RC, true>(a, grid, s);
  return launch_smooth2d_tile<RC, false>(a, grid, s);
}

__global__ __launch_bounds__(256) void k_member_max(MemberMaxArgs a) {
  __shared__ float wmax[4];
  const int m = blockIdx.x;
  float mx = 0.f;
  for (int i = threadIdx.x; i < a.blocks_per_member; i += blockDim.x)
    mx = fmaxf(mx, a.block_max[(size_t)m * a.blocks_per_member + i]);
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    float v = wmax[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = fmaxf(v, wmax[w]);
    a.maxv[m] = v;
  }
}

// S' = {a_sigma > tau * max a_sigma}, compared in double; unchanged if max = 0.
// One thread per four pixels; eight lanes form one support word.
__global__ __launch_bounds__(256) void k_threshold(ThresholdArgs a) {
  const long nn = (long)a.n * a.n;
  const int m = blockIdx.y;
  const long p0 = ((long)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  const float mx = a.maxv[m];
  if (!(mx > 0.f)) return;  // uniform over the workgroup
  const double thr = a.tau * (double)mx;
  const float* in = a.in + (size_t)m * nn;
  float v[4];
  if (p0 + 4 <= nn) {
    const float4 q = *reinterpret_cast<const float4*>(in + p0);
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
  } else {
    for (int j = 0; j < 4; ++j) v[j] = p0 + j < nn ? in[p0 + j] : 0.f;
  }
  uint32_t nib = 0;
  for (int j = 0; j < 4; ++j) nib |= (p0 + j < nn && (double)v[j] > thr ? 1u : 0u) << j;
  const int lane = threadIdx.x & 63;
  uint32_t word = nib << (4 * (lane & 7));
  word |= __shfl_xor(word, 1, 64);
  word |= __shfl_xor(word, 2, 64);
  word |= __shfl_xor(word, 4, 64);
  const long wi = p0 >> 5;
  if ((lane & 7) == 0 && wi < a.W) a.desc[a.slots[m]].S[wi] = word;
}

// ---------------------------------------------------------------------------
// UpdateSupportSize: exact top-k of the smoothed modulus, ties to the lower
// linear index.  One workgroup per member: MSB-first radix select on the
// float bit patterns (order-preserving for values >= 0) with per-wavefront
// histograms, then an index-ordered pass that takes the remaining ties in
// index order (wavefront ballots and a workgroup prefix count).
// ---------------------------------------------------------------------------
constexpr int TOPK_THREADS = 1024;

// Add one count per lane to hist[bin] (bin < 0: none).  The smoothed modulus
// is concentrated in a few bins (most pixels are near zero), so lanes with the
// same bin are first combined with ballots (a few rounds, one atomic per
// group); the rest add individually.
__device__ __forceinline__ void wave_histogram_add(uint32_t* hist, int bin, int lane) {
  bool pending = bin >= 0;
#pragma unroll
  for (int round = 0; round < 4; ++round) {
    const unsigned long long pend = __ballot(pending);
    if (pend == 0ull) return;
    const int leader = __ffsll((long long)pend) - 1;
    const int lb = __shfl(bin, leader, 64);
    const unsigned long long same = __ballot(pending && bin == lb);
    if (lane == leader) atomicAdd(&hist[lb], (uint32_t)__popcll(same));
    if (bin == lb) pending = false;
  }
  if (pending) atomicAdd(&hist[bin], 1u);
}
constexpr int TOPK_WAVES = TOPK_THREADS / 64;

constexpr int TOPK_PER_THREAD = 8;  // contiguous keys per thread (N^2 is a multiple of 16)

__device__ __forceinline__ void load8(const uint32_t* __restrict__ keys, long i, long nn, uint32_t (&k)[8]) {
  if (i + 8 <= nn) {
    const uint4 a = *reinterpret_cast<const uint4*>(keys + i);
    const uint4 b = *reinterpret_cast<const uint4*>(keys + i + 4);
    k[0] = a.x; k[1] = a.y; k[2] = a.z; k[3] = a.w;
    k[4] = b.x; k[5] = b.y; k[6] = b.z; k[7] = b.w;
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) k[j] = i + j < nn ? keys[i + j] : 0u;
  }
}

__global__ __launch_bounds__(TOPK_THREADS) void k_topk(TopkArgs a) {
  __shared__ uint32_t hist[TOPK_WAVES][256];
  __shared__ uint32_t tot[256];
  __shared__ uint32_t sh_prefix, sh_rem;
  __shared__ int scan_sh[TOPK_WAVES];
  const int m = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long nn = (long)a.n * a.n;
  const uint32_t* keys = reinterpret_cast<const uint32_t*>(a.in + (size_t)m * nn);
  uint8_t* Sb = reinterpret_cast<uint8_t*>(a.desc[a.slots[m]].S);
  const double alpha = a.alpha_src ? a.alpha_src[a.alpha_index] : a.alpha_abs;
  double kd = floor(alpha + 0.5);
  if (!(kd >= 1.0)) kd = 1.0;
  if (kd > (double)nn) kd = (double)nn;
  const uint32_t k = (uint32_t)kd;
  constexpr long CHUNK = (long)TOPK_THREADS * TOPK_PER_THREAD;

  uint32_t prefix = 0, pmask = 0, rem = k;
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    for (int i = threadIdx.x; i < TOPK_WAVES * 256; i += blockDim.x) (&hist[0][0])[i] = 0;
    __syncthreads();
    for (long base = 0; base < nn; base += CHUNK) {
      const long i = base + (long)threadIdx.x * TOPK_PER_THREAD;
      uint32_t kk[8];
      load8(keys, i, nn, kk);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int bin = (i + j < nn && (kk[j] & pmask) == prefix) ? (int)((kk[j] >> shift) & 255u) : -1;
        wave_histogram_add(hist[wv], bin, lane);
      }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < 256; b += blockDim.x) {
      uint32_t sum = 0;
      for (int w = 0; w < TOPK_WAVES; ++w) sum += hist[w][b];
      tot[b] = sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t cum = 0;
      int digit = 0;
      for (int b = 255; b >= 0; --b) {
        if (cum + tot[b] >= rem) {
          digit = b;
          break;
        }
        cum += tot[b];
      }
      sh_prefix = prefix | ((uint32_t)digit << shift);
      sh_rem = rem - cum;
    }
    __syncthreads();
    prefix = sh_prefix;
    rem = sh_rem;
    pmask |= 255u << shift;
  }
  // prefix = k-th largest key; rem = number of keys equal to it to take, in
  // index order.  Thread t owns pixels base + 8t .. base + 8t + 7, i.e. one
  // byte of the support words.
  uint32_t taken = 0;
  for (long base = 0; base < nn; base += CHUNK) {
    const long i = base + (long)threadIdx.x * TOPK_PER_THREAD;
    uint32_t kk[8];
    load8(keys, i, nn, kk);
    int ties = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) ties += (i + j < nn && kk[j] == prefix) ? 1 : 0;
    int total;
    const int before = block_exclusive_scan(ties, scan_sh, &total);
    uint32_t rank = taken + (uint32_t)before;
    uint32_t byte = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (i + j >= nn) continue;
      if (kk[j] > prefix) {
        byte |= 1u << j;
      } else if (kk[j] == prefix) {
        if (rank < rem) byte |= 1u << j;
        ++rank;
      }
    }
    if (i < nn) Sb[i >> 3] = (uint8_t)byte;
    taken += (uint32_t)total;
  }
}

// ---------------------------------------------------------------------------
// UpdateSupportSize on large images: the same selection spread over many
// workgroups per member.  Three digit passes (bits 31..20, 19..8, 7..0 of the
// float keys) each build the member's histogram of the keys that match the
// digits found so far (per-workgroup LDS histograms added into a global one),
// and a one-workgroup step per member picks the digit holding the k-th
// largest key.  Then every workgroup counts its keys equal to the k-th
// largest, and writes its support bytes, taking the equal keys in index order
// after those of the earlier workgroups.
// ---------------------------------------------------------------------------
constexpr int TKM_THREADS = 256;
constexpr int TKM_KEYS = TKM_THREADS * 32;  // keys per workgroup
constexpr int TKM_BINS = 4096;

struct TopkPass {
  int shift, bits;
};
__host__ __device__ constexpr TopkPass topk_pass(int pass) {
  return pass == 0 ? TopkPass{20, 12} : pass == 1 ? TopkPass{8, 12} : TopkPass{0, 8};
}

struct TopkMArgs {
  TopkArgs a;
  int bpm;          // workgroups per member
  uint32_t* hist;   // [nm][TKM_BINS]
  uint32_t* state;  // [nm][4]: digits found (prefix), their mask, keys still to take (rem)
  uint32_t* ties;   // [nm][bpm]
};

__global__ __launch_bounds__(TKM_THREADS) void k_topkm_zero(TopkMArgs t) {
  uint32_t* h = t.hist + (size_t)blockIdx.x * TKM_BINS;
  for (int b = threadIdx.x; b < TKM_BINS; b += TKM_THREADS) h[b] = 0u;
}

template <int PASS>
__global__ __launch_bounds__(TKM_THREADS) void k_topkm_hist(TopkMArgs t) {
  constexpr TopkPass tp = topk_pass(PASS);
  constexpr uint32_t dmask = (1u << tp.bits) - 1u;
  __shared__ uint32_t lh[1 << tp.bits];
  const int m = blockIdx.y, lane = threadIdx.x & 63;
  const long nn = (long)t.a.n * t.a.n;
  const uint32_t* keys = reinterpret_cast<const uint32_t*>(t.a.in + (size_t)m * nn);
  const uint32_t prefix = PASS ? t.state[m * 4 + 0] : 0u, pmask = PASS ? t.state[m * 4 + 1] : 0u;
  for (int b = threadIdx.x; b < (1 << tp.bits); b += TKM_THREADS) lh[b] = 0u;
  __syncthreads();
  const long base = (long)blockIdx.x * TKM_KEYS;
#pragma unroll
  for (int c = 0; c < TKM_KEYS / (TKM_THREADS * 8); ++c) {
    const long i = base + (long)c * TKM_THREADS * 8 + (long)threadIdx.x * 8;
    uint32_t kk[8];
    load8(keys, i, nn, kk);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int bin = (i + j < nn && (kk[j] & pmask) == prefix) ? (int)((kk[j] >> tp.shift) & dmask) : -1;
      wave_histogram_add(lh, bin, lane);
    }
  }
  __syncthreads();
  uint32_t* h = t.hist + (size_t)m * TKM_BINS;
  for (int b = threadIdx.x; b < (1 << tp.bits); b += TKM_THREADS)
    if (lh[b]) atomicAdd(&h[b], lh[b]);
}

template <int PASS>
__global__ __launch_bounds__(TKM_THREADS) void k_topkm_select(TopkMArgs t) {
  constexpr TopkPass tp = topk_pass(PASS);
  constexpr int NB = 1 << tp.bits, PER = NB / TKM_THREADS;
  __shared__ int scan_sh[TKM_THREADS / 64];
  const int m = blockIdx.x;
  uint32_t* h = t.hist + (size_t)m * TKM_BINS;
  uint32_t* st = t.state + m * 4;
  uint32_t rem;
  if (PASS == 0) {
    const long nn = (long)t.a.n * t.a.n;
    const double alpha = t.a.alpha_src ? t.a.alpha_src[t.a.alpha_index] : t.a.alpha_abs;
    double kd = floor(alpha + 0.5);
    if (!(kd >= 1.0)) kd = 1.0;
    if (kd > (double)nn) kd = (double)nn;
    rem = (uint32_t)kd;
  } else {
    rem = st[2];
  }
  // thread u owns bins (TKM_THREADS - 1 - u) * PER ... + PER - 1, so that an
  // exclusive scan over u counts the keys in higher bins
  const int u = threadIdx.x;
  const int lo = (TKM_THREADS - 1 - u) * PER;
  uint32_t cnt[PER];
  int part = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    cnt[q] = h[lo + q];
    part += (int)cnt[q];
  }
  int total;
  const int above = block_exclusive_scan(part, scan_sh, &total);
  if ((uint32_t)above < rem && rem <= (uint32_t)(above + part)) {
    uint32_t cum = (uint32_t)above;
    int digit = lo;
#pragma unroll
    for (int q = PER - 1; q >= 0; --q) {
      if (cum + cnt[q] >= rem) {
        digit = lo + q;
        break;
      }
      cum += cnt[q];
    }
    const uint32_t prefix = PASS ? st[0] : 0u, pmask = PASS ? st[1] : 0u;
    st[0] = prefix | ((uint32_t)digit << tp.shift);
    st[1] = pmask | (((1u << tp.bits) - 1u) << tp.shift);
    st[2] = rem - cum;
  }
  // leave the histogram cleared for the next pass
#pragma unroll
  for (int q = 0; q < PER; ++q) h[lo + q] = 0u;
}

__global__ __launch_bounds__(TKM_THREADS) void k_topkm_ties(TopkMArgs t) {
  __shared__ int scan_sh[TKM_THREADS / 64];
  const int m = blockIdx.y;
  const long nn = (long)t.a.n * t.a.n;
  const uint32_t* keys = reinterpret_cast<const uint32_t*>(t.a.in + (size_t)m * nn);
  const uint32_t kth = t.state[m * 4 + 0];
  const long base = (long)blockIdx.x * TKM_KEYS;
  int c = 0;
#pragma unroll
  for (int r = 0; r < TKM_KEYS / (TKM_THREADS * 8); ++r) {
    const long i = base + (long)r * TKM_THREADS * 8 + (long)threadIdx.x * 8;
    uint32_t kk[8];
    load8(keys, i, nn, kk);
#pragma unroll
    for (int j = 0; j < 8; ++j) c += (i + j < nn && kk[j] == kth) ? 1 : 0;
  }
  int total;
  block_exclusive_scan(c, scan_sh, &total);
  if (threadIdx.x == 0) t.ties[(size_t)m * t.bpm + blockIdx.x] = (uint32_t)total;
}

__global__ __launch_bounds__(TKM_THREADS) void k_topkm_write(TopkMArgs t) {
  __shared__ int scan_sh[TKM_THREADS / 64];
  const int m = blockIdx.y;
  const long nn = (long)t.a.n * t.a.n;
  const uint32_t* keys = reinterpret_cast<const uint32_t*>(t.a.in + (size_t)m * nn);
  uint8_t* Sb = reinterpret_cast<uint8_t*>(t.a.desc[t.a.slots[m]].S);
  const uint32_t kth = t.state[m * 4 + 0], rem = t.state[m * 4 + 2];
  uint32_t taken = 0;  // equal keys in earlier workgroups
  for (int b = 0; b < (int)blockIdx.x; ++b) taken += t.ties[(size_t)m * t.bpm + b];
  const long base = (long)blockIdx.x * TKM_KEYS;
  for (int r = 0; r < TKM_KEYS / (TKM_THREADS * 8); ++r) {
    const long i = base + (long)r * TKM_THREADS * 8 + (long)threadIdx.x * 8;
    uint32_t kk[8];
    load8(keys, i, nn, kk);
    int ties = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) ties += (i + j < nn && kk[j] == kth) ? 1 : 0;
    int total;
    const int before = block_exclusive_scan(ties, scan_sh, &total);
    uint32_t rank = taken + (uint32_t)before;
    uint32_t byte = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (i + j >= nn) continue;
      if (kk[j] > kth) {
        byte |= 1u << j;
      } else if (kk[j] == kth) {
        if (rank < rem) byte |= 1u << j;
        ++rank;
      }
    }
    if (i < nn) Sb[i >> 3] = (uint8_t)byte;
    taken += (uint32_t)total;
  }
}

// ---------------------------------------------------------------------------
// Generation statistics of Alg. improve (parents only): best = lowest error
// (ties to the lowest index), alpha_best, alpha_all (union), alpha_eval.
// ---------------------------------------------------------------------------
__host__ __device__ int stats_workgroups_of(int W) { return (W + 255) / 256; }
// Best parent: lowest error, ties to the lowest index.
__device__ int stats_best(const StatsArgs& a) {
  int best = 0;
  double be = a.E[a.table[0]];
  for (int p = 1; p < a.P; ++p) {
    const double e = a.E[a.table[p]];
    if (e < be) {
      be = e;
      best = p;
    }
  }
  return best;
}

constexpr int STATS_THREADS = 256;

// Support counts over a range of words, one word per thread: the best
// parent's bits and the union of every parent's bits.
__global__ __launch_bounds__(STATS_THREADS) void k_stats_part(StatsArgs a) {
  __shared__ int sh[STATS_THREADS / 64];
  __shared__ int sh_best;
  if (threadIdx.x == 0) sh_best = stats_best(a);
  __syncthreads();
  const int w = blockIdx.x * STATS_THREADS + threadIdx.x;
  int cb = 0, ca = 0;
  if (w < a.W) {
    cb = __popc(a.S[(size_t)a.table[sh_best] * a.W + w]);
    uint32_t u = 0;
    int p = 0;
    for (; p + 8 <= a.P; p += 8) {  // eight loads in flight
      uint32_t v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = a.S[(size_t)a.table[p + q] * a.W + w];
#pragma unroll
      for (int q = 0; q < 8; ++q) u |= v[q];
    }
    for (; p < a.P; ++p) u |= a.S[(size_t)a.table[p] * a.W + w];
    ca = __popc(u);
  }
  cb = block_sum_int(cb, sh);
  ca = block_sum_int(ca, sh);
  if (threadIdx.x == 0) {
    a.part[2 * blockIdx.x] = cb;
    a.part[2 * blockIdx.x + 1] = ca;
  }
}

__global__ __launch_bounds__(64) void k_stats(StatsArgs a) {
  if (threadIdx.x != 0) return;
  const int best = stats_best(a);
  int cb = 0, ca = 0;
  for (int b = 0; b < stats_workgroups_of(a.W); ++b) {
    cb += a.part[2 * b];
    ca += a.part[2 * b + 1];
  }
  const double fr = (double)a.gen / (double)a.gens;
  const double ev = fr * (double)cb + (1.0 - fr) * (double)ca;
  a.scal->alpha[0] = (double)cb;
  a.scal->alpha[1] = ev;
  a.scal->alpha_all = (double)ca;
  a.scal->best = best;
  GenStatsDev* rec = a.rec;
  rec->gen = a.gen;
  rec->best = best;
  rec->alpha_best = cb;
  rec->alpha_all = ca;
  rec->alpha_eval = ev;
}

// Alg. select: child p replaces parent p iff E_child < E_parent (strict); the
// slot table entries are swapped instead of copying the reconstructions.
__global__ void k_select(SelectArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int repl = 0;
  for (int p = 0; p < a.P; ++p) {
    const int sp = a.table[p], sc = a.table[a.P + p];
    if (a.E[sc] < a.E[sp]) {
      a.table[p] = sc;
      a.table[a.P + p] = sp;
      ++repl;
    }
  }
  double lo = a.E[a.table[0]], hi = lo, sum = 0.0;
  for (int p = 0; p < a.P; ++p) {
    const double e = a.E[a.table[p]];
    lo = e < lo ? e : lo;
    hi = e > hi ? e : hi;
    sum += e;
  }
  GenStatsDev* rec = a.rec;
  rec->gen = a.gen;
  rec->replaced = repl;
  rec->err_best = lo;
  rec->err_mean = sum / a.P;
  rec->err_worst = hi;
}

// RandomChoice (three distinct parents other than p, by skip-mapping uniform
// draws past the excluded indices) and the crossover-map parameters.
__global__ void k_choice(ChoiceArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.P) return;
  int ex[4] = {p, 0, 0, 0};
  int nex = 1;
  for (int i = 0; i < 3; ++i) {
    uint32_t r = uniform_int(philox_draw(a.seed, PURPOSE_CHOICE, (uint32_t)a.gen, (uint32_t)p, (uint32_t)i),
                             (uint32_t)(a.P - 1 - i));
    // ascending order of the excluded set
    int srt[4];
    for (int q = 0; q < nex; ++q) srt[q] = ex[q];
    for (int q = 1; q < nex; ++q)
      for (int z = q; z > 0 && srt[z - 1] > srt[z]; --z) {
        int tmp = srt[z];
        srt[z] = srt[z - 1];
        srt[z - 1] = tmp;
      }
    for (int q = 0; q < nex; ++q)
      if ((int)r >= srt[q]) ++r;
    a.abc[3 * p + i] = (int)r;
    ex[nex++] = (int)r;
  }
  uint32_t d[5];
  for (int i = 0; i < 5; ++i) d[i] = philox_draw(a.seed, PURPOSE_MAPPARAM, (uint32_t)a.gen, (uint32_t)p, (uint32_t)i);
  const int span = a.t_max - a.t_min + 1;
  const int tx = a.t_min + (int)uniform_int(d[0], (uint32_t)span);
  const int ty = a.t_min + (int)uniform_int(d[1], (uint32_t)span);
  a.mapprm[5 * p + 0] = tx;
  a.mapprm[5 * p + 1] = ty;
  a.mapprm[5 * p + 2] = (int)uniform_int(d[2], (uint32_t)tx);
  a.mapprm[5 * p + 3] = (int)uniform_int(d[3], (uint32_t)ty);
  a.mapprm[5 * p + 4] = (int)uniform_int(d[4], (uint32_t)N_ROTATIONS);
}

// Reshift decision per (child, parent) pair from the per-block argmax records:
// shift = argmax index, twin iff its peak is strictly higher, phase of C(d).
__device__ __forceinline__ bool better_rec(const ArgmaxRec& x, const ArgmaxRec& y) {
  return x.val > y.val || (x.val == y.val && x.idx < y.idx);
}

// One wavefront per pair: each lane takes a stride of the row partials, then
// a butterfly reduction under the same order (larger value, then lower index).
__device__ ArgmaxRec wave_best(const ArgmaxRec* src, int count) {
  const int lane = threadIdx.x & 63;
  ArgmaxRec best = src[0];
  for (int i = lane; i < count; i += 64)
    if (better_rec(src[i], best)) best = src[i];
  for (int o = 32; o > 0; o >>= 1) {
    ArgmaxRec other;
    other.val = __shfl_xor(best.val, o, 64);
    other.idx = __shfl_xor(best.idx, o, 64);
    other.re = __shfl_xor(best.re, o, 64);
    other.im = __shfl_xor(best.im, o, 64);
    if (better_rec(other, best)) best = other;
  }
  return best;
}

__global__ __launch_bounds__(64) void k_align(AlignArgs a) {
  const int pair = blockIdx.x;
  ArgmaxRec b[2];
  for (int tw = 0; tw < 2; ++tw) b[tw] = wave_best(a.partial + (size_t)(2 * pair + tw) * a.blocks, a.blocks);
  if (threadIdx.x != 0) return;
  const int twin = b[1].val > b[0].val ? 1 : 0;
  const ArgmaxRec& c = b[twin];
  AlignRec r;
  r.dr = c.idx / a.n;
  r.dc = c.idx % a.n;
  r.twin = twin;
  r.pad = 0;
  const float mag = sqrtf(c.re * c.re + c.im * c.im);
  if (mag > 0.f) {
    r.pr = c.re / mag;
    r.pi = c.im / mag;
  } else {
    r.pr = 1.f;
    r.pi = 0.f;
  }
  r.peak1 = b[0].val;
  r.peak2 = b[1].val;
  r.second = 0.f;
  r.pad2 = 0.f;
  a.align[pair] = r;
}

// Crossover support logic: S_new = S_a' OR (S_b' AND S_c' AND S_p), where the
// aligned supports are S(y - d) (or S(d - y) for the twin).
__global__ void k_support_mix(SupportMixArgs a) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)a.P * a.W) return;
  const int p = (int)(gid / a.W);
  const int w = (int)(gid % a.W);
  const long nn = (long)a.n * a.n;
  const uint32_t* Sq[3];
  AlignRec al[3];
  for (int k = 0; k < 3; ++k) {
    Sq[k] = a.S + (size_t)a.table[a.abc[3 * p + k]] * a.W;
    al[k] = a.align[3 * p + k];
  }
  const uint32_t* Sp = a.S + (size_t)a.table[p] * a.W;
  if (a.n % 32 == 0) {
    // the word's 32 pixels lie in one row; each aligned support supplies a
    // 32-bit window of one of its rows (reversed for the twin)
    const int n = a.n, wr = n / 32;
    const int yr = (int)(((long)w * 32) / n), yc0 = (int)(((long)w * 32) % n);
    uint32_t s[3];
    for (int k = 0; k < 3; ++k) {
      const bool twin = al[k].twin;
      int sr = twin ? al[k].dr - yr : yr - al[k].dr;
      sr = ((sr % n) + n) % n;
      int c0 = twin ? al[k].dc - yc0 - 31 : yc0 - al[k].dc;
      c0 = ((c0 % n) + n) % n;
      const uint32_t* row = Sq[k] + (size_t)sr * wr;
      const int i = c0 >> 5, o = c0 & 31;
      const uint32_t lo = row[i], hi = row[(i + 1) % wr];
      const uint32_t win = o ? (lo >> o) | (hi << (32 - o)) : lo;
      s[k] = twin ? __builtin_bitreverse32(win) : win;
    }
    a.S[(size_t)a.table[a.P + p] * a.W + w] = s[0] | (s[1] & s[2] & Sp[w]);
    return;
  }
  uint32_t bits = 0;
  for (int b = 0; b < 32; ++b) {
    const long idx = (long)w * 32 + b;
    if (idx >= nn) break;
    const int yr = (int)(idx / a.n), yc = (int)(idx % a.n);
    bool s[3];
    for (int k = 0; k < 3; ++k) {
      int sr, sc;
      if (al[k].twin) {
        sr = al[k].dr - yr;
        sc = al[k].dc - yc;
      } else {
        sr = yr - al[k].dr;
        sc = yc - al[k].dc;
      }
      sr = ((sr % a.n) + a.n) % a.n;
      sc = ((sc % a.n) + a.n) % a.n;
      s[k] = bit_at(Sq[k], (long)sr * a.n + sc);
    }
    const bool sp = bit_at(Sp, idx);
    if (s[0] || (s[1] && s[2] && sp)) bits |= 1u << b;
  }
  a.S[(size_t)a.table[a.P + p] * a.W + w] = bits;
}

// uint8 supports [member][n*n] <-> bit words [slot][W]
__global__ void k_pack(PackArgs a) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)a.nm * a.W) return;
  const int m = (int)(gid / a.W);
  const int w = (int)(gid % a.W);
  const long nn = (long)a.n * a.n;
  const uint8_t* src = a.bytes + (a.broadcast ? 0 : (size_t)m * nn);
  uint32_t bits = 0;
  for (int b = 0; b < 32; ++b) {
    const long idx = (long)w * 32 + b;
    if (idx < nn && src[idx]) bits |= 1u << b;
  }
  a.S[(size_t)a.slots[m] * a.W + w] = bits;
}

__global__ void k_unpack(PackArgs a) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nn = (long)a.n * a.n;
  if (gid >= (long)a.nm * nn) return;
  const int m = (int)(gid / nn);
  const long idx = gid % nn;
  const uint32_t* Sm = a.S + (size_t)a.slots[m] * a.W;
  a.bytes[gid] = bit_at(Sm, idx) ? 1 : 0;
}

// One Philox block per thread gives the phases of four consecutive pixels.
// The angle and its sine/cosine are taken in FP64 and rounded once.
__global__ void k_init_phase(InitPhaseArgs a) {
  const long nn = (long)a.n * a.n;
  const long nb = (nn + 3) / 4;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (gid >= nb || m >= a.nm) return;
  const U4 u = philox4x32_10((uint32_t)gid, (uint32_t)m, 0u, PURPOSE_INIT, (uint32_t)a.seed,
                             (uint32_t)(a.seed >> 32));
  float2* X = a.X + (size_t)m * nn;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const long k = gid * 4 + w;
    if (k >= nn) break;
    const float av = amp_load(a.amp, a.amp16, k);
    const double v = signbit(av) ? 0.0 : (double)av * (double)a.amp_scale;
    const double phi = 6.283185307179586476925 * ((double)u.v[w] + 0.5) * 2.3283064365386962890625e-10;
    double sn, cs;
    sincos(phi, &sn, &cs);
    X[k] = make_float2((float)(v * cs), (float)(v * sn));
  }
}

__global__ void k_gather_best(GatherBestArgs a) {
  __shared__ int sbest;
  if (threadIdx.x == 0) {
    int b = 0;
    double bv = a.E[0];
    for (int p = 1; p < a.P; ++p) {
      const double e = a.E[p];
      // strict: ties keep the lower index; a NaN never replaces, and is replaced
      if (e < bv || (bv != bv && e == e)) {
        bv = e;
        b = p;
      }
    }
    sbest = b;
  }
  __syncthreads();
  const int best = sbest;
  const long nn = (long)a.n * a.n;
  const size_t offX = 32 + 8 * (size_t)a.P;
  const size_t offS = offX + 8 * (size_t)nn;
  float2* X = reinterpret_cast<float2*>(a.out + offX);
  uint32_t* S = reinterpret_cast<uint32_t*>(a.out + offS);
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < nn) X[gid] = a.X[(size_t)best * nn + gid];
  if (gid < a.W) S[gid] = a.S[(size_t)best * a.W + gid];
  if (gid < a.P) reinterpret_cast<double*>(a.out + 32)[gid] = a.E[gid];
  if (gid == 0) {
    reinterpret_cast<int*>(a.out)[0] = best;
    reinterpret_cast<int*>(a.out)[1] = *a.status;
  }
}

// Best parent: lowest E, ties to the lower index, a NaN never chosen over a number.
__global__ void k_avg_best(AvgArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int b = 0;
  double bv = a.E[a.table[0]];
  for (int p = 1; p < a.P; ++p) {
    const double e = a.E[a.table[p]];
    if (e < bv || (bv != bv && e == e)) {
      bv = e;
      b = p;
    }
  }
  *a.ref = b;
}

// Per Fourier pixel: the mean of the aligned parent spectra and the mean of
// their moduli (Eq. avgint1, Eq. avgint2), folded into Mavg.
__global__ void k_avg_spectra(AvgArgs a) {
  const long nn = (long)a.n * a.n;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  const int e = (int)(i / a.n), col = (int)(i % a.n);
  float sx = 0.f, sy = 0.f, ms = 0.f;
  for (int q = 0; q < a.P; ++q) {
    const AlignRec al = a.align[q];
    float2 x = a.F[(size_t)q * nn + i];
    ms += sqrtf(fmaf(x.x, x.x, __fmul_rn(x.y, x.y)));
    if (al.twin) x = make_float2(x.x, -x.y);
    const int ridx = (int)(((long long)e * al.dr + (long long)col * al.dc) % a.n);
    const float2 w = a.tw[ridx];
    const float2 wx = make_float2(fmaf(w.x, x.x, -__fmul_rn(w.y, x.y)), fmaf(w.x, x.y, __fmul_rn(w.y, x.x)));
    sx += fmaf(al.pr, wx.x, -__fmul_rn(al.pi, wx.y));
    sy += fmaf(al.pr, wx.y, __fmul_rn(al.pi, wx.x));
  }
  const float inv = 1.f / (float)a.P;
  const float2 m = make_float2(sx * inv, sy * inv);
  a.avgF[i] = m;
  a.Mavg[i] = 0.5f * (sqrtf(fmaf(m.x, m.x, __fmul_rn(m.y, m.y))) + ms * inv);
}

// Union of the aligned supports: S'(y) = S(y - d), or S(d - y) for a twin.
__global__ void k_avg_support(AvgArgs a) {
  const long w = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= a.W) return;
  const long nn = (long)a.n * a.n;
  uint32_t bits = 0;
  for (int b = 0; b < 32; ++b) {
    const long idx = w * 32 + b;
    if (idx >= nn) break;
    const int yr = (int)(idx / a.n), yc = (int)(idx % a.n);
    bool on = false;
    for (int q = 0; q < a.P && !on; ++q) {
      const AlignRec al = a.align[q];
      int sr = al.twin ? al.dr - yr : yr - al.dr;
      int sc = al.twin ? al.dc - yc : yc - al.dc;
      sr = ((sr % a.n) + a.n) % a.n;
      sc = ((sc % a.n) + a.n) % a.n;
      on = bit_at(a.S + (size_t)a.table[q] * a.W, (long)sr * a.n + sc);
    }
    if (on) bits |= 1u << b;
  }
  a.avgS[w] = bits;
}

// One pixel of one member: the sum of the projected spheres (FP64), its
// modulus raised to gamma with the phase kept.
__global__ void k_init_spheres(SphereArgs a) {
  const long nn = (long)a.n * a.n;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (i >= nn || m >= a.nm) return;
  const double y = (double)(i / a.n) - 0.5 * a.n, x = (double)(i % a.n) - 0.5 * a.n;
  const double half = 0.5 * a.sigma_init, inv32 = 2.3283064365386962890625e-10;
  double re = 0.0, im = 0.0;
  for (int k = 0; k < a.n_init; ++k) {
    const U4 u = philox4x32_10((uint32_t)k, (uint32_t)m, 0u, PURPOSE_SPHERES, (uint32_t)a.seed,
                               (uint32_t)(a.seed >> 32));
    const double R = 0.5 * (a.dmin + (a.dmax - a.dmin) * (u.v[0] * inv32)) * a.sigma_init;
    double cy = 0.0, cx = 0.0;
    if (half > R) {
      cy = -half + R + 2.0 * (half - R) * (u.v[1] * inv32);
      cx = -half + R + 2.0 * (half - R) * (u.v[2] * inv32);
    }
    const double ph = a.phmin + (a.phmax - a.phmin) * (u.v[3] * inv32);
    const double r2 = (y - cy) * (y - cy) + (x - cx) * (x - cx);
    const double d = R * R - r2;
    if (d > 0.0) {
      const double t = 2.0 * sqrt(d);
      double sn, cs;
      sincos(ph, &sn, &cs);
      re += t * cs;
      im += t * sn;
    }
  }
  const double A = sqrt(re * re + im * im);
  float2 v = make_float2(0.f, 0.f);
  if (A > 0.0) {
    const double g = pow(A, a.gamma) / A;
    v = make_float2((float)(re * g), (float)(im * g));
  }
  a.X[(size_t)a.slots[m] * nn + i] = v;
}

// Known-pixel power of each member's spectrum: fixed-order block partial sums.
__global__ void k_norm_partial(NormArgs a) {
  __shared__ double red[256];
  const long nn = (long)a.n * a.n;
  const int m = blockIdx.y;
  const long chunk = (nn + a.blocks - 1) / a.blocks;
  const long beg = blockIdx.x * chunk, end = beg + chunk < nn ? beg + chunk : nn;
  double s = 0.0;
  for (long i = beg + threadIdx.x; i < end; i += blockDim.x) {
    if (signbit(amp_load(a.amp, a.amp16, i))) continue;
    const float2 f = a.F[(size_t)m * nn + i];
    s += (double)f.x * f.x + (double)f.y * f.y;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partial[(size_t)m * a.blocks + blockIdx.x] = red[0];
}

__global__ void k_norm_factor(NormArgs a) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= a.nm) return;
  double p = 0.0;
  for (int b = 0; b < a.blocks; ++b) p += a.partial[(size_t)m * a.blocks + b];
  a.fac[m] = p > 0.0 ? (float)sqrt(a.den / p) : 1.f;
}

__global__ void k_norm_scale(NormArgs a) {
  const long nn = (long)a.n * a.n;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (i >= nn) return;
  float2* X = a.X + (size_t)a.slots[m] * nn;
  const float f = a.fac[m];
  X[i] = make_float2(X[i].x * f, X[i].y * f);
}

// Sum of rho and of |rho| of one member (or of the average, member P), in
// FP64 with a fixed-order tree.
__global__ void k_member_sums(MonitorArgs a) {
  __shared__ double red[3][256];
  const int m = blockIdx.x;
  const long nn = (long)a.n * a.n;
  const float2* X = m < a.P ? a.X + (size_t)a.table[m] * nn : a.avgX;
  double re = 0.0, im = 0.0, ab = 0.0;
  for (long i = threadIdx.x; i < nn; i += blockDim.x) {
    const float2 v = X[i];
    re += v.x;
    im += v.y;
    ab += sqrt((double)v.x * v.x + (double)v.y * v.y);
  }
  red[0][threadIdx.x] = re;
  red[1][threadIdx.x] = im;
  red[2][threadIdx.x] = ab;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 3) a.sums[(size_t)m * 3 + threadIdx.x] = red[threadIdx.x][0];
}

// Ranks of the parents' errors (ties to the lower index, a NaN ranked last)
// give the best, lower-median and worst values; the sums give the mean
// complexity and the mean and relative spread of |sum rho|.
__global__ void k_monitor_final(MonitorArgs a) {
  __shared__ double med[3];
  const int P = a.P;
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    double ei = a.E[a.table[i]];
    if (ei != ei) ei = __builtin_huge_val();
    int rank = 0;
    for (int j = 0; j < P; ++j) {
      double ej = a.E[a.table[j]];
      if (ej != ej) ej = __builtin_huge_val();
      if (ej < ei || (ej == ei && j < i)) ++rank;
    }
    if (rank == 0) med[0] = ei;
    if (rank == (P - 1) / 2) med[1] = ei;
    if (rank == P - 1) med[2] = ei;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double esum = 0.0, gsum = 0.0, ssum = 0.0, s2 = 0.0;
  for (int p = 0; p < P; ++p) {
    esum += a.E[a.table[p]];
    const double* q = a.sums + (size_t)p * 3;
    const double sa = sqrt(q[0] * q[0] + q[1] * q[1]);
    gsum += q[2] > 0.0 ? 1.0 - sa / q[2] : 0.0;
    ssum += sa;
  }
  const double smean = ssum / P;
  for (int p = 0; p < P; ++p) {  // second pass: no cancellation in the spread
    const double* q = a.sums + (size_t)p * 3;
    const double d = sqrt(q[0] * q[0] + q[1] * q[1]) - smean;
    s2 += d * d;
  }
  MonitorDev r;
  r.gen = a.gen;
  r.P = P;
  r.err_best = med[0];
  r.err_median = med[1];
  r.err_worst = med[2];
  r.err_mean = esum / P;
  r.gamma_mean = gsum / P;
  r.sum_mean = smean;
  r.sum_rel_std = smean > 0.0 ? sqrt(s2 / P) / smean : 0.0;
  r.has_avg = a.avgX != nullptr;
  r.gamma_avg = 0.0;
  r.err_avg = 0.0;
  if (a.avgX) {
    const double* q = a.sums + (size_t)P * 3;
    const double sa = sqrt(q[0] * q[0] + q[1] * q[1]);
    r.gamma_avg = q[2] > 0.0 ? 1.0 - sa / q[2] : 0.0;
    r.err_avg = a.avgE ? *a.avgE : 0.0;
  }
  r.pad = 0;
  *a.rec = r;
}

inline unsigned blocks_for(long n, int tpb) { return (unsigned)((n + tpb - 1) / tpb); }

}  // namespace

hipError_t launch_trace_final(const TraceFinalArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_trace_final, dim3(blocks_for(a.nm, 64)), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_fill(const FillArgs& a, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(a.count, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_err_final(const ErrFinalArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_err_final, dim3(blocks_for(a.nm, 64)), dim3(64), 0, s, a);
  return hipGetLastError();
}
int smooth_blocks_per_member(int n) {
  const int t = n < SM_TILE ? n : SM_TILE;
  return ((n + t - 1) / t) * ((n + t - 1) / t);
}

hipError_t launch_smooth(const SmoothArgs& sa, const MemberMaxArgs& mx, hipStream_t s) {
  const int n = sa.n, r = sa.r;
  if (n > 1024 || r > (MAX_TAPS - 1) / 2) return hipErrorInvalidValue;
  const int t = n < SM_TILE ? n : SM_TILE;
  const dim3 grid((n + t - 1) / t, (n + t - 1) / t, sa.nm);
  Smooth2dArgs a{};
  a.slots = sa.slots;
  a.desc = sa.desc;
  a.nm = sa.nm;
  a.n = n;
  a.out = sa.out;
  a.block_max = sa.block_max;
  hipError_t e;
  if (r == 0) e = launch_smooth2d_rc<0>(a, sa.w, r, grid, s);
  else if (r <= 2) e = launch_smooth2d_rc<2>(a, sa.w, r, grid, s);
  else if (r <= 4) e = launch_smooth2d_rc<4>(a, sa.w, r, grid, s);
  else if (r <= 8) e = launch_smooth2d_rc<8>(a, sa.w, r, grid, s);
  else if (r <= 16) e = launch_smooth2d_rc<16>(a, sa.w, r, grid, s);
  else e = launch_smooth2d_rc<32>(a, sa.w, r, grid, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_member_max, dim3(mx.nm), dim3(256), 0, s, mx);
  return hipGetLastError();
}
hipError_t launch_threshold(const ThresholdArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_threshold, dim3(blocks_for(((long)a.n * a.n + 3) / 4, 256), a.nm), dim3(256), 0, s, a);
  return hipGetLastError();
}
// Sizes from 96 up spread the selection over workgroups (their work area fits
// the member's row-transform buffer); smaller ones use one workgroup per member.
size_t topk_scratch_words(int n) {
  if (n < 96) return 0;
  const size_t bpm = ((size_t)n * n + TKM_KEYS - 1) / TKM_KEYS;
  return TKM_BINS + 4 + bpm;
}

hipError_t launch_topk(const TopkArgs& a, hipStream_t s) {
  if (topk_scratch_words(a.n) == 0 || !a.scratch) {
    hipLaunchKernelGGL(k_topk, dim3(a.nm), dim3(TOPK_THREADS), 0, s, a);
    return hipGetLastError();
  }
  TopkMArgs t{};
  t.a = a;
  t.bpm = (int)(((long)a.n * a.n + TKM_KEYS - 1) / TKM_KEYS);
  t.hist = a.scratch;
  t.state = a.scratch + (size_t)a.nm * TKM_BINS;
  t.ties = t.state + (size_t)a.nm * 4;
  const dim3 grid(t.bpm, a.nm), block(TKM_THREADS);
  hipLaunchKernelGGL(k_topkm_zero, dim3(a.nm), block, 0, s, t);
  hipLaunchKernelGGL(k_topkm_hist<0>, grid, block, 0, s, t);
  hipLaunchKernelGGL(k_topkm_select<0>, dim3(a.nm), block, 0, s, t);
  hipLaunchKernelGGL(k_topkm_hist<1>, grid, block, 0, s, t);
  hipLaunchKernelGGL(k_topkm_select<1>, dim3(a.nm), block, 0, s, t);
  hipLaunchKernelGGL(k_topkm_hist<2>, grid, block, 0, s, t);
  hipLaunchKernelGGL(k_topkm_select<2>, dim3(a.nm), block, 0, s, t);
  hipLaunchKernelGGL(k_topkm_ties, grid, block, 0, s, t);
  hipLaunchKernelGGL(k_topkm_write, grid, block, 0, s, t);
  return hipGetLastError();
}
int stats_workgroups(int W) { return stats_workgroups_of(W); }

hipError_t launch_stats(const StatsArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_stats_part, dim3(stats_workgroups_of(a.W)), dim3(STATS_THREADS), 0, s, a);
  hipLaunchKernelGGL(k_stats, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_select(const SelectArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_choice(const ChoiceArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_choice, dim3(blocks_for(a.P, 64)), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_align(const AlignArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_align, dim3(a.npairs), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_support_mix(const SupportMixArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_support_mix, dim3(blocks_for((long)a.P * a.W, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_init_phase(const InitPhaseArgs& a, hipStream_t s) {
  const long nb = ((long)a.n * a.n + 3) / 4;
  hipLaunchKernelGGL(k_init_phase, dim3(blocks_for(nb, 256), a.nm), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gather_best(const GatherBestArgs& a, hipStream_t s) {
  const long work = std::max<long>((long)a.n * a.n, std::max(a.W, a.P));
  hipLaunchKernelGGL(k_gather_best, dim3(blocks_for(work, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_avg_best(const AvgArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_avg_best, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_avg_spectra(const AvgArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_avg_spectra, dim3(blocks_for((long)a.n * a.n, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_avg_support(const AvgArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_avg_support, dim3(blocks_for(a.W, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_init_spheres(const SphereArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_init_spheres, dim3(blocks_for((long)a.n * a.n, 256), a.nm), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_norm(const NormArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_partial, dim3(a.blocks, a.nm), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_norm_factor, dim3(blocks_for(a.nm, 64)), dim3(64), 0, s, a);
  hipLaunchKernelGGL(k_norm_scale, dim3(blocks_for((long)a.n * a.n, 256), a.nm), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_monitor(const MonitorArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_member_sums, dim3(a.P + (a.avgX ? 1 : 0)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_monitor_final, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pack(const PackArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(blocks_for((long)a.nm * a.W, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_unpack(const PackArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack, dim3(blocks_for((long)a.nm * a.n * a.n, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace spr
