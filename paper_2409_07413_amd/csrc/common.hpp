// Shared declarations of the MPR hot-path library: kernel argument blocks,
// the per-size kernel table, Philox4x32-10 and small device helpers.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spr {

// Real-space constraint modes (phase constraint of the real-space constraints
// appendix): off (chi <= 0 or >= 1), positivity (chi = 0.5, Re >= 0 exactly),
// general cone |arg z| <= chi*pi with cos/sin of the half-angle supplied.
enum PhaseMode : int { PHASE_OFF = 0, PHASE_POS = 1, PHASE_CONE = 2 };

// Row-ingest modes: what is applied to the real-space density before the row FFT.
enum IngestMode : int { INGEST_PLAIN = 0, INGEST_PC = 1, INGEST_SMASK = 2 };

// Iterative algorithms.
enum Alg : int { ALG_ER = 0, ALG_HIO = 1, ALG_RAAR = 2 };

// Row-update output: next row-FFT'd iterate (plain or after P_C for a following
// ER step), or the final real-space density.
enum OutMode : int { OUT_T_PLAIN = 0, OUT_T_PC = 1, OUT_REAL = 2 };

struct Phase {
  int mode;
  float c, s;  // cos(chi pi), sin(chi pi) for PHASE_CONE
};

// Storage of one reconstruction, reached through slots[m] -> desc[slot]: its
// density and support words, the measured modulus of its shot and where its
// fitness goes.  A launch may mix members of several shots of one size.
struct SlotDesc {
  float2* X;             // real-space density, N*N complex
  float2* T;             // the member's own row-transform buffer (launches with t_by_slot)
  uint32_t* S;           // support bits, W words
  const float* amp;      // measured modulus of its shot, FFT order, sign bit set = unknown
  const __half* amp16;   // or the same stored as M / amp_scale in FP16 (amp then null)
  double* E;             // fitness slot
  double den;            // sum of Xi M^2 of its shot
  int* flags;            // status word of its population (bit 0: non-finite fitness)
  float amp_scale;
  int pad;
};

// Stored amplitude i (FP32 or FP16 storage; the sign bit marks unknown pixels).
__device__ __forceinline__ float amp_load(const float* a32, const __half* a16, size_t i) {
  return a16 ? __half2float(a16[i]) : a32[i];
}

// Per-member iteration parameters (members at different schedule positions).
struct IterParam {
  int alg;
  float beta;
  Phase ph;
  int out_mode;
  Phase ph_next;
};

// Densities and supports are addressed by storage slot (slots[m]); the work
// buffers T and Y by the member's position m in the launch, so a launch over
// any subset of members works in one compact region.
struct RowIngestArgs {
  const int* slots;      // launch member -> storage slot
  int nm;                // members
  const SlotDesc* desc;  // per slot
  float2* T;             // out: row-FFT of the ingested density [member][N*N]
  int W;
  int t_by_slot;         // 1: T is desc[slot].T instead of T + member*N*N
  int mode;              // IngestMode
  Phase ph;
  const float2* tw;
};

struct ColProjArgs {
  const int* slots;
  int nm;
  const SlotDesc* desc;  // measured modulus of each member's shot
  int t_by_slot;
  const float2* T;       // row-FFT'd iterate [member][N*N]
  float2* Y;             // out: column-IFFT of the projected spectrum [member][N*N]
  const float2* tw;
  double* trace_partial; // null, or out: FP64 sums of Xi (|X| - M)^2 per [member][column tile]
};

struct RowUpdateArgs {
  const int* slots;
  int nm;
  const SlotDesc* desc;
  const float2* Y;       // rowFFT(P_M x) from the column pass
  float2* T;             // in: rowFFT(x) (HIO/RAAR); out: next iterate's row FFT
  int W;
  int t_by_slot;
  const IterParam* ip;   // per-member parameters, or null: the uniform ones below
  int alg;               // Alg
  float beta;
  Phase ph;              // constraint of this step
  int out_mode;          // OutMode
  Phase ph_next;         // constraint used by OUT_T_PC
  const float2* tw;
};

struct ColErrArgs {
  const int* slots;
  int nm;
  const SlotDesc* desc;
  int t_by_slot;
  const float2* T;       // row-FFT of S*x [member][N*N]
  double* partial;       // out: [member][N/C] partial sums of Xi (|X| - M)^2
  const float2* tw;
};

struct RowFftArgs {
  const int* slots_in;   // may be null: identity
  const int* slots_out;  // may be null: identity
  int nm;
  const float2* in;
  float2* out;
  int dir;               // -1 forward, +1 inverse
  float scale;
  const float2* tw;
};

struct ColFftArgs {
  const int* slots_in;
  const int* slots_out;
  int nm;
  const float2* in;
  float2* out;
  int dir;
  float scale;
  const float2* tw;
};

// Reshift cross-correlations: pair (child p, parent q) for q in {a, b, c}.
struct ColCorrArgs {
  int npairs;            // 3 P (crossover) or P (average)
  const int* abc;        // [P][3] chosen parents (population indices)
  const int* ref_idx;    // null: pair k aligns abc[k] to k / 3; else pair k aligns k to *ref_idx
  const float2* F;       // parent spectra, indexed by population index [P][N*N]
  const float* amp;      // mask = sign bit (FP32 or FP16 storage)
  const __half* amp16;
  float2* C;             // out: [pair][2][N*N] column-IFFT of Xi conj(Xq) Xp and Xi Xq Xp
  const float2* tw;
};

struct ArgmaxRec {
  float val;             // |C|^2 at the maximum
  int idx;               // linear FFT-order index (lowest on ties)
  float re, im;          // C at the maximum
};

struct RowArgmaxArgs {
  int nimg;              // 2 * 3P images
  const float2* C;
  ArgmaxRec* partial;    // out: [img][blocks per image]
  const float2* tw;
};

struct AlignRec {
  int dr, dc;            // shift
  int twin;              // 1 if the twin image was kept
  int pad;
  float pr, pi;          // e^{i phi}
  float peak1, peak2;    // |C1| and |C2| maxima (squared)
  float second;          // unused (kept for layout)
  float pad2;
};

struct ColMixArgs {
  int P;
  const int* abc;        // [P][3]
  const int* mapprm;     // [P][5]: tx, ty, sx, sy, rotation index
  const AlignRec* align; // [P][3]
  const float2* F;       // parent spectra [P][N*N]
  const int* table;      // slot table: children at table[P + p]
  float2* out;           // out: column-IFFT of the mixed spectrum, at child slots
  float c_w;
  uint64_t seed;
  int gen;
  uint64_t cp_thr;       // Bernoulli threshold (may be 2^32)
  float inv_n;           // unitary inverse scaling folded into the column pass
  const float2* tw;
  float c_a;             // weight of the population's average modulus on parent a (0: none)
  const float* Mavg;     // (|F[rho_avg]| + mean |F[rho_p]|) / 2, FFT order (used when c_a > 0)
};

// Optional events that the dispatch of a kernel records at its start and end
// (its own execution interval, as a kernel trace reports it).
struct LaunchEvents {
  hipEvent_t start, stop;
};

// Per-size kernel table.  The projection-loop launchers take optional
// LaunchEvents (null: none).
// Resident Sequence: the ingest and up to kResMaxIters iterations of a
// Sequence in one cooperative launch (sizes whose single launches are
// latency-bound).  res_bar holds two words per launch position (arrivals,
// sense), zero before the first launch; a barrier wait that runs out sets
// bit 1 of the population's status word and ends the launch.
constexpr int kResMaxIters = 48;
struct ResIter {
  int alg;
  float beta;
  Phase ph;
  int out_mode;
  Phase ph_next;
};
struct SeqResArgs {
  const int* slots;
  int nm;
  const SlotDesc* desc;
  float2* T;
  float2* Y;
  int W;
  int t_by_slot;
  const float2* tw;
  int ingest;         // 1: the launch starts with the ingest of the densities
  int ingest_mode;    // IngestMode
  Phase ingest_ph;
  unsigned* res_bar;  // [nm][2]
  long long wait_ticks;  // longest barrier wait, in ticks of the device's constant-rate clock
  int iters;
  ResIter it[kResMaxIters];
};

struct SizeKernels {
  int n, E, T, C, RW;
  int RWI;               // rows per workgroup of the correlation argmax
  size_t col_lds, row_lds;
  hipError_t (*row_ingest)(const RowIngestArgs&, hipStream_t, const LaunchEvents*);
  hipError_t (*col_proj)(const ColProjArgs&, hipStream_t, const LaunchEvents*);
  hipError_t (*row_update)(const RowUpdateArgs&, hipStream_t, const LaunchEvents*);
  hipError_t (*col_err)(const ColErrArgs&, hipStream_t);
  hipError_t (*row_fft)(const RowFftArgs&, hipStream_t);
  hipError_t (*col_fft)(const ColFftArgs&, hipStream_t);
  hipError_t (*col_corr)(const ColCorrArgs&, hipStream_t);
  hipError_t (*row_argmax)(const RowArgmaxArgs&, hipStream_t);
  hipError_t (*col_mix)(const ColMixArgs&, hipStream_t);
  hipError_t (*seq_res)(const SeqResArgs&, hipStream_t);  // null where there is no resident form
};

// Compiled kernels of size n: variant 0 (default plan) or another variant
// (size_variants(n) of them); null for an unsupported size or variant.
const SizeKernels* size_kernels(int n, int variant = 0);
int size_variants(int n);
bool has_resident(int n);  // some variant of size n has the resident Sequence

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): multipliers 0xD2511F53, 0xCD9E8D57,
// Weyl key increments 0x9E3779B9, 0xBB67AE85.  counter = (block, member,
// generation, purpose); key = (seed low, seed high).
// ---------------------------------------------------------------------------
enum Purpose : uint32_t {
  PURPOSE_CHOICE = 1,
  PURPOSE_MAPPARAM = 2,
  PURPOSE_TILE = 3,
  PURPOSE_INIT = 4,
  PURPOSE_SPHERES = 5
};

struct U4 {
  uint32_t v[4];
};

__host__ __device__ inline U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
  uint32_t c[4] = {c0, c1, c2, c3};
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c[0] = hi1 ^ c[1] ^ k0;
    c[1] = lo1;
    c[2] = hi0 ^ c[3] ^ k1;
    c[3] = lo0;
  }
  U4 r;
  for (int i = 0; i < 4; ++i) r.v[i] = c[i];
  return r;
}

// Draw `index` of the stream (seed, purpose, generation, member).
__host__ __device__ inline uint32_t philox_draw(uint64_t seed, uint32_t purpose, uint32_t gen,
                                                uint32_t member, uint32_t index) {
  U4 o = philox4x32_10(index >> 2, member, gen, purpose, (uint32_t)seed, (uint32_t)(seed >> 32));
  return o.v[index & 3];
}

// Uniform integer in [0, n): high word of the 64-bit product.
__host__ __device__ inline uint32_t uniform_int(uint32_t u, uint32_t n) {
  return (uint32_t)(((uint64_t)u * (uint64_t)n) >> 32);
}

// Floor division for a positive divisor.
__host__ __device__ inline int floor_div(int a, int b) {
  int q = a / b;
  return (a % b != 0 && a < 0) ? q - 1 : q;
}

// Integer Pythagorean rotations (a, b, h), a^2 + b^2 = h^2, angles in [0, 90).
__host__ __device__ inline void rotation(int i, int& a, int& b, int& h) {
  const int t[9][3] = {{1, 0, 1},  {24, 7, 25}, {12, 5, 13}, {15, 8, 17}, {4, 3, 5},
                       {3, 4, 5},  {8, 15, 17}, {5, 12, 13}, {7, 24, 25}};
  a = t[i][0];
  b = t[i][1];
  h = t[i][2];
}
constexpr int N_ROTATIONS = 9;

}  // namespace spr
