// Argument blocks and launchers of the size-independent kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace spr {

constexpr int MAX_TAPS = 65;  // Gaussian radius ceil(4 sigma) <= 32

// Device-side scalars of a population: areas from the last STATS.
struct PopScalars {
  double alpha[2];   // [0] alpha_best, [1] alpha_eval
  double alpha_all;
  int best;
  int pad;
};

// Device record of one generation (mirrors spr_gen_stats).
struct GenStatsDev {
  int gen, best, alpha_best, alpha_all;
  double alpha_eval, err_best, err_mean, err_worst;
  int replaced, pad;
};

struct ErrFinalArgs {
  const double* partial;
  int ntiles;
  int nm;
  const int* slots;
  const SlotDesc* desc;  // fitness slot, sum of Xi M^2 and status word per member
};

// Per-iteration Fourier error of nm members into one trace row:
// row[pos0 + m] = sqrt(sum of the member's tile partials / sum Xi M^2).
struct TraceFinalArgs {
  const double* partial;
  int ntiles, nm;
  const int* slots;
  const SlotDesc* desc;
  double* row;
  int pos0;
};
struct FillArgs {
  double* dst;
  long count;
  double value;
};

// Shrink-wrap smoothing of |x| (Gaussian of radius r, periodic, rows then
// columns) for nm members; also the maximum per tile (block_max).
struct SmoothArgs {
  const int* slots;
  int nm, n, r;
  const SlotDesc* desc;
  float* out;        // [member][n*n]
  float* block_max;  // [member][tiles per member]
  float w[MAX_TAPS]; // taps k = 0..2r
};

struct MemberMaxArgs {
  int nm, blocks_per_member;
  const float* block_max;
  float* maxv;
};

struct ThresholdArgs {
  const int* slots;
  int nm, n, W;
  const float* in;
  const float* maxv;
  double tau;
  const SlotDesc* desc;
};

struct TopkArgs {
  const int* slots;
  int nm, n, W;
  const float* in;
  const double* alpha_src;  // device scalars or null
  int alpha_index;
  double alpha_abs;
  const SlotDesc* desc;
  // work area of at least nm * topk_scratch_words(n) words (sizes that use
  // the multi-workgroup selection), or null
  uint32_t* scratch;
};
// Words of top-k work area per member (0: the size uses one workgroup per member).
size_t topk_scratch_words(int n);

struct StatsArgs {
  int P, W, gen, gens;
  const int* table;
  const double* E;
  const uint32_t* S;
  PopScalars* scal;
  GenStatsDev* rec;
  int* part;  // 2 * stats_workgroups(W) counts
};
int stats_workgroups(int W);

struct SelectArgs {
  int P, gen;
  int* table;
  const double* E;
  GenStatsDev* rec;
};

struct ChoiceArgs {
  int P, gen, t_min, t_max;
  uint64_t seed;
  int* abc;
  int* mapprm;
};

struct AlignArgs {
  int npairs, blocks, n;
  const ArgmaxRec* partial;
  AlignRec* align;
};

struct SupportMixArgs {
  int P, n, W;
  const int* table;
  const int* abc;
  const AlignRec* align;
  uint32_t* S;
};

struct PackArgs {
  const int* slots;
  int nm, n, W, broadcast;
  uint8_t* bytes;
  uint32_t* S;
};

// Random-phase start, Fourier side: X[m][k] = Xi M e^{i phi}, phi drawn from
// (seed, INIT, generation 0, member m, draw k) at FFT-order pixel k.
struct InitPhaseArgs {
  int nm, n;
  const float* amp;  // FFT order, sign bit set = unknown
  const __half* amp16;  // or FP16 storage of M / amp_scale (amp then null)
  float amp_scale;
  uint64_t seed;
  float2* X;         // [member][n*n], contiguous
};

// Best member of one shot (lowest E, ties to the lower index, non-finite E
// never chosen over a finite one) gathered into one contiguous record:
// [int best][int status][24 bytes pad][double E[P]][float2 X[n*n]][uint32 S[W]].
struct GatherBestArgs {
  int P, n, W;
  const double* E;      // [P]
  const float2* X;      // [P][n*n]
  const uint32_t* S;    // [P][W]
  const int* status;
  unsigned char* out;
};

// Population average (members aligned to the best parent).
struct AvgArgs {
  int P, n, W;
  const int* table;        // slot table (parents first)
  const double* E;         // fitness by slot
  int* ref;                // out: index of the best parent (lowest E, ties to the lower index)
  const float2* F;         // parent spectra [P][n*n], unitary, FFT order
  const AlignRec* align;   // [P]: alignment of parent q to the best one
  float2* avgF;            // out: mean aligned spectrum
  float* Mavg;             // out: (|avgF| + mean |F|) / 2
  const uint32_t* S;       // support words by slot
  uint32_t* avgS;          // out: union of the aligned supports
  const float2* tw;        // exp(-2 pi i e / n)
};

// Sphere start (the paper's Initialize): densities of nm members at slots.
struct SphereArgs {
  int nm, n, n_init;
  uint64_t seed;
  double sigma_init, dmin, dmax;  // diameters in [dmin, dmax] * sigma_init
  double phmin, phmax, gamma;
  const int* slots;
  float2* X;                      // [slot][n*n]
};

// Eq. norm scaling: members' unitary spectra F [m][n*n] (contiguous), the
// known-pixel power per member, and the factor sqrt(sum Xi M^2 / power).
struct NormArgs {
  int nm, n, blocks;              // blocks per member of the partial sums
  const float2* F;
  const float* amp;
  const __half* amp16;
  double den;
  double* partial;                // [m][blocks]
  float* fac;                     // [m]
  const int* slots;
  float2* X;
};

// Per-generation monitor record (mirrors spr_monitor).
struct MonitorDev {
  int gen, P;
  double err_best, err_median, err_worst, err_mean;
  double gamma_mean, sum_mean, sum_rel_std;
  double gamma_avg, err_avg;
  int has_avg, pad;
};

struct MonitorArgs {
  int P, n;
  const int* table;     // parents: slots table[0..P)
  const float2* X;      // densities by slot
  const float2* avgX;   // the average density, or null
  const double* E;      // fitness by slot
  const double* avgE;   // fitness of the average, or null
  double* sums;         // [P + 1][3]: Re sum, Im sum, sum of moduli (FP64)
  MonitorDev* rec;
  int gen;
};

// Blocks per member of the column smoothing pass (size of the block-max array).
int smooth_blocks_per_member(int n);

hipError_t launch_err_final(const ErrFinalArgs& a, hipStream_t s);
hipError_t launch_trace_final(const TraceFinalArgs& a, hipStream_t s);
hipError_t launch_fill(const FillArgs& a, hipStream_t s);
hipError_t launch_smooth(const SmoothArgs& a, const MemberMaxArgs& mx,
                         hipStream_t s);
hipError_t launch_threshold(const ThresholdArgs& a, hipStream_t s);
hipError_t launch_topk(const TopkArgs& a, hipStream_t s);
hipError_t launch_stats(const StatsArgs& a, hipStream_t s);
hipError_t launch_select(const SelectArgs& a, hipStream_t s);
hipError_t launch_choice(const ChoiceArgs& a, hipStream_t s);
hipError_t launch_align(const AlignArgs& a, hipStream_t s);
hipError_t launch_support_mix(const SupportMixArgs& a, hipStream_t s);
hipError_t launch_pack(const PackArgs& a, hipStream_t s);
hipError_t launch_unpack(const PackArgs& a, hipStream_t s);
hipError_t launch_init_phase(const InitPhaseArgs& a, hipStream_t s);
hipError_t launch_gather_best(const GatherBestArgs& a, hipStream_t s);
hipError_t launch_avg_best(const AvgArgs& a, hipStream_t s);
hipError_t launch_init_spheres(const SphereArgs& a, hipStream_t s);
hipError_t launch_norm(const NormArgs& a, hipStream_t s);
hipError_t launch_monitor(const MonitorArgs& a, hipStream_t s);
hipError_t launch_avg_spectra(const AvgArgs& a, hipStream_t s);
hipError_t launch_avg_support(const AvgArgs& a, hipStream_t s);

}  // namespace spr
