// Internal declarations of the host runtime shared by the C ABI (runtime.cpp)
// and the serving engine (server.cpp): handle structures, launch groups and
// the enqueueing helpers.  Helpers have internal linkage (one copy per
// translation unit); the live-handle registry is a single inline object.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels_common.hpp"
#include "spr.h"

using namespace spr;

// Work buffers of batched launches, per detector size, grown on demand.
struct Workspace {
  size_t members = 0;
  float2* T = nullptr;
  float2* Y = nullptr;
  double* err_partial = nullptr;
  float* block_max = nullptr;
  float* maxv = nullptr;
  SlotDesc* desc = nullptr;
  int* slots = nullptr;
  hipStream_t last = nullptr;  // stream of the last batch that used these buffers
};

// Default byte budget of an iteration run's work buffers (spr_ctx): the
// memory-side cache of one MI355X.
constexpr size_t kDefaultCacheBudget = (size_t)256 << 20;

struct spr_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  // iteration runs whose two work buffers fit in this many bytes run as one
  // launch per pass; larger ones are split into member chunks whose buffers
  // fill three quarters of it (0: no split), so that they stay in the
  // memory-side cache (see chunk_for)
  size_t cache_budget = kDefaultCacheBudget;
  // per-size choices of the tuner (or of the caller): kernel variant for
  // shots created from now on, members per iteration launch (0: the budget rule)
  std::map<int, int> variant;
  std::map<int, int> chunk_members;
  std::string err;
  std::map<int, float2*> tw;
  std::map<int, Workspace> ws;
  std::set<spr_shot*> shots;  // live shots, populations and servers created on this context
  std::set<spr_pop*> pops;
  std::set<spr_server*> servers;
  std::set<spr_graph*> graphs;
  std::vector<hipStream_t> side;  // streams of the size groups of a batch after the first (default priority)
  std::mutex mu;
};

struct spr_shot {
  spr_ctx* ctx = nullptr;
  int n = 0;
  const SizeKernels* K = nullptr;
  float* amp = nullptr;  // FFT order, sign bit = unknown
  __half* amp16 = nullptr;  // FP16 storage of amp / amp_scale instead (SPR_AMP_FP16)
  float amp_scale = 1.f;
  double den = 0.0;      // sum of Xi M^2
  int live = 0;
};

struct spr_pop {
  spr_shot* shot = nullptr;
  spr_ctx* ctx = nullptr;
  const SizeKernels* K = nullptr;
  int n = 0, P = 0, nslots = 0, W = 0;
  bool memetic = false;
  int graphs = 0;  // captured graphs that replay work on this population
  uint64_t seed = 0;
  int gen_offset = 0;
  float2 *X = nullptr, *T = nullptr, *Y = nullptr;
  uint32_t* S = nullptr;
  double* E = nullptr;
  int* table = nullptr;
  SlotDesc* desc = nullptr;  // per storage slot
  double* err_partial = nullptr;
  float* block_max = nullptr;
  float* maxv = nullptr;
  int* flags = nullptr;
  unsigned* res_bar = nullptr;  // resident-Sequence barrier words, two per slot (sizes with that form)
  PopScalars* scal = nullptr;
  int* stats_part = nullptr;  // per-workgroup support counts of STATS
  // per-iteration Fourier error of traced iterations: [row][slot position]
  double* trace = nullptr;
  int trace_cap = 0;   // rows allocated
  int trace_rows = 0;  // rows written by the last run
  GenStatsDev* hist = nullptr;
  int hist_cap = 4096;
  float2* F = nullptr;
  float2* Cc = nullptr;
  ArgmaxRec* amax = nullptr;
  AlignRec* align = nullptr;
  int* abc = nullptr;
  int* mapprm = nullptr;
  // population average (allocated by the first AVERAGE): density, support
  // words, fitness, the mean aligned spectrum, the average modulus for the
  // crossover, the best parent's index and a one-slot descriptor table
  float2* avgX = nullptr;
  uint32_t* avgS = nullptr;
  double* avgE = nullptr;
  float2* avgF = nullptr;
  float* Mavg = nullptr;
  int* avg_ref = nullptr;
  SlotDesc* avg_desc = nullptr;
  int* avg_slot = nullptr;
  bool avg_done = false;
  // per-generation monitor records (allocated by the first MONITOR)
  MonitorDev* mon = nullptr;
  double* mon_sums = nullptr;
  int mon_cap = 4096;
  uint8_t* stage = nullptr;
  size_t stage_bytes = 0;
  hipStream_t last = nullptr;
  hipEvent_t done = nullptr;  // recorded after the population's latest enqueued work
  // optional per-kernel timing: HIP events recorded around each launch
  uint32_t timing = 0;  // bit k: time kernel k
  int timing_every = 1;  // time one launch in every timing_every of each kernel
  int64_t timing_seen[SPR_KERNEL_COUNT] = {};
  struct Stamp {
    int kernel;
    hipEvent_t start, stop;
  };
  std::vector<Stamp> stamps;
  std::vector<hipEvent_t> event_pool;
  double kernel_ms[SPR_KERNEL_COUNT] = {};
  int64_t kernel_launches[SPR_KERNEL_COUNT] = {};
};

struct spr_sched {
  std::vector<spr_op> ops;
};

namespace spr_live {
// Live handles of the process.  Destroy calls on unknown (already destroyed)
// handles are rejected instead of touching freed memory, and a context being
// destroyed first destroys the populations and shots still created on it.
inline std::mutex g_live_mu;
inline std::set<const void*> g_live;

inline void live_add(const void* h) {
  std::lock_guard<std::mutex> g(g_live_mu);
  g_live.insert(h);
}
inline bool live_remove(const void* h) {
  std::lock_guard<std::mutex> g(g_live_mu);
  return g_live.erase(h) > 0;
}
inline bool live_has(const void* h) {
  std::lock_guard<std::mutex> g(g_live_mu);
  return g_live.count(h) > 0;
}
}  // namespace spr_live
using namespace spr_live;

// Device address of the allocation-free entry point's scratch array on this
// device (noalloc.cpp), looked up once per device at context creation.
spr_status noalloc_setup(int device, std::string* err);

namespace {

struct Fail {
  spr_status code;
  std::string msg;
};

[[noreturn]] void fail(spr_status code, const std::string& msg) { throw Fail{code, msg}; }

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) fail(SPR_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T_>
T_* dalloc(size_t count) {
  void* p = nullptr;
  size_t bytes = std::max<size_t>(count * sizeof(T_), 256);
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    fail(SPR_E_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  return static_cast<T_*>(p);
}

template <class T_>
void dfree(T_*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

template <class Fn>
spr_status guarded(spr_ctx* ctx, Fn&& fn) {
  try {
    fn();
    return SPR_OK;
  } catch (const Fail& f) {
    if (ctx) ctx->err = f.msg;
    return f.code;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->err = "host allocation failed";
    return SPR_E_OOM;
  } catch (...) {
    if (ctx) ctx->err = "unexpected internal error";
    return SPR_E_INVALID_ARG;
  }
}

void use_device(spr_ctx* ctx) { HIPCHK(hipSetDevice(ctx->device)); }

// Kernels of size n in the variant selected on the context (default 0).
const SizeKernels* ctx_kernels(spr_ctx* ctx, int n) {
  auto it = ctx->variant.find(n);
  return size_kernels(n, it == ctx->variant.end() ? 0 : it->second);
}

const float2* twiddles(spr_ctx* ctx, int n) {
  std::lock_guard<std::mutex> g(ctx->mu);
  auto it = ctx->tw.find(n);
  if (it != ctx->tw.end()) return it->second;
  std::vector<float2> h(n);
  const double two_pi = 6.283185307179586476925286766559;
  for (int e = 0; e < n; ++e) {
    const double ang = two_pi * (double)e / (double)n;
    h[e] = make_float2((float)std::cos(ang), (float)-std::sin(ang));
  }
  float2* d = dalloc<float2>(n);
  HIPCHK(hipMemcpy(d, h.data(), n * sizeof(float2), hipMemcpyHostToDevice));
  ctx->tw[n] = d;
  return d;
}

Phase phase_of(double chi) {
  Phase p;
  p.c = 0.f;
  p.s = 0.f;
  if (!(chi > 0.0) || chi >= 1.0) {
    p.mode = PHASE_OFF;
  } else if (chi == 0.5) {
    p.mode = PHASE_POS;
  } else {
    p.mode = PHASE_CONE;
    const double th = chi * 3.14159265358979323846264338327950288;
    p.c = (float)std::cos(th);
    p.s = (float)std::sin(th);
  }
  return p;
}

void to_host(std::vector<uint8_t>& dst, const void* src, size_t bytes, bool device) {
  dst.resize(bytes);
  if (device) HIPCHK(hipMemcpy(dst.data(), src, bytes, hipMemcpyDeviceToHost));
  else std::memcpy(dst.data(), src, bytes);
}

// Measured modulus in FFT order with the mask in the sign bit (known <=>
// stored value >= +0), and the normaliser sum of Xi M^2 of Eq. error_calc.
double encode_shot(int n, const float* a, const uint8_t* mask, uint32_t flags, float* enc) {
  double den = 0.0;
  const int h = (flags & SPR_LAYOUT_FFT) ? 0 : n / 2;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      // FFT-order index (i, j) reads the centred image at (i + n/2, j + n/2) mod n
      const size_t src = (size_t)((i + h) % n) * n + (size_t)((j + h) % n);
      const float v = a[src];
      if (mask[src] != 0) {
        if (!std::isfinite(v) || v < 0.f) fail(SPR_E_NUMERIC, "measured amplitude is negative or not finite");
        enc[(size_t)i * n + j] = v == 0.f ? 0.f : v;
        den += (double)v * (double)v;
      } else {
        enc[(size_t)i * n + j] = -0.f;
      }
    }
  if (!(den > 0.0)) fail(SPR_E_INVALID_ARG, "sum of measured M^2 must be positive");
  return den;
}

// Smallest positive normal FP16 value (a zero bound in FP16 storage).
constexpr float kHalfTiny = 6.103515625e-05f;

// FP16 storage of the encoded modulus: M / s rounded to nearest even, with s
// the power of two that puts the largest measured value in [2^13, 2^14], so
// that no stored value overflows and small ones stay clear of the subnormal
// range; the sign bit (unknown pixels) is kept.
// The normaliser of Eq. error_calc is recomputed from the stored values, so
// that numerator and denominator see the same modulus.
float fp16_encode(const float* enc, size_t nn, std::vector<__half>& out, double& den) {
  float mx = 0.f;
  for (size_t k = 0; k < nn; ++k)
    if (!std::signbit(enc[k])) mx = std::max(mx, enc[k]);
  const float s = mx > 0.f ? std::ldexp(1.0f, (int)std::ceil(std::log2((double)mx)) - 14) : 1.0f;
  out.resize(nn);
  den = 0.0;
  for (size_t k = 0; k < nn; ++k) {
    // unknown pixels keep their (scaled) amplitude bound, or -0
    out[k] = __float2half(std::signbit(enc[k]) ? -std::min(-enc[k] / s, 65504.0f) : enc[k] / s);
    if (!std::signbit(enc[k])) {
      const double v = (double)__half2float(out[k]) * (double)s;
      den += v * v;
    }
  }
  return s;
}

// Upper bounds of the unknown amplitudes from the radial profile of the known
// intensities (Eq. avgint, Eq. stdint, Eq. upperbound): per ring q (distance
// of the signed frequency from zero, rounded half up), mu and sigma of I = M^2
// over the ring's known pixels and U = mu + eta sigma; a ring with more than
// max_unknown of its pixels unknown gets none.  The amplitude bound sqrt(U)
// goes into the unknown pixels of `enc` (stored values, FFT order) as -sqrt(U)
// / scale, keeping the sign bit that marks them; -0 means no bound, and a zero
// bound is kept as the smallest positive normal value.  eta <= 0 clears every
// bound.  With `sat` (FFT order, nonzero = saturated, all unknown), the
// saturation rules of the same appendix apply: a saturated pixel gets no bound
// and a ring with more than max_sat of its pixels saturated gets none.
// Returns the number of rings with a bound.
int apply_upper_bounds(int n, float* enc, float scale, double eta, double max_unknown,
                       float tiny = std::numeric_limits<float>::min(), const uint8_t* sat = nullptr,
                       double max_sat = 1.0) {
  const size_t nn = (size_t)n * n;
  std::vector<int> bin(nn);
  int nb = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double u = i < (n + 1) / 2 ? i : i - n, v = j < (n + 1) / 2 ? j : j - n;
      const int b = (int)std::floor(std::sqrt(u * u + v * v) + 0.5);
      bin[(size_t)i * n + j] = b;
      nb = std::max(nb, b + 1);
    }
  std::vector<double> s1(nb, 0.0), s2(nb, 0.0);
  std::vector<int64_t> known(nb, 0), total(nb, 0), nsat(nb, 0);
  for (size_t k = 0; k < nn; ++k) {
    total[bin[k]]++;
    if (sat && sat[k]) nsat[bin[k]]++;
    if (!std::signbit(enc[k])) {
      const double I = (double)enc[k] * scale * ((double)enc[k] * scale);
      s1[bin[k]] += I;
      s2[bin[k]] += I * I;
      known[bin[k]]++;
    }
  }
  std::vector<double> bound(nb, -1.0);
  int rings = 0;
  for (int b = 0; b < nb; ++b) {
    if (!(eta > 0.0) || known[b] == 0) continue;
    if ((double)(total[b] - known[b]) > max_unknown * (double)total[b]) continue;
    if ((double)nsat[b] > max_sat * (double)total[b]) continue;
    const double mu = s1[b] / (double)known[b];
    const double var = std::max(s2[b] / (double)known[b] - mu * mu, 0.0);
    bound[b] = std::sqrt(mu + eta * std::sqrt(var));
    ++rings;
  }
  for (size_t k = 0; k < nn; ++k) {
    if (!std::signbit(enc[k])) continue;
    const double b = bound[bin[k]];
    if (b < 0.0 || (sat && sat[k])) enc[k] = -0.0f;
    else enc[k] = -std::max((float)(b / scale), tiny);
  }
  return rings;
}

// A saturation mask (layout as the shot's mask) in FFT order; every saturated
// pixel must be unknown in the encoded modulus.
std::vector<uint8_t> saturation_fft(int n, const uint8_t* sat, uint32_t flags, const float* enc) {
  const int h = (flags & SPR_LAYOUT_FFT) ? 0 : n / 2;
  std::vector<uint8_t> out((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const size_t k = (size_t)i * n + j;
      out[k] = sat[(size_t)((i + h) % n) * n + (size_t)((j + h) % n)] != 0;
      if (out[k] && !std::signbit(enc[k])) fail(SPR_E_INVALID_ARG, "a saturated pixel is marked as measured");
    }
  return out;
}

uint8_t* stage(spr_pop* pop, size_t bytes) {
  if (pop->stage_bytes < bytes) {
    dfree(pop->stage);
    pop->stage = dalloc<uint8_t>(bytes);
    pop->stage_bytes = bytes;
  }
  return pop->stage;
}

struct Scope {
  const int* slots;
  int nm;
};

Scope scope_of(spr_pop* pop, int scope) {
  switch (scope) {
    case SPR_SCOPE_ALL:
      return {pop->table, pop->nslots};
    case SPR_SCOPE_PARENTS:
      return {pop->table, pop->P};
    case SPR_SCOPE_CHILDREN:
      if (!pop->memetic) fail(SPR_E_INVALID_ARG, "children scope on a population without children");
      return {pop->table + pop->P, pop->P};
    default:
      fail(SPR_E_INVALID_ARG, "unknown scope " + std::to_string(scope));
  }
}

void launch_ok(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(SPR_E_HIP, std::string("launch of ") + what + " failed: " + hipGetErrorString(e));
}

hipEvent_t pooled_event(spr_pop* pop) {
  if (!pop->event_pool.empty()) {
    hipEvent_t e = pop->event_pool.back();
    pop->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  return e;
}

// Launch through `fn(const LaunchEvents*)`; when timing is enabled the
// dispatch itself records a pair of events at the kernel's start and end.
template <class Fn>
void timed(spr_pop* pop, int kernel, hipStream_t s, const char* what, Fn&& fn) {
  if (!(pop->timing & (1u << kernel)) || pop->timing_seen[kernel]++ % pop->timing_every != 0) {
    launch_ok(fn(nullptr), what);
    return;
  }
  const LaunchEvents ev{pooled_event(pop), pooled_event(pop)};
  launch_ok(fn(&ev), what);
  pop->stamps.push_back({kernel, ev.start, ev.stop});
}

// Fold finished stamps into the per-kernel totals (after a synchronisation).
void collect_stamps(spr_pop* pop) {
  for (auto& st : pop->stamps) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, st.start, st.stop));
    pop->kernel_ms[st.kernel] += ms;
    pop->kernel_launches[st.kernel] += 1;
    pop->event_pool.push_back(st.start);
    pop->event_pool.push_back(st.stop);
  }
  pop->stamps.clear();
}

struct Iter {
  int alg;
  float beta;
  double chi;
  bool trace = false;  // record the Fourier error of the spectrum this iteration projects
};

// A launch group: members of one size reached through slot descriptors, and
// the work buffers they use.  A population's scope and a batch of shots both
// run through groups.
struct Group {
  spr_ctx* ctx = nullptr;
  const SizeKernels* K = nullptr;
  int n = 0, W = 0;
  const int* slots = nullptr;
  int nm = 0;
  const SlotDesc* desc = nullptr;
  float2* T = nullptr;           // work buffers: >= chunk members (>= nm for smoothing/fitness)
  float2* Y = nullptr;
  double* err_partial = nullptr; // >= nm * n / C
  float* block_max = nullptr;    // >= nm * smoothing blocks per member
  float* maxv = nullptr;         // >= nm
  int* flags = nullptr;
  spr_pop* timing = nullptr;     // where launch timings are kept (may be null)
  int chunk = 0;                 // members per iteration launch
  int t_by_slot = 0;             // row transforms in each member's own buffer (desc.T)
  double* trace = nullptr;       // trace rows of the population (traced iterations only)
  int trace_cols = 0;            // slot positions per trace row
  int pos0 = 0;                  // slot position of slots[0]
  unsigned* res_bar = nullptr;   // barrier words of the resident Sequence (>= 2 per chunk member), or null
};

int chunk_for(spr_ctx* ctx, int n, int nm) {
  auto it = ctx->chunk_members.find(n);
  if (it != ctx->chunk_members.end() && it->second > 0) return std::min(nm, it->second);
  if (ctx->cache_budget == 0) return nm;
  const size_t per_member = 2 * (size_t)n * n * sizeof(float2);
  if ((size_t)nm * per_member <= ctx->cache_budget) return nm;
  // Chunks of three quarters of the budget, measured over 128 members at
  // 384^2-1024^2: 0-4 % faster than chunks of the whole budget (a chunk's
  // iterations then leave room in the cache for the modulus, supports and
  // twiddles every pass also reads); one launch stays best while the whole
  // population fits.
  return (int)std::min<size_t>((size_t)nm, std::max<size_t>(1, ctx->cache_budget / 4 * 3 / per_member));
}

Group pop_group(spr_pop* pop, int scope) {
  Scope sc = scope_of(pop, scope);
  Group g;
  g.ctx = pop->ctx;
  g.K = pop->K;
  g.n = pop->n;
  g.W = pop->W;
  g.slots = sc.slots;
  g.nm = sc.nm;
  g.desc = pop->desc;
  g.T = pop->T;
  g.Y = pop->Y;
  g.err_partial = pop->err_partial;
  g.block_max = pop->block_max;
  g.maxv = pop->maxv;
  g.flags = pop->flags;
  g.timing = pop;
  g.chunk = chunk_for(pop->ctx, pop->n, sc.nm);
  g.trace = pop->trace;
  g.trace_cols = pop->nslots;
  g.pos0 = scope == SPR_SCOPE_CHILDREN ? pop->P : 0;
  g.res_bar = pop->res_bar;
  return g;
}

template <class Fn>
void launch_timed(spr_pop* tp, int kernel, hipStream_t s, const char* what, Fn&& fn) {
  if (tp) timed(tp, kernel, s, what, fn);
  else launch_ok(fn(nullptr), what);
}

// The resident form of a Sequence over members slots[0..nm), where the size
// has one: no iteration is traced and the stream is not being captured.  The
// iterations go kResMaxIters to a launch; returns false when the Sequence
// must run as launch pairs.
bool run_resident(const Group& g, const std::vector<Iter>& its, int c0, int nm, hipStream_t s) {
  if (!g.K->seq_res || !g.res_bar || g.t_by_slot) return false;
  for (const auto& it : its)
    if (it.trace) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
  SeqResArgs a{};
  a.slots = g.slots + c0;
  a.nm = nm;
  a.desc = g.desc;
  a.T = g.T;
  a.Y = g.Y;
  a.W = g.W;
  a.t_by_slot = 0;
  a.tw = twiddles(g.ctx, g.n);
  a.ingest_mode = its[0].alg == ALG_ER ? INGEST_PC : INGEST_PLAIN;
  a.ingest_ph = phase_of(its[0].chi);
  a.res_bar = g.res_bar;
  for (size_t i0 = 0; i0 < its.size(); i0 += kResMaxIters) {
    const size_t i1 = std::min(its.size(), i0 + (size_t)kResMaxIters);
    a.ingest = i0 == 0;
    a.iters = (int)(i1 - i0);
    for (size_t i = i0; i < i1; ++i) {
      const bool last = i + 1 == its.size();
      ResIter& q = a.it[i - i0];
      q.alg = its[i].alg;
      q.beta = its[i].beta;
      q.ph = phase_of(its[i].chi);
      q.out_mode = last ? OUT_REAL : (its[i + 1].alg == ALG_ER ? OUT_T_PC : OUT_T_PLAIN);
      q.ph_next = last ? phase_of(1.0) : phase_of(its[i + 1].chi);
    }
    launch_ok(g.K->seq_res(a, s), "seq_res");
  }
  return true;
}

// One Sequence over members slots[0..nm): ingest, then per iteration a column
// pass and a row pass.
void run_iterations_on(const Group& g, const std::vector<Iter>& its, int c0, int nm, int trace_row0,
                       hipStream_t s) {
  if (run_resident(g, its, c0, nm, s)) return;
  const int* slots = g.slots + c0;
  const SizeKernels* K = g.K;
  const float2* tw = twiddles(g.ctx, g.n);
  RowIngestArgs ia{slots, nm, g.desc, g.T, g.W, g.t_by_slot,
                   its[0].alg == ALG_ER ? INGEST_PC : INGEST_PLAIN, phase_of(its[0].chi), tw};
  launch_timed(g.timing, SPR_KERNEL_ROW_INGEST, s, "row_ingest",
               [&](const LaunchEvents* ev) { return K->row_ingest(ia, s, ev); });
  int trace_row = trace_row0;
  for (size_t i = 0; i < its.size(); ++i) {
    ColProjArgs ca{slots, nm, g.desc, g.t_by_slot, g.T, g.Y, tw, its[i].trace ? g.err_partial : nullptr};
    launch_timed(g.timing, SPR_KERNEL_COL_PROJ, s, "col_proj",
                 [&](const LaunchEvents* ev) { return K->col_proj(ca, s, ev); });
    if (its[i].trace) {
      if (!g.trace) fail(SPR_E_INVALID_ARG, "iteration traces are recorded for single populations only");
      TraceFinalArgs ta{g.err_partial, g.n / K->C, nm, slots, g.desc,
                        g.trace + (size_t)trace_row * g.trace_cols, g.pos0 + c0};
      launch_ok(launch_trace_final(ta, s), "trace_final");
      ++trace_row;
    }
    const bool last = i + 1 == its.size();
    RowUpdateArgs ra;
    ra.slots = slots;
    ra.nm = nm;
    ra.desc = g.desc;
    ra.Y = g.Y;
    ra.T = g.T;
    ra.W = g.W;
    ra.t_by_slot = g.t_by_slot;
    ra.ip = nullptr;
    ra.alg = its[i].alg;
    ra.beta = its[i].beta;
    ra.ph = phase_of(its[i].chi);
    ra.out_mode = last ? OUT_REAL : (its[i + 1].alg == ALG_ER ? OUT_T_PC : OUT_T_PLAIN);
    ra.ph_next = last ? phase_of(1.0) : phase_of(its[i + 1].chi);
    ra.tw = tw;
    const int kid = ra.alg == ALG_ER ? SPR_KERNEL_ROW_UPDATE_ER : SPR_KERNEL_ROW_UPDATE_IA;
    launch_timed(g.timing, kid, s, "row_update", [&](const LaunchEvents* ev) { return K->row_update(ra, s, ev); });
  }
}

// Members are independent inside a Sequence, so the run may proceed chunk by
// chunk; with a cache budget the chunk's buffers stay cache-resident across
// its iterations.
void run_iterations(const Group& g, const std::vector<Iter>& its, hipStream_t s, int trace_row0 = 0) {
  if (its.empty() || g.nm == 0) return;
  const int chunk = g.chunk > 0 ? g.chunk : g.nm;
  for (int c0 = 0; c0 < g.nm; c0 += chunk) run_iterations_on(g, its, c0, std::min(chunk, g.nm - c0), trace_row0, s);
}

int traced_iterations(const spr_sched* sch) {
  int rows = 0;
  for (const auto& o : sch->ops)
    if ((o.kind == SPR_OP_ER || o.kind == SPR_OP_HIO || o.kind == SPR_OP_RAAR) && (o.which & SPR_ITER_TRACE))
      rows += o.count;
  return rows;
}

void trace_buffers(spr_pop* pop, int rows) {
  if (rows <= pop->trace_cap) return;
  double* t = dalloc<double>((size_t)rows * pop->nslots);
  dfree(pop->trace);
  pop->trace = t;
  pop->trace_cap = rows;
}

void smooth(const Group& g, double sigma, hipStream_t s) {
  SmoothArgs sa{};
  int r = 0;
  std::vector<double> w(1, 1.0);
  if (sigma > 0) {
    r = (int)std::ceil(4.0 * sigma);
    if (r > (MAX_TAPS - 1) / 2) fail(SPR_E_INVALID_ARG, "shrink-wrap sigma above 8 pixels is not supported");
    w.assign(2 * r + 1, 0.0);
    double sum = 0.0;
    for (int k = -r; k <= r; ++k) {
      w[k + r] = std::exp(-(double)(k * k) / (2.0 * sigma * sigma));
      sum += w[k + r];
    }
    for (auto& v : w) v /= sum;
  }
  sa.slots = g.slots;
  sa.nm = g.nm;
  sa.n = g.n;
  sa.r = r;
  sa.desc = g.desc;
  sa.out = reinterpret_cast<float*>(g.Y);
  sa.block_max = g.block_max;
  for (int k = 0; k <= 2 * r; ++k) sa.w[k] = (float)w[k];
  MemberMaxArgs ma{g.nm, smooth_blocks_per_member(g.n), g.block_max, g.maxv};
  launch_ok(launch_smooth(sa, ma, s), "smooth");
}

void shrinkwrap(const Group& g, double sigma, double tau, hipStream_t s) {
  if (g.nm == 0) return;
  smooth(g, sigma, s);
  ThresholdArgs ta{g.slots, g.nm, g.n, g.W, reinterpret_cast<const float*>(g.Y), g.maxv, tau, g.desc};
  launch_ok(launch_threshold(ta, s), "threshold");
}

void support_area(const Group& g, double sigma, const double* alpha_src, int alpha_index, double alpha_abs,
                  hipStream_t s) {
  if (g.nm == 0) return;
  smooth(g, sigma, s);
  TopkArgs ta{};
  ta.slots = g.slots;
  ta.nm = g.nm;
  ta.n = g.n;
  ta.W = g.W;
  ta.in = reinterpret_cast<const float*>(g.Y);
  ta.alpha_src = alpha_src;
  ta.alpha_index = alpha_index;
  ta.alpha_abs = alpha_abs;
  ta.desc = g.desc;
  // the row-transform buffer is free between sequences: it holds the
  // selection's histograms (at least nm * n * n floats)
  ta.scratch = reinterpret_cast<uint32_t*>(g.T);
  launch_ok(launch_topk(ta, s), "topk");
}

void get_error(const Group& g, hipStream_t s) {
  if (g.nm == 0) return;
  const SizeKernels* K = g.K;
  const float2* tw = twiddles(g.ctx, g.n);
  RowIngestArgs ia{g.slots, g.nm, g.desc, g.T, g.W, g.t_by_slot, INGEST_SMASK, phase_of(1.0), tw};
  launch_ok(K->row_ingest(ia, s, nullptr), "row_ingest");
  ColErrArgs ea{g.slots, g.nm, g.desc, g.t_by_slot, g.T, g.err_partial, tw};
  launch_ok(K->col_err(ea, s), "col_err");
  ErrFinalArgs fa{g.err_partial, g.n / K->C, g.nm, g.slots, g.desc};
  launch_ok(launch_err_final(fa, s), "err_final");
}

// Random-phase start of P members stored contiguously at X: Fourier-side
// values, then the unitary inverse 2D transform in place.
void random_phase_start(spr_ctx* ctx, const SizeKernels* K, int n, int P, const float* amp, const __half* amp16,
                        float amp_scale, uint64_t seed, float2* X, hipStream_t s) {
  if (P == 0) return;
  const float2* tw = twiddles(ctx, n);
  InitPhaseArgs ia{P, n, amp, amp16, amp_scale, seed, X};
  launch_ok(launch_init_phase(ia, s), "init_phase");
  ColFftArgs c{nullptr, nullptr, P, X, X, +1, 1.f, tw};
  launch_ok(K->col_fft(c, s), "col_fft");
  RowFftArgs r{nullptr, nullptr, P, X, X, +1, 1.f / (float)n, tw};
  launch_ok(K->row_fft(r, s), "row_fft");
}

const double* alpha_source(spr_pop* pop, const spr_op& op, int& index, double& abs_alpha) {
  index = 0;
  abs_alpha = 0.0;
  if (op.which == SPR_AREA_ABS) {
    abs_alpha = op.alpha;
    return nullptr;
  }
  if (op.which == SPR_AREA_BEST || op.which == SPR_AREA_EVAL) {
    if (!pop) fail(SPR_E_INVALID_ARG, "areas from generation statistics need a population");
    index = op.which;
    return pop->scal->alpha;
  }
  fail(SPR_E_INVALID_ARG, "unknown support-area source");
}

void need_memetic(spr_pop* pop, const char* what) {
  if (!pop->memetic) fail(SPR_E_INVALID_ARG, std::string(what) + " needs a population created with SPR_POP_MEMETIC");
}

// Parent spectra, correlation images and alignment records (first use).
void correlation_buffers(spr_pop* pop) {
  if (pop->F) return;
  const int n = pop->n, P = pop->P;
  const size_t nn = (size_t)n * n;
  const int blocks = n / pop->K->RWI;
  pop->F = dalloc<float2>((size_t)P * nn);
  pop->Cc = dalloc<float2>((size_t)6 * P * nn);
  pop->amax = dalloc<ArgmaxRec>((size_t)6 * P * blocks);
  pop->align = dalloc<AlignRec>((size_t)3 * P);
  pop->abc = dalloc<int>((size_t)3 * P);
  pop->mapprm = dalloc<int>((size_t)5 * P);
}

void monitor_buffers(spr_pop* pop) {
  if (pop->mon) return;
  pop->mon = dalloc<MonitorDev>(pop->mon_cap);
  pop->mon_sums = dalloc<double>((size_t)(pop->P + 1) * 3);
  HIPCHK(hipMemset(pop->mon, 0, sizeof(MonitorDev) * pop->mon_cap));
}

void average_buffers(spr_pop* pop) {
  if (pop->avgX) return;
  const size_t nn = (size_t)pop->n * pop->n;
  pop->avgX = dalloc<float2>(nn);
  pop->avgS = dalloc<uint32_t>(pop->W);
  pop->avgE = dalloc<double>(1);
  pop->avgF = dalloc<float2>(nn);
  pop->Mavg = dalloc<float>(nn);
  pop->avg_ref = dalloc<int>(1);
  pop->avg_slot = dalloc<int>(1);
  pop->avg_desc = dalloc<SlotDesc>(1);
  SlotDesc d{};
  d.X = pop->avgX;
  d.T = pop->T;
  d.S = pop->avgS;
  d.amp = pop->shot->amp;
  d.amp16 = pop->shot->amp16;
  d.E = pop->avgE;
  d.den = pop->shot->den;
  d.flags = pop->flags;
  d.amp_scale = pop->shot->amp_scale;
  const int zero = 0;
  HIPCHK(hipMemcpy(pop->avg_desc, &d, sizeof(d), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(pop->avg_slot, &zero, sizeof(int), hipMemcpyHostToDevice));
}

// Population average of the parents (Alg. mpr's Average, Eq. avgrec): every
// parent aligned to the best one (Reshift, Eq. crosscorr), the mean aligned
// density and the union of the aligned supports, its fitness (Eq.
// error_calc), and the average modulus (Eq. avgint1, Eq. avgint2) used by a
// crossover with c_a > 0.
void average(spr_pop* pop, hipStream_t s) {
  const SizeKernels* K = pop->K;
  const int n = pop->n, P = pop->P;
  const float2* tw = twiddles(pop->ctx, n);
  correlation_buffers(pop);
  average_buffers(pop);
  RowFftArgs r1{pop->table, pop->table, P, pop->X, pop->T, -1, 1.f, tw};
  launch_ok(K->row_fft(r1, s), "row_fft");
  ColFftArgs c1{pop->table, nullptr, P, pop->T, pop->F, -1, 1.f / (float)n, tw};
  launch_ok(K->col_fft(c1, s), "col_fft");
  AvgArgs aa{P, n, pop->W, pop->table, pop->E, pop->avg_ref, pop->F, pop->align, pop->avgF, pop->Mavg,
             pop->S, pop->avgS, tw};
  launch_ok(launch_avg_best(aa, s), "avg_best");
  ColCorrArgs cc{P, nullptr, pop->avg_ref, pop->F, pop->shot->amp, pop->shot->amp16, pop->Cc, tw};
  launch_ok(K->col_corr(cc, s), "col_corr");
  RowArgmaxArgs am{2 * P, pop->Cc, pop->amax, tw};
  launch_ok(K->row_argmax(am, s), "row_argmax");
  AlignArgs al{P, n / K->RWI, n, pop->amax, pop->align};
  launch_ok(launch_align(al, s), "align");
  launch_ok(launch_avg_spectra(aa, s), "avg_spectra");
  launch_ok(launch_avg_support(aa, s), "avg_support");
  // rho_avg = unitary inverse transform of the mean aligned spectrum
  ColFftArgs c2{nullptr, nullptr, 1, pop->avgF, pop->T, +1, 1.f, tw};
  launch_ok(K->col_fft(c2, s), "col_fft");
  RowFftArgs r2{nullptr, nullptr, 1, pop->T, pop->avgX, +1, 1.f / (float)n, tw};
  launch_ok(K->row_fft(r2, s), "row_fft");
  Group g;
  g.ctx = pop->ctx;
  g.K = K;
  g.n = n;
  g.W = pop->W;
  g.slots = pop->avg_slot;
  g.nm = 1;
  g.desc = pop->avg_desc;
  g.T = pop->T;
  g.Y = pop->Y;
  g.err_partial = pop->err_partial;
  g.block_max = pop->block_max;
  g.maxv = pop->maxv;
  g.flags = pop->flags;
  get_error(g, s);
  pop->avg_done = true;
}

void crossover(spr_pop* pop, const spr_op& op, hipStream_t s) {
  need_memetic(pop, "CROSSOVER");
  if (pop->P < 4) fail(SPR_E_INVALID_ARG, "crossover needs P >= 4");
  const SizeKernels* K = pop->K;
  const int n = pop->n, P = pop->P;
  const float2* tw = twiddles(pop->ctx, n);
  int t_min = op.t_min > 0 ? op.t_min : 4;
  int t_max = op.t_max > 0 ? op.t_max : std::max(t_min, n / 8);
  if (t_max < t_min) fail(SPR_E_INVALID_ARG, "crossover t_max < t_min");
  if (!(op.c_p >= 0.0 && op.c_p <= 1.0)) fail(SPR_E_INVALID_ARG, "crossover probability outside [0, 1]");
  const int blocks = n / K->RWI;
  correlation_buffers(pop);
  if (op.c_a > 0.0 && !pop->avg_done)
    fail(SPR_E_INVALID_ARG, "a crossover with c_a > 0 needs an AVERAGE of the parents first");
  // parent spectra F[p] (unitary)
  RowFftArgs r1{pop->table, pop->table, P, pop->X, pop->T, -1, 1.f, tw};
  launch_ok(K->row_fft(r1, s), "row_fft");
  ColFftArgs c1{pop->table, nullptr, P, pop->T, pop->F, -1, 1.f / (float)n, tw};
  launch_ok(K->col_fft(c1, s), "col_fft");
  ChoiceArgs ch{P, op.gen, t_min, t_max, pop->seed, pop->abc, pop->mapprm};
  launch_ok(launch_choice(ch, s), "choice");
  ColCorrArgs cc{3 * P, pop->abc, nullptr, pop->F, pop->shot->amp, pop->shot->amp16, pop->Cc, tw};
  launch_ok(K->col_corr(cc, s), "col_corr");
  RowArgmaxArgs am{6 * P, pop->Cc, pop->amax, tw};
  launch_ok(K->row_argmax(am, s), "row_argmax");
  AlignArgs al{3 * P, blocks, n, pop->amax, pop->align};
  launch_ok(launch_align(al, s), "align");
  double thr = std::floor(op.c_p * 4294967296.0);
  thr = std::min(std::max(thr, 0.0), 4294967296.0);
  ColMixArgs mx{P, pop->abc, pop->mapprm, pop->align, pop->F, pop->table, pop->T, (float)op.c_w,
                pop->seed, op.gen, (uint64_t)thr, 1.f / (float)n, tw,
                op.c_a > 0.0 ? (float)op.c_a : 0.f, op.c_a > 0.0 ? pop->Mavg : nullptr};
  launch_ok(K->col_mix(mx, s), "col_mix");
  RowFftArgs r2{pop->table + P, pop->table + P, P, pop->T, pop->X, +1, 1.f, tw};
  launch_ok(K->row_fft(r2, s), "row_fft");
  SupportMixArgs sm{P, n, pop->W, pop->table, pop->abc, pop->align, pop->S};
  launch_ok(launch_support_mix(sm, s), "support_mix");
}

GenStatsDev* record(spr_pop* pop, int gen) {
  int g = gen - 1;
  if (g < 0) g = 0;
  return pop->hist + (g % pop->hist_cap);
}

void validate_op(const spr_op& o) {
  switch (o.kind) {
    case SPR_OP_ER:
    case SPR_OP_HIO:
    case SPR_OP_RAAR:
      if (o.count < 0) fail(SPR_E_INVALID_ARG, "negative iteration count");
      if (o.which & ~SPR_ITER_TRACE) fail(SPR_E_INVALID_ARG, "unknown iteration flags");
      if (o.kind != SPR_OP_ER && !(o.beta > 0.0 && o.beta <= 1.0)) fail(SPR_E_INVALID_ARG, "beta outside (0, 1]");
      break;
    case SPR_OP_SHRINKWRAP:
      if (!(o.sigma >= 0.0 && o.sigma <= 8.0)) fail(SPR_E_INVALID_ARG, "sigma outside [0, 8]");
      if (!(o.tau >= 0.0 && o.tau <= 1.0)) fail(SPR_E_INVALID_ARG, "tau outside [0, 1]");
      break;
    case SPR_OP_SUPPORT_AREA:
      if (!(o.sigma >= 0.0 && o.sigma <= 8.0)) fail(SPR_E_INVALID_ARG, "sigma outside [0, 8]");
      if (o.which < 0 || o.which > 2) fail(SPR_E_INVALID_ARG, "unknown area source");
      break;
    case SPR_OP_GET_ERROR:
      break;
    case SPR_OP_STATS:
      if (o.gen < 1 || o.gens < 1) fail(SPR_E_INVALID_ARG, "STATS needs gen >= 1 and gens >= 1");
      break;
    case SPR_OP_CROSSOVER:
      if (o.gen < 1) fail(SPR_E_INVALID_ARG, "CROSSOVER needs gen >= 1");
      if (!(o.c_w >= 0.0 && o.c_w <= 2.0)) fail(SPR_E_INVALID_ARG, "c_w outside [0, 2]");
      if (!(o.c_a >= 0.0 && o.c_a <= 1.0)) fail(SPR_E_INVALID_ARG, "c_a outside [0, 1]");
      break;
    case SPR_OP_AVERAGE:
      break;
    case SPR_OP_MONITOR:
      if (o.gen < 1) fail(SPR_E_INVALID_ARG, "MONITOR needs gen >= 1");
      break;
    case SPR_OP_SELECT:
      if (o.gen < 1) fail(SPR_E_INVALID_ARG, "SELECT needs gen >= 1");
      break;
    default:
      fail(SPR_E_INVALID_ARG, "unknown op kind " + std::to_string(o.kind));
  }
  if (o.scope < 0 || o.scope > 2) fail(SPR_E_INVALID_ARG, "unknown scope");
}

void run_schedule(spr_pop* pop, const spr_sched* sch, hipStream_t s) {
  const auto& ops = sch->ops;
  for (const auto& o : ops) {
    if ((o.kind == SPR_OP_CROSSOVER || o.kind == SPR_OP_SELECT || o.kind == SPR_OP_STATS ||
         o.scope == SPR_SCOPE_CHILDREN) && !pop->memetic)
      fail(SPR_E_INVALID_ARG, "schedule needs a population created with SPR_POP_MEMETIC");
    if (o.kind == SPR_OP_CROSSOVER && pop->P < 4) fail(SPR_E_INVALID_ARG, "crossover needs P >= 4");
  }
  // traced iterations: one row per traced iteration, NaN where a slot is not traced
  const int rows = traced_iterations(sch);
  if (rows > 0) {
    trace_buffers(pop, rows);
    FillArgs fa{pop->trace, (long)rows * pop->nslots, std::numeric_limits<double>::quiet_NaN()};
    launch_ok(launch_fill(fa, s), "fill");
    pop->trace_rows = rows;
  }
  int trace_row = 0;
  size_t i = 0;
  while (i < ops.size()) {
    const spr_op& o = ops[i];
    if (o.kind == SPR_OP_ER || o.kind == SPR_OP_HIO || o.kind == SPR_OP_RAAR) {
      std::vector<Iter> its;
      const int scope = o.scope;
      while (i < ops.size() &&
             (ops[i].kind == SPR_OP_ER || ops[i].kind == SPR_OP_HIO || ops[i].kind == SPR_OP_RAAR) &&
             ops[i].scope == scope) {
        const spr_op& q = ops[i];
        const int alg = q.kind == SPR_OP_ER ? ALG_ER : (q.kind == SPR_OP_HIO ? ALG_HIO : ALG_RAAR);
        for (int c = 0; c < q.count; ++c) its.push_back({alg, (float)q.beta, q.chi, (q.which & SPR_ITER_TRACE) != 0});
        ++i;
      }
      int traced = 0;
      for (const auto& it : its) traced += it.trace ? 1 : 0;
      run_iterations(pop_group(pop, scope), its, s, trace_row);
      trace_row += traced;
      continue;
    }
    switch (o.kind) {
      case SPR_OP_SHRINKWRAP:
        shrinkwrap(pop_group(pop, o.scope), o.sigma, o.tau, s);
        break;
      case SPR_OP_SUPPORT_AREA: {
        int idx;
        double ab;
        const double* src = alpha_source(pop, o, idx, ab);
        support_area(pop_group(pop, o.scope), o.sigma, src, idx, ab, s);
        break;
      }
      case SPR_OP_GET_ERROR:
        get_error(pop_group(pop, o.scope), s);
        break;
      case SPR_OP_STATS: {
        need_memetic(pop, "STATS");
        StatsArgs sa{pop->P, pop->W, o.gen, o.gens, pop->table, pop->E, pop->S, pop->scal, record(pop, o.gen),
                     pop->stats_part};
        launch_ok(launch_stats(sa, s), "stats");
        break;
      }
      case SPR_OP_CROSSOVER:
        crossover(pop, o, s);
        break;
      case SPR_OP_AVERAGE:
        average(pop, s);
        break;
      case SPR_OP_MONITOR: {
        monitor_buffers(pop);
        const int g = o.gen > 0 ? o.gen - 1 : 0;
        MonitorArgs ma{pop->P, pop->n, pop->table, pop->X, pop->avg_done ? pop->avgX : nullptr, pop->E,
                       pop->avg_done ? pop->avgE : nullptr, pop->mon_sums, pop->mon + (g % pop->mon_cap), o.gen};
        launch_ok(launch_monitor(ma, s), "monitor");
        break;
      }
      case SPR_OP_SELECT: {
        need_memetic(pop, "SELECT");
        SelectArgs se{pop->P, o.gen, pop->table, pop->E, record(pop, o.gen)};
        launch_ok(launch_select(se, s), "select");
        break;
      }
      default:
        fail(SPR_E_INVALID_ARG, "unknown op kind");
    }
    ++i;
  }
}

void sched_at(int g, int G, int j, int j_er, int j_end, double sigma, double sigma_end, double tau,
              double tau_end, int& jg, int& jer, double& sg, double& tg) {
  const double t = G <= 1 ? 0.0 : (double)(g - 1) / (double)(G - 1);
  jg = (int)std::floor((double)j + t * (double)(j_end - j) + 0.5);
  jer = j + j_er - jg;
  sg = sigma + t * (sigma_end - sigma);
  tg = tau + t * (tau_end - tau);
}

spr_op make_op(int kind) {
  spr_op o;
  std::memset(&o, 0, sizeof(o));
  o.kind = kind;
  o.chi = 0.5;
  return o;
}

void push_seq(std::vector<spr_op>& ops, int alg, int jg, int jer, double beta, double chi) {
  if (jg > 0) {
    spr_op o = make_op(alg == SPR_ALG_RAAR ? SPR_OP_RAAR : SPR_OP_HIO);
    o.count = jg;
    o.beta = beta;
    o.chi = chi;
    ops.push_back(o);
  }
  if (jer > 0) {
    spr_op o = make_op(SPR_OP_ER);
    o.count = jer;
    o.chi = chi;
    ops.push_back(o);
  }
}

void destroy_pop(spr_pop* p) {
  for (auto& st : p->stamps) {
    (void)hipEventDestroy(st.start);
    (void)hipEventDestroy(st.stop);
  }
  p->stamps.clear();
  for (auto e : p->event_pool) (void)hipEventDestroy(e);
  p->event_pool.clear();
  if (p->done) (void)hipEventDestroy(p->done);
  p->done = nullptr;
  dfree(p->X);
  dfree(p->T);
  dfree(p->Y);
  dfree(p->S);
  dfree(p->E);
  dfree(p->table);
  dfree(p->desc);
  dfree(p->err_partial);
  dfree(p->block_max);
  dfree(p->maxv);
  dfree(p->flags);
  dfree(p->res_bar);
  dfree(p->scal);
  dfree(p->stats_part);
  dfree(p->trace);
  dfree(p->hist);
  dfree(p->F);
  dfree(p->Cc);
  dfree(p->amax);
  dfree(p->align);
  dfree(p->abc);
  dfree(p->mapprm);
  dfree(p->avgX);
  dfree(p->avgS);
  dfree(p->avgE);
  dfree(p->avgF);
  dfree(p->Mavg);
  dfree(p->avg_ref);
  dfree(p->avg_desc);
  dfree(p->avg_slot);
  dfree(p->mon);
  dfree(p->mon_sums);
  dfree(p->stage);
}

std::vector<int> host_table(spr_pop* pop) {
  std::vector<int> t(pop->nslots);
  HIPCHK(hipMemcpy(t.data(), pop->table, sizeof(int) * pop->nslots, hipMemcpyDeviceToHost));
  return t;
}

void sync_pop(spr_pop* pop) {
  if (pop->done) HIPCHK(hipEventSynchronize(pop->done));
  HIPCHK(hipStreamSynchronize(pop->ctx->stream));
  if (!pop->stamps.empty()) collect_stamps(pop);
}

void workspace_alloc(Workspace& w, int n, size_t members, const SizeKernels* K);
void workspace_free(Workspace& w);

Workspace& workspace(spr_ctx* ctx, int n, size_t members, const SizeKernels* K) {
  Workspace& w = ctx->ws[n];
  if (w.members >= members) return w;
  HIPCHK(hipDeviceSynchronize());  // the old buffers may still be in use
  workspace_free(w);
  workspace_alloc(w, n, members, K);
  return w;
}

bool same_op(const spr_op& a, const spr_op& b) {
  return a.kind == b.kind && a.count == b.count && a.scope == b.scope && a.which == b.which && a.gen == b.gen &&
         a.gens == b.gens && a.t_min == b.t_min && a.t_max == b.t_max && a.beta == b.beta && a.chi == b.chi &&
         a.sigma == b.sigma && a.tau == b.tau && a.alpha == b.alpha && a.c_p == b.c_p && a.c_w == b.c_w &&
         a.c_a == b.c_a;
}

// Populations of one size advancing through one schedule together: every
// operation is a single launch over all their members.
void run_group_schedule(const Group& g, const spr_sched* sch, hipStream_t s) {
  const auto& ops = sch->ops;
  size_t i = 0;
  while (i < ops.size()) {
    const spr_op& o = ops[i];
    if (o.kind == SPR_OP_ER || o.kind == SPR_OP_HIO || o.kind == SPR_OP_RAAR) {
      std::vector<Iter> its;
      while (i < ops.size() &&
             (ops[i].kind == SPR_OP_ER || ops[i].kind == SPR_OP_HIO || ops[i].kind == SPR_OP_RAAR)) {
        const spr_op& q = ops[i];
        if (q.which & SPR_ITER_TRACE)
          fail(SPR_E_INVALID_ARG, "iteration traces are recorded for single populations only");
        const int alg = q.kind == SPR_OP_ER ? ALG_ER : (q.kind == SPR_OP_HIO ? ALG_HIO : ALG_RAAR);
        for (int c = 0; c < q.count; ++c) its.push_back({alg, (float)q.beta, q.chi});
        ++i;
      }
      run_iterations(g, its, s);
      continue;
    }
    switch (o.kind) {
      case SPR_OP_SHRINKWRAP:
        shrinkwrap(g, o.sigma, o.tau, s);
        break;
      case SPR_OP_SUPPORT_AREA:
        if (o.which != SPR_AREA_ABS) fail(SPR_E_INVALID_ARG, "batched runs take absolute support areas only");
        support_area(g, o.sigma, nullptr, 0, o.alpha, s);
        break;
      case SPR_OP_GET_ERROR:
        get_error(g, s);
        break;
      default:
        fail(SPR_E_INVALID_ARG, "batched runs take ER/HIO/RAAR, SHRINKWRAP, SUPPORT_AREA and GET_ERROR only");
    }
    ++i;
  }
}

// Crossover buffers allocated ahead of a capture (no allocation may happen
// while a stream is being captured).
void prepare_buffers(spr_pop* pop, const spr_sched* sch) {
  trace_buffers(pop, traced_iterations(sch));
  for (const auto& o : sch->ops) {
    if ((o.kind == SPR_OP_CROSSOVER && pop->memetic && pop->P >= 4) || o.kind == SPR_OP_AVERAGE)
      correlation_buffers(pop);
    if (o.kind == SPR_OP_AVERAGE) {
      average_buffers(pop);
      pop->avg_done = true;  // the captured AVERAGE precedes any crossover that uses it
    }
    if (o.kind == SPR_OP_MONITOR) monitor_buffers(pop);
  }
}

// Populations of one size in a batch: their schedule and where their
// descriptors and slot list live.
struct BatchGroup {
  int n = 0;
  std::vector<int> idx;  // indices into the batch
  const spr_sched* sched = nullptr;
  Group g;
};

// Validate a batch and group it by size; descriptors and slot lists are
// written (synchronously) into the given workspaces, one per size.
std::vector<BatchGroup> plan_batch(spr_ctx* ctx, spr_pop* const* pops, const spr_sched* const* scheds, int n,
                                   const std::function<Workspace&(int, size_t, const SizeKernels*)>& ws_for) {
  std::map<int, std::vector<int>> by_size;
  for (int i = 0; i < n; ++i) {
    if (!pops[i] || !scheds[i]) fail(SPR_E_INVALID_ARG, "null population or schedule");
    if (!live_has(pops[i])) fail(SPR_E_INVALID_ARG, "population already destroyed");
    if (pops[i]->ctx != ctx) fail(SPR_E_INVALID_ARG, "population of another context");
    for (int j = 0; j < i; ++j)
      if (pops[j] == pops[i]) fail(SPR_E_INVALID_ARG, "population listed twice");
    for (const auto& o : scheds[i]->ops)
      if (o.scope != SPR_SCOPE_ALL) fail(SPR_E_INVALID_ARG, "batched runs act on every member (scope ALL)");
    by_size[pops[i]->n].push_back(i);
  }
  std::vector<BatchGroup> out;
  for (auto& kv : by_size) {
    BatchGroup bg;
    bg.n = kv.first;
    bg.idx = kv.second;
    bg.sched = scheds[bg.idx[0]];
    for (int i : bg.idx) {
      const auto& a = scheds[i]->ops;
      if (a.size() != bg.sched->ops.size()) fail(SPR_E_INVALID_ARG, "schedules of one size must be equal");
      for (size_t k = 0; k < a.size(); ++k)
        if (!same_op(a[k], bg.sched->ops[k])) fail(SPR_E_INVALID_ARG, "schedules of one size must be equal");
    }
    size_t total = 0;
    for (int i : bg.idx) total += pops[i]->nslots;
    const SizeKernels* K = pops[bg.idx[0]]->K;
    for (int i : bg.idx)
      if (pops[i]->K != K) fail(SPR_E_INVALID_ARG, "populations of one size were created with different kernel variants");
    Workspace& w = ws_for(bg.n, total, K);
    std::vector<int> slots;
    std::vector<SlotDesc> descs;
    size_t off = 0;
    for (int i : bg.idx) {
      spr_pop* pop = pops[i];
      sync_pop(pop);
      std::vector<SlotDesc> d(pop->nslots);
      HIPCHK(hipMemcpy(d.data(), pop->desc, sizeof(SlotDesc) * pop->nslots, hipMemcpyDeviceToHost));
      descs.insert(descs.end(), d.begin(), d.end());
      std::vector<int> t = host_table(pop);
      for (int v : t) slots.push_back((int)off + v);
      off += pop->nslots;
    }
    HIPCHK(hipMemcpy(w.desc, descs.data(), sizeof(SlotDesc) * descs.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(w.slots, slots.data(), sizeof(int) * slots.size(), hipMemcpyHostToDevice));
    Group& g = bg.g;
    g.ctx = ctx;
    g.K = K;
    g.n = bg.n;
    g.W = pops[bg.idx[0]]->W;
    g.slots = w.slots;
    g.nm = (int)total;
    g.desc = w.desc;
    g.T = w.T;
    g.Y = w.Y;
    g.err_partial = w.err_partial;
    g.block_max = w.block_max;
    g.maxv = w.maxv;
    g.timing = nullptr;
    g.chunk = chunk_for(ctx, bg.n, (int)total);
    out.push_back(bg);
  }
  return out;
}

// Run the size groups of a batch.  Groups touch disjoint members and work
// buffers, so their order does not matter.  When the groups' iteration
// chunks together fit the cache budget (small shots, whose launches cannot
// fill the device alone), they overlap on the device: the first on s, each
// other one on a stream of its own that starts when s reaches this point,
// and s then waits for all of them.  Otherwise they run one after another:
// each group's chunk already fills the memory-side cache, and overlapping
// groups would evict each other's work buffers (measured: 32 shots of
// 256^2..1024^2 ran 5 % slower overlapped).  Under stream capture the side
// streams join the capture through the events, and the graph gets the same
// fork and join.
void run_groups(spr_ctx* ctx, std::vector<BatchGroup>& groups, hipStream_t s) {
  size_t resident = 0;
  for (const auto& bg : groups) resident += 2 * (size_t)bg.g.chunk * bg.n * bg.n * sizeof(float2);
  if (groups.size() <= 1 || ctx->cache_budget == 0 || resident > ctx->cache_budget) {
    for (auto& bg : groups) run_group_schedule(bg.g, bg.sched, s);
    return;
  }
  while (ctx->side.size() + 1 < groups.size()) {
    hipStream_t t = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&t, hipStreamNonBlocking));
    ctx->side.push_back(t);
  }
  std::vector<hipEvent_t> ev;
  auto event = [&]() {
    hipEvent_t e = nullptr;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ev.push_back(e);
    return e;
  };
  try {
    hipEvent_t fork = event();
    HIPCHK(hipEventRecord(fork, s));
    std::vector<hipEvent_t> joins;
    for (size_t k = 1; k < groups.size(); ++k) {
      hipStream_t t = ctx->side[k - 1];
      HIPCHK(hipStreamWaitEvent(t, fork, 0));
      run_group_schedule(groups[k].g, groups[k].sched, t);
      hipEvent_t j = event();
      HIPCHK(hipEventRecord(j, t));
      joins.push_back(j);
    }
    run_group_schedule(groups[0].g, groups[0].sched, s);
    for (hipEvent_t j : joins) HIPCHK(hipStreamWaitEvent(s, j, 0));
  } catch (...) {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    throw;
  }
  for (hipEvent_t e : ev) HIPCHK(hipEventDestroy(e));
}

// Work buffers of a batch of `members` members of size n.
void workspace_alloc(Workspace& w, int n, size_t members, const SizeKernels* K) {
  const size_t nn = (size_t)n * n;
  w.T = dalloc<float2>(members * nn);
  w.Y = dalloc<float2>(members * nn);
  w.err_partial = dalloc<double>(members * (n / K->C));
  w.block_max = dalloc<float>(members * smooth_blocks_per_member(n));
  w.maxv = dalloc<float>(members);
  w.desc = dalloc<SlotDesc>(members);
  w.slots = dalloc<int>(members);
  w.members = members;
}

void workspace_free(Workspace& w) {
  for (void* q : {(void*)w.T, (void*)w.Y, (void*)w.err_partial, (void*)w.block_max, (void*)w.maxv,
                  (void*)w.desc, (void*)w.slots})
    if (q) (void)hipFree(q);
  w = Workspace();
}

}  // namespace

