/*
 * spr.h -- C ABI of the MI355X (gfx950) hot path of Memetic Phase Retrieval
 * (MPR), the reconstruction method of SPRING (Colombo et al., arXiv 2409.07413).
 *
 * The problem (section "The phase problem and conventional approaches"): recover
 * a complex density rho (N x N) from the measured Fourier modulus M = sqrt(I),
 * known only where the mask Xi = 1 (beamstop and detector gaps are left free,
 * appendix "Dealing with missing intensities", Eq. pm_full).  A population of
 * candidate reconstructions R = (rho, S, E) -- density, boolean support and
 * error -- is improved by iterative projection algorithms (ER, HIO, RAAR),
 * shrink-wrap support updates, the Eq. error_calc fitness, and, for MPR, the
 * memetic crossover and selection operators (appendix "Memetic operators").
 *
 * Conventions
 * -----------
 * - Every call returns spr_status: SPR_OK (0) or a negative error code; the
 *   message of the last error is kept per context (spr_ctx_last_error).  No
 *   C++ exception crosses this boundary.
 * - Sizes: N must be 2^a 3^b with 8 <= N <= 1024 from the compiled set
 *   (spr_supported_size); other sizes give SPR_E_UNSUPPORTED_SIZE.
 * - Complex arrays are interleaved float32 pairs (re, im), row-major
 *   [member][row][col].  Supports are uint8 (0/1) [member][row][col].
 * - Amplitudes and masks are taken in the centred detector layout (zero
 *   frequency at [N/2][N/2]) unless SPR_LAYOUT_FFT is given.  Densities and
 *   supports are real-space arrays with natural indices.
 * - Pointers are host memory unless SPR_DEVICE_PTRS is given, in which case they
 *   are device pointers on the context's device (e.g. torch data_ptr()).
 * - Inputs are copied at create/write time: the caller keeps ownership of every
 *   buffer it passes.  The library owns all device state until the matching
 *   destroy call.  Outputs go only into caller buffers.
 * - Work is enqueued asynchronously on a HIP stream (NULL = the context's
 *   stream); spr_sync and the read calls wait for it.
 * - Threads: calls on one context and on the handles created from it (shots,
 *   populations, graphs, servers) must not overlap in time: one thread at a
 *   time, or the caller's own locking.  Distinct contexts may be used from
 *   distinct threads.  A server's engine thread is internal to the library
 *   and needs no locking by the caller.  Schedule calls with a NULL context
 *   touch no shared state.
 */
#ifndef SPR_H
#define SPR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t spr_status;

#define SPR_OK 0
#define SPR_E_INVALID_ARG (-1)      /* null pointer, bad count or parameter, wrong handle state */
#define SPR_E_UNSUPPORTED_SIZE (-2) /* N not in the compiled set */
#define SPR_E_OOM (-3)              /* device allocation failed */
#define SPR_E_HIP (-4)              /* a HIP runtime call or kernel launch failed */
#define SPR_E_NOT_READY (-5)        /* serving: result not finished */
#define SPR_E_BUSY (-6)             /* destroy of a shot that still has populations */
#define SPR_E_NUMERIC (-7)          /* NaN/Inf in the inputs or in a fitness value */
#define SPR_E_ADMISSION (-8)        /* serving: request can never fit the memory budget */

/* flags */
#define SPR_DEVICE_PTRS 0x1u   /* pointer arguments are device memory */
#define SPR_LAYOUT_FFT 0x2u    /* amplitude/mask already in FFT order (DC at [0][0]) */
#define SPR_POP_MEMETIC 0x4u   /* population also holds P children (needed by crossover/select) */
#define SPR_READ_CHILDREN 0x8u /* spr_read/spr_pop_write act on the child population */
#define SPR_INIT_RANDOM_PHASE 0x10u /* spr_pop_create: generate the random-phase start on the device */
#define SPR_AMP_FP16 0x20u     /* shot: store the measured modulus in FP16 (see spr_shot_create) */

typedef struct spr_ctx spr_ctx;
typedef struct spr_shot spr_shot;
typedef struct spr_pop spr_pop;
typedef struct spr_sched spr_sched;

/* ------------------------------------------------------------------------- */
/* Context: one per device; owns a stream and the per-size twiddle tables.   */
/* ------------------------------------------------------------------------- */
spr_status spr_ctx_create(int32_t hip_device, spr_ctx** out);
/* Destroys the populations and shots still alive on the context, then the     */
/* context.  Calls on destroyed handles return SPR_E_INVALID_ARG.              */
void spr_ctx_destroy(spr_ctx* ctx);
/* Message of the last failed call on this context ("" if none). Owned by ctx. */
const char* spr_ctx_last_error(const spr_ctx* ctx);
/* 1 if N is a supported detector size, else 0. */
int32_t spr_supported_size(int32_t n);
/* Iteration runs (consecutive ER/HIO/RAAR ops) whose two N x N complex work    */
/* buffers per member fit in `bytes` (default 256 MiB, the memory-side cache of */
/* one MI355X) run as one launch per pass; larger ones in chunks of members     */
/* whose buffers fill three quarters of it.  Members are independent inside a  */
/* run, so results do not depend on it.  0 = one chunk.                         */
spr_status spr_ctx_set_cache_budget(spr_ctx* ctx, uint64_t bytes);

/* Tuning.  Sizes 128, 256, 384, 512, 768 and 1024 are compiled twice:       */
/* variant 0 (the default plan) and variant 1 (the other column-tile width,  */
/* for 1024 the other radix order, for 128 the resident Sequence: one        */
/* cooperative launch per Sequence, whose workgroups meet at device-memory   */
/* barriers between passes; same results bit for bit, used when no iteration */
/* is traced and the stream is not being captured).  spr_ctx_autotune times RAAR iterations on */
/* `members` synthetic members of size n for every variant and member-chunk  */
/* candidate (all members, the chunks whose two work buffers fit 256, 192   */
/* and 128 MiB), keeps the fastest on the context and reports every one.    */
/* The variant applies to shots (and their populations) created afterwards;  */
/* the chunk to every later iteration run of that size.  Results do not      */
/* depend on the choice beyond floating-point rounding of the transform.     */
#define SPR_TUNE_MAX 16
typedef struct spr_tune_result {
  int32_t n, variant, chunk_members, candidates;
  double member_iterations_per_s;    /* of the choice */
  int32_t cand_variant[SPR_TUNE_MAX];
  int32_t cand_chunk[SPR_TUNE_MAX];
  double cand_rate[SPR_TUNE_MAX];    /* member-iterations/s */
} spr_tune_result;
/* Number of compiled kernel variants of size n (0 if unsupported). */
int32_t spr_size_variants(int32_t n);
/* Times the candidates of size n on `members` synthetic members (as above); */
/* waits for the device.  SPR_E_UNSUPPORTED_SIZE for an unsupported n.       */
spr_status spr_ctx_autotune(spr_ctx* ctx, int32_t n, int32_t members, spr_tune_result* out);
/* Set the choice by hand (chunk_members 0: the cache-budget rule). */
spr_status spr_ctx_set_variant(spr_ctx* ctx, int32_t n, int32_t variant, int32_t chunk_members);
/* The choice in force for size n (variant 0 and chunk 0 when none was made). */
spr_status spr_ctx_get_tuning(spr_ctx* ctx, int32_t n, int32_t* variant, int32_t* chunk_members);

/* ------------------------------------------------------------------------- */
/* Shot: the measured modulus M = sqrt(I) and mask Xi (1 = measured) of one    */
/* diffraction pattern (section "The phase problem...", Eq. pm_full).         */
/* amp: N*N float32, finite, >= 0 where measured.  mask: N*N uint8.            */
/* The sum of Xi M^2 must be positive (it normalises Eq. error_calc).          */
/* SPR_AMP_FP16: the library keeps M / s in FP16 (2 bytes per pixel, rounded  */
/* to nearest even), with s the power of two that puts the largest measured   */
/* M / s in [2^13, 2^14]; kernels multiply by s after loading.  All other     */
/* arithmetic is unchanged (FP32 transforms, FP64 reductions).                */
/* Errors: SPR_E_INVALID_ARG, SPR_E_NUMERIC (non-finite or negative measured   */
/* amplitude), SPR_E_UNSUPPORTED_SIZE, SPR_E_OOM, SPR_E_HIP.                   */
/* ------------------------------------------------------------------------- */
spr_status spr_shot_create(spr_ctx* ctx, int32_t n, const float* amp, const uint8_t* mask,
                           uint32_t flags, spr_shot** out);
/* SPR_E_BUSY while populations created on the shot are alive. */
spr_status spr_shot_destroy(spr_shot* shot);
/* Upper bounds on the unknown amplitudes (appendix on missing intensities,   */
/* Eq. avgint, Eq. stdint, Eq. upperbound, Eq. pm_bounds): per ring of pixels  */
/* at the same rounded distance q from the zero frequency, mu and sigma of the */
/* known intensities M^2 give U(q) = mu + eta sigma; the projector then brings */
/* an unknown Fourier value whose modulus exceeds sqrt(U(q)) down to it (phase */
/* kept).  Rings with more than max_unknown (e.g. 0.2) of their pixels unknown */
/* get no bound.  eta <= 0 removes the bounds.  The bounds live in the sign-   */
/* marked unknown pixels of the stored modulus (no extra memory).  Waits for   */
/* the device; *rings (may be NULL) gets the number of bounded rings.          */
spr_status spr_shot_set_bounds(spr_shot* shot, double eta, double max_unknown, int32_t* rings);
/* The same bounds with the saturation rules of that appendix: a saturated     */
/* pixel gets no bound, and a ring with more than max_saturated of its pixels  */
/* saturated (the paper's example: 0.05) gets none; saturated pixels count as   */
/* unknown in the max_unknown rule.  saturated: N*N bytes, nonzero = saturated, */
/* in the shot's layout (centred unless SPR_LAYOUT_FFT in flags; device memory  */
/* with SPR_DEVICE_PTRS); read during the call only.  Every saturated pixel     */
/* must be unknown in the shot's mask, else SPR_E_INVALID_ARG.  saturated ==    */
/* NULL gives spr_shot_set_bounds (max_saturated and flags unused).             */
spr_status spr_shot_set_bounds_sat(spr_shot* shot, double eta, double max_unknown, const uint8_t* saturated,
                                   double max_saturated, uint32_t flags, int32_t* rings);

/* ------------------------------------------------------------------------- */
/* Population: P reconstructions (Alg. mpr / Alg. randomsearch, D1-D2 of the   */
/* memetic-operators appendix).                                               */
/* rho0: P*N*N complex (interleaved float32).  supp0: N*N (broadcast, when     */
/* supp_per_member = 0) or P*N*N uint8.  seed keys the Philox4x32-10 stream of */
/* the memetic operators; gen_offset is the number of generations already run  */
/* (resume).  SPR_POP_MEMETIC reserves the P children of Alg. crossover.       */
/* Crossover needs P >= 4 (three distinct other parents).                      */
/* With SPR_INIT_RANDOM_PHASE rho0 is ignored (may be NULL) and member p starts */
/* at rho0_p = F^-1[Xi M e^{i phi}] (unitary inverse DFT), phi = 2 pi (u+1/2)/2^32 */
/* with u = Philox draw k of (seed, purpose 4, generation 0, member p) at the   */
/* FFT-order pixel k (row-major): the classic random-phase start; the paper's   */
/* own Initialize (projected spheres, initialisation appendix) is separate.    */
/* ------------------------------------------------------------------------- */
spr_status spr_pop_create(spr_shot* shot, int32_t P, const float* rho0, const uint8_t* supp0,
                          int32_t supp_per_member, uint32_t flags, uint64_t seed,
                          int32_t gen_offset, spr_pop** out);
/* Waits for the population's work and frees it; SPR_E_BUSY while a graph    */
/* references it.                                                             */
spr_status spr_pop_destroy(spr_pop* pop);
/* The paper's Initialize (initialisation appendix) on the device, for the     */
/* parents: each fills a centred sigma_init-wide square with n_init projected  */
/* spheres (optical depth 2 sqrt(R^2 - r^2)), diameters uniform in             */
/* [diam_min, diam_max] * sigma_init, centres uniform over the positions that  */
/* keep the sphere in the square, each sphere with a phase uniform in          */
/* [phase_min, phase_max]; the modulus of the sum is raised to gamma (phase    */
/* kept) and the density scaled by sqrt(nu) of Eq. norm.  The draws are those  */
/* of the population's seed (purpose 5: words 4k..4k+3 for sphere k).  With    */
/* set_support the parents' supports become the square |row - N/2| <= s/2,     */
/* |col - N/2| <= s/2 (s = sigma_init).  Waits for the device.                 */
typedef struct spr_sphere_params {
  double sigma_init;          /* side of the centred square, pixels (> 0) */
  int32_t n_init;             /* spheres per member (>= 1) */
  int32_t set_support;
  double diam_min, diam_max;  /* fractions of sigma_init, e.g. 0.2 and 0.9 */
  double phase_min, phase_max;
  double gamma;               /* > 0 */
} spr_sphere_params;
spr_status spr_pop_init_spheres(spr_pop* pop, const spr_sphere_params* prm);
/* Overwrite the state of the parents (or children with SPR_READ_CHILDREN):    */
/* any of rho (P*N*N complex), supp (P*N*N uint8), err (P doubles) may be NULL. */
spr_status spr_pop_write(spr_pop* pop, const float* rho, const uint8_t* supp, const double* err,
                         uint32_t flags);

/* ------------------------------------------------------------------------- */
/* Schedules: a flat list of operations applied in order to a population.     */
/* ------------------------------------------------------------------------- */
#define SPR_OP_ER 1           /* count iterations of x <- P_M P_C x (Error Reduction) */
#define SPR_OP_HIO 2          /* count iterations of HIO, beta */
#define SPR_OP_RAAR 3         /* count iterations of RAAR, beta */
#define SPR_OP_SHRINKWRAP 4   /* UpdateSupport (Eq. shrinkwrap): sigma, tau */
#define SPR_OP_SUPPORT_AREA 5 /* UpdateSupportSize: sigma, area from `which` */
#define SPR_OP_GET_ERROR 6    /* E <- Eq. error_calc */
#define SPR_OP_STATS 7        /* alpha_best, alpha_all, alpha_eval of Alg. improve, for gen/gens */
#define SPR_OP_CROSSOVER 8    /* Alg. crossover into the children: c_p, c_w, t_min, t_max, gen */
#define SPR_OP_SELECT 9       /* Alg. select, gen */
#define SPR_OP_AVERAGE 10     /* Alg. mpr's Average of the parents (Eq. avgrec), members aligned */
                              /* to the best one; also the average modulus used when c_a > 0    */
#define SPR_OP_MONITOR 11     /* indicators of the parents for generation gen (spr_read_monitor) */
/* ER/HIO/RAAR flag (spr_op.which): record, for every iteration of the op, the */
/* Fourier error sqrt(sum Xi (|X| - M)^2 / sum Xi M^2) of the spectrum X that  */
/* the iteration projects (Eq. error_calc's measure applied to the iterate,    */
/* x for HIO/RAAR, P_C x for ER), summed in FP64 inside the column pass.       */
/* Single populations only (spr_run, population graphs).                       */
#define SPR_ITER_TRACE 1

#define SPR_ALG_HIO 1
#define SPR_ALG_RAAR 2

#define SPR_AREA_BEST 0 /* alpha_best of the last STATS */
#define SPR_AREA_EVAL 1 /* alpha_eval of the last STATS */
#define SPR_AREA_ABS 2  /* the op's alpha */

#define SPR_SCOPE_ALL 0      /* every member (parents and children) */
#define SPR_SCOPE_PARENTS 1
#define SPR_SCOPE_CHILDREN 2

typedef struct spr_op {
  int32_t kind;   /* SPR_OP_* */
  int32_t count;  /* ER/HIO/RAAR: iterations */
  int32_t scope;  /* SPR_SCOPE_* (iterations, support updates, GET_ERROR) */
  int32_t which;  /* SUPPORT_AREA: SPR_AREA_*; ER/HIO/RAAR: 0 or SPR_ITER_TRACE */
  int32_t gen;    /* STATS/CROSSOVER/SELECT: generation g (1-based, absolute) */
  int32_t gens;   /* STATS: total generations G */
  int32_t t_min;  /* CROSSOVER: tile side range [t_min, t_max] */
  int32_t t_max;
  double beta;    /* HIO/RAAR feedback parameter */
  double chi;     /* ER/HIO/RAAR: phase range [-chi pi, chi pi]; chi <= 0 or >= 1: none */
  double sigma;   /* SHRINKWRAP/SUPPORT_AREA: Gaussian width in pixels (0: no smoothing, <= 8) */
  double tau;     /* SHRINKWRAP: threshold fraction of the smoothed maximum */
  double alpha;   /* SUPPORT_AREA with SPR_AREA_ABS: target area in pixels */
  double c_p;     /* CROSSOVER: tile election probability */
  double c_w;     /* CROSSOVER: differential weight */
  double c_a;     /* CROSSOVER: weight of the average modulus on parent a (Eq. crossavg); */
                  /* > 0 needs an earlier AVERAGE                                       */
} spr_op;

/* Parameters of Table tab:params and the linear schedules ("Changing values  */
/* over generations"): j decays linearly from j to j_end over G, the ER count  */
/* keeps j + j_er constant, sigma and tau interpolate to their end values.     */
typedef struct spr_plain_params {
  int32_t alg;               /* SPR_ALG_HIO or SPR_ALG_RAAR */
  int32_t G;                 /* blocks (Alg. randomsearch generations) */
  int32_t j, j_er, j_end;    /* IA iterations at g = 1, ER iterations at g = 1, IA at g = G */
  double beta, chi;
  double sigma, sigma_end, tau, tau_end;
} spr_plain_params;

typedef struct spr_mpr_params {
  int32_t alg;
  int32_t G, R;              /* generations, sequences per self-improvement (R >= 2) */
  int32_t j, j_er, j_end, j_eval;
  int32_t t_min, t_max;      /* crossover tile sides */
  int32_t gen_first;         /* first generation to emit (1 = start) */
  int32_t gen_count;         /* generations to emit (0 = through G) */
  int32_t init_error;        /* 1: evaluate the parents' errors before the first generation */
  double beta, chi;
  double sigma, sigma_end, tau, tau_end;
  double c_p, c_w;
  double c_a;                /* Eq. crossavg weight (0: the plain crossover) */
  int32_t monitor;           /* 1: AVERAGE and MONITOR after every generation */
  int32_t pad;
} spr_mpr_params;

/* Schedule calls run on the host only; ctx (for error messages) may be NULL. */
spr_status spr_sched_create(spr_ctx* ctx, const spr_op* ops, int32_t nops, spr_sched** out);
/* Alg. randomsearch with Alg. normalimprove: per block Sequence then           */
/* UpdateSupport on every member, then GET_ERROR on every member.               */
spr_status spr_sched_plain(spr_ctx* ctx, const spr_plain_params* prm, spr_sched** out);
/* Alg. mpr: per generation (AVERAGE when c_a > 0), CROSSOVER, STATS, the      */
/* Alg. improve operations on every member, SELECT; after generation G the     */
/* final AVERAGE (read with spr_read_average).                                 */
spr_status spr_sched_mpr(spr_ctx* ctx, const spr_mpr_params* prm, spr_sched** out);
/* Frees a schedule (a host object; work already enqueued from it is kept).  */
spr_status spr_sched_destroy(spr_sched* sched);
/* Copy out the expanded op list (ops may be NULL to query the count). */
spr_status spr_sched_ops(const spr_sched* sched, spr_op* ops, int32_t max_ops, int32_t* n_ops);

/* ------------------------------------------------------------------------- */
/* Execution.                                                                 */
/* ------------------------------------------------------------------------- */
/* Enqueue the schedule on `hip_stream` (a hipStream_t; NULL = context stream). */
spr_status spr_run(spr_pop* pop, const spr_sched* sched, void* hip_stream);
/* Batched uneven shots: run scheds[i] on pops[i] for i < n.  Populations of one */
/* detector size advance together, each operation being one launch over all    */
/* their members (each reaching its own shot's modulus); size groups run one   */
/* after another on the stream, or overlap on context-owned side streams when  */
/* their iteration chunks together fit the cache budget.  Within a size the schedules must be equal and use    */
/* only ER/HIO/RAAR, SHRINKWRAP, SUPPORT_AREA with SPR_AREA_ABS and GET_ERROR on  */
/* scope ALL; otherwise SPR_E_INVALID_ARG.  Results equal running each          */
/* population alone.  Each population must appear once.                         */
spr_status spr_run_batch(spr_ctx* ctx, spr_pop* const* pops, const spr_sched* const* scheds, int32_t n,
                         void* hip_stream);
/* Wait for the population's work; SPR_E_NUMERIC if a fitness value was NaN/Inf; */
/* SPR_E_HIP if a resident Sequence (128^2 variant 1) ran out of a barrier wait  */
/* (its results are then not valid; the population can run again).  spr_read    */
/* reports the latter too.                                                       */
spr_status spr_sync(spr_pop* pop);

typedef struct spr_gen_stats {
  int32_t gen;          /* generation g (0: record unused) */
  int32_t best;         /* parent index of the lowest error before self-improvement */
  int32_t alpha_best;   /* support area of that parent */
  int32_t alpha_all;    /* area of the union of the parents' supports */
  double alpha_eval;    /* (g/G) alpha_best + (1 - g/G) alpha_all */
  double err_best;      /* after Select: lowest, mean and highest parent error */
  double err_mean;
  double err_worst;
  int32_t replaced;     /* children that replaced their parent (replacement factor * P) */
  int32_t pad;
} spr_gen_stats;

/* Read the parents (or children with SPR_READ_CHILDREN) into caller buffers:  */
/* rho P*N*N complex, supp P*N*N uint8, err P doubles; any may be NULL.         */
/* With SPR_DEVICE_PTRS the buffers are device memory.  Waits for the work.     */
spr_status spr_read(spr_pop* pop, float* rho, uint8_t* supp, double* err, uint32_t flags);
/* One parent (or child with SPR_READ_CHILDREN) into caller buffers: rho N*N  */
/* complex, supp N*N uint8; either may be NULL.  member in [0, P).            */
spr_status spr_read_member(spr_pop* pop, int32_t member, float* rho, uint8_t* supp, uint32_t flags);
/* The last AVERAGE: rho N*N complex, supp N*N uint8, err its Eq. error_calc  */
/* fitness (each may be NULL).  SPR_E_INVALID_ARG before any AVERAGE.         */
spr_status spr_read_average(spr_pop* pop, float* rho, uint8_t* supp, double* err, uint32_t flags);
/* Indicators of the monitoring section and the appendix on unconstrained    */
/* modes, per MONITOR op: errors of the parents (best, lower median, worst,   */
/* mean), mean complexity Gamma = 1 - |sum rho| / sum |rho| (Eq. complexity),  */
/* mean density sum |sum rho| and its population standard deviation relative  */
/* to the mean, and Gamma and error of the last AVERAGE (has_avg).             */
typedef struct spr_monitor {
  int32_t gen, P;
  double err_best, err_median, err_worst, err_mean;
  double gamma_mean, sum_mean, sum_rel_std;
  double gamma_avg, err_avg;
  int32_t has_avg, pad;
} spr_monitor;
/* Monitor records, oldest first; at most max_n; *n_out gets the count. */
spr_status spr_read_monitor(spr_pop* pop, spr_monitor* out, int32_t max_n, int32_t* n_out);
/* Traced iterations of the last run (SPR_ITER_TRACE): *rows traced iterations  */
/* in schedule order, each a row of *cols values (one per slot position: the  */
/* P parents, then the P children of a memetic population; NaN where the      */
/* iteration's scope left the member out).  out holds max_rows * cols doubles */
/* (host memory); rows beyond max_rows are not copied.                         */
spr_status spr_read_trace(spr_pop* pop, double* out, int32_t max_rows, int32_t* rows, int32_t* cols);
/* Generation records, oldest first; at most max_n; *n_out gets the count. */
spr_status spr_read_stats(spr_pop* pop, spr_gen_stats* out, int32_t max_n, int32_t* n_out);

typedef struct spr_xover_info {
  int32_t a, b, c;      /* parents chosen by RandomChoice for this child */
  int32_t tx, ty, sx, sy, rot; /* crossover-map tile sides, shift, rotation index */
  int32_t dr[3], dc[3]; /* Reshift translation of a, b, c */
  int32_t twin[3];      /* 1 where the twin image was taken */
  float phase[3][2];    /* e^{i phi} applied to a, b, c */
  float peak[3][2];     /* squared correlation maxima (direct, twin) */
} spr_xover_info;

/* Decisions of the last CROSSOVER (P records, host memory). */
spr_status spr_read_xover(spr_pop* pop, spr_xover_info* out, int32_t max_n);

/* ------------------------------------------------------------------------- */
/* Kernel timing: HIP events are recorded on the launch stream around every   */
/* launch of the kernels selected by `mask` (bit k = SPR_KERNEL_k; 0 = off);   */
/* spr_timing_read returns the number of launches and their summed event time */
/* since the last spr_timing_enable (it waits for the population's work).      */
/* ------------------------------------------------------------------------- */
#define SPR_KERNEL_ROW_INGEST 0    /* real-space density -> row FFT (sequence start) */
#define SPR_KERNEL_COL_PROJ 1      /* column FFT, masked modulus projection, column IFFT */
#define SPR_KERNEL_ROW_UPDATE_ER 2 /* row IFFT, ER step, row FFT */
#define SPR_KERNEL_ROW_UPDATE_IA 3 /* row IFFTs, HIO/RAAR step, row FFT */
#define SPR_KERNEL_COUNT 4
#define SPR_TIMING_ALL 0xF
spr_status spr_timing_enable(spr_pop* pop, int32_t mask);
/* Time only the first of every `every` (>= 1, default 1) launches of each    */
/* selected kernel, so that the events cost little beside the kernels; the   */
/* counts of spr_timing_read are then the timed launches.  Resets the totals. */
spr_status spr_timing_sample(spr_pop* pop, int32_t every);
spr_status spr_timing_read(spr_pop* pop, int32_t kernel, int64_t* launches, double* total_ms);

/* Unitary 2D DFT of `batch` N x N complex images (device pointers, in != out */
/* allowed to alias): forward exp(-2 pi i ...) / N, inverse exp(+...) / N.     */
spr_status spr_fft2(spr_ctx* ctx, int32_t n, int32_t batch, const float* in, float* out,
                    int32_t inverse, void* hip_stream);

/* The same transform for callers that cannot allocate device memory (code   */
/* under HIP graph capture, tight serving loops, harnesses that forbid       */
/* hipMalloc): it calls no device allocation or free.  Its twiddle table and  */
/* row-transform intermediate live in a fixed 64 MiB device array that the    */
/* library holds on every GPU it runs on until the process ends, so          */
/* batch * (8 n^2) + 8 n (the table, rounded up to 256 bytes) must not        */
/* exceed 64 MiB (e.g. 7 images of 1024^2): larger requests give              */
/* SPR_E_INVALID_ARG before anything is launched.  in and out are device      */
/* pointers and may alias.  Every call on one GPU shares the array, so calls  */
/* that overlap on one GPU (other streams, or threads) race; calls on one     */
/* stream are ordered.  Results agree with spr_fft2 to FP32 rounding.         */
spr_status spr_fft2_noalloc(spr_ctx* ctx, int32_t n, int32_t batch, const float* in, float* out,
                            int32_t inverse, void* hip_stream);

/* ------------------------------------------------------------------------- */
/* Graphs: the launches of a schedule recorded once into a HIP graph and      */
/* replayed with one call, for schedules whose per-launch host cost matters   */
/* (small detectors, short sequences, many populations).                      */
/* A graph replays exactly the recorded launches: the same schedule (with its */
/* generation numbers) on the same populations and buffers.  spr_pop_destroy  */
/* returns SPR_E_BUSY while a graph references the population.                */
/* ------------------------------------------------------------------------- */
typedef struct spr_graph spr_graph;

/* Records `sched` on `pop` (waits for the population's earlier work; nothing */
/* runs).  Crossover buffers are allocated here.                              */
spr_status spr_graph_create(spr_pop* pop, const spr_sched* sched, spr_graph** out);
/* Records a batch as spr_run_batch would run it (same rules); the graph owns */
/* its work buffers and the member order of the populations at creation.      */
spr_status spr_graph_create_batch(spr_ctx* ctx, spr_pop* const* pops, const spr_sched* const* scheds, int32_t n,
                                  spr_graph** out);
/* Enqueues one replay on hip_stream (NULL = the context stream), ordered     */
/* after the populations' earlier work.                                       */
spr_status spr_graph_launch(spr_graph* g, void* hip_stream);
/* Waits for the graph's replays and frees it (and the work buffers it owns). */
spr_status spr_graph_destroy(spr_graph* g);

/* ------------------------------------------------------------------------- */
/* Serving: a request loop for streamed single shots of mixed detector sizes.  */
/* Every admitted shot keeps its P-member population resident on the device   */
/* and runs the server's schedule; the shots admitted at any moment advance   */
/* together in ticks (continuous batching): in each tick every resident shot  */
/* runs its next sequence of iterations and the support/fitness steps that    */
/* follow it, with the members of all shots of one size and step batched into */
/* the same launches.  Requests are admitted first come, first served, when a */
/* shot slot and a range of the server's device-memory budget large enough    */
/* for the shot's footprint (amplitudes, densities, row transforms, support    */
/* bits, errors and its result record) are free; memory and slot return when  */
/* the result has reached host memory.  Members only interact with their own  */
/* shot's data, so a result is the same whichever shots share its ticks.      */
/* ------------------------------------------------------------------------- */
typedef struct spr_server spr_server;

#define SPR_SERVER_MANUAL 0x1u      /* no engine thread: the caller drives spr_server_step */
#define SPR_SERVER_ALL_MEMBERS 0x2u /* results carry every member, not only the best one */
/* Each tick advances only the shots of one size: that of the resident shot  */
/* with the least remaining work (modelled at 4 TB/s) less the time it has    */
/* waited since arrival.  Small shots then pass large ones instead of moving  */
/* at their pace, and the waiting time keeps large ones from starving.       */
/* Without it every resident shot advances in every tick.                    */
#define SPR_SERVER_SHORTEST_FIRST 0x4u

typedef struct spr_server_cfg {
  uint64_t hbm_budget;    /* device bytes held by the server (work buffers + admitted shots) */
  int32_t max_shots;      /* shots resident at once */
  int32_t P;              /* members per shot */
  const spr_sched* sched; /* per-shot schedule: ER/HIO/RAAR, SHRINKWRAP, SUPPORT_AREA with */
                          /* SPR_AREA_ABS and GET_ERROR, scope ALL (copied at create)      */
  uint32_t flags;         /* SPR_SERVER_* */
  int32_t max_inflight;   /* ticks enqueued ahead of the device (0: 2) */
  uint64_t max_queue;     /* waiting requests before submit returns SPR_E_BUSY (0: unbounded) */
  double sim_bytes_per_s; /* ctx NULL only: modelled device bandwidth of the simulated executor */
  double sim_launch_s;    /* ctx NULL only: modelled cost of one launch */
} spr_server_cfg;

typedef struct spr_shot_desc {
  int32_t n;              /* detector size */
  const float* amp;       /* N*N float32 M = sqrt(I), centred layout unless SPR_LAYOUT_FFT */
  const uint8_t* mask;    /* N*N, 1 = measured */
  const uint8_t* supp0;   /* N*N (broadcast) or P*N*N (supp_per_member) initial supports */
  int32_t supp_per_member;
  uint32_t flags;         /* SPR_LAYOUT_FFT, SPR_AMP_FP16; SPR_INIT_RANDOM_PHASE (else rho0 is the start) */
  const float* rho0;      /* P*N*N complex start, or NULL with SPR_INIT_RANDOM_PHASE */
  uint64_t seed;          /* keys the random-phase start */
  double arrival;         /* < 0: stamped at submit; else the arrival time on the server clock */
                          /* (the simulated executor admits no request before its arrival)  */
  double bound_eta;       /* > 0: upper bounds on unknown amplitudes as spr_shot_set_bounds */
  double bound_max_unknown;
  const uint8_t* saturated;   /* NULL, or N*N saturation mask (host, layout of amp): the */
  double bound_max_saturated; /* saturation rules of spr_shot_set_bounds_sat           */
} spr_shot_desc;

typedef struct spr_result {
  float* rho;             /* caller buffer or NULL: members * N*N complex */
  uint8_t* supp;          /* caller buffer or NULL: members * N*N */
  double* err;            /* caller buffer or NULL: P fitness values (Eq. error_calc) */
  int32_t n, P;
  int32_t members;        /* 1 (best member) or P (SPR_SERVER_ALL_MEMBERS) */
  int32_t best;           /* member with the lowest error, ties to the lower index */
  double t_arrival, t_admit, t_finish; /* seconds on the server clock */
  spr_status status;      /* SPR_OK, or SPR_E_NUMERIC when a fitness value was not finite */
  int32_t pad;
} spr_result;

typedef struct spr_server_stats {
  double now;             /* server clock, seconds since create */
  int64_t queued, active, finishing, done;
  int64_t admitted, completed, ticks, launches;
  int64_t max_active;     /* most shots resident at once */
  uint64_t bytes_capacity, bytes_in_use, bytes_peak; /* shot memory of the budget */
} spr_server_stats;

/* ctx NULL selects the simulated executor: no device work, time advances by   */
/* the modelled cost of each tick (for testing the scheduling logic; results  */
/* carry no data).  Requires SPR_SERVER_MANUAL.  SPR_E_INVALID_ARG when the    */
/* budget cannot hold the work buffers.                                        */
spr_status spr_server_create(spr_ctx* ctx, const spr_server_cfg* cfg, spr_server** out);
/* Copies the request and returns at once with its ticket.  SPR_E_ADMISSION    */
/* when the shot could never fit the budget, SPR_E_BUSY when the queue is      */
/* full, SPR_E_UNSUPPORTED_SIZE, SPR_E_NUMERIC / SPR_E_INVALID_ARG for bad data. */
spr_status spr_server_submit(spr_server* sv, const spr_shot_desc* shot, uint64_t* ticket);
/* SPR_E_NOT_READY until the shot is done; then fills *res (copying into its   */
/* non-NULL buffers) and forgets the ticket.  Unknown ticket: SPR_E_INVALID_ARG. */
spr_status spr_server_poll(spr_server* sv, uint64_t ticket, spr_result* res);
/* SPR_SERVER_MANUAL: one round of the engine (collect finished shots, admit,  */
/* plan and enqueue one tick).  *pending = requests not yet done.              */
spr_status spr_server_step(spr_server* sv, int64_t* pending);
/* Wait until every submitted request is done (driving the engine in manual    */
/* mode); SPR_E_NOT_READY after timeout_s seconds (< 0: no limit).             */
spr_status spr_server_drain(spr_server* sv, double timeout_s);
/* Counters and memory figures of the server so far (see spr_server_stats). */
spr_status spr_server_stats_get(spr_server* sv, spr_server_stats* st);
/* Message of the last failed call on this server (owned by the server).      */
const char* spr_server_last_error(const spr_server* sv);
/* Stops the engine, waits for the device and frees everything (pending       */
/* results included).                                                          */
spr_status spr_server_destroy(spr_server* sv);

#ifdef __cplusplus
}
#endif

#endif /* SPR_H */
