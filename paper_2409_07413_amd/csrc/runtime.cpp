// Host runtime and C ABI (include/spr.h): contexts, shots, populations,
// schedules and the enqueueing of the hot-path kernels on a HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
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

namespace spr {

// sizes with one compiled plan (V1) and with a tunable alternative (V2)
#define SPR_SIZES(V1, V2)                                                                  \
  V1(8) V1(12) V1(16) V1(24) V1(32) V1(48) V1(64) V1(96) V2(128) V1(192) V2(256) V2(384) \
      V2(512) V2(768) V2(1024)
#define SPR_DECL1(n) const SizeKernels* size_kernels_##n##_0();
#define SPR_DECL2(n) SPR_DECL1(n) const SizeKernels* size_kernels_##n##_1();
SPR_SIZES(SPR_DECL1, SPR_DECL2)
#undef SPR_DECL1
#undef SPR_DECL2

const SizeKernels* size_kernels(int n, int v) {
  switch (n) {
#define SPR_CASE1(n) \
  case n:            \
    return v == 0 ? size_kernels_##n##_0() : nullptr;
#define SPR_CASE2(n) \
  case n:            \
    return v == 0 ? size_kernels_##n##_0() : (v == 1 ? size_kernels_##n##_1() : nullptr);
    SPR_SIZES(SPR_CASE1, SPR_CASE2)
#undef SPR_CASE1
#undef SPR_CASE2
    default:
      return nullptr;
  }
}

int size_variants(int n) {
  int v = 0;
  while (size_kernels(n, v)) ++v;
  return v;
}

bool has_resident(int n) {
  for (int v = 0; v < size_variants(n); ++v)
    if (size_kernels(n, v)->seq_res) return true;
  return false;
}

}  // namespace spr

using namespace spr;

#include "internal.hpp"

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int32_t spr_supported_size(int32_t n) { return size_kernels(n) ? 1 : 0; }

spr_status spr_ctx_create(int32_t hip_device, spr_ctx** out) {
  if (!out) return SPR_E_INVALID_ARG;
  *out = nullptr;
  spr_ctx* ctx = new (std::nothrow) spr_ctx();
  if (!ctx) return SPR_E_OOM;
  spr_status st = guarded(ctx, [&] {
    int count = 0;
    HIPCHK(hipGetDeviceCount(&count));
    if (hip_device < 0 || hip_device >= count) fail(SPR_E_INVALID_ARG, "no such device");
    ctx->device = hip_device;
    use_device(ctx);
    std::string why;
    if (noalloc_setup(hip_device, &why) != SPR_OK) fail(SPR_E_HIP, why);
    HIPCHK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
  });
  if (st != SPR_OK) {
    delete ctx;
    return st;
  }
  live_add(ctx);
  *out = ctx;
  return SPR_OK;
}

void spr_ctx_destroy(spr_ctx* ctx) {
  if (!ctx || !live_has(ctx)) return;
  // servers, populations, then shots still alive on this context
  std::vector<spr_server*> servers(ctx->servers.begin(), ctx->servers.end());
  for (spr_server* sv : servers) spr_server_destroy(sv);
  std::vector<spr_graph*> graphs(ctx->graphs.begin(), ctx->graphs.end());
  for (spr_graph* g : graphs) spr_graph_destroy(g);
  std::vector<spr_pop*> pops;
  std::vector<spr_shot*> shots;
  for (spr_pop* p : ctx->pops) pops.push_back(p);
  for (spr_shot* sh : ctx->shots) shots.push_back(sh);
  for (spr_pop* p : pops) spr_pop_destroy(p);
  for (spr_shot* sh : shots) spr_shot_destroy(sh);
  live_remove(ctx);
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (hipStream_t t : ctx->side) (void)hipStreamSynchronize(t);
  for (auto& kv : ctx->tw) (void)hipFree(kv.second);
  for (auto& kv : ctx->ws) workspace_free(kv.second);
  for (hipStream_t t : ctx->side) (void)hipStreamDestroy(t);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

const char* spr_ctx_last_error(const spr_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

spr_status spr_shot_create(spr_ctx* ctx, int32_t n, const float* amp, const uint8_t* mask, uint32_t flags,
                           spr_shot** out) {
  if (!ctx || !out || !amp || !mask) return SPR_E_INVALID_ARG;
  if (!live_has(ctx)) return SPR_E_INVALID_ARG;
  *out = nullptr;
  return guarded(ctx, [&] {
    const SizeKernels* K = ctx_kernels(ctx, n);
    if (!K) fail(SPR_E_UNSUPPORTED_SIZE, "unsupported detector size " + std::to_string(n));
    use_device(ctx);
    const size_t nn = (size_t)n * n;
    const bool dev = flags & SPR_DEVICE_PTRS;
    std::vector<uint8_t> ab, mb;
    to_host(ab, amp, nn * sizeof(float), dev);
    to_host(mb, mask, nn, dev);
    std::vector<float> enc(nn);
    double den = encode_shot(n, reinterpret_cast<const float*>(ab.data()), mb.data(), flags, enc.data());
    std::vector<__half> h16;
    float scale16 = 1.f;
    if (flags & SPR_AMP_FP16) {
      scale16 = fp16_encode(enc.data(), nn, h16, den);
      if (!(den > 0.0)) fail(SPR_E_INVALID_ARG, "sum of measured M^2 must be positive");
    }
    spr_shot* sh = new spr_shot();
    sh->ctx = ctx;
    sh->n = n;
    sh->K = K;
    sh->den = den;
    try {
      if (flags & SPR_AMP_FP16) {
        sh->amp_scale = scale16;
        sh->amp16 = dalloc<__half>(nn);
        HIPCHK(hipMemcpy(sh->amp16, h16.data(), nn * sizeof(__half), hipMemcpyHostToDevice));
      } else {
        sh->amp = dalloc<float>(nn);
        HIPCHK(hipMemcpy(sh->amp, enc.data(), nn * sizeof(float), hipMemcpyHostToDevice));
      }
      (void)twiddles(ctx, n);
    } catch (...) {
      dfree(sh->amp);
      dfree(sh->amp16);
      delete sh;
      throw;
    }
    live_add(sh);
    ctx->shots.insert(sh);
    *out = sh;
  });
}

spr_status spr_shot_destroy(spr_shot* shot) {
  if (!shot || !live_has(shot)) return SPR_E_INVALID_ARG;
  if (shot->live > 0) {
    shot->ctx->err = "shot still has live populations";
    return SPR_E_BUSY;
  }
  live_remove(shot);
  shot->ctx->shots.erase(shot);
  (void)hipSetDevice(shot->ctx->device);
  dfree(shot->amp);
  dfree(shot->amp16);
  delete shot;
  return SPR_OK;
}

spr_status spr_pop_create(spr_shot* shot, int32_t P, const float* rho0, const uint8_t* supp0,
                          int32_t supp_per_member, uint32_t flags, uint64_t seed, int32_t gen_offset,
                          spr_pop** out) {
  const bool init_phase = (flags & SPR_INIT_RANDOM_PHASE) != 0;
  if (!shot || !out || (!rho0 && !init_phase) || !supp0) return SPR_E_INVALID_ARG;
  if (!live_has(shot)) return SPR_E_INVALID_ARG;
  *out = nullptr;
  spr_ctx* ctx = shot->ctx;
  return guarded(ctx, [&] {
    if (P < 1) fail(SPR_E_INVALID_ARG, "P must be >= 1");
    if (gen_offset < 0) fail(SPR_E_INVALID_ARG, "negative generation offset");
    use_device(ctx);
    spr_pop* pop = new spr_pop();
    pop->shot = shot;
    pop->ctx = ctx;
    pop->K = shot->K;
    pop->n = shot->n;
    pop->P = P;
    pop->memetic = (flags & SPR_POP_MEMETIC) != 0;
    pop->nslots = pop->memetic ? 2 * P : P;
    const size_t nn = (size_t)pop->n * pop->n;
    pop->W = (int)((nn + 31) / 32);
    pop->seed = seed;
    pop->gen_offset = gen_offset;
    try {
      const size_t ns = pop->nslots;
      pop->X = dalloc<float2>(ns * nn);
      pop->T = dalloc<float2>(ns * nn);
      pop->Y = dalloc<float2>(ns * nn);
      pop->S = dalloc<uint32_t>(ns * pop->W);
      pop->E = dalloc<double>(ns);
      pop->table = dalloc<int>(ns);
      pop->err_partial = dalloc<double>(ns * (pop->n / pop->K->C));
      pop->block_max = dalloc<float>(ns * smooth_blocks_per_member(pop->n));
      pop->maxv = dalloc<float>(ns);
      pop->flags = dalloc<int>(1);
      if (has_resident(pop->n)) pop->res_bar = dalloc<unsigned>(2 * ns);
      pop->scal = dalloc<PopScalars>(1);
      pop->stats_part = dalloc<int>(2 * stats_workgroups(pop->W));
      pop->hist = dalloc<GenStatsDev>(pop->hist_cap);
      std::vector<int> tbl(ns);
      for (size_t i = 0; i < ns; ++i) tbl[i] = (int)i;
      HIPCHK(hipMemcpy(pop->table, tbl.data(), ns * sizeof(int), hipMemcpyHostToDevice));
      pop->desc = dalloc<SlotDesc>(ns);
      std::vector<SlotDesc> dh(ns);
      for (size_t i = 0; i < ns; ++i) {
        dh[i].X = pop->X + i * nn;
        dh[i].S = pop->S + i * pop->W;
        dh[i].amp = shot->amp;
        dh[i].amp16 = shot->amp16;
        dh[i].E = pop->E + i;
        dh[i].den = shot->den;
        dh[i].flags = pop->flags;
        dh[i].amp_scale = shot->amp_scale;
        dh[i].pad = 0;
      }
      HIPCHK(hipMemcpy(pop->desc, dh.data(), ns * sizeof(SlotDesc), hipMemcpyHostToDevice));
      std::vector<double> e(ns, std::numeric_limits<double>::infinity());
      HIPCHK(hipMemcpy(pop->E, e.data(), ns * sizeof(double), hipMemcpyHostToDevice));
      // on the context stream, ahead of the start-up kernels below
      hipStream_t cs = ctx->stream;
      HIPCHK(hipMemsetAsync(pop->flags, 0, sizeof(int), cs));
      if (pop->res_bar) HIPCHK(hipMemsetAsync(pop->res_bar, 0, 2 * ns * sizeof(unsigned), cs));
      HIPCHK(hipMemsetAsync(pop->scal, 0, sizeof(PopScalars), cs));
      HIPCHK(hipMemsetAsync(pop->hist, 0, sizeof(GenStatsDev) * pop->hist_cap, cs));
      HIPCHK(hipMemsetAsync(pop->S, 0, ns * pop->W * sizeof(uint32_t), cs));
      HIPCHK(hipMemsetAsync(pop->X, 0, ns * nn * sizeof(float2), cs));
      HIPCHK(hipStreamSynchronize(cs));
      const bool dev = flags & SPR_DEVICE_PTRS;
      if (init_phase) random_phase_start(ctx, pop->K, pop->n, P, shot->amp, shot->amp16, shot->amp_scale, seed, pop->X,
                                         ctx->stream);
      else
        HIPCHK(hipMemcpy(pop->X, rho0, (size_t)P * nn * sizeof(float2),
                         dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
      const size_t sb = supp_per_member ? (size_t)P * nn : nn;
      uint8_t* st = stage(pop, sb);
      HIPCHK(hipMemcpy(st, supp0, sb, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
      PackArgs pa{pop->table, P, pop->n, pop->W, supp_per_member ? 0 : 1, st, pop->S};
      launch_ok(launch_pack(pa, ctx->stream), "pack");
      HIPCHK(hipStreamSynchronize(ctx->stream));
    } catch (...) {
      destroy_pop(pop);
      delete pop;
      throw;
    }
    HIPCHK(hipEventCreateWithFlags(&pop->done, hipEventDisableTiming));
    shot->live++;
    live_add(pop);
    ctx->pops.insert(pop);
    *out = pop;
  });
}

spr_status spr_pop_destroy(spr_pop* pop) {
  if (!pop || !live_has(pop)) return SPR_E_INVALID_ARG;
  if (pop->graphs > 0) {
    pop->ctx->err = "population still has captured graphs";
    return SPR_E_BUSY;
  }
  live_remove(pop);
  pop->ctx->pops.erase(pop);
  (void)hipSetDevice(pop->ctx->device);
  if (pop->done) (void)hipEventSynchronize(pop->done);
  (void)hipStreamSynchronize(pop->ctx->stream);
  destroy_pop(pop);
  pop->shot->live--;
  delete pop;
  return SPR_OK;
}

spr_status spr_pop_init_spheres(spr_pop* pop, const spr_sphere_params* prm) {
  if (!pop || !prm || !live_has(pop)) return SPR_E_INVALID_ARG;
  spr_ctx* ctx = pop->ctx;
  return guarded(ctx, [&] {
    if (!(prm->sigma_init > 0.0) || prm->n_init < 1 || prm->n_init > 4096 || !(prm->gamma > 0.0) ||
        !(prm->diam_min > 0.0) || prm->diam_max < prm->diam_min || prm->phase_max < prm->phase_min)
      fail(SPR_E_INVALID_ARG, "bad sphere parameters");
    use_device(ctx);
    sync_pop(pop);
    hipStream_t s = ctx->stream;
    const int n = pop->n, P = pop->P;
    const size_t nn = (size_t)n * n;
    const SizeKernels* K = pop->K;
    const float2* tw = twiddles(ctx, n);
    SphereArgs sa{P, n, prm->n_init, pop->seed, prm->sigma_init, prm->diam_min, prm->diam_max,
                  prm->phase_min, prm->phase_max, prm->gamma, pop->table, pop->X};
    launch_ok(launch_init_spheres(sa, s), "init_spheres");
    // unitary spectra of the parents into the row-transform buffers
    RowFftArgs r1{pop->table, nullptr, P, pop->X, pop->T, -1, 1.f, tw};
    launch_ok(K->row_fft(r1, s), "row_fft");
    ColFftArgs c1{nullptr, nullptr, P, pop->T, pop->T, -1, 1.f / (float)n, tw};
    launch_ok(K->col_fft(c1, s), "col_fft");
    const int blocks = (int)std::min<size_t>(64, (nn + 4095) / 4096);
    double* partial = dalloc<double>((size_t)P * blocks);
    float* fac = dalloc<float>(P);
    NormArgs na{P, n, blocks, pop->T, pop->shot->amp, pop->shot->amp16, pop->shot->den, partial, fac, pop->table,
                pop->X};
    hipError_t e = launch_norm(na, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dfree(partial);
    dfree(fac);
    launch_ok(e, "norm");
    if (prm->set_support) {
      std::vector<uint8_t> sq(nn, 0);
      const double half = 0.5 * prm->sigma_init;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
          if (std::fabs(i - 0.5 * n) <= half && std::fabs(j - 0.5 * n) <= half) sq[(size_t)i * n + j] = 1;
      uint8_t* st = stage(pop, nn);
      HIPCHK(hipMemcpy(st, sq.data(), nn, hipMemcpyHostToDevice));
      PackArgs pa{pop->table, P, n, pop->W, 1, st, pop->S};
      launch_ok(launch_pack(pa, s), "pack");
      HIPCHK(hipStreamSynchronize(s));
    }
  });
}

spr_status spr_pop_write(spr_pop* pop, const float* rho, const uint8_t* supp, const double* err,
                         uint32_t flags) {
  if (!pop) return SPR_E_INVALID_ARG;
  if (!live_has(pop)) return SPR_E_INVALID_ARG;
  spr_ctx* ctx = pop->ctx;
  return guarded(ctx, [&] {
    use_device(ctx);
    sync_pop(pop);
    const bool kids = flags & SPR_READ_CHILDREN;
    if (kids) need_memetic(pop, "writing children");
    const bool dev = flags & SPR_DEVICE_PTRS;
    const size_t nn = (size_t)pop->n * pop->n;
    std::vector<int> tbl = host_table(pop);
    const int base = kids ? pop->P : 0;
    if (rho) {
      for (int p = 0; p < pop->P; ++p)
        HIPCHK(hipMemcpy(pop->X + (size_t)tbl[base + p] * nn, rho + (size_t)p * nn * 2, nn * sizeof(float2),
                         dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
    }
    if (supp) {
      uint8_t* st = stage(pop, (size_t)pop->P * nn);
      HIPCHK(hipMemcpy(st, supp, (size_t)pop->P * nn, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
      PackArgs pa{pop->table + base, pop->P, pop->n, pop->W, 0, st, pop->S};
      launch_ok(launch_pack(pa, ctx->stream), "pack");
      HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    if (err) {
      std::vector<double> e(pop->nslots), in(pop->P);
      HIPCHK(hipMemcpy(e.data(), pop->E, sizeof(double) * pop->nslots, hipMemcpyDeviceToHost));
      if (dev) HIPCHK(hipMemcpy(in.data(), err, sizeof(double) * pop->P, hipMemcpyDeviceToHost));
      else std::memcpy(in.data(), err, sizeof(double) * pop->P);
      for (int p = 0; p < pop->P; ++p) e[tbl[base + p]] = in[p];
      HIPCHK(hipMemcpy(pop->E, e.data(), sizeof(double) * pop->nslots, hipMemcpyHostToDevice));
    }
  });
}

spr_status spr_sched_create(spr_ctx* ctx, const spr_op* ops, int32_t nops, spr_sched** out) {
  if (!out || (nops > 0 && !ops) || nops < 0) return SPR_E_INVALID_ARG;
  *out = nullptr;
  return guarded(ctx, [&] {
    spr_sched* s = new spr_sched();
    s->ops.assign(ops, ops + nops);
    try {
      for (const auto& o : s->ops) validate_op(o);
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
  });
}

spr_status spr_sched_plain(spr_ctx* ctx, const spr_plain_params* prm, spr_sched** out) {
  if (!prm || !out) return SPR_E_INVALID_ARG;
  *out = nullptr;
  return guarded(ctx, [&] {
    if (prm->G < 1 || prm->j < 0 || prm->j_er < 0 || prm->j_end < 0) fail(SPR_E_INVALID_ARG, "bad plain schedule counts");
    if (prm->alg != SPR_ALG_HIO && prm->alg != SPR_ALG_RAAR) fail(SPR_E_INVALID_ARG, "alg must be HIO or RAAR");
    spr_sched* s = new spr_sched();
    for (int g = 1; g <= prm->G; ++g) {
      int jg, jer;
      double sg, tg;
      sched_at(g, prm->G, prm->j, prm->j_er, prm->j_end, prm->sigma, prm->sigma_end, prm->tau, prm->tau_end,
               jg, jer, sg, tg);
      push_seq(s->ops, prm->alg, jg, jer, prm->beta, prm->chi);
      spr_op sw = make_op(SPR_OP_SHRINKWRAP);
      sw.sigma = sg;
      sw.tau = tg;
      s->ops.push_back(sw);
    }
    s->ops.push_back(make_op(SPR_OP_GET_ERROR));
    try {
      for (const auto& o : s->ops) validate_op(o);
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
  });
}

spr_status spr_sched_mpr(spr_ctx* ctx, const spr_mpr_params* prm, spr_sched** out) {
  if (!prm || !out) return SPR_E_INVALID_ARG;
  *out = nullptr;
  return guarded(ctx, [&] {
    if (prm->G < 1 || prm->R < 2 || prm->j < 0 || prm->j_er < 0 || prm->j_end < 0 || prm->j_eval < 0)
      fail(SPR_E_INVALID_ARG, "bad MPR schedule counts");
    if (prm->alg != SPR_ALG_HIO && prm->alg != SPR_ALG_RAAR) fail(SPR_E_INVALID_ARG, "alg must be HIO or RAAR");
    const int g0 = prm->gen_first > 0 ? prm->gen_first : 1;
    const int g1 = prm->gen_count > 0 ? g0 + prm->gen_count - 1 : prm->G;
    spr_sched* s = new spr_sched();
    auto& ops = s->ops;
    if (prm->init_error) {
      spr_op e = make_op(SPR_OP_GET_ERROR);
      e.scope = SPR_SCOPE_PARENTS;
      ops.push_back(e);
    }
    if (!(prm->c_a >= 0.0 && prm->c_a <= 1.0)) fail(SPR_E_INVALID_ARG, "c_a outside [0, 1]");
    for (int g = g0; g <= g1; ++g) {
      if (prm->c_a > 0.0) {
        spr_op av = make_op(SPR_OP_AVERAGE);
        av.scope = SPR_SCOPE_PARENTS;
        ops.push_back(av);
      }
      spr_op x = make_op(SPR_OP_CROSSOVER);
      x.gen = g;
      x.c_p = prm->c_p;
      x.c_w = prm->c_w;
      x.c_a = prm->c_a;
      x.t_min = prm->t_min;
      x.t_max = prm->t_max;
      ops.push_back(x);
      spr_op st = make_op(SPR_OP_STATS);
      st.gen = g;
      st.gens = prm->G;
      ops.push_back(st);
      int jg, jer;
      double sg, tg;
      sched_at(g, prm->G, prm->j, prm->j_er, prm->j_end, prm->sigma, prm->sigma_end, prm->tau, prm->tau_end,
               jg, jer, sg, tg);
      spr_op sw = make_op(SPR_OP_SHRINKWRAP);
      sw.sigma = sg;
      sw.tau = tg;
      for (int r = 0; r < prm->R - 2; ++r) {
        push_seq(ops, prm->alg, jg, jer, prm->beta, prm->chi);
        ops.push_back(sw);
      }
      push_seq(ops, prm->alg, jg, jer, prm->beta, prm->chi);
      spr_op ab = make_op(SPR_OP_SUPPORT_AREA);
      ab.sigma = sg;
      ab.which = SPR_AREA_BEST;
      ops.push_back(ab);
      push_seq(ops, prm->alg, jg, jer, prm->beta, prm->chi);
      spr_op ae = ab;
      ae.which = SPR_AREA_EVAL;
      ops.push_back(ae);
      push_seq(ops, prm->alg, 0, prm->j_eval, prm->beta, prm->chi);
      ops.push_back(make_op(SPR_OP_GET_ERROR));
      ops.push_back(sw);
      spr_op se = make_op(SPR_OP_SELECT);
      se.gen = g;
      ops.push_back(se);
      if (g == prm->G || prm->monitor) {
        spr_op av = make_op(SPR_OP_AVERAGE);
        av.scope = SPR_SCOPE_PARENTS;
        ops.push_back(av);
      }
      if (prm->monitor) {
        spr_op mo = make_op(SPR_OP_MONITOR);
        mo.gen = g;
        ops.push_back(mo);
      }
    }
    for (auto& o : ops)
      if (o.kind == SPR_OP_ER || o.kind == SPR_OP_HIO || o.kind == SPR_OP_RAAR) o.chi = prm->chi;
    try {
      for (const auto& o : ops) validate_op(o);
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
  });
}

spr_status spr_sched_destroy(spr_sched* sched) {
  if (!sched) return SPR_E_INVALID_ARG;
  delete sched;
  return SPR_OK;
}

spr_status spr_sched_ops(const spr_sched* sched, spr_op* ops, int32_t max_ops, int32_t* n_ops) {
  if (!sched || !n_ops) return SPR_E_INVALID_ARG;
  *n_ops = (int32_t)sched->ops.size();
  if (ops) {
    const int32_t k = std::min<int32_t>(max_ops, *n_ops);
    for (int32_t i = 0; i < k; ++i) ops[i] = sched->ops[i];
  }
  return SPR_OK;
}

spr_status spr_run(spr_pop* pop, const spr_sched* sched, void* hip_stream) {
  if (!pop || !sched) return SPR_E_INVALID_ARG;
  if (!live_has(pop)) return SPR_E_INVALID_ARG;
  spr_ctx* ctx = pop->ctx;
  return guarded(ctx, [&] {
    use_device(ctx);
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    // order after work previously enqueued on another stream
    if (pop->last && pop->last != s) HIPCHK(hipStreamWaitEvent(s, pop->done, 0));
    pop->last = s;
    try {
      run_schedule(pop, sched, s);
    } catch (...) {
      (void)hipEventRecord(pop->done, s);
      throw;
    }
    HIPCHK(hipEventRecord(pop->done, s));
  });
}

spr_status spr_run_batch(spr_ctx* ctx, spr_pop* const* pops, const spr_sched* const* scheds, int32_t n,
                         void* hip_stream) {
  if (!ctx || (n > 0 && (!pops || !scheds)) || n < 0) return SPR_E_INVALID_ARG;
  return guarded(ctx, [&] {
    use_device(ctx);
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    // descriptors and slot lists of every size group go into the context's
    // work buffers; earlier batches on other streams must be done with them
    for (auto& kv : ctx->ws)
      if (kv.second.last && kv.second.last != s) HIPCHK(hipStreamSynchronize(kv.second.last));
    std::vector<BatchGroup> groups =
        plan_batch(ctx, pops, scheds, n, [&](int sz, size_t members, const SizeKernels* K) -> Workspace& {
          Workspace& w = workspace(ctx, sz, members, K);
          if (w.last) HIPCHK(hipStreamSynchronize(w.last));
          w.last = s;
          return w;
        });
    for (int i = 0; i < n; ++i) pops[i]->last = s;
    try {
      run_groups(ctx, groups, s);
    } catch (...) {
      for (int i = 0; i < n; ++i) (void)hipEventRecord(pops[i]->done, s);
      throw;
    }
    for (int i = 0; i < n; ++i) HIPCHK(hipEventRecord(pops[i]->done, s));
  });
}

// The population's status word after its work: a resident Sequence that ran
// out of its barrier wait (bit 1) left results that are not valid; the barrier
// words are reset so the population can run again, and the call fails.
int check_resident_status(spr_pop* pop) {
  int f = 0;
  HIPCHK(hipMemcpy(&f, pop->flags, sizeof(int), hipMemcpyDeviceToHost));
  if (f & 2) {
    HIPCHK(hipMemset(pop->res_bar, 0, 2 * (size_t)pop->nslots * sizeof(unsigned)));
    const int keep = f & ~2;
    HIPCHK(hipMemcpy(pop->flags, &keep, sizeof(int), hipMemcpyHostToDevice));
    fail(SPR_E_HIP, "a resident Sequence's barrier wait timed out");
  }
  return f;
}

spr_status spr_sync(spr_pop* pop) {
  if (!pop) return SPR_E_INVALID_ARG;
  if (!live_has(pop)) return SPR_E_INVALID_ARG;
  spr_ctx* ctx = pop->ctx;
  return guarded(ctx, [&] {
    use_device(ctx);
    sync_pop(pop);
    const int f = check_resident_status(pop);
    if (f & 1) fail(SPR_E_NUMERIC, "a fitness value is not finite");
  });
}

spr_status spr_read(spr_pop* pop, float* rho, uint8_t* supp, double* err, uint32_t flags) {
  if (!pop) return SPR_E_INVALID_ARG;
  if (!live_has(pop)) return SPR_E_INVALID_ARG;
  spr_ctx* ctx = pop->ctx;
  return guarded(ctx, [&] {
    use_device(ctx);
    sync_pop(pop);
    if (pop->res_bar) check_resident_status(pop);
    const bool kids = flags & SPR_READ_CHILDREN;
    if (kids) need_memetic(pop, "reading children");
    const bool dev = flags & SPR_DEVICE_PTRS;
    const size_t nn = (size_t)pop->n * pop->n;
    std::vector<int> tbl = host_table(pop);
    const int base = kids ? pop->P : 0;
    if (rho) {
      for (int p = 0; p < pop->P; ++p)
        HIPCHK(hipMemcpy(rho + (size_t)p * nn * 2, pop->X + (size_t)tbl[base + p] * nn, nn * sizeof(float2),
                         dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    }
    if (supp) {
      uint8_t* st = stage(pop, (size_t)pop->P * nn);
      PackArgs pa{pop->table + base, pop->P, pop->n, pop->W, 0, st, pop->S};
      launch_ok(launch_unpack(pa, ctx->stream), "unpack");
      HIPCHK(hipStreamSynchronize(ctx->stream));
      HIPCHK(hipMemcpy(supp, st, (size_t)pop->P * nn, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    }
    if (err) {
      std::vector<double> e(pop->nslots), o(pop->P);
      HIPCHK(hipMemcpy(e.data(), pop->E, sizeof(double) * pop->nslots, hipMemcpyDeviceToHost));
      for (int p = 0; p < pop->P; ++p) o[p] = e[tbl[base + p]];
      if (dev) HIPCHK(hipMemcpy(err, o.data(), sizeof(double) * pop->P, hipMemcpyHostToDevice));
      else std::memcpy(err, o.data(), sizeof(double) * pop->P);
    }
  });
}

spr_status spr_read_member(spr_pop* pop, int32_t member, float* rho, uint8_t* supp, uint32_t flags) {
  if (!pop || !live_has(pop)) return SPR_E_INVALID_ARG;
  spr_ctx* ctx = pop->ctx;
  return guarded(ctx, [&] {
    if (member < 0 || member >= pop->P) fail(SPR_E_INVALID_ARG, "member out of range");
    use_device(ctx);
    sync_pop(pop);
    const bool kids = flags & SPR_READ_CHILDREN;
    if (kids) need_memetic(pop, "reading children");
    const bool dev = flags & SPR_DEVICE_PTRS;
    const size_t nn = (size_t)pop->n * pop->n;
    const int slot_index = (kids ? pop->P : 0) + member;
    int slot = 0;
    HIPCHK(hipMemcpy(&slot, pop->table + slot_index, sizeof(int), hipMemcpyDeviceToHost));
    if (rho)
      HIPCHK(hipMemcpy(rho, pop->X + (size_t)slot * nn, nn * sizeof(float2),
                       dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    if (supp) {
      uint8_t* st = stage(pop, nn);
      PackArgs pa{pop->table + slot_index, 1, pop->n, pop->W, 0, st, pop->S};
      launch_ok(launch_unpack(pa, ctx->stream), "unpack");
      HIPCHK(hipStreamSynchronize(ctx->stream));
      HIPCHK(hipMemcpy(supp, st, nn, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    }
  });
}

spr_status spr_read_average(spr_pop* pop, float* rho, uint8_t* supp, double* err, uint32_t flags) {
  if (!pop || !live_has(pop)) return SPR_E_INVALID_ARG;
  spr_ctx* ctx = pop->ctx;
  return guarded(ctx, [&] {
    if (!pop->avg_done) fail(SPR_E_INVALID_ARG, "no AVERAGE has run on this population");
    use_device(ctx);
    sync_pop(pop);
    const bool dev = flags & SPR_DEVICE_PTRS;
    const size_t nn = (size_t)pop->n * pop->n;
    const auto kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (rho) HIPCHK(hipMemcpy(rho, pop->avgX, nn * sizeof(float2), kind));
    if (supp) {
      uint8_t* st = stage(pop, nn);
      PackArgs pa{pop->avg_slot, 1, pop->n, pop->W, 0, st, pop->avgS};
      launch_ok(launch_unpack(pa, ctx->stream), "unpack");
      HIPCHK(hipStreamSynchronize(ctx->stream));
      HIPCHK(hipMemcpy(supp, st, nn, kind));
    }
    if (err) HIPCHK(hipMemcpy(err, pop->avgE, sizeof(double), kind));
  });
}

spr_status spr_read_trace(spr_pop* pop, double* out, int32_t max_rows, int32_t* rows, int32_t* cols) {
  if (!pop || !rows || !cols || max_rows < 0 || (max_rows > 0 && !out) || !live_has(pop)) return SPR_E_INVALID_ARG;
  spr_ctx* ctx = pop->ctx;
  return guarded(ctx, [&] {
    use_device(ctx);
    sync_pop(pop);
    *rows = pop->trace_rows;
    *cols = pop->nslots;
    const int k = std::min(max_rows, pop->trace_rows);
    if (k > 0)
      HIPCHK(hipMemcpy(out, pop->trace, sizeof(double) * (size_t)k * pop->nslots, hipMemcpyDeviceToHost));
  });
}

spr_status spr_read_monitor(spr_pop* pop, spr_monitor* out, int32_t max_n, int32_t* n_out) {
  if (!pop || !n_out || (max_n > 0 && !out) || !live_has(pop)) return SPR_E_INVALID_ARG;
  spr_ctx* ctx = pop->ctx;
  return guarded(ctx, [&] {
    use_device(ctx);
    sync_pop(pop);
    *n_out = 0;
    if (!pop->mon) return;
    std::vector<MonitorDev> h(pop->mon_cap);
    HIPCHK(hipMemcpy(h.data(), pop->mon, sizeof(MonitorDev) * pop->mon_cap, hipMemcpyDeviceToHost));
    std::vector<MonitorDev> used;
    for (auto& r : h)
      if (r.gen > 0) used.push_back(r);
    std::sort(used.begin(), used.end(), [](const MonitorDev& a, const MonitorDev& b) { return a.gen < b.gen; });
    int32_t k = 0;
    for (auto& r : used) {
      if (k >= max_n) break;
      spr_monitor o;
      o.gen = r.gen;
      o.P = r.P;
      o.err_best = r.err_best;
      o.err_median = r.err_median;
      o.err_worst = r.err_worst;
      o.err_mean = r.err_mean;
      o.gamma_mean = r.gamma_mean;
      o.sum_mean = r.sum_mean;
      o.sum_rel_std = r.sum_rel_std;
      o.gamma_avg = r.gamma_avg;
      o.err_avg = r.err_avg;
      o.has_avg = r.has_avg;
      o.pad = 0;
      out[k++] = o;
    }
    *n_out = k;
  });
}

spr_status spr_read_stats(spr_pop* pop, spr_gen_stats* out, int32_t max_n, int32_t* n_out) {
  if (!pop || !n_out || (max_n > 0 && !out)) return SPR_E_INVALID_ARG;
  if (!live_has(pop)) return SPR_E_INVALID_ARG;
  spr_ctx* ctx = pop->ctx;
  return guarded(ctx, [&] {
    use_device(ctx);
    sync_pop(pop);
    std::vector<GenStatsDev> h(pop->hist_cap);
    HIPCHK(hipMemcpy(h.data(), pop->hist, sizeof(GenStatsDev) * pop->hist_cap, hipMemcpyDeviceToHost));
    std::vector<GenStatsDev> used;
    for (auto& r : h)
      if (r.gen > 0) used.push_back(r);
    std::sort(used.begin(), used.end(), [](const GenStatsDev& a, const GenStatsDev& b) { return a.gen < b.gen; });
    int32_t k = 0;
    for (auto& r : used) {
      if (k >= max_n) break;
      spr_gen_stats o;
      o.gen = r.gen;
      o.best = r.best;
      o.alpha_best = r.alpha_best;
      o.alpha_all = r.alpha_all;
      o.alpha_eval = r.alpha_eval;
      o.err_best = r.err_best;
      o.err_mean = r.err_mean;
      o.err_worst = r.err_worst;
      o.replaced = r.replaced;
      o.pad = 0;
      out[k++] = o;
    }
    *n_out = k;
  });
}

spr_status spr_read_xover(spr_pop* pop, spr_xover_info* out, int32_t max_n) {
  if (!pop || !out) return SPR_E_INVALID_ARG;
  if (!live_has(pop)) return SPR_E_INVALID_ARG;
  spr_ctx* ctx = pop->ctx;
  return guarded(ctx, [&] {
    use_device(ctx);
    if (!pop->abc) fail(SPR_E_INVALID_ARG, "no crossover has run on this population");
    sync_pop(pop);
    const int P = pop->P;
    std::vector<int> abc(3 * P), mp(5 * P);
    std::vector<AlignRec> al(3 * P);
    HIPCHK(hipMemcpy(abc.data(), pop->abc, sizeof(int) * 3 * P, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(mp.data(), pop->mapprm, sizeof(int) * 5 * P, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(al.data(), pop->align, sizeof(AlignRec) * 3 * P, hipMemcpyDeviceToHost));
    for (int p = 0; p < std::min(P, max_n); ++p) {
      spr_xover_info& o = out[p];
      o.a = abc[3 * p];
      o.b = abc[3 * p + 1];
      o.c = abc[3 * p + 2];
      o.tx = mp[5 * p];
      o.ty = mp[5 * p + 1];
      o.sx = mp[5 * p + 2];
      o.sy = mp[5 * p + 3];
      o.rot = mp[5 * p + 4];
      for (int k = 0; k < 3; ++k) {
        const AlignRec& r = al[3 * p + k];
        o.dr[k] = r.dr;
        o.dc[k] = r.dc;
        o.twin[k] = r.twin;
        o.phase[k][0] = r.pr;
        o.phase[k][1] = r.pi;
        o.peak[k][0] = r.peak1;
        o.peak[k][1] = r.peak2;
      }
    }
  });
}

spr_status spr_timing_enable(spr_pop* pop, int32_t enable) {
  if (!pop) return SPR_E_INVALID_ARG;
  if (!live_has(pop)) return SPR_E_INVALID_ARG;
  return guarded(pop->ctx, [&] {
    use_device(pop->ctx);
    sync_pop(pop);
    pop->timing = (uint32_t)enable & ((1u << SPR_KERNEL_COUNT) - 1);
    for (int k = 0; k < SPR_KERNEL_COUNT; ++k) {
      pop->kernel_ms[k] = 0.0;
      pop->kernel_launches[k] = 0;
      pop->timing_seen[k] = 0;
    }
  });
}

spr_status spr_timing_sample(spr_pop* pop, int32_t every) {
  if (!pop || every < 1 || !live_has(pop)) return SPR_E_INVALID_ARG;
  return guarded(pop->ctx, [&] {
    use_device(pop->ctx);
    sync_pop(pop);
    pop->timing_every = every;
    for (int k = 0; k < SPR_KERNEL_COUNT; ++k) {
      pop->kernel_ms[k] = 0.0;
      pop->kernel_launches[k] = 0;
      pop->timing_seen[k] = 0;
    }
  });
}

spr_status spr_ctx_set_cache_budget(spr_ctx* ctx, uint64_t bytes) {
  if (!ctx) return SPR_E_INVALID_ARG;
  ctx->cache_budget = (size_t)bytes;
  return SPR_OK;
}

spr_status spr_timing_read(spr_pop* pop, int32_t kernel, int64_t* launches, double* total_ms) {
  if (!pop || !launches || !total_ms || kernel < 0 || kernel >= SPR_KERNEL_COUNT) return SPR_E_INVALID_ARG;
  if (!live_has(pop)) return SPR_E_INVALID_ARG;
  return guarded(pop->ctx, [&] {
    use_device(pop->ctx);
    sync_pop(pop);
    *launches = pop->kernel_launches[kernel];
    *total_ms = pop->kernel_ms[kernel];
  });
}

spr_status spr_fft2(spr_ctx* ctx, int32_t n, int32_t batch, const float* in, float* out, int32_t inverse,
                    void* hip_stream) {
  if (!ctx || !in || !out || batch < 0) return SPR_E_INVALID_ARG;
  return guarded(ctx, [&] {
    const SizeKernels* K = ctx_kernels(ctx, n);
    if (!K) fail(SPR_E_UNSUPPORTED_SIZE, "unsupported size " + std::to_string(n));
    if (batch == 0) return;
    use_device(ctx);
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    const float2* tw = twiddles(ctx, n);
    const int dir = inverse ? +1 : -1;
    RowFftArgs r{nullptr, nullptr, batch, reinterpret_cast<const float2*>(in), reinterpret_cast<float2*>(out),
                 dir, 1.f, tw};
    launch_ok(K->row_fft(r, s), "row_fft");
    ColFftArgs c{nullptr, nullptr, batch, reinterpret_cast<float2*>(out), reinterpret_cast<float2*>(out), dir,
                 1.f / (float)n, tw};
    launch_ok(K->col_fft(c, s), "col_fft");
  });
}

int32_t spr_size_variants(int32_t n) { return size_variants(n); }

spr_status spr_ctx_set_variant(spr_ctx* ctx, int32_t n, int32_t variant, int32_t chunk_members) {
  if (!ctx || !live_has(ctx)) return SPR_E_INVALID_ARG;
  return guarded(ctx, [&] {
    if (!size_kernels(n)) fail(SPR_E_UNSUPPORTED_SIZE, "unsupported size " + std::to_string(n));
    if (variant < 0 || variant >= size_variants(n))
      fail(SPR_E_INVALID_ARG, "size " + std::to_string(n) + " has " + std::to_string(size_variants(n)) +
                                  " kernel variants");
    if (chunk_members < 0) fail(SPR_E_INVALID_ARG, "negative chunk");
    ctx->variant[n] = variant;
    ctx->chunk_members[n] = chunk_members;
  });
}

spr_status spr_ctx_get_tuning(spr_ctx* ctx, int32_t n, int32_t* variant, int32_t* chunk_members) {
  if (!ctx || !variant || !chunk_members || !live_has(ctx)) return SPR_E_INVALID_ARG;
  auto v = ctx->variant.find(n);
  auto c = ctx->chunk_members.find(n);
  *variant = v == ctx->variant.end() ? 0 : v->second;
  *chunk_members = c == ctx->chunk_members.end() ? 0 : c->second;
  return SPR_OK;
}

spr_status spr_ctx_autotune(spr_ctx* ctx, int32_t n, int32_t members, spr_tune_result* out) {
  if (!ctx || !out || members < 1 || !live_has(ctx)) return SPR_E_INVALID_ARG;
  return guarded(ctx, [&] {
    if (!size_kernels(n)) fail(SPR_E_UNSUPPORTED_SIZE, "unsupported size " + std::to_string(n));
    use_device(ctx);
    std::memset(out, 0, sizeof(*out));
    const size_t nn = (size_t)n * n;
    const int W = (int)((nn + 31) / 32);
    hipStream_t s = ctx->stream;
    // a synthetic shot (unit modulus, all measured) and a random-phase population
    std::vector<float> one(nn, 1.0f);
    std::vector<uint32_t> bits((size_t)W * members, 0xffffffffu);
    std::vector<int> ident(members);
    for (int m = 0; m < members; ++m) ident[m] = m;
    float* amp = nullptr;
    float2 *X = nullptr, *T = nullptr, *Y = nullptr;
    uint32_t* S = nullptr;
    double *E = nullptr, *errp = nullptr;
    float *bmax = nullptr, *maxv = nullptr;
    int *flags = nullptr, *slots = nullptr;
    unsigned* rbar = nullptr;
    SlotDesc* desc = nullptr;
    std::vector<hipEvent_t> ev;
    auto cleanup = [&] {
      (void)hipStreamSynchronize(s);
      for (void* q : {(void*)amp, (void*)X, (void*)T, (void*)Y, (void*)S, (void*)E, (void*)errp, (void*)bmax,
                      (void*)maxv, (void*)flags, (void*)slots, (void*)desc, (void*)rbar})
        if (q) (void)hipFree(q);
      for (auto e : ev) (void)hipEventDestroy(e);
    };
    try {
      const SizeKernels* K0 = size_kernels(n, 0);
      amp = dalloc<float>(nn);
      X = dalloc<float2>(nn * members);
      T = dalloc<float2>(nn * members);
      Y = dalloc<float2>(nn * members);
      S = dalloc<uint32_t>((size_t)W * members);
      E = dalloc<double>(members);
      errp = dalloc<double>((size_t)members * n);
      bmax = dalloc<float>((size_t)members * smooth_blocks_per_member(n));
      maxv = dalloc<float>(members);
      flags = dalloc<int>(1);
      slots = dalloc<int>(members);
      desc = dalloc<SlotDesc>(members);
      HIPCHK(hipMemset(flags, 0, sizeof(int)));
      if (has_resident(n)) {
        rbar = dalloc<unsigned>(2 * (size_t)members);
        HIPCHK(hipMemset(rbar, 0, 2 * (size_t)members * sizeof(unsigned)));
      }
      HIPCHK(hipMemcpy(amp, one.data(), nn * sizeof(float), hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(S, bits.data(), bits.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(slots, ident.data(), sizeof(int) * members, hipMemcpyHostToDevice));
      std::vector<SlotDesc> dh(members);
      for (int m = 0; m < members; ++m) {
        dh[m].X = X + (size_t)m * nn;
        dh[m].T = T + (size_t)m * nn;
        dh[m].S = S + (size_t)m * W;
        dh[m].amp = amp;
        dh[m].amp16 = nullptr;
        dh[m].E = E + m;
        dh[m].den = (double)nn;
        dh[m].flags = flags;
        dh[m].amp_scale = 1.f;
        dh[m].pad = 0;
      }
      HIPCHK(hipMemcpy(desc, dh.data(), sizeof(SlotDesc) * members, hipMemcpyHostToDevice));
      (void)twiddles(ctx, n);
      random_phase_start(ctx, K0, n, members, amp, nullptr, 1.f, 12345, X, s);
      for (int k = 0; k < 2; ++k) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        ev.push_back(e);
      }
      const std::vector<Iter> its(10, Iter{ALG_RAAR, 0.9f, 0.5});
      // chunks whose two work buffers fill the 256 MiB memory-side cache, three
      // quarters of it (the default budget) and half of it
      std::vector<int> chunks = {members};
      for (size_t mib : {(size_t)256, (size_t)192, (size_t)128}) {
        const int c = (int)std::max<size_t>(1, (mib << 20) / (2 * nn * sizeof(float2)));
        if (c < members && std::find(chunks.begin(), chunks.end(), c) == chunks.end()) chunks.push_back(c);
      }
      double best = -1;
      int nc = 0;
      for (int v = 0; v < size_variants(n); ++v) {
        for (int c : chunks) {
          Group g;
          g.ctx = ctx;
          g.K = size_kernels(n, v);
          g.n = n;
          g.W = W;
          g.slots = slots;
          g.nm = members;
          g.desc = desc;
          g.T = T;
          g.Y = Y;
          g.err_partial = errp;
          g.block_max = bmax;
          g.maxv = maxv;
          g.flags = flags;
          g.timing = nullptr;
          g.chunk = c;
          g.res_bar = rbar;
          run_iterations(g, its, s);  // warm-up
          HIPCHK(hipEventRecord(ev[0], s));
          for (int rep = 0; rep < 3; ++rep) run_iterations(g, its, s);
          HIPCHK(hipEventRecord(ev[1], s));
          HIPCHK(hipEventSynchronize(ev[1]));
          float ms = 0.f;
          HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
          double rate = (double)members * its.size() * 3 / (ms * 1e-3);
          if (rbar) {
            // a resident candidate whose barrier wait ran out did no valid work
            int f = 0;
            HIPCHK(hipMemcpy(&f, flags, sizeof(int), hipMemcpyDeviceToHost));
            if (f & 2) {
              rate = 0.0;
              HIPCHK(hipMemset(flags, 0, sizeof(int)));
              HIPCHK(hipMemset(rbar, 0, 2 * (size_t)members * sizeof(unsigned)));
            }
          }
          if (nc < SPR_TUNE_MAX) {
            out->cand_variant[nc] = v;
            out->cand_chunk[nc] = c;
            out->cand_rate[nc] = rate;
            ++nc;
          }
          if (rate > best) {
            best = rate;
            out->variant = v;
            out->chunk_members = c;
          }
        }
      }
      out->n = n;
      out->candidates = nc;
      out->member_iterations_per_s = best;
      ctx->variant[n] = out->variant;
      ctx->chunk_members[n] = out->chunk_members;
    } catch (...) {
      cleanup();
      throw;
    }
    cleanup();
  });
}

spr_status spr_shot_set_bounds_sat(spr_shot* shot, double eta, double max_unknown, const uint8_t* saturated,
                                   double max_saturated, uint32_t flags, int32_t* rings) {
  if (!shot || !live_has(shot)) return SPR_E_INVALID_ARG;
  spr_ctx* ctx = shot->ctx;
  return guarded(ctx, [&] {
    if (!(max_unknown >= 0.0 && max_unknown <= 1.0)) fail(SPR_E_INVALID_ARG, "max_unknown must lie in [0, 1]");
    if (saturated && !(max_saturated >= 0.0 && max_saturated <= 1.0))
      fail(SPR_E_INVALID_ARG, "max_saturated must lie in [0, 1]");
    use_device(ctx);
    HIPCHK(hipDeviceSynchronize());  // populations may be reading the modulus
    const int n = shot->n;
    const size_t nn = (size_t)n * n;
    std::vector<uint8_t> sat_in;
    if (saturated) to_host(sat_in, saturated, nn, flags & SPR_DEVICE_PTRS);
    std::vector<float> enc(nn);
    std::vector<__half> h;
    if (shot->amp16) {
      h.resize(nn);
      HIPCHK(hipMemcpy(h.data(), shot->amp16, nn * sizeof(__half), hipMemcpyDeviceToHost));
      for (size_t k = 0; k < nn; ++k) enc[k] = __half2float(h[k]);
    } else {
      HIPCHK(hipMemcpy(enc.data(), shot->amp, nn * sizeof(float), hipMemcpyDeviceToHost));
    }
    std::vector<uint8_t> sat;
    if (saturated) sat = saturation_fft(n, sat_in.data(), flags, enc.data());
    const uint8_t* sp = saturated ? sat.data() : nullptr;
    const double ms = saturated ? max_saturated : 1.0;
    int r = 0;
    if (shot->amp16) {
      r = apply_upper_bounds(n, enc.data(), shot->amp_scale, eta, max_unknown, kHalfTiny, sp, ms);
      for (size_t k = 0; k < nn; ++k)
        h[k] = __float2half(std::signbit(enc[k]) ? -std::min(-enc[k], 65504.0f) : enc[k]);
      HIPCHK(hipMemcpy(shot->amp16, h.data(), nn * sizeof(__half), hipMemcpyHostToDevice));
    } else {
      r = apply_upper_bounds(n, enc.data(), 1.0f, eta, max_unknown, std::numeric_limits<float>::min(), sp, ms);
      HIPCHK(hipMemcpy(shot->amp, enc.data(), nn * sizeof(float), hipMemcpyHostToDevice));
    }
    if (rings) *rings = r;
  });
}

spr_status spr_shot_set_bounds(spr_shot* shot, double eta, double max_unknown, int32_t* rings) {
  return spr_shot_set_bounds_sat(shot, eta, max_unknown, nullptr, 0.0, 0u, rings);
}

}  // extern "C"
