// Captured schedules (include/spr.h, "Graphs"): the launches of a schedule on
// one population, or on a batch of populations, recorded once into a HIP
// graph and replayed with a single launch call.
#include <hip/hip_runtime.h>

#include "common.hpp"

using namespace spr;

#include "internal.hpp"

struct spr_graph {
  spr_ctx* ctx = nullptr;
  std::vector<spr_pop*> pops;
  std::map<int, Workspace> ws;  // batch graphs: their own work buffers and descriptor tables
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void release(spr_graph* g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  for (auto& kv : g->ws) workspace_free(kv.second);
  g->exec = nullptr;
  g->graph = nullptr;
}

// Record `enqueue` on a private stream into g's graph and instantiate it.
template <class Fn>
void capture(spr_graph* g, Fn&& enqueue) {
  hipStream_t cs = nullptr;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  bool capturing = false;
  try {
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    capturing = true;
    enqueue(cs);
    capturing = false;
    HIPCHK(hipStreamEndCapture(cs, &g->graph));
    HIPCHK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
  } catch (...) {
    if (capturing) {
      hipGraph_t junk = nullptr;
      (void)hipStreamEndCapture(cs, &junk);
      if (junk) (void)hipGraphDestroy(junk);
      (void)hipGetLastError();
    }
    (void)hipStreamDestroy(cs);
    throw;
  }
  HIPCHK(hipStreamDestroy(cs));
}

void check_capturable(const spr_sched* sch) {
  for (const auto& o : sch->ops) validate_op(o);
}

}  // namespace

extern "C" {

spr_status spr_graph_create(spr_pop* pop, const spr_sched* sched, spr_graph** out) {
  if (!pop || !sched || !out || !live_has(pop)) return SPR_E_INVALID_ARG;
  *out = nullptr;
  spr_ctx* ctx = pop->ctx;
  return guarded(ctx, [&] {
    use_device(ctx);
    check_capturable(sched);
    sync_pop(pop);
    prepare_buffers(pop, sched);
    spr_graph* g = new spr_graph();
    g->ctx = ctx;
    g->pops.push_back(pop);
    const uint32_t timing = pop->timing;
    pop->timing = 0;  // no timing events inside a graph
    try {
      capture(g, [&](hipStream_t cs) { run_schedule(pop, sched, cs); });
    } catch (...) {
      pop->timing = timing;
      release(g);
      delete g;
      throw;
    }
    pop->timing = timing;
    pop->graphs++;
    live_add(g);
    ctx->graphs.insert(g);
    *out = g;
  });
}

spr_status spr_graph_create_batch(spr_ctx* ctx, spr_pop* const* pops, const spr_sched* const* scheds, int32_t n,
                                  spr_graph** out) {
  if (!ctx || !out || n < 1 || !pops || !scheds || !live_has(ctx)) return SPR_E_INVALID_ARG;
  *out = nullptr;
  return guarded(ctx, [&] {
    use_device(ctx);
    spr_graph* g = new spr_graph();
    g->ctx = ctx;
    try {
      std::vector<BatchGroup> groups =
          plan_batch(ctx, pops, scheds, n, [&](int sz, size_t members, const SizeKernels* K) -> Workspace& {
            Workspace& w = g->ws[sz];
            workspace_alloc(w, sz, members, K);
            return w;
          });
      for (auto& bg : groups)
        for (const auto& o : bg.sched->ops)
          if (o.kind != SPR_OP_ER && o.kind != SPR_OP_HIO && o.kind != SPR_OP_RAAR && o.kind != SPR_OP_SHRINKWRAP &&
              o.kind != SPR_OP_SUPPORT_AREA && o.kind != SPR_OP_GET_ERROR)
            fail(SPR_E_INVALID_ARG, "batched runs take ER/HIO/RAAR, SHRINKWRAP, SUPPORT_AREA and GET_ERROR only");
      capture(g, [&](hipStream_t cs) { run_groups(ctx, groups, cs); });
    } catch (...) {
      release(g);
      delete g;
      throw;
    }
    for (int i = 0; i < n; ++i) {
      g->pops.push_back(pops[i]);
      pops[i]->graphs++;
    }
    live_add(g);
    ctx->graphs.insert(g);
    *out = g;
  });
}

spr_status spr_graph_launch(spr_graph* g, void* hip_stream) {
  if (!g || !live_has(g)) return SPR_E_INVALID_ARG;
  spr_ctx* ctx = g->ctx;
  return guarded(ctx, [&] {
    use_device(ctx);
    hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    for (spr_pop* p : g->pops)
      if (p->last && p->last != s) HIPCHK(hipStreamWaitEvent(s, p->done, 0));
    HIPCHK(hipGraphLaunch(g->exec, s));
    for (spr_pop* p : g->pops) {
      p->last = s;
      HIPCHK(hipEventRecord(p->done, s));
    }
  });
}

spr_status spr_graph_destroy(spr_graph* g) {
  if (!g || !live_remove(g)) return SPR_E_INVALID_ARG;
  (void)hipSetDevice(g->ctx->device);
  for (spr_pop* p : g->pops) {
    if (p->done) (void)hipEventSynchronize(p->done);
    p->graphs--;
  }
  g->ctx->graphs.erase(g);
  release(g);
  delete g;
  return SPR_OK;
}

}  // extern "C"
