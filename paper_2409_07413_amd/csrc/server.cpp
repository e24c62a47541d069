// Serving engine: continuous batching of streamed shots (include/spr.h,
// "Serving").  The host scheduler (serve_sched.hpp) decides admissions and
// plans ticks; an executor carries the plans out, either on the device (HIP
// stream, one arena allocation, pinned staging) or in modelled time.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <functional>
#include <memory>
#include <thread>

#include "common.hpp"

using namespace spr;

#include "internal.hpp"
#include "serve_sched.hpp"

using namespace spr_serve;

namespace {

// ---------------------------------------------------------------------------
// Schedule -> per-shot program
// ---------------------------------------------------------------------------
Program compile_program(const spr_sched* sch) {
  Program pg;
  const auto& ops = sch->ops;
  size_t i = 0;
  int run = 0;
  while (i < ops.size()) {
    const spr_op& o = ops[i];
    validate_op(o);
    if (o.scope != SPR_SCOPE_ALL) fail(SPR_E_INVALID_ARG, "served schedules act on every member (scope ALL)");
    if (o.kind == SPR_OP_ER || o.kind == SPR_OP_HIO || o.kind == SPR_OP_RAAR) {
      Step st;
      st.kind = STEP_SEQ;
      st.it0 = (int)pg.its.size();
      while (i < ops.size() &&
             (ops[i].kind == SPR_OP_ER || ops[i].kind == SPR_OP_HIO || ops[i].kind == SPR_OP_RAAR)) {
        const spr_op& q = ops[i];
        if (q.scope != SPR_SCOPE_ALL) fail(SPR_E_INVALID_ARG, "served schedules act on every member (scope ALL)");
        if (q.which & SPR_ITER_TRACE)
          fail(SPR_E_INVALID_ARG, "iteration traces are recorded for single populations only");
        const int alg = q.kind == SPR_OP_ER ? ALG_ER : (q.kind == SPR_OP_HIO ? ALG_HIO : ALG_RAAR);
        for (int c = 0; c < q.count; ++c) pg.its.push_back({alg, (float)q.beta, q.chi});
        ++i;
      }
      st.nit = (int)pg.its.size() - st.it0;
      if (st.nit > 0) {
        pg.steps.push_back(st);
        pg.max_seq = std::max(pg.max_seq, st.nit);
        pg.member_its += st.nit;
        run = 0;
      }
      continue;
    }
    Step st;
    switch (o.kind) {
      case SPR_OP_SHRINKWRAP:
        st.kind = STEP_SW;
        st.sigma = o.sigma;
        st.tau = o.tau;
        break;
      case SPR_OP_SUPPORT_AREA:
        if (o.which != SPR_AREA_ABS) fail(SPR_E_INVALID_ARG, "served schedules take absolute support areas only");
        st.kind = STEP_AREA;
        st.sigma = o.sigma;
        st.alpha = o.alpha;
        break;
      case SPR_OP_GET_ERROR:
        st.kind = STEP_ERR;
        break;
      default:
        fail(SPR_E_INVALID_ARG, "served schedules take ER/HIO/RAAR, SHRINKWRAP, SUPPORT_AREA and GET_ERROR only");
    }
    pg.steps.push_back(st);
    pg.max_non_seq_run = std::max(pg.max_non_seq_run, ++run);
    ++i;
  }
  return pg;
}

// ---------------------------------------------------------------------------
// Requests' host data
// ---------------------------------------------------------------------------
struct Pinned {
  void* p = nullptr;
  size_t bytes = 0;
};

// Pinned host blocks for uploads and results, reused across requests.
class PinnedPool {
 public:
  ~PinnedPool() {
    for (auto& kv : free_) (void)hipHostFree(kv.second);
  }
  Pinned get(size_t bytes) {
    bytes = (bytes + (64 << 10) - 1) / (64 << 10) * (64 << 10);
    auto it = free_.lower_bound(bytes);
    if (it != free_.end() && it->first <= 2 * bytes) {
      Pinned b{it->second, it->first};
      free_.erase(it);
      return b;
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      fail(SPR_E_OOM, "pinned host allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return Pinned{p, bytes};
  }
  void put(Pinned& b) {
    if (b.p) free_.emplace(b.bytes, b.p);
    b = Pinned();
  }

 private:
  std::multimap<size_t, void*> free_;
};

struct ShotData {
  std::vector<float> enc;  // FFT order, sign bit = unknown
  std::vector<__half> enc16;  // SPR_AMP_FP16: FP16 storage of enc / amp_scale (enc then empty)
  float amp_scale = 1.f;
  double den = 0;
  std::vector<uint8_t> supp;
  int supp_per_member = 0;
  std::vector<float> rho0;  // empty: random-phase start
  uint64_t seed = 0;
  Pinned upload, result;
  hipEvent_t done = nullptr;
};

ShotData* data_of(Req* r) { return static_cast<ShotData*>(r->payload.get()); }

// Byte offsets of one shot's device data inside its arena range, in the
// order of shot_footprint().
struct ShotLayout {
  size_t amp, X, T, S, E, status, res;
  ShotLayout(int n, int P, size_t base) {
    auto A = [](size_t b) { return Arena::align_up(b); };
    const size_t nn = (size_t)n * n, W = (nn + 31) / 32;
    amp = base;
    X = amp + A(4 * nn);
    T = X + A(8 * nn * P);
    S = T + A(8 * nn * P);
    E = S + A(4 * W * P);
    status = E + A(8 * (size_t)P);
    res = status + A(16);
  }
};

size_t result_bytes(int n, int P, bool all) {
  const size_t nn = (size_t)n * n, W = (nn + 31) / 32;
  return all ? 32 + 8 * (size_t)P + 8 * nn * P + 4 * W * P : 32 + 8 * (size_t)P + 8 * nn + 4 * W;
}

// ---------------------------------------------------------------------------
// Executors
// ---------------------------------------------------------------------------
class Exec {
 public:
  virtual ~Exec() {}
  virtual double now() = 0;
  // back-pressure: wait (without the server lock) until a tick may be enqueued
  virtual void wait_slot() {}
  virtual void issue(TickPlan& tp) = 0;
  virtual bool finished(Req* r) = 0;
  virtual void fetch(Req* r, spr_result* res, int members) = 0;
  virtual void discard(Req* r) = 0;
  virtual bool simulated() const { return false; }
  int64_t launches = 0;
};

class SimExec : public Exec {
 public:
  SimExec(double bw, double launch_s, int P) : bw_(bw), launch_(launch_s), P_(P) {}
  double now() override { return clock_; }
  bool simulated() const override { return true; }
  void advance_to(double t) { clock_ = std::max(clock_, t); }
  void issue(TickPlan& tp) override {
    double cost = 0;
    auto add = [&](int nl, double bytes) {
      cost += nl * launch_ + bytes / bw_;
      launches += nl;
    };
    for (Req* r : tp.started) add(5, (double)r->n * r->n * (5.0 + 16.0 * P_));
    for (auto& round : tp.rounds)
      for (auto& L : round) {
        const double px = (double)L.n * L.n * P_ * (double)L.shots.size();
        switch (L.kind) {
          case STEP_SEQ:
            add(1 + 2 * L.nit, px * (16.0 + 40.0 * L.nit));
            break;
          case STEP_SW:
            add(3, px * 24.0);
            break;
          case STEP_AREA:
            add(4, px * 40.0);
            break;
          default:
            add(3, px * 24.0);
        }
      }
    for (Req* r : tp.ending) add(2, (double)r->n * r->n * 16.0);
    clock_ += cost;
    for (Req* r : tp.ending) r->sim_done = clock_;
  }
  bool finished(Req* r) override { return clock_ >= r->sim_done; }
  void fetch(Req* r, spr_result* res, int) override {
    // modelled execution carries no data: errors read as NaN
    res->best = 0;
    res->status = SPR_OK;
    if (res->err)
      for (int p = 0; p < r->P; ++p) res->err[p] = std::numeric_limits<double>::quiet_NaN();
  }
  void discard(Req*) override {}

 private:
  double clock_ = 0, bw_, launch_;
  int P_;
};

class HipExec : public Exec {
 public:
  HipExec(spr_ctx* ctx, const Program& pg, const spr_server_cfg& cfg)
      : ctx_(ctx), pg_(pg), all_(cfg.flags & SPR_SERVER_ALL_MEMBERS),
        R_(cfg.max_inflight > 0 ? cfg.max_inflight : 2), t0_(std::chrono::steady_clock::now()) {
    use_device(ctx);
    members_ = (size_t)cfg.max_shots * cfg.P;
    // twiddles of every size up front: no synchronous upload while serving
    for (int n = 8; n <= 1024; ++n)
      if (size_kernels(n)) (void)twiddles(ctx, n);
    max_tiles_ = 1;
    max_blocks_ = 1;
    for (int n = 8; n <= 1024; ++n)
      if (const SizeKernels* K = ctx_kernels(ctx, n)) {
        Ks_[n] = K;  // the context's kernel variant of each size, fixed for the server's life
        max_tiles_ = std::max(max_tiles_, n / K->C);
        max_blocks_ = std::max(max_blocks_, smooth_blocks_per_member(n));
      }
    // two work buffers filling three quarters of the cache budget, as the
    // member chunks of populations larger than it (>= one 1024^2 member)
    ws_bytes_ = std::max<size_t>(ctx->cache_budget / 8 * 3, (size_t)8 << 20);
    const size_t lists = members_ * (size_t)(pg.max_non_seq_run + 3);
    meta_cap_ = Arena::align_up(lists * (4 + 16) + members_ * (size_t)std::max(pg.max_seq, 1) * sizeof(IterParam) +
                                4096);
    // reserved part of the arena
    size_t off = 0;
    auto take = [&](size_t b) {
      const size_t o = off;
      off = Arena::align_up(off + std::max<size_t>(b, 1));
      return o;
    };
    o_table_ = take(members_ * sizeof(SlotDesc));
    o_ident_ = take(sizeof(int) * (size_t)std::max(cfg.P, 1));
    o_ring_ = take(meta_cap_ * R_);
    o_wsA_ = take(ws_bytes_);
    o_wsB_ = take(ws_bytes_);
    o_errp_ = take(members_ * max_tiles_ * sizeof(double));
    o_bmax_ = take(members_ * max_blocks_ * sizeof(float));
    o_maxv_ = take(members_ * sizeof(float));
    reserved_ = off;
    if (reserved_ >= cfg.hbm_budget)
      fail(SPR_E_INVALID_ARG, "the memory budget must exceed the " + std::to_string(reserved_ >> 20) +
                                  " MiB of work buffers");
    budget_ = cfg.hbm_budget;
    HIPCHK(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
    base_ = reinterpret_cast<char*>(dalloc<uint8_t>(budget_));
    std::vector<int> id(std::max(cfg.P, 1));
    for (size_t i = 0; i < id.size(); ++i) id[i] = (int)i;
    HIPCHK(hipMemcpy(base_ + o_ident_, id.data(), sizeof(int) * id.size(), hipMemcpyHostToDevice));
    ring_.resize(R_);
    for (int k = 0; k < R_; ++k) {
      Pinned b = pool_.get(meta_cap_);
      ring_[k].host = static_cast<char*>(b.p);
      ring_[k].pin = b;
      ring_[k].dev = base_ + o_ring_ + (size_t)k * meta_cap_;
      HIPCHK(hipEventCreateWithFlags(&ring_[k].ev, hipEventDisableTiming));
    }
  }
  ~HipExec() override {
    (void)hipSetDevice(ctx_->device);
    if (s_) (void)hipStreamSynchronize(s_);
    for (auto& e : ring_) {
      if (e.ev) (void)hipEventDestroy(e.ev);
      pool_.put(e.pin);
    }
    for (hipEvent_t e : events_) (void)hipEventDestroy(e);
    if (base_) (void)hipFree(base_);
    if (s_) (void)hipStreamDestroy(s_);
  }
  size_t reserved() const { return reserved_; }
  size_t budget() const { return budget_; }

  double now() override {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
  }

  void wait_slot() override {
    RingEntry& e = ring_[(last_tick_ + 1) % R_];
    if (e.used) HIPCHK(hipEventSynchronize(e.ev));
  }

  void issue(TickPlan& tp) override {
    use_device(ctx_);
    RingEntry& e = ring_[tp.id % R_];
    if (e.used) HIPCHK(hipEventSynchronize(e.ev));
    meta_used_ = 0;
    meta_host_ = e.host;
    meta_dev_ = e.dev;
    ops_.clear();
    for (Req* r : tp.started) plan_start(r);
    for (auto& round : tp.rounds)
      for (auto& L : round) plan_launch(L);
    for (Req* r : tp.ending) plan_end(r);
    if (meta_used_) HIPCHK(hipMemcpyAsync(e.dev, e.host, meta_used_, hipMemcpyHostToDevice, s_));
    for (auto& op : ops_) op();
    ops_.clear();
    HIPCHK(hipEventRecord(e.ev, s_));
    e.used = true;
    last_tick_ = tp.id;
  }

  bool finished(Req* r) override {
    ShotData* d = data_of(r);
    const hipError_t q = hipEventQuery(d->done);
    if (q == hipErrorNotReady) return false;
    if (q != hipSuccess) fail(SPR_E_HIP, std::string("serving stream: ") + hipGetErrorString(q));
    pool_.put(d->upload);
    recycle(d->done);
    d->done = nullptr;
    return true;
  }

  void fetch(Req* r, spr_result* res, int members) override {
    ShotData* d = data_of(r);
    const int n = r->n, P = r->P;
    const size_t nn = (size_t)n * n, W = (nn + 31) / 32;
    const char* b = static_cast<const char*>(d->result.p);
    int best = reinterpret_cast<const int*>(b)[0];
    const int status = reinterpret_cast<const int*>(b)[1];
    const double* E = reinterpret_cast<const double*>(b + 32);
    if (best < 0) {
      // every member was returned: the best one by the same rule as on the device
      best = 0;
      double bv = E[0];
      for (int p = 1; p < P; ++p)
        if (E[p] < bv || (bv != bv && E[p] == E[p])) {
          bv = E[p];
          best = p;
        }
    }
    const char* X = b + 32 + 8 * (size_t)P;
    const uint32_t* S = reinterpret_cast<const uint32_t*>(X + 8 * nn * members);
    res->best = best;
    res->status = (status & 1) ? SPR_E_NUMERIC : SPR_OK;
    if (res->err) std::memcpy(res->err, E, sizeof(double) * P);
    if (res->rho) std::memcpy(res->rho, X, 8 * nn * members);
    if (res->supp)
      for (int m = 0; m < members; ++m)
        for (size_t k = 0; k < nn; ++k) res->supp[m * nn + k] = (S[m * W + k / 32] >> (k % 32)) & 1u;
    pool_.put(d->result);
  }

  void discard(Req* r) override {
    ShotData* d = data_of(r);
    if (!d) return;
    if (d->done) {
      (void)hipEventSynchronize(d->done);
      recycle(d->done);
      d->done = nullptr;
    }
    pool_.put(d->upload);
    pool_.put(d->result);
  }

 private:
  struct RingEntry {
    char* host = nullptr;
    char* dev = nullptr;
    Pinned pin;
    hipEvent_t ev = nullptr;
    bool used = false;
  };

  template <class T_>
  T_* dev(size_t off) const {
    return reinterpret_cast<T_*>(base_ + off);
  }

  // Host staging of one tick's launch metadata; returns the device address.
  template <class T_>
  T_* meta(const T_* src, size_t count) {
    const size_t off = (meta_used_ + 15) / 16 * 16;
    const size_t bytes = sizeof(T_) * count;
    if (off + bytes > meta_cap_) fail(SPR_E_INVALID_ARG, "tick metadata exceeds its buffer");
    std::memcpy(meta_host_ + off, src, bytes);
    meta_used_ = off + bytes;
    return reinterpret_cast<T_*>(meta_dev_ + off);
  }

  hipEvent_t event() {
    if (!events_.empty()) {
      hipEvent_t e = events_.back();
      events_.pop_back();
      return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return e;
  }
  void recycle(hipEvent_t e) {
    if (e) events_.push_back(e);
  }

  void launch(hipError_t e, const char* what) {
    launch_ok(e, what);
    ++launches;
  }

  Group group(int n, const int* slots, int nm) {
    Group g;
    g.ctx = ctx_;
    g.K = Ks_.at(n);
    g.n = n;
    g.W = (int)(((size_t)n * n + 31) / 32);
    g.slots = slots;
    g.nm = nm;
    g.desc = dev<SlotDesc>(o_table_);
    g.T = dev<float2>(o_wsA_);
    g.Y = dev<float2>(o_wsB_);
    g.err_partial = dev<double>(o_errp_);
    g.block_max = dev<float>(o_bmax_);
    g.maxv = dev<float>(o_maxv_);
    g.timing = nullptr;
    g.chunk = 0;
    g.t_by_slot = 1;
    return g;
  }

  // Uploads of a newly admitted shot: descriptors, initial errors and status,
  // amplitudes, supports (packed), and the start densities.
  void plan_start(Req* r) {
    ShotData* d = data_of(r);
    const int n = r->n, P = r->P;
    const size_t nn = (size_t)n * n, W = (nn + 31) / 32;
    const ShotLayout L(n, P, reserved_ + r->arena_off);
    const size_t sb = d->supp.size();
    auto A = [](size_t b) { return Arena::align_up(b); };
    const size_t o_desc = 0, o_E = A(sizeof(SlotDesc) * P), o_st = o_E + A(8 * (size_t)P), o_amp = o_st + A(16),
                 o_supp = o_amp + A(4 * nn), o_rho = o_supp + A(sb);
    const size_t up_bytes = o_rho + (d->rho0.empty() ? 0 : 8 * nn * P);
    d->upload = pool_.get(up_bytes);
    char* u = static_cast<char*>(d->upload.p);
    SlotDesc* desc = reinterpret_cast<SlotDesc*>(u + o_desc);
    for (int m = 0; m < P; ++m) {
      desc[m].X = dev<float2>(L.X) + (size_t)m * nn;
      desc[m].T = dev<float2>(L.T) + (size_t)m * nn;
      desc[m].S = dev<uint32_t>(L.S) + (size_t)m * W;
      desc[m].amp = d->enc16.empty() ? dev<float>(L.amp) : nullptr;
      desc[m].amp16 = d->enc16.empty() ? nullptr : dev<__half>(L.amp);
      desc[m].E = dev<double>(L.E) + m;
      desc[m].den = d->den;
      desc[m].flags = dev<int>(L.status);
      desc[m].amp_scale = d->amp_scale;
      desc[m].pad = 0;
    }
    double* E0 = reinterpret_cast<double*>(u + o_E);
    for (int m = 0; m < P; ++m) E0[m] = std::numeric_limits<double>::infinity();
    std::memset(u + o_st, 0, 16);
    const size_t amp_bytes = d->enc16.empty() ? 4 * nn : 2 * nn;
    if (d->enc16.empty()) std::memcpy(u + o_amp, d->enc.data(), amp_bytes);
    else std::memcpy(u + o_amp, d->enc16.data(), amp_bytes);
    const float amp_scale = d->amp_scale;
    const bool fp16 = !d->enc16.empty();
    std::memcpy(u + o_supp, d->supp.data(), sb);
    if (!d->rho0.empty()) std::memcpy(u + o_rho, d->rho0.data(), 8 * nn * P);
    const int slot0 = r->slot * P;
    const bool bcast = d->supp_per_member == 0;
    const uint64_t seed = d->seed;
    const bool init = d->rho0.empty();
    ops_.push_back([=] {
      HIPCHK(hipMemcpyAsync(dev<SlotDesc>(o_table_) + slot0, u + o_desc, sizeof(SlotDesc) * P,
                            hipMemcpyHostToDevice, s_));
      HIPCHK(hipMemcpyAsync(base_ + L.E, u + o_E, 8 * (size_t)P, hipMemcpyHostToDevice, s_));
      HIPCHK(hipMemcpyAsync(base_ + L.status, u + o_st, 16, hipMemcpyHostToDevice, s_));
      HIPCHK(hipMemcpyAsync(base_ + L.amp, u + o_amp, amp_bytes, hipMemcpyHostToDevice, s_));
      // supports through the first work buffer, as many members at a time as fit
      const int per = bcast ? P : (int)std::max<size_t>(1, std::min<size_t>(P, ws_bytes_ / nn));
      for (int m0 = 0; m0 < P; m0 += per) {
        const int cnt = std::min(per, P - m0);
        const size_t bytes = bcast ? nn : nn * cnt;
        HIPCHK(hipMemcpyAsync(base_ + o_wsA_, u + o_supp + (bcast ? 0 : nn * m0), bytes, hipMemcpyHostToDevice, s_));
        PackArgs pa{dev<int>(o_ident_) + m0, cnt, n, (int)W, bcast ? 1 : 0, dev<uint8_t>(o_wsA_), dev<uint32_t>(L.S)};
        launch(launch_pack(pa, s_), "pack");
      }
      if (init) {
        random_phase_start(ctx_, Ks_.at(n), n, P, fp16 ? nullptr : dev<float>(L.amp),
                           fp16 ? dev<__half>(L.amp) : nullptr, amp_scale, seed, dev<float2>(L.X), s_);
        launches += 3;
      } else {
        HIPCHK(hipMemcpyAsync(base_ + L.X, u + o_rho, 8 * nn * P, hipMemcpyHostToDevice, s_));
      }
    });
  }

  void member_slots(const Launch& L, std::vector<int>& slots, std::vector<int>& step_of) {
    slots.clear();
    step_of.clear();
    for (auto& sp : L.shots)
      for (int m = 0; m < sp.first->P; ++m) {
        slots.push_back(sp.first->slot * sp.first->P + m);
        step_of.push_back(sp.second);
      }
  }

  void plan_launch(const Launch& L) {
    std::vector<int> slots, step_of;
    member_slots(L, slots, step_of);
    const int n = L.n;
    const size_t nn = (size_t)n * n;
    const int total = (int)slots.size();
    const SizeKernels* K = Ks_.at(n);
    const float2* tw = twiddles(ctx_, n);
    if (L.kind == STEP_SEQ) {
      const int chunk = (int)std::max<size_t>(1, ws_bytes_ / (8 * nn));
      for (int c0 = 0; c0 < total; c0 += chunk) {
        const int cm = std::min(chunk, total - c0);
        const int* dslots = meta(slots.data() + c0, cm);
        // ingest, one launch per distinct (mode, chi) of the members' first iteration
        std::map<std::pair<int, double>, std::vector<int>> ing;
        for (int k = 0; k < cm; ++k) {
          const ItStep& f = pg_.its[pg_.steps[step_of[c0 + k]].it0];
          ing[{f.alg == ALG_ER ? INGEST_PC : INGEST_PLAIN, f.chi}].push_back(slots[c0 + k]);
        }
        for (auto& kv : ing) {
          const int* ds = meta(kv.second.data(), kv.second.size());
          RowIngestArgs ia{ds, (int)kv.second.size(), dev<SlotDesc>(o_table_), nullptr, 0, 1, kv.first.first,
                           phase_of(kv.first.second), tw};
          ia.W = (int)((nn + 31) / 32);
          ops_.push_back([=] { launch(K->row_ingest(ia, s_, nullptr), "row_ingest"); });
        }
        std::vector<IterParam> ip(cm);
        for (int i = 0; i < L.nit; ++i) {
          for (int k = 0; k < cm; ++k) {
            const Step& st = pg_.steps[step_of[c0 + k]];
            const ItStep& it = pg_.its[st.it0 + i];
            const bool last = i + 1 == st.nit;
            IterParam& q = ip[k];
            q.alg = it.alg;
            q.beta = it.beta;
            q.ph = phase_of(it.chi);
            if (last) {
              q.out_mode = OUT_REAL;
              q.ph_next = phase_of(1.0);
            } else {
              const ItStep& nx = pg_.its[st.it0 + i + 1];
              q.out_mode = nx.alg == ALG_ER ? OUT_T_PC : OUT_T_PLAIN;
              q.ph_next = phase_of(nx.chi);
            }
          }
          // members sharing one set of parameters take the launch-wide form
          // (and the algorithm's own kernel); the arithmetic is the same
          bool uniform = true;
          for (int k = 1; k < cm && uniform; ++k) uniform = std::memcmp(&ip[k], &ip[0], sizeof(IterParam)) == 0;
          const IterParam* dip = uniform ? nullptr : meta(ip.data(), cm);
          ColProjArgs ca{dslots, cm, dev<SlotDesc>(o_table_), 1, nullptr, dev<float2>(o_wsB_), tw};
          RowUpdateArgs ra;
          std::memset(&ra, 0, sizeof(ra));
          ra.slots = dslots;
          ra.nm = cm;
          ra.desc = dev<SlotDesc>(o_table_);
          ra.Y = dev<float2>(o_wsB_);
          ra.T = nullptr;
          ra.W = (int)((nn + 31) / 32);
          ra.t_by_slot = 1;
          ra.ip = dip;
          ra.alg = ip[0].alg;
          ra.beta = ip[0].beta;
          ra.ph = ip[0].ph;
          ra.out_mode = ip[0].out_mode;
          ra.ph_next = ip[0].ph_next;
          ra.tw = tw;
          ops_.push_back([=] {
            launch(K->col_proj(ca, s_, nullptr), "col_proj");
            launch(K->row_update(ra, s_, nullptr), "row_update");
          });
        }
      }
      return;
    }
    // support and fitness steps: chunks sized by the smoothing scratch
    const int chunk = L.kind == STEP_ERR ? total : (int)std::max<size_t>(1, ws_bytes_ / (4 * nn));
    for (int c0 = 0; c0 < total; c0 += chunk) {
      const int cm = std::min(chunk, total - c0);
      const int* dslots = meta(slots.data() + c0, cm);
      Group g = group(n, dslots, cm);
      const int kind = L.kind;
      const double sigma = L.sigma, tau = L.tau, alpha = L.alpha;
      ops_.push_back([=] {
        if (kind == STEP_SW) {
          shrinkwrap(g, sigma, tau, s_);
          launches += 3;
        } else if (kind == STEP_AREA) {
          support_area(g, sigma, nullptr, 0, alpha, s_);
          launches += 2 + (topk_scratch_words(n) ? 9 : 1);  // smoothing, then the selection
        } else {
          get_error(g, s_);
          launches += 3;
        }
      });
    }
  }

  // Results to pinned host memory, then the completion event.
  void plan_end(Req* r) {
    ShotData* d = data_of(r);
    const int n = r->n, P = r->P;
    const size_t nn = (size_t)n * n, W = (nn + 31) / 32;
    const ShotLayout L(n, P, reserved_ + r->arena_off);
    d->result = pool_.get(result_bytes(n, P, all_));
    d->done = event();
    char* h = static_cast<char*>(d->result.p);
    const bool all = all_;
    hipEvent_t done = d->done;
    ops_.push_back([=] {
      if (!all) {
        GatherBestArgs ga{P, n, (int)W, dev<double>(L.E), dev<float2>(L.X), dev<uint32_t>(L.S), dev<int>(L.status),
                          dev<unsigned char>(L.res)};
        launch(launch_gather_best(ga, s_), "gather_best");
        HIPCHK(hipMemcpyAsync(h, base_ + L.res, result_bytes(n, P, false), hipMemcpyDeviceToHost, s_));
      } else {
        const size_t oX = 32 + 8 * (size_t)P;
        HIPCHK(hipMemcpyAsync(h + 4, base_ + L.status, sizeof(int), hipMemcpyDeviceToHost, s_));
        HIPCHK(hipMemcpyAsync(h + 32, base_ + L.E, 8 * (size_t)P, hipMemcpyDeviceToHost, s_));
        HIPCHK(hipMemcpyAsync(h + oX, base_ + L.X, 8 * nn * P, hipMemcpyDeviceToHost, s_));
        HIPCHK(hipMemcpyAsync(h + oX + 8 * nn * P, base_ + L.S, 4 * W * P, hipMemcpyDeviceToHost, s_));
      }
      HIPCHK(hipEventRecord(done, s_));
    });
    if (all) {
      // the host picks the best member once the errors have arrived
      reinterpret_cast<int*>(h)[0] = -1;
    }
  }

  spr_ctx* ctx_;
  const Program& pg_;
  bool all_;
  int R_;
  std::chrono::steady_clock::time_point t0_;
  size_t members_ = 0, ws_bytes_ = 0, meta_cap_ = 0, reserved_ = 0, budget_ = 0;
  int max_tiles_ = 1, max_blocks_ = 1;
  size_t o_table_ = 0, o_ident_ = 0, o_ring_ = 0, o_wsA_ = 0, o_wsB_ = 0, o_errp_ = 0, o_bmax_ = 0, o_maxv_ = 0;
  hipStream_t s_ = nullptr;
  char* base_ = nullptr;
  std::vector<RingEntry> ring_;
  uint64_t last_tick_ = 0;
  char* meta_host_ = nullptr;
  char* meta_dev_ = nullptr;
  size_t meta_used_ = 0;
  std::vector<std::function<void()>> ops_;
  std::vector<hipEvent_t> events_;
  std::map<int, const SizeKernels*> Ks_;
  PinnedPool pool_;
};

}  // namespace

// ---------------------------------------------------------------------------
// The server handle
// ---------------------------------------------------------------------------
struct spr_server {
  spr_ctx* ctx = nullptr;
  spr_server_cfg cfg{};
  Program prog;
  std::unique_ptr<Scheduler> sch;
  std::unique_ptr<Exec> ex;
  std::mutex mu;
  std::condition_variable cv;       // wakes the engine (submit, stop)
  std::condition_variable cv_done;  // wakes drain (a request finished)
  std::thread th;
  bool stop = false;
  std::string err;
  spr_status engine_status = SPR_OK;
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  uint64_t next_ticket = 1;
  int64_t done_waiting = 0;
};

namespace {

template <class Fn>
spr_status server_guarded(spr_server* sv, Fn&& fn) {
  try {
    fn();
    return SPR_OK;
  } catch (const Fail& f) {
    sv->err = f.msg;
    return f.code;
  } catch (const std::bad_alloc&) {
    sv->err = "host allocation failed";
    return SPR_E_OOM;
  } catch (...) {
    sv->err = "unexpected internal error";
    return SPR_E_INVALID_ARG;
  }
}

int64_t pending(spr_server* sv) {
  return (int64_t)(sv->sch->queued() + sv->sch->active() + sv->sch->finishing());
}

// One engine round under the server lock: collect finished shots, admit,
// plan and enqueue a tick.  Returns whether anything happened.
bool engine_round(spr_server* sv) {
  bool did = false;
  std::vector<Req*> fin = sv->sch->finishing_list();
  for (Req* r : fin)
    if (sv->ex->finished(r)) {
      sv->sch->complete(r, sv->ex->now());
      ++sv->done_waiting;
      did = true;
    }
  if (did) sv->cv_done.notify_all();
  if (sv->ex->simulated() && sv->sch->active() == 0 && sv->sch->finishing() == 0 && sv->sch->queued() > 0) {
    // modelled time: jump to the next arrival when the device would be idle
    static_cast<SimExec*>(sv->ex.get())->advance_to(sv->sch->queue().front()->t_arrival);
  }
  std::vector<Req*> started = sv->sch->admit(sv->ex->now());
  if (sv->sch->active() > 0) {
    TickPlan tp = sv->sch->plan(started, sv->ex->now());
    sv->ex->issue(tp);
    did = true;
  }
  return did;
}

void engine_thread(spr_server* sv) {
  if (sv->ctx) (void)hipSetDevice(sv->ctx->device);
  for (;;) {
    try {
      sv->ex->wait_slot();
    } catch (const Fail& f) {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->engine_status = f.code;
      sv->err = f.msg;
      sv->cv_done.notify_all();
      return;
    }
    std::unique_lock<std::mutex> lk(sv->mu);
    if (sv->stop) return;
    bool did = false;
    try {
      did = engine_round(sv);
    } catch (const Fail& f) {
      sv->engine_status = f.code;
      sv->err = f.msg;
      sv->cv_done.notify_all();
      return;
    }
    if (did) continue;
    if (sv->sch->finishing() > 0 || sv->sch->active() > 0)
      sv->cv.wait_for(lk, std::chrono::microseconds(50));
    else
      sv->cv.wait(lk, [&] { return sv->stop || sv->sch->queued() > 0; });
  }
}

}  // namespace

extern "C" {

spr_status spr_server_create(spr_ctx* ctx, const spr_server_cfg* cfg, spr_server** out) {
  if (!cfg || !out || !cfg->sched) return SPR_E_INVALID_ARG;
  *out = nullptr;
  if (ctx && !live_has(ctx)) return SPR_E_INVALID_ARG;
  std::unique_ptr<spr_server> sv(new (std::nothrow) spr_server());
  if (!sv) return SPR_E_OOM;
  spr_status st = server_guarded(sv.get(), [&] {
    if (cfg->P < 1 || cfg->max_shots < 1) fail(SPR_E_INVALID_ARG, "P and max_shots must be >= 1");
    if (cfg->max_inflight < 0) fail(SPR_E_INVALID_ARG, "negative max_inflight");
    sv->ctx = ctx;
    sv->cfg = *cfg;
    sv->cfg.sched = nullptr;
    sv->prog = compile_program(cfg->sched);
    const bool all = cfg->flags & SPR_SERVER_ALL_MEMBERS;
    size_t base = 0, cap = 0;
    if (!ctx) {
      if (!(cfg->flags & SPR_SERVER_MANUAL)) fail(SPR_E_INVALID_ARG, "the simulated executor needs SPR_SERVER_MANUAL");
      if (!(cfg->sim_bytes_per_s > 0) || cfg->sim_launch_s < 0)
        fail(SPR_E_INVALID_ARG, "the simulated executor needs a positive bandwidth");
      sv->ex.reset(new SimExec(cfg->sim_bytes_per_s, cfg->sim_launch_s, cfg->P));
      cap = cfg->hbm_budget;
    } else {
      HipExec* he = new HipExec(ctx, sv->prog, sv->cfg);
      sv->ex.reset(he);
      base = 0;
      cap = he->budget() - he->reserved();
    }
    const int policy = (cfg->flags & SPR_SERVER_SHORTEST_FIRST) ? POLICY_SHORTEST : POLICY_ALL;
    sv->sch.reset(new Scheduler(sv->prog, cfg->max_shots, cfg->P, base, cap, all, (size_t)cfg->max_queue, policy,
                                ctx ? 4e12 : cfg->sim_bytes_per_s));
  });
  if (st != SPR_OK) {
    if (ctx) ctx->err = sv->err;
    return st;
  }
  spr_server* h = sv.release();
  if (!(cfg->flags & SPR_SERVER_MANUAL)) h->th = std::thread(engine_thread, h);
  live_add(h);
  if (ctx) ctx->servers.insert(h);
  *out = h;
  return SPR_OK;
}

spr_status spr_server_submit(spr_server* sv, const spr_shot_desc* sd, uint64_t* ticket) {
  if (!sv || !sd || !ticket || !live_has(sv)) return SPR_E_INVALID_ARG;
  const double t_in = sv->ex->now();
  // host preparation outside the lock
  std::unique_ptr<Req> r(new (std::nothrow) Req());
  if (!r) return SPR_E_OOM;
  std::shared_ptr<ShotData> d;
  std::string msg;
  spr_status st = [&]() -> spr_status {
    try {
      if (!sd->amp || !sd->mask || !sd->supp0) fail(SPR_E_INVALID_ARG, "amp, mask and supp0 are required");
      if (!size_kernels(sd->n)) fail(SPR_E_UNSUPPORTED_SIZE, "unsupported detector size " + std::to_string(sd->n));
      const bool init = sd->flags & SPR_INIT_RANDOM_PHASE;
      if (!init && !sd->rho0) fail(SPR_E_INVALID_ARG, "rho0 is required without SPR_INIT_RANDOM_PHASE");
      const int n = sd->n, P = sv->cfg.P;
      const size_t nn = (size_t)n * n;
      d = std::make_shared<ShotData>();
      d->enc.resize(nn);
      d->den = encode_shot(n, sd->amp, sd->mask, sd->flags, d->enc.data());
      if (sd->bound_eta > 0.0) {
        if (!(sd->bound_max_unknown >= 0.0 && sd->bound_max_unknown <= 1.0))
          fail(SPR_E_INVALID_ARG, "bound_max_unknown must lie in [0, 1]");
        std::vector<uint8_t> sat;
        if (sd->saturated) {
          if (!(sd->bound_max_saturated >= 0.0 && sd->bound_max_saturated <= 1.0))
            fail(SPR_E_INVALID_ARG, "bound_max_saturated must lie in [0, 1]");
          sat = saturation_fft(n, sd->saturated, sd->flags, d->enc.data());
        }
        apply_upper_bounds(n, d->enc.data(), 1.0f, sd->bound_eta, sd->bound_max_unknown,
                           std::numeric_limits<float>::min(), sd->saturated ? sat.data() : nullptr,
                           sd->saturated ? sd->bound_max_saturated : 1.0);
      }
      if (sd->flags & SPR_AMP_FP16) {
        d->amp_scale = fp16_encode(d->enc.data(), nn, d->enc16, d->den);
        if (!(d->den > 0.0)) fail(SPR_E_INVALID_ARG, "sum of measured M^2 must be positive");
        std::vector<float>().swap(d->enc);
      }
      d->supp_per_member = sd->supp_per_member ? 1 : 0;
      d->supp.assign(sd->supp0, sd->supp0 + (d->supp_per_member ? nn * P : nn));
      if (!init) d->rho0.assign(sd->rho0, sd->rho0 + 2 * nn * P);
      d->seed = sd->seed;
      return SPR_OK;
    } catch (const Fail& f) {
      msg = f.msg;
      return f.code;
    } catch (const std::bad_alloc&) {
      msg = "host allocation failed";
      return SPR_E_OOM;
    }
  }();
  std::lock_guard<std::mutex> lk(sv->mu);
  if (st != SPR_OK) {
    sv->err = msg;
    return st;
  }
  if (sv->engine_status != SPR_OK) return sv->engine_status;
  const int c = sv->sch->check_submit(sd->n);
  if (c == 1) {
    sv->err = "a shot of size " + std::to_string(sd->n) + " needs more memory than the server's budget";
    return SPR_E_ADMISSION;
  }
  if (c == 2) {
    sv->err = "request queue is full";
    return SPR_E_BUSY;
  }
  r->ticket = sv->next_ticket++;
  r->n = sd->n;
  r->t_arrival = sd->arrival >= 0 ? sd->arrival : t_in;
  r->payload = d;
  Req* rp = r.get();
  sv->reqs[rp->ticket] = std::move(r);
  sv->sch->enqueue(rp);
  *ticket = rp->ticket;
  sv->cv.notify_all();
  return SPR_OK;
}

spr_status spr_server_poll(spr_server* sv, uint64_t ticket, spr_result* res) {
  if (!sv || !res || !live_has(sv)) return SPR_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) {
    sv->err = "unknown ticket";
    return SPR_E_INVALID_ARG;
  }
  Req* r = it->second.get();
  if (r->state != REQ_DONE) return sv->engine_status != SPR_OK ? sv->engine_status : SPR_E_NOT_READY;
  return server_guarded(sv, [&] {
    const int members = (sv->cfg.flags & SPR_SERVER_ALL_MEMBERS) ? r->P : 1;
    res->n = r->n;
    res->P = r->P;
    res->members = members;
    res->t_arrival = r->t_arrival;
    res->t_admit = r->t_admit;
    res->t_finish = r->t_finish;
    sv->ex->fetch(r, res, members);
    sv->reqs.erase(it);
    --sv->done_waiting;
  });
}

spr_status spr_server_step(spr_server* sv, int64_t* pend) {
  if (!sv || !live_has(sv)) return SPR_E_INVALID_ARG;
  if (!(sv->cfg.flags & SPR_SERVER_MANUAL)) {
    sv->err = "spr_server_step drives servers created with SPR_SERVER_MANUAL";
    return SPR_E_INVALID_ARG;
  }
  if (sv->ctx) (void)hipSetDevice(sv->ctx->device);
  spr_status st = server_guarded(sv, [&] { sv->ex->wait_slot(); });
  if (st != SPR_OK) return st;
  std::lock_guard<std::mutex> lk(sv->mu);
  st = server_guarded(sv, [&] { engine_round(sv); });
  if (pend) *pend = pending(sv);
  return st;
}

spr_status spr_server_drain(spr_server* sv, double timeout_s) {
  if (!sv || !live_has(sv)) return SPR_E_INVALID_ARG;
  const auto t0 = std::chrono::steady_clock::now();
  auto expired = [&] {
    return timeout_s >= 0 &&
           std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > timeout_s;
  };
  if (sv->cfg.flags & SPR_SERVER_MANUAL) {
    for (;;) {
      int64_t p = 0;
      spr_status st = spr_server_step(sv, &p);
      if (st != SPR_OK) return st;
      if (p == 0) return SPR_OK;
      if (expired()) return SPR_E_NOT_READY;
      if (!sv->ex->simulated()) {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->sch->active() == 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
      }
    }
  }
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    if (sv->engine_status != SPR_OK) return sv->engine_status;
    if (pending(sv) == 0) return SPR_OK;
    if (expired()) return SPR_E_NOT_READY;
    sv->cv_done.wait_for(lk, std::chrono::milliseconds(5));
  }
}

spr_status spr_server_stats_get(spr_server* sv, spr_server_stats* o) {
  if (!sv || !o || !live_has(sv)) return SPR_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  o->now = sv->ex->now();
  o->queued = (int64_t)sv->sch->queued();
  o->active = (int64_t)sv->sch->active();
  o->finishing = (int64_t)sv->sch->finishing();
  o->done = sv->done_waiting;
  o->admitted = (int64_t)sv->sch->admitted();
  o->completed = (int64_t)sv->sch->completed();
  o->ticks = (int64_t)sv->sch->ticks();
  o->launches = sv->ex->launches;
  o->max_active = sv->sch->max_active_seen();
  o->bytes_capacity = sv->sch->capacity();
  o->bytes_in_use = sv->sch->used();
  o->bytes_peak = sv->sch->peak();
  return SPR_OK;
}

const char* spr_server_last_error(const spr_server* sv) { return sv ? sv->err.c_str() : "null server"; }

spr_status spr_server_destroy(spr_server* sv) {
  if (!sv || !live_remove(sv)) return SPR_E_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  if (sv->th.joinable()) sv->th.join();
  if (sv->ctx) {
    (void)hipSetDevice(sv->ctx->device);
    sv->ctx->servers.erase(sv);
  }
  try {
    for (auto& kv : sv->reqs) sv->ex->discard(kv.second.get());
  } catch (...) {
  }
  sv->reqs.clear();
  sv->sch.reset();
  sv->ex.reset();
  delete sv;
  return SPR_OK;
}

}  // extern "C"
