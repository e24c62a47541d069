// Host scheduler of the serving engine: request queue, admission by device
// memory footprint, shot slots, per-shot program counters and the planning of
// continuous-batching ticks.  Free of HIP so that the same logic runs under
// the device executor and under the simulated (modelled-time) executor.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

namespace spr_serve {

// ---------------------------------------------------------------------------
// Arena: first-fit allocation of byte ranges inside one device allocation.
// ---------------------------------------------------------------------------
class Arena {
 public:
  static constexpr size_t kAlign = 256;
  Arena() = default;
  Arena(size_t base, size_t size) { reset(base, size); }
  void reset(size_t base, size_t size) {
    free_.clear();
    base_ = align_up(base);
    end_ = base + size;
    if (end_ > base_) free_[base_] = end_ - base_;
    used_ = peak_ = 0;
  }
  static size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
  size_t capacity() const { return end_ > base_ ? end_ - base_ : 0; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  // offset of a range of `bytes`, or SIZE_MAX when no free range is large enough
  size_t alloc(size_t bytes) {
    bytes = align_up(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      live_[off] = bytes;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return off;
    }
    return SIZE_MAX;
  }
  void release(size_t off) {
    auto it = live_.find(off);
    if (it == live_.end()) return;
    size_t start = off, len = it->second;
    used_ -= len;
    live_.erase(it);
    auto nx = free_.lower_bound(start);
    if (nx != free_.end() && start + len == nx->first) {
      len += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == start) {
        start = pv->first;
        len += pv->second;
        free_.erase(pv);
      }
    }
    free_[start] = len;
  }
  size_t largest_free() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  size_t base_ = 0, end_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  std::map<size_t, size_t> live_;
};

// ---------------------------------------------------------------------------
// The per-shot program: a schedule compiled into steps.
// ---------------------------------------------------------------------------
enum StepKind { STEP_SEQ = 0, STEP_SW = 1, STEP_AREA = 2, STEP_ERR = 3 };

struct ItStep {
  int alg;  // 0 ER, 1 HIO, 2 RAAR (values of the iteration kernels)
  float beta;
  double chi;
};

struct Step {
  int kind = STEP_SEQ;
  int it0 = 0, nit = 0;  // STEP_SEQ: iterations its[it0 .. it0+nit)
  double sigma = 0, tau = 0, alpha = 0;
};

struct Program {
  std::vector<Step> steps;
  std::vector<ItStep> its;
  int max_seq = 0;         // longest sequence
  int max_non_seq_run = 0; // longest run of consecutive non-sequence steps
  double member_its = 0;   // iterations per member
};

// Device bytes held by one admitted shot (all sub-allocations 256-aligned).
inline size_t shot_footprint(int n, int P, bool all_members) {
  auto A = [](size_t b) { return Arena::align_up(b); };
  const size_t nn = (size_t)n * n, W = (nn + 31) / 32;
  size_t b = A(4 * nn)           // amplitudes
             + A(8 * nn * P)     // densities
             + A(8 * nn * P)     // row-transform buffers
             + A(4 * W * P)      // support bits
             + A(8 * (size_t)P)  // errors
             + A(16);            // status word
  if (!all_members) b += A(32 + 8 * (size_t)P + 8 * nn + 4 * W);  // best-member result
  return b;
}

// ---------------------------------------------------------------------------
// Requests and tick plans.
// ---------------------------------------------------------------------------
enum ReqState { REQ_QUEUED = 0, REQ_ACTIVE = 1, REQ_FINISHING = 2, REQ_DONE = 3 };

struct Req {
  uint64_t ticket = 0;
  int n = 0, P = 0;
  size_t footprint = 0;
  size_t arena_off = SIZE_MAX;
  int slot = -1;  // shot slot: member descriptors [slot*P, slot*P + P)
  int pc = 0;
  int state = REQ_QUEUED;
  double t_arrival = 0, t_admit = 0, t_finish = 0;
  double sim_done = 0;  // simulated executor: completion time
  int status = 0;
  std::shared_ptr<void> payload;  // executor-owned inputs/results
};

// One batched operation of a tick over every member of the listed shots.
struct Launch {
  int kind = STEP_SEQ;
  int n = 0;
  int nit = 0;  // STEP_SEQ: iterations
  double sigma = 0, tau = 0, alpha = 0;
  std::vector<std::pair<Req*, int>> shots;  // (request, step index it executes)
};

struct TickPlan {
  uint64_t id = 0;
  std::vector<Req*> started;          // admitted this tick: uploads come first
  std::vector<std::vector<Launch>> rounds;
  std::vector<Req*> ending;           // programs complete at the end of this tick
  bool empty() const { return started.empty() && rounds.empty() && ending.empty(); }
};

// Which resident shots a tick advances.
enum TickPolicy {
  POLICY_ALL = 0,       // every resident shot (lockstep continuous batching)
  POLICY_SHORTEST = 1,  // the shots of one size: that of the shot with the least remaining
                        // work, less the time it has waited (aging), first
};

class Scheduler {
 public:
  Scheduler(const Program& prog, int max_shots, int P, size_t shot_bytes_base, size_t shot_bytes,
            bool all_members, size_t max_queue, int policy = POLICY_ALL, double bytes_per_s = 4e12)
      : prog_(prog), P_(P), all_members_(all_members), max_queue_(max_queue), policy_(policy),
        bytes_per_s_(bytes_per_s), free_slots_() {
    arena_.reset(shot_bytes_base, shot_bytes);
    for (int s = max_shots - 1; s >= 0; --s) free_slots_.push_back(s);
  }

  const Program& program() const { return prog_; }
  size_t capacity() const { return arena_.capacity(); }
  size_t used() const { return arena_.used(); }
  size_t peak() const { return arena_.peak(); }
  size_t queued() const { return queue_.size(); }
  size_t active() const { return active_.size(); }
  size_t finishing() const { return finishing_.size(); }
  uint64_t admitted() const { return admitted_; }
  uint64_t completed() const { return completed_; }
  uint64_t ticks() const { return tick_id_; }
  int max_active_seen() const { return max_active_; }
  const std::deque<Req*>& queue() const { return queue_; }
  const std::vector<Req*>& active_list() const { return active_; }
  std::vector<Req*>& finishing_list() { return finishing_; }

  // 0: accepted; 1: can never fit (admission); 2: queue full (back-pressure)
  int check_submit(int n) const {
    const size_t fp = shot_footprint(n, P_, all_members_);
    if (fp > arena_.capacity()) return 1;
    if (max_queue_ && queue_.size() >= max_queue_) return 2;
    return 0;
  }
  void enqueue(Req* r) {
    r->P = P_;
    r->footprint = shot_footprint(r->n, P_, all_members_);
    r->state = REQ_QUEUED;
    queue_.push_back(r);
  }

  // Admit from the head of the queue while a slot and a memory range are free
  // (first come, first served: a head that does not fit blocks the rest).
  std::vector<Req*> admit(double now) {
    std::vector<Req*> out;
    while (!queue_.empty() && !free_slots_.empty()) {
      Req* r = queue_.front();
      if (r->t_arrival > now) break;
      const size_t off = arena_.alloc(r->footprint);
      if (off == SIZE_MAX) break;
      queue_.pop_front();
      r->arena_off = off;
      r->slot = free_slots_.back();
      free_slots_.pop_back();
      r->state = REQ_ACTIVE;
      r->t_admit = now;
      r->pc = 0;
      active_.push_back(r);
      out.push_back(r);
      ++admitted_;
    }
    max_active_ = std::max<int>(max_active_, (int)active_.size());
    return out;
  }

  // Modelled seconds of device work left for a request (iterations dominate).
  double remaining_s(const Req* r) const {
    double its = 0;
    for (size_t k = (size_t)r->pc; k < prog_.steps.size(); ++k)
      if (prog_.steps[k].kind == STEP_SEQ) its += prog_.steps[k].nit;
    return its * (double)r->n * r->n * P_ * 40.0 / bytes_per_s_;
  }

  // Plan one tick: every advancing shot runs its steps up to and including
  // one sequence (or to its end); steps of equal kind, size and parameters
  // taken by several shots in the same round become one launch.
  TickPlan plan(const std::vector<Req*>& started, double now = 0.0) {
    TickPlan tp;
    tp.id = ++tick_id_;
    tp.started = started;
    std::vector<char> did_seq(active_.size(), 0), stop(active_.size(), 0);
    if (policy_ == POLICY_SHORTEST && !active_.empty()) {
      size_t pick = 0;
      double best = 0;
      for (size_t i = 0; i < active_.size(); ++i) {
        const double key = remaining_s(active_[i]) - (now - active_[i]->t_arrival);
        if (i == 0 || key < best) {
          best = key;
          pick = i;
        }
      }
      for (size_t i = 0; i < active_.size(); ++i)
        if (active_[i]->n != active_[pick]->n) stop[i] = 1;  // waits for a later tick
    }
    const auto& steps = prog_.steps;
    for (;;) {
      std::map<std::tuple<int, int, int, double, double, double>, size_t> key_of;
      std::vector<Launch> round;
      for (size_t i = 0; i < active_.size(); ++i) {
        if (stop[i]) continue;
        Req* r = active_[i];
        if (r->pc >= (int)steps.size()) {
          stop[i] = 1;
          continue;
        }
        const Step& st = steps[r->pc];
        if (st.kind == STEP_SEQ && did_seq[i]) {
          stop[i] = 1;
          continue;
        }
        auto key = std::make_tuple(st.kind, r->n, st.kind == STEP_SEQ ? st.nit : 0, st.sigma, st.tau, st.alpha);
        auto it = key_of.find(key);
        if (it == key_of.end()) {
          Launch L;
          L.kind = st.kind;
          L.n = r->n;
          L.nit = st.kind == STEP_SEQ ? st.nit : 0;
          L.sigma = st.sigma;
          L.tau = st.tau;
          L.alpha = st.alpha;
          it = key_of.emplace(key, round.size()).first;
          round.push_back(L);
        }
        round[it->second].shots.push_back({r, r->pc});
        if (st.kind == STEP_SEQ) did_seq[i] = 1;
        r->pc++;
      }
      if (round.empty()) break;
      tp.rounds.push_back(std::move(round));
    }
    std::vector<Req*> keep;
    for (Req* r : active_) {
      if (r->pc >= (int)steps.size()) {
        r->state = REQ_FINISHING;
        tp.ending.push_back(r);
        finishing_.push_back(r);
      } else {
        keep.push_back(r);
      }
    }
    active_.swap(keep);
    return tp;
  }

  // A finishing request whose results are on the host: release its slot and memory.
  void complete(Req* r, double now) {
    r->state = REQ_DONE;
    r->t_finish = now;
    arena_.release(r->arena_off);
    r->arena_off = SIZE_MAX;
    free_slots_.push_back(r->slot);
    finishing_.erase(std::remove(finishing_.begin(), finishing_.end(), r), finishing_.end());
    ++completed_;
  }

 private:
  Program prog_;
  int P_;
  bool all_members_;
  size_t max_queue_;
  int policy_;
  double bytes_per_s_;
  Arena arena_;
  std::vector<int> free_slots_;
  std::deque<Req*> queue_;
  std::vector<Req*> active_;
  std::vector<Req*> finishing_;
  uint64_t tick_id_ = 0, admitted_ = 0, completed_ = 0;
  int max_active_ = 0;
};

}  // namespace spr_serve
