// Continuous-batching request loop over one fn_batch (fn_server_*).
//
// Loop: admit visible requests into free slots while their events fit the
// device-memory budget (first-fit arena for generated events, caller-owned
// events charged by size; no hipMalloc/hipFree in the loop), generate their
// events on the batch stream, advance the batch poll_every steps, read the
// per-slot status mirror, retire finished fits (result rows, timestamps,
// arena space, budget and slot released), repeat.  New requests join at step
// boundaries while earlier ones are still running.
//
// Admission order: arrival order, with backfilling -- a request whose events
// do not fit the free budget does not stop later (smaller) arrivals from
// being admitted, until kMaxBypass requests have been admitted past it; from
// then on nothing more is admitted until it fits, so a large request cannot
// be starved by a stream of small ones.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "internal.hpp"
#include "serve.hpp"

using namespace fn;

namespace {

// First-fit allocator over [0, size) with coalescing, in 256-byte units.
class Arena {
 public:
  explicit Arena(int64_t size = 0) { reset(size); }
  void reset(int64_t size) {
    free_.clear();
    if (size > 0) free_[0] = size;
    size_ = size;
  }
  int64_t alloc(int64_t bytes) {
    bytes = (bytes + 255) & ~int64_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest > 0) free_[off + bytes] = rest;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t bytes) {
    bytes = (bytes + 255) & ~int64_t(255);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  int64_t size() const { return size_; }

 private:
  std::map<int64_t, int64_t> free_;
  int64_t size_ = 0;
};

struct Pending {
  fn_request r;
  int64_t off = -1;     // arena offset of generated events (-1: caller events)
  int64_t bytes = 0;    // budget charge: the request's event bytes
  double t_admit = -1.0;
  int bypassed = 0;     // requests admitted past this one while it was blocked
};

// Requests admitted past a blocked one before admission waits for it.
constexpr int kMaxBypass = 256;

}  // namespace

struct fn_server {
  fn_model* m = nullptr;
  fn_batch* b = nullptr;
  int slots = 0;
  int P = 0;
  int64_t max_ev = 0;
  int64_t budget = 0;
  int64_t in_use = 0;                   // budget charged by admitted, unfinished requests
  DevBuf arena_mem;
  Arena arena;
  DevBuf gen_count;
  bool started = false;                 // server clock: starts with the first fn_server_run
  std::chrono::steady_clock::time_point t0;
  std::vector<Pending> queue;           // submitted, not yet admitted (sorted by arrival)
  std::vector<int> slot_req;            // slot -> 1 while a request runs in it, -1 free
  std::vector<int> free_slots;          // stack of free slots
  std::vector<Pending> running;         // by slot
  std::vector<fn_result> done;
  int* h_stat = nullptr;
  double* h_rows = nullptr;
  AdmitRec* h_adm = nullptr;            // admission records of one round (pinned)
  ~fn_server() {
    if (b) fn_batch_destroy(b);
    if (h_stat) (void)hipHostFree(h_stat);
    if (h_rows) (void)hipHostFree(h_rows);
    if (h_adm) (void)hipHostFree(h_adm);
  }
};

extern "C" {

fn_status fn_server_create(fn_model* m, int32_t max_slots, int64_t max_events_per_fit, int64_t budget_bytes,
                           fn_server** out) {
  fn_server* s = nullptr;
  const fn_status st = guard([&] {
    if (!m || !out) throw Error(FN_E_INVALID, "NULL argument");
    if (budget_bytes < 256) throw Error(FN_E_INVALID, "budget too small");
    s = new fn_server;
    s->m = m;
    const fn_status bs = fn_batch_create(m, max_slots, max_events_per_fit, &s->b);
    if (bs != FN_OK) throw Error(bs, fn_last_error());
    s->slots = max_slots;
    s->P = m->P;
    s->max_ev = max_events_per_fit;
    s->budget = budget_bytes;
    s->arena_mem.reserve((size_t)budget_bytes);
    s->arena.reset(budget_bytes);
    s->gen_count.reserve(sizeof(unsigned int));
    s->slot_req.assign(max_slots, -1);
    for (int k = max_slots - 1; k >= 0; --k) s->free_slots.push_back(k);  // lowest slot on top
    s->running.resize(max_slots);
    if (hipHostMalloc((void**)&s->h_stat, sizeof(int) * max_slots, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&s->h_rows, sizeof(double) * max_slots * (3 + 2 * s->P), hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void**)&s->h_adm, sizeof(AdmitRec) * max_slots, hipHostMallocDefault) != hipSuccess)
      throw Error(FN_E_NOMEM, "hipHostMalloc failed");
    *out = s;
  });
  if (st != FN_OK) delete s;
  return st;
}

fn_status fn_server_destroy(fn_server* s) {
  return guard([&] { delete s; });
}

fn_status fn_server_submit(fn_server* s, const fn_request* reqs, int32_t n) {
  return guard([&] {
    if (!s || (n > 0 && !reqs)) throw Error(FN_E_INVALID, "NULL argument");
    for (int i = 0; i < n; ++i) {
      Pending p;
      p.r = reqs[i];
      if (p.r.n_events < 1 || p.r.n_events > s->max_ev) throw Error(FN_E_INVALID, "request event count out of range");
      p.bytes = p.r.n_events * (int64_t)sizeof(double);
      s->queue.push_back(p);
    }
    std::stable_sort(s->queue.begin(), s->queue.end(),
                     [](const Pending& a, const Pending& c) { return a.r.arrival_s < c.r.arrival_s; });
  });
}

fn_status fn_server_run(fn_server* s, int32_t poll_every, double max_seconds, int32_t* n_done) {
  return guard([&] {
    if (!s) throw Error(FN_E_INVALID, "server is NULL");
    hip_check(hipSetDevice(s->m->device), "hipSetDevice");
    if (poll_every < 1) poll_every = 1;
    const Mix1dConst& mc = s->m->mix;
    const bool can_generate = mc.K == 2 && mc.type[0] == kGauss && mc.type[1] == kExp;
    if (!s->started) {
      s->t0 = std::chrono::steady_clock::now();
      s->started = true;
    }
    const auto t_call = std::chrono::steady_clock::now();
    auto now = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count(); };
    auto call_s = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_call).count(); };
    const int W = 3 + 2 * s->P;
    // fits still running from an earlier call that stopped on max_seconds
    int n_running = 0;
    for (int k = 0; k < s->slots; ++k) n_running += s->slot_req[k] >= 0;
    std::vector<int> fin_slots;
    std::vector<char> taken;
    while (true) {
      if (max_seconds > 0.0 && call_s() > max_seconds) break;
      const double t = now();
      // admission: arrivals visible now, in arrival order with backfilling,
      // while a slot is free and the events fit the budget; the round's
      // records go to the device in one copy and one launch (state reset,
      // status, event pointers, event generation)
      int n_adm = 0;
      int64_t gen_blocks = 0;
      taken.assign(s->queue.size(), 0);
      Pending* blocked = nullptr;  // earliest arrival that did not fit
      for (size_t i = 0; i < s->queue.size() && !s->free_slots.empty(); ++i) {
        Pending& p = s->queue[i];
        if (p.r.arrival_s > t) break;
        const double* ev = p.r.events;
        const bool gen = ev == nullptr;
        // generated events take whole 256-byte arena units
        if ((gen ? (p.bytes + 255) & ~int64_t(255) : p.bytes) > s->budget) {
          fn_result r;
          std::memset(&r, 0, sizeof(r));
          r.id = p.r.id;
          r.status = FN_E_BUDGET;
          r.t_arrival = p.r.arrival_s;
          r.t_admit = r.t_done = t;
          s->done.push_back(r);
          taken[i] = 1;
          continue;
        }
        if (gen && !can_generate) throw Error(FN_E_INVALID, "generation needs a (gauss, exp) mixture model");
        bool fits = s->in_use + p.bytes <= s->budget;
        int64_t off = -1;
        if (fits && gen) {
          off = s->arena.alloc(p.bytes);
          fits = off >= 0;
        }
        if (!fits) {
          if (!blocked) blocked = &p;
          continue;
        }
        if (blocked) {
          if (blocked->bypassed >= kMaxBypass) {
            if (off >= 0) s->arena.release(off, p.bytes);
            break;  // wait for the starved request
          }
          ++blocked->bypassed;
        }
        if (gen) ev = (const double*)((char*)s->arena_mem.ptr + off);
        p.off = off;
        s->in_use += p.bytes;
        const int slot = s->free_slots.back();
        s->free_slots.pop_back();
        AdmitRec& a = s->h_adm[n_adm++];
        a.slot = slot;
        a.generate = gen ? 1 : 0;
        a.n = p.r.n_events;
        a.ev = const_cast<double*>(ev);
        a.block0 = gen_blocks;
        a.seed = p.r.seed;
        a.fit = p.r.fit;
        for (int j = 0; j < 4; ++j) a.theta_gen[j] = p.r.theta_gen[j];
        for (int j = 0; j < kBatchMaxP; ++j) a.theta0[j] = j < s->P ? p.r.theta0[j] : 0.0;
        if (gen) gen_blocks += (p.r.n_events + kBlock - 1) / kBlock;
        p.t_admit = t;
        s->running[slot] = p;
        s->slot_req[slot] = 1;
        ++n_running;
        taken[i] = 1;
      }
      if (std::find(taken.begin(), taken.end(), 1) != taken.end()) {
        size_t w = 0;
        for (size_t i = 0; i < s->queue.size(); ++i)
          if (!taken[i]) s->queue[w++] = s->queue[i];
        s->queue.resize(w);
      }
      batch_admit_async(s->b, s->h_adm, n_adm, gen_blocks, mc.lo, mc.hi, (unsigned int*)s->gen_count.ptr);
      if (n_running == 0) {
        if (s->queue.empty()) break;
        // idle until the next arrival (a request that is still waiting here
        // has arrived and fits once nothing runs, so only a future arrival
        // can be pending)
        const double wait = s->queue.front().r.arrival_s - now();
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 1e-3)));
        continue;
      }
      batch_steps(s->b, poll_every);
      batch_poll(s->b, s->h_stat);
      fin_slots.clear();
      for (int k = 0; k < s->slots; ++k)
        if (s->slot_req[k] >= 0 && (s->h_stat[k] == kFitConverged || s->h_stat[k] == kFitFailed))
          fin_slots.push_back(k);
      if (!fin_slots.empty()) {
        batch_read_rows(s->b, fin_slots.data(), (int)fin_slots.size(), s->h_rows);
        const double td = now();
        for (size_t i = 0; i < fin_slots.size(); ++i) {
          const int k = fin_slots[i];
          Pending& p = s->running[k];
          const double* row = s->h_rows + i * W;
          fn_result r;
          std::memset(&r, 0, sizeof(r));
          r.id = p.r.id;
          r.status = s->h_stat[k];
          r.nll = row[0];
          r.iters = (int32_t)row[1];
          r.n_evals = (int32_t)row[2];
          for (int j = 0; j < s->P; ++j) {
            r.theta[j] = row[3 + j];
            r.errors[j] = row[3 + s->P + j];
          }
          r.t_arrival = p.r.arrival_s;
          r.t_admit = p.t_admit;
          r.t_done = td;
          s->done.push_back(r);
          if (p.off >= 0) s->arena.release(p.off, p.bytes);
          s->in_use -= p.bytes;
          s->slot_req[k] = -1;
          s->free_slots.push_back(k);
          --n_running;
        }
      }
    }
    // Requests admitted but unfinished when max_seconds ran out keep their
    // slots, memory and device state; the next fn_server_run continues them.
    if (n_done) *n_done = (int32_t)s->done.size();
  });
}

fn_status fn_server_results(fn_server* s, fn_result* out, int32_t max, int32_t* n_out) {
  return guard([&] {
    if (!s || (max > 0 && !out)) throw Error(FN_E_INVALID, "NULL argument");
    const int n = std::min<int>(max, (int)s->done.size());
    for (int i = 0; i < n; ++i) out[i] = s->done[i];
    if (n_out) *n_out = n;
  });
}

}  // extern "C"
