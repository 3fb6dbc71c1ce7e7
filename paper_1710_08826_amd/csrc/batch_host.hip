// Host side of batched fits (fn_batch_*) and device toy generation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "batch.hpp"
#include "internal.hpp"

using namespace fn;

struct fn_batch {
  fn_model* m = nullptr;
  int max_fits = 0;
  int64_t max_ev = 0;
  int P = 0;
  int chunk = 0;
  int64_t rows_per_slot = 0;
  int eval_grid = 0;
  double tol = 1e-7;
  int max_iter = 500;
  bool use_graph = true;
  hipStream_t stream = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t step_done = nullptr;  // recorded after each fn_batch_step outside a capture
  bool step_pending = false;
  DevBuf st, tabs, evp, nev, item_base, part_base, part, out, nrun, stat, rres;
  DevBuf adm, fin_slots, fin_rows;  // serving: admission records, finished-slot list and gathered rows
  // pinned staging of per-slot inputs (stable sources for async copies)
  BfgsState* h_st = nullptr;
  const double** h_ev = nullptr;
  int64_t* h_nev = nullptr;
  int* h_nrun = nullptr;
  int* h_fin = nullptr;  // finished-slot list staging
  BatchDev dev() {
    BatchDev d;
    d.st = (BfgsState*)st.ptr;
    d.tabs = (Mix1dTable*)tabs.ptr;
    d.ev = (const double**)evp.ptr;
    d.nev = (int64_t*)nev.ptr;
    d.item_base = (int64_t*)item_base.ptr;
    d.part_base = (int64_t*)part_base.ptr;
    d.part = (double*)part.ptr;
    d.out = (double*)out.ptr;
    d.n_running = (int*)nrun.ptr;
    d.stat = (int*)stat.ptr;
    d.rres = (double*)rres.ptr;
    return d;
  }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
  }
  ~fn_batch() {
    drop_graph();
    if (step_done) (void)hipEventDestroy(step_done);
    if (stream) (void)hipStreamDestroy(stream);
    if (h_st) (void)hipHostFree(h_st);
    if (h_ev) (void)hipHostFree(h_ev);
    if (h_nev) (void)hipHostFree(h_nev);
    if (h_nrun) (void)hipHostFree(h_nrun);
    if (h_fin) (void)hipHostFree(h_fin);
  }
};

static void* pinned(size_t bytes) {
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) throw Error(FN_E_NOMEM, "hipHostMalloc failed");
  std::memset(p, 0, bytes);
  return p;
}

// The step graph (the five step launches captured once on the batch stream).
static hipGraphExec_t step_graph(fn_batch* b) {
  if (!b->exec) {
    hipGraph_t g = nullptr;
    hip_check(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    batch_launch_step(b->dev(), b->m->mix, b->max_fits, b->P, b->chunk, b->eval_grid, b->tol, b->max_iter,
                      b->stream);
    hip_check(hipStreamEndCapture(b->stream, &g), "hipStreamEndCapture");
    const hipError_t e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    hip_check(e, "hipGraphInstantiate");
  }
  return b->exec;
}

static void step(fn_batch* b) {
  if (b->use_graph) {
    hip_check(hipGraphLaunch(step_graph(b), b->stream), "hipGraphLaunch");
  } else {
    batch_launch_step(b->dev(), b->m->mix, b->max_fits, b->P, b->chunk, b->eval_grid, b->tol, b->max_iter,
                      b->stream);
    hip_check(hipGetLastError(), "kernel launch");
  }
}

// Work on the batch stream starts after the steps fn_batch_step enqueued on
// caller streams.
static void after_caller_steps(fn_batch* b) {
  if (b->step_pending) {
    hip_check(hipStreamWaitEvent(b->stream, b->step_done, 0), "hipStreamWaitEvent");
    b->step_pending = false;
  }
}

extern "C" {

fn_status fn_batch_create(fn_model* m, int32_t max_fits, int64_t max_events_per_fit, fn_batch** out) {
  fn_batch* b = nullptr;
  const fn_status st = guard([&] {
    if (!m || !out) throw Error(FN_E_INVALID, "NULL argument");
    if (m->kind != kKindMix1d) throw Error(FN_E_INVALID, "batches support mix1d models");
    if (m->P > kBatchMaxP) throw Error(FN_E_INVALID, "batched fits take at most 24 parameters");
    if (max_fits < 1 || max_fits > (1 << 20)) throw Error(FN_E_INVALID, "max_fits out of range");
    if (max_events_per_fit < 1) throw Error(FN_E_INVALID, "max_events_per_fit must be >= 1");
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    b = new fn_batch;
    b->m = m;
    b->max_fits = max_fits;
    b->max_ev = max_events_per_fit;
    b->P = m->P;
    b->chunk = m->chunk;
    b->rows_per_slot = (max_events_per_fit + m->chunk - 1) / m->chunk;
    const int kmax = mix1d_kmax(m->mix.K);
    const int nv = mix1d_nv(kmax, true);
    hip_check(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking), "hipStreamCreate");
    b->st.reserve(sizeof(BfgsState) * max_fits);
    b->tabs.reserve(sizeof(Mix1dTable) * max_fits);
    b->evp.reserve(sizeof(double*) * max_fits);
    b->nev.reserve(sizeof(int64_t) * max_fits);
    b->item_base.reserve(sizeof(int64_t) * (max_fits + 1));
    b->part_base.reserve(sizeof(int64_t) * max_fits);
    b->part.reserve(sizeof(double) * (size_t)b->rows_per_slot * max_fits * nv);
    b->out.reserve(sizeof(double) * (size_t)max_fits * (2 + 2 * b->P));
    b->nrun.reserve(sizeof(int));
    b->stat.reserve(sizeof(int) * max_fits);
    b->rres.reserve(sizeof(double) * (size_t)max_fits * (3 + 2 * b->P));
    hip_check(hipMemsetAsync(b->stat.ptr, 0, sizeof(int) * max_fits, b->stream), "hipMemsetAsync");
    b->h_st = (BfgsState*)pinned(sizeof(BfgsState) * max_fits);
    b->h_ev = (const double**)pinned(sizeof(double*) * max_fits);
    b->h_nev = (int64_t*)pinned(sizeof(int64_t) * max_fits);
    b->h_nrun = (int*)pinned(sizeof(int));
    b->h_fin = (int*)pinned(sizeof(int) * max_fits);
    std::vector<int64_t> pb(max_fits);
    for (int f = 0; f < max_fits; ++f) pb[f] = (int64_t)f * b->rows_per_slot;
    // all slots idle, no events
    hip_check(hipMemcpyAsync(b->st.ptr, b->h_st, sizeof(BfgsState) * max_fits, hipMemcpyHostToDevice, b->stream),
              "hipMemcpyAsync");
    hip_check(hipMemcpyAsync(b->evp.ptr, b->h_ev, sizeof(double*) * max_fits, hipMemcpyHostToDevice, b->stream),
              "hipMemcpyAsync");
    hip_check(hipMemcpyAsync(b->nev.ptr, b->h_nev, sizeof(int64_t) * max_fits, hipMemcpyHostToDevice, b->stream),
              "hipMemcpyAsync");
    hip_check(hipMemcpyAsync(b->part_base.ptr, pb.data(), sizeof(int64_t) * max_fits, hipMemcpyHostToDevice,
                             b->stream),
              "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    int cus = 0;
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device), "hipDeviceGetAttribute");
    b->eval_grid = cus * batch_eval_blocks_per_cu(m->mix);
    *out = b;
  });
  if (st != FN_OK) delete b;
  return st;
}

fn_status fn_batch_destroy(fn_batch* b) {
  return guard([&] {
    if (b) {
      if (b->step_pending) (void)hipEventSynchronize(b->step_done);
      (void)hipStreamSynchronize(b->stream);
      delete b;
    }
  });
}

fn_status fn_batch_config(fn_batch* b, double tol, int32_t max_iter, int32_t use_graph) {
  return guard([&] {
    if (!b) throw Error(FN_E_INVALID, "batch is NULL");
    b->tol = tol > 0.0 ? tol : 1e-7;
    b->max_iter = max_iter > 0 ? max_iter : 500;
    b->use_graph = use_graph != 0;
    // a step graph launched on a caller stream may still run
    if (b->step_pending) hip_check(hipEventSynchronize(b->step_done), "hipEventSynchronize");
    b->step_pending = false;
    b->drop_graph();
  });
}

fn_status fn_batch_set_slot(fn_batch* b, int32_t slot, const double* ev, int64_t n, const double* theta0,
                            const int32_t* free_mask) {
  return guard([&] {
    if (!b || !theta0) throw Error(FN_E_INVALID, "NULL argument");
    if (slot < 0 || slot >= b->max_fits) throw Error(FN_E_INVALID, "slot out of range");
    if (n < 1 || n > b->max_ev) throw Error(FN_E_INVALID, "event count must be in [1, max_events_per_fit]");
    if (!ev) throw Error(FN_E_INVALID, "events pointer is NULL");
    hip_check(hipSetDevice(b->m->device), "hipSetDevice");
    after_caller_steps(b);
    // the previous copy out of this staging entry must have completed
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    BfgsState& s = b->h_st[slot];
    std::memset(&s, 0, sizeof(s));
    for (int i = 0; i < b->P; ++i) {
      s.xt[i] = theta0[i];
      s.mask[i] = free_mask ? (free_mask[i] != 0) : 1;
    }
    s.status = kFitRunning;
    s.phase = kPhaseStart;
    b->h_ev[slot] = ev;
    b->h_nev[slot] = n;
    hip_check(hipMemcpyAsync((BfgsState*)b->st.ptr + slot, &s, sizeof(BfgsState), hipMemcpyHostToDevice, b->stream),
              "hipMemcpyAsync");
    // the per-slot status mirror is what the step kernels consult
    hip_check(hipMemcpyAsync((int*)b->stat.ptr + slot, &s.status, sizeof(int), hipMemcpyHostToDevice, b->stream),
              "hipMemcpyAsync");
    hip_check(hipMemcpyAsync((const double**)b->evp.ptr + slot, &b->h_ev[slot], sizeof(double*),
                             hipMemcpyHostToDevice, b->stream),
              "hipMemcpyAsync");
    hip_check(hipMemcpyAsync((int64_t*)b->nev.ptr + slot, &b->h_nev[slot], sizeof(int64_t), hipMemcpyHostToDevice,
                             b->stream),
              "hipMemcpyAsync");
  });
}

fn_status fn_batch_clear_slot(fn_batch* b, int32_t slot) {
  return guard([&] {
    if (!b) throw Error(FN_E_INVALID, "batch is NULL");
    if (slot < 0 || slot >= b->max_fits) throw Error(FN_E_INVALID, "slot out of range");
    hip_check(hipSetDevice(b->m->device), "hipSetDevice");
    after_caller_steps(b);
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    // status lives at a fixed offset: write only that int
    b->h_st[slot].status = kFitIdle;
    hip_check(hipMemcpyAsync(&((BfgsState*)b->st.ptr)[slot].status, &b->h_st[slot].status, sizeof(int),
                             hipMemcpyHostToDevice, b->stream),
              "hipMemcpyAsync");
    hip_check(hipMemcpyAsync((int*)b->stat.ptr + slot, &b->h_st[slot].status, sizeof(int), hipMemcpyHostToDevice,
                             b->stream),
              "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  });
}

fn_status fn_batch_run(fn_batch* b, int32_t max_steps, int32_t poll_every, int32_t* steps_done,
                       int32_t* n_running) {
  return guard([&] {
    if (!b) throw Error(FN_E_INVALID, "batch is NULL");
    hip_check(hipSetDevice(b->m->device), "hipSetDevice");
    after_caller_steps(b);
    if (poll_every < 1) poll_every = 1;
    int done = 0;
    int running = -1;
    while (done < max_steps) {
      const int k = std::min(poll_every, max_steps - done);
      for (int i = 0; i < k; ++i) step(b);
      done += k;
      hip_check(hipMemcpyAsync(b->h_nrun, b->nrun.ptr, sizeof(int), hipMemcpyDeviceToHost, b->stream),
                "hipMemcpyAsync");
      hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
      running = *b->h_nrun;
      if (running == 0) break;
    }
    if (steps_done) *steps_done = done;
    if (n_running) *n_running = running;
  });
}

fn_status fn_batch_results(fn_batch* b, int32_t* status, double* theta, double* nll, double* errors,
                           int32_t* iters, int32_t* n_evals) {
  return guard([&] {
    if (!b) throw Error(FN_E_INVALID, "batch is NULL");
    hip_check(hipSetDevice(b->m->device), "hipSetDevice");
    after_caller_steps(b);
    std::vector<BfgsState> hs(b->max_fits);
    hip_check(hipMemcpyAsync(hs.data(), b->st.ptr, sizeof(BfgsState) * b->max_fits, hipMemcpyDeviceToHost,
                             b->stream),
              "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    const int P = b->P;
    for (int f = 0; f < b->max_fits; ++f) {
      const BfgsState& s = hs[f];
      if (status) status[f] = s.status;
      if (theta)
        for (int i = 0; i < P; ++i) theta[(size_t)f * P + i] = s.x[i];
      if (nll) nll[f] = s.f;
      if (errors)
        for (int i = 0; i < P; ++i)
          errors[(size_t)f * P + i] = s.mask[i] ? std::sqrt(std::fabs(s.H[i * kBatchMaxP + i])) : 0.0;
      if (iters) iters[f] = s.iter;
      if (n_evals) n_evals[f] = s.n_eval;
    }
  });
}

fn_status fn_batch_set(fn_batch* b, int32_t n_fits, const double* const* ev, const int64_t* n, const int64_t* ld,
                       const double* theta0_dev) {
  return guard([&] {
    if (!b) throw Error(FN_E_INVALID, "batch is NULL");
    if (n_fits < 0 || n_fits > b->max_fits) throw Error(FN_E_INVALID, "n_fits must be in [0, max_fits]");
    if (n_fits > 0 && (!ev || !n || !theta0_dev)) throw Error(FN_E_INVALID, "NULL argument");
    for (int f = 0; f < n_fits; ++f) {
      if (n[f] < 1 || n[f] > b->max_ev)
        throw Error(FN_E_INVALID, "fit " + std::to_string(f) + ": event count must be in [1, max_events_per_fit]");
      if (!ev[f]) throw Error(FN_E_INVALID, "fit " + std::to_string(f) + ": events pointer is NULL");
      if (ld && ld[f] < n[f]) throw Error(FN_E_INVALID, "fit " + std::to_string(f) + ": ld must be >= n");
    }
    hip_check(hipSetDevice(b->m->device), "hipSetDevice");
    after_caller_steps(b);
    // the staging arrays may still feed an earlier copy
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    for (int f = 0; f < b->max_fits; ++f) {
      b->h_ev[f] = f < n_fits ? ev[f] : nullptr;
      b->h_nev[f] = f < n_fits ? n[f] : 0;
    }
    hip_check(hipMemcpyAsync(b->evp.ptr, b->h_ev, sizeof(double*) * b->max_fits, hipMemcpyHostToDevice, b->stream),
              "hipMemcpyAsync");
    hip_check(hipMemcpyAsync(b->nev.ptr, b->h_nev, sizeof(int64_t) * b->max_fits, hipMemcpyHostToDevice, b->stream),
              "hipMemcpyAsync");
    batch_launch_set(b->dev(), theta0_dev, n_fits, b->max_fits, b->P, b->stream);
    hip_check(hipGetLastError(), "kernel launch");
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  });
}

fn_status fn_batch_step(fn_batch* b, void* stream) {
  return guard([&] {
    if (!b) throw Error(FN_E_INVALID, "batch is NULL");
    hip_check(hipSetDevice(b->m->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hip_check(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing");
    if (cs == hipStreamCaptureStatusActive) {
      // recorded into the caller's graph: the step's kernels themselves
      batch_launch_step(b->dev(), b->m->mix, b->max_fits, b->P, b->chunk, b->eval_grid, b->tol, b->max_iter, s);
      hip_check(hipGetLastError(), "kernel launch");
      return;
    }
    if (b->use_graph) {
      hip_check(hipGraphLaunch(step_graph(b), s), "hipGraphLaunch");
    } else {
      batch_launch_step(b->dev(), b->m->mix, b->max_fits, b->P, b->chunk, b->eval_grid, b->tol, b->max_iter, s);
      hip_check(hipGetLastError(), "kernel launch");
    }
    if (!b->step_done) hip_check(hipEventCreateWithFlags(&b->step_done, hipEventDisableTiming), "hipEventCreate");
    hip_check(hipEventRecord(b->step_done, s), "hipEventRecord");
    b->step_pending = true;
  });
}

fn_status fn_batch_status(fn_batch* b, int32_t* status_host, double* theta_host, double* nll_host,
                          double* err_host) {
  return fn_batch_results(b, status_host, theta_host, nll_host, err_host, nullptr, nullptr);
}

fn_status fn_generate_mix1d(uint32_t seed, uint32_t fit, int64_t n, const double* theta_gen, double lo, double hi,
                            double* x, void* stream) {
  return guard([&] {
    if (!theta_gen) throw Error(FN_E_INVALID, "theta_gen is NULL");
    if (n < 0 || (n > 0 && !x)) throw Error(FN_E_INVALID, "bad output");
    if (!(hi > lo) || !(theta_gen[1] > 0.0)) throw Error(FN_E_INVALID, "need hi > lo and sigma > 0");
    if (n == 0) return;
    hipStream_t s = (hipStream_t)stream;
    DevBuf cnt;
    cnt.reserve(sizeof(unsigned int));
    hip_check(hipMemsetAsync(cnt.ptr, 0, sizeof(unsigned int), s), "hipMemsetAsync");
    batch_launch_gen_mix1d(seed, fit, 0u, n, theta_gen, lo, hi, x, (unsigned int*)cnt.ptr, s);
    hip_check(hipGetLastError(), "kernel launch");
    unsigned int bad = 0;
    hip_check(hipMemcpyAsync(&bad, cnt.ptr, sizeof(bad), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (bad) throw Error(FN_E_DOMAIN, std::to_string(bad) + " events not resolved within the attempt limit");
  });
}

}  // extern "C"

// ------------------------------------------------ internal hooks for serving
namespace fn {

hipStream_t batch_stream(fn_batch* b) { return b->stream; }
int batch_params(fn_batch* b) { return b->P; }
int batch_slots(fn_batch* b) { return b->max_fits; }

// Admit n records (staging entries in pinned host memory, left untouched
// until the caller has synchronised the batch stream) in one copy and one
// launch.
void batch_admit_async(fn_batch* b, const AdmitRec* recs_host, int n, int64_t gen_blocks, double lo, double hi,
                       unsigned int* n_unresolved) {
  if (n == 0) return;
  if (n > b->max_fits) throw Error(FN_E_INVALID, "more admissions than slots");
  b->adm.reserve(sizeof(AdmitRec) * (size_t)b->max_fits);
  hip_check(hipMemcpyAsync(b->adm.ptr, recs_host, sizeof(AdmitRec) * n, hipMemcpyHostToDevice, b->stream),
            "hipMemcpyAsync");
  batch_launch_admit(b->dev(), (const AdmitRec*)b->adm.ptr, n, gen_blocks, b->P, lo, hi, n_unresolved, b->stream);
  hip_check(hipGetLastError(), "kernel launch");
}

void batch_steps(fn_batch* b, int k) {
  for (int i = 0; i < k; ++i) step(b);
}

// Copy the per-slot status mirror to pinned host memory and wait.
void batch_poll(fn_batch* b, int* stat_host) {
  hip_check(hipMemcpyAsync(stat_host, b->stat.ptr, sizeof(int) * b->max_fits, hipMemcpyDeviceToHost, b->stream),
            "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
}

// Copy the result rows (3 + 2P doubles) of the given slots and wait: a few
// rows by one copy each, more by one gather launch and one copy.
void batch_read_rows(fn_batch* b, const int* slots, int n, double* rows_host) {
  const int w = 3 + 2 * b->P;
  if (n <= 2) {
    for (int i = 0; i < n; ++i)
      hip_check(hipMemcpyAsync(rows_host + (size_t)i * w, (double*)b->rres.ptr + (size_t)slots[i] * w,
                               sizeof(double) * w, hipMemcpyDeviceToHost, b->stream),
                "hipMemcpyAsync");
  } else {
    if (n > b->max_fits) throw Error(FN_E_INVALID, "more rows than slots");
    b->fin_slots.reserve(sizeof(int) * (size_t)b->max_fits);
    b->fin_rows.reserve(sizeof(double) * (size_t)b->max_fits * w);
    std::memcpy(b->h_fin, slots, sizeof(int) * n);
    hip_check(hipMemcpyAsync(b->fin_slots.ptr, b->h_fin, sizeof(int) * n, hipMemcpyHostToDevice, b->stream),
              "hipMemcpyAsync");
    batch_launch_gather_rows(b->dev(), (const int*)b->fin_slots.ptr, n, b->P, (double*)b->fin_rows.ptr, b->stream);
    hip_check(hipGetLastError(), "kernel launch");
    hip_check(hipMemcpyAsync(rows_host, b->fin_rows.ptr, sizeof(double) * (size_t)n * w, hipMemcpyDeviceToHost,
                             b->stream),
              "hipMemcpyAsync");
  }
  hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
}

}  // namespace fn
