// Systematic-variation batches of the time-dependent four-body model: many
// fits of one event sample that differ in their fixed constants (lineshape
// masses and widths, time resolution) and start points, advanced together.
//
// One step = for every running fit: prologue (trial point -> table), the
// events pass (one workgroup per (event chunk, fit), fits fastest so the
// workgroups of a chunk share it through L2), the per-fit finalize (level-2 sum
// + normalization), and one BFGS state-machine step.  The per-fit
// normalization matrices M_f = <B_i conj(B_j)> over the phase-space sample are
// built once per batch (they depend on the fixed constants only).  A fit's
// partial rows are the same as the single-fit path's, so its NLL bits do not
// depend on the other fits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "bfgs_device.hpp"
#include "internal.hpp"

using namespace fn;

namespace {

constexpr int kVbMaxP = 4 * kTd4MaxAmp + 2;
using VState = BfgsStateT<kVbMaxP>;
static_assert(sizeof(VState) % sizeof(double) == 0, "trial points are read with a double stride");

void* pinned(size_t bytes) {
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) throw Error(FN_E_NOMEM, "hipHostMalloc failed");
  std::memset(p, 0, bytes);
  return p;
}

}  // namespace

struct fn_vbatch {
  fn_model* m = nullptr;
  int F = 0;
  int P = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ready = nullptr;
  hipGraphExec_t exec = nullptr;
  const double* g_ev = nullptr;  // the event sample the graph was captured for
  int64_t g_n = -1, g_ld = -1;
  double g_tol = 0.0;
  int g_iter = 0;
  bool M_valid = false;
  int64_t mc_gen = -1;           // normalization sample the matrices were built from
  DevBuf fc, tabs, Mc, part, mpart, out, theta, st, stat, rres, sel;
  Td4FitConst* h_fc = nullptr;
  VState* h_st = nullptr;
  double* h_theta = nullptr;
  double* h_out = nullptr;
  int* h_stat = nullptr;
  int* h_sel = nullptr;  // serving: fits admitted in one round

  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
  }
  ~fn_vbatch() {
    drop_graph();
    if (ready) (void)hipEventDestroy(ready);
    if (stream) (void)hipStreamDestroy(stream);
    if (h_fc) (void)hipHostFree(h_fc);
    if (h_st) (void)hipHostFree(h_st);
    if (h_theta) (void)hipHostFree(h_theta);
    if (h_out) (void)hipHostFree(h_out);
    if (h_stat) (void)hipHostFree(h_stat);
    if (h_sel) (void)hipHostFree(h_sel);
  }
};

namespace {

// The caller's stream must have produced the events: order the batch stream after it.
void wait_caller(fn_vbatch* b, void* stream) {
  hip_check(hipEventRecord(b->ready, (hipStream_t)stream), "hipEventRecord");
  hip_check(hipStreamWaitEvent(b->stream, b->ready, 0), "hipStreamWaitEvent");
}

void check_events(fn_vbatch* b, const double* ev, int64_t n, int64_t ld) {
  if (n < 1) throw Error(FN_E_INVALID, "need at least one event");
  if (!ev) throw Error(FN_E_INVALID, "events pointer is NULL");
  if (ld < n) throw Error(FN_E_INVALID, "ld must be >= n");
  if (b->m->n_mc <= 0) throw Error(FN_E_INVALID, "td4: normalization sample not set (fn_model_set_norm_sample)");
}

void reserve_part(fn_vbatch* b, int64_t n) {
  const int64_t nch = (n + b->m->chunk - 1) / b->m->chunk;
  const void* before = b->part.ptr;
  b->part.reserve(sizeof(double) * (size_t)nch * b->F * td4_nv(b->m->td4, true));
  if (b->part.ptr != before) b->drop_graph();  // a captured step holds the old address
}

// Normalization matrices of every fit (tables must be current for the fixed constants).
void build_matrices(fn_vbatch* b) {
  fn_model* m = b->m;
  if (b->M_valid && b->mc_gen == m->mc_gen) return;
  const int mchunk = 1024;
  const int64_t rows = (m->n_mc + mchunk - 1) / mchunk;
  b->mpart.reserve(sizeof(double) * (size_t)rows * b->F * 2 * td4_row_block(m->td4.K) * td4_kmax(m->td4.K));
  td4_launch_mmatrix(*m->td4_jit, m->td4, (const Td4Table*)b->tabs.ptr, b->F, (const double*)m->d_mc.ptr, m->n_mc,
                     m->n_mc, mchunk, (double*)b->mpart.ptr, (double*)b->Mc.ptr, b->stream);
  hip_check(hipGetLastError(), "kernel launch");
  b->M_valid = true;
  b->mc_gen = m->mc_gen;
}

void upload_fixed(fn_vbatch* b) {
  hip_check(hipMemcpyAsync(b->fc.ptr, b->h_fc, sizeof(Td4FitConst) * b->F, hipMemcpyHostToDevice, b->stream),
            "hipMemcpyAsync");
}

void launch_step(fn_vbatch* b, const double* ev, int64_t n, int64_t ld, double tol, int max_iter) {
  fn_model* m = b->m;
  const Td4Const& tc = m->td4;
  const int64_t nch = (n + m->chunk - 1) / m->chunk;
  const int stride = (int)(sizeof(VState) / sizeof(double));
  auto* tabs = (Td4Table*)b->tabs.ptr;
  auto* stat = (const int*)b->stat.ptr;
  td4_launch_prologue(tc, nullptr, (const double*)b->st.ptr, stride, (const Td4FitConst*)b->fc.ptr, stat, b->F, tabs,
                      b->stream);
  td4_launch_events(*m->td4_jit, tc, tabs, stat, b->F, ev, ld, n, m->chunk, true, (double*)b->part.ptr,
                    b->stream);
  td4_launch_finalize(tc, tabs, stat, b->F, (const double*)b->part.ptr, nch, true, (const double*)b->Mc.ptr,
                      (double)n, (double*)b->out.ptr, 2 + 2 * b->P, nullptr, b->stream);
  bfgs_launch<kVbMaxP>((VState*)b->st.ptr, (const double*)b->out.ptr, 2 + 2 * b->P, b->F, b->P, tol, max_iter,
                       (int*)b->stat.ptr, (double*)b->rres.ptr, b->stream);
}

void step(fn_vbatch* b, bool use_graph, const double* ev, int64_t n, int64_t ld, double tol, int max_iter) {
  if (!use_graph) {
    launch_step(b, ev, n, ld, tol, max_iter);
    hip_check(hipGetLastError(), "kernel launch");
    return;
  }
  if (b->exec && (b->g_ev != ev || b->g_n != n || b->g_ld != ld || b->g_tol != tol || b->g_iter != max_iter))
    b->drop_graph();
  if (!b->exec) {
    hipGraph_t g = nullptr;
    hip_check(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    launch_step(b, ev, n, ld, tol, max_iter);
    hip_check(hipStreamEndCapture(b->stream, &g), "hipStreamEndCapture");
    const hipError_t e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    hip_check(e, "hipGraphInstantiate");
    b->g_ev = ev;
    b->g_n = n;
    b->g_ld = ld;
    b->g_tol = tol;
    b->g_iter = max_iter;
  }
  hip_check(hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch");
}

}  // namespace

extern "C" {

fn_status fn_vbatch_create(fn_model* m, int32_t n_fits, fn_vbatch** out) {
  fn_vbatch* b = nullptr;
  const fn_status st = guard([&] {
    if (!m || !out) throw Error(FN_E_INVALID, "NULL argument");
    if (m->kind != kKindTd4) throw Error(FN_E_INVALID, "variation batches support td4 models");
    if (n_fits < 1 || n_fits > 4096) throw Error(FN_E_INVALID, "n_fits must be in [1, 4096]");
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    b = new fn_vbatch;
    b->m = m;
    b->F = n_fits;
    b->P = m->P;
    hip_check(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking), "hipStreamCreate");
    hip_check(hipEventCreateWithFlags(&b->ready, hipEventDisableTiming), "hipEventCreate");
    b->fc.reserve(sizeof(Td4FitConst) * n_fits);
    b->tabs.reserve(sizeof(Td4Table) * n_fits);
    b->Mc.reserve(sizeof(double) * 2 * kTd4MaxAmp * kTd4MaxAmp * n_fits);
    b->out.reserve(sizeof(double) * (size_t)n_fits * (2 + 2 * b->P));
    b->theta.reserve(sizeof(double) * (size_t)n_fits * b->P);
    b->st.reserve(sizeof(VState) * n_fits);
    b->stat.reserve(sizeof(int) * n_fits);
    b->rres.reserve(sizeof(double) * (size_t)n_fits * (3 + 2 * b->P));
    b->h_fc = (Td4FitConst*)pinned(sizeof(Td4FitConst) * n_fits);
    b->h_st = (VState*)pinned(sizeof(VState) * n_fits);
    b->h_theta = (double*)pinned(sizeof(double) * (size_t)n_fits * b->P);
    b->h_out = (double*)pinned(sizeof(double) * (size_t)n_fits * (2 + 2 * b->P));
    b->h_stat = (int*)pinned(sizeof(int) * n_fits);
    b->h_sel = (int*)pinned(sizeof(int) * n_fits);
    b->sel.reserve(sizeof(int) * n_fits);
    const Td4FitConst dflt = td4_fit_const(m->td4, m->fixed_ls.data());
    for (int f = 0; f < n_fits; ++f) b->h_fc[f] = dflt;
    *out = b;
  });
  if (st != FN_OK) delete b;
  return st;
}

fn_status fn_vbatch_destroy(fn_vbatch* b) {
  return guard([&] {
    if (b) {
      (void)hipStreamSynchronize(b->stream);
      delete b;
    }
  });
}

fn_status fn_vbatch_set_fixed(fn_vbatch* b, int32_t fit, const double* fixed_host) {
  return guard([&] {
    if (!b) throw Error(FN_E_INVALID, "batch is NULL");
    if (fit < 0 || fit >= b->F) throw Error(FN_E_INVALID, "fit index out of range");
    const Td4FitConst fc = td4_fit_const(b->m->td4, fixed_host ? fixed_host : b->m->fixed_ls.data());
    hip_check(hipSetDevice(b->m->device), "hipSetDevice");
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");  // staging may be in flight
    b->h_fc[fit] = fc;
    b->M_valid = false;
  });
}

fn_status fn_vbatch_nll(fn_vbatch* b, const double* theta_host, const double* ev, int64_t n, int64_t ld,
                        double* nll_host, double* grad_host, void* stream) {
  return guard([&] {
    if (!b || !theta_host) throw Error(FN_E_INVALID, "NULL argument");
    check_events(b, ev, n, ld);
    fn_model* m = b->m;
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    const int F = b->F, P = b->P;
    std::memcpy(b->h_theta, theta_host, sizeof(double) * (size_t)F * P);
    wait_caller(b, stream);
    upload_fixed(b);
    hip_check(hipMemcpyAsync(b->theta.ptr, b->h_theta, sizeof(double) * (size_t)F * P, hipMemcpyHostToDevice,
                             b->stream),
              "hipMemcpyAsync");
    auto* tabs = (Td4Table*)b->tabs.ptr;
    const bool grad = grad_host != nullptr;
    reserve_part(b, n);
    td4_launch_prologue(m->td4, nullptr, (const double*)b->theta.ptr, P, (const Td4FitConst*)b->fc.ptr, nullptr, F,
                        tabs, b->stream);
    build_matrices(b);
    td4_launch_events(*m->td4_jit, m->td4, tabs, nullptr, F, ev, ld, n, m->chunk, grad, (double*)b->part.ptr,
                      b->stream);
    const int64_t nch = (n + m->chunk - 1) / m->chunk;
    td4_launch_finalize(m->td4, tabs, nullptr, F, (const double*)b->part.ptr, nch, grad, (const double*)b->Mc.ptr,
                        (double)n, (double*)b->out.ptr, 2 + 2 * P, nullptr, b->stream);
    hip_check(hipGetLastError(), "kernel launch");
    hip_check(hipMemcpyAsync(b->h_out, b->out.ptr, sizeof(double) * (size_t)F * (2 + 2 * P), hipMemcpyDeviceToHost,
                             b->stream),
              "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    bool bad = false;
    for (int f = 0; f < F; ++f) {
      const double* o = b->h_out + (size_t)f * (2 + 2 * P);
      if (nll_host) nll_host[f] = o[0];
      bad |= !std::isfinite(o[0]);
      if (grad)
        for (int i = 0; i < P; ++i) grad_host[(size_t)f * P + i] = o[1 + i];
    }
    if (bad) throw Error(FN_E_NONFINITE, "NLL is not finite for at least one fit");
  });
}

fn_status fn_vbatch_fit(fn_vbatch* b, const double* theta0_host, const int32_t* free_mask, const double* ev,
                        int64_t n, int64_t ld, double tol, int32_t max_iter, int32_t use_graph, int32_t* status_out,
                        double* theta_out, double* err_out, double* nll_out, int32_t* iters_out,
                        int32_t* n_evals_out, void* stream) {
  return guard([&] {
    if (!b || !theta0_host) throw Error(FN_E_INVALID, "NULL argument");
    check_events(b, ev, n, ld);
    fn_model* m = b->m;
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    const int F = b->F, P = b->P;
    if (tol <= 0.0) tol = 1e-7;
    if (max_iter <= 0) max_iter = 500;
    for (int f = 0; f < F; ++f) {
      VState& s = b->h_st[f];
      std::memset(&s, 0, sizeof(s));
      for (int i = 0; i < P; ++i) {
        s.xt[i] = theta0_host[(size_t)f * P + i];
        s.mask[i] = free_mask ? (free_mask[i] != 0) : 1;
      }
      s.status = kFitRunning;
      s.phase = kPhaseStart;
      b->h_stat[f] = kFitRunning;
    }
    wait_caller(b, stream);
    upload_fixed(b);
    hip_check(hipMemcpyAsync(b->st.ptr, b->h_st, sizeof(VState) * F, hipMemcpyHostToDevice, b->stream),
              "hipMemcpyAsync");
    hip_check(hipMemcpyAsync(b->stat.ptr, b->h_stat, sizeof(int) * F, hipMemcpyHostToDevice, b->stream),
              "hipMemcpyAsync");
    reserve_part(b, n);
    if (!(b->M_valid && b->mc_gen == m->mc_gen)) {
      // tables for the matrices: lineshape constants only depend on the fixed constants
      td4_launch_prologue(m->td4, nullptr, (const double*)b->st.ptr, (int)(sizeof(VState) / sizeof(double)),
                          (const Td4FitConst*)b->fc.ptr, nullptr, F, (Td4Table*)b->tabs.ptr, b->stream);
      build_matrices(b);
    }
    const long max_steps = (long)max_iter * (kMaxLineSearch + 2) + 2;
    const int poll_every = 8;
    long done = 0;
    for (;;) {
      for (int i = 0; i < poll_every; ++i) step(b, use_graph != 0, ev, n, ld, tol, max_iter);
      done += poll_every;
      hip_check(hipMemcpyAsync(b->h_stat, b->stat.ptr, sizeof(int) * F, hipMemcpyDeviceToHost, b->stream),
                "hipMemcpyAsync");
      hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
      int running = 0;
      for (int f = 0; f < F; ++f) running += b->h_stat[f] == kFitRunning;
      if (running == 0 || done >= max_steps) break;
    }
    std::vector<VState> hs(F);
    hip_check(hipMemcpyAsync(hs.data(), b->st.ptr, sizeof(VState) * F, hipMemcpyDeviceToHost, b->stream),
              "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    for (int f = 0; f < F; ++f) {
      const VState& s = hs[f];
      if (status_out) status_out[f] = s.status;
      if (nll_out) nll_out[f] = s.f;
      if (iters_out) iters_out[f] = s.iter;
      if (n_evals_out) n_evals_out[f] = s.n_eval;
      for (int i = 0; i < P; ++i) {
        if (theta_out) theta_out[(size_t)f * P + i] = s.x[i];
        if (err_out) err_out[(size_t)f * P + i] = s.mask[i] ? std::sqrt(std::fabs(s.H[i * kVbMaxP + i])) : 0.0;
      }
    }
  });
}

fn_status fn_vbatch_serve(fn_vbatch* b, const fn_vrequest* reqs, int32_t n_req, const int32_t* free_mask,
                          const double* ev, int64_t n, int64_t ld, double tol, int32_t max_iter, int32_t poll_every,
                          int32_t* status_out, double* theta_out, double* err_out, double* nll_out,
                          int32_t* iters_out, int32_t* n_evals_out, double* t_admit_out, double* t_done_out,
                          void* stream) {
  return guard([&] {
    if (!b || (n_req > 0 && !reqs)) throw Error(FN_E_INVALID, "NULL argument");
    if (n_req < 0) throw Error(FN_E_INVALID, "n_req must be >= 0");
    check_events(b, ev, n, ld);
    fn_model* m = b->m;
    const Td4Const& tc = m->td4;
    const int F = b->F, P = b->P;
    if (tol <= 0.0) tol = 1e-7;
    if (max_iter <= 0) max_iter = 500;
    if (poll_every < 1) poll_every = 1;
    // every request's constants are checked before anything runs
    std::vector<Td4FitConst> fcs(n_req);
    std::vector<int> order(n_req);
    for (int r = 0; r < n_req; ++r) {
      if (!reqs[r].theta0) throw Error(FN_E_INVALID, "request without a start point");
      if (!(reqs[r].arrival_s >= 0.0) || !std::isfinite(reqs[r].arrival_s))
        throw Error(FN_E_INVALID, "arrival times must be finite and >= 0");
      fcs[r] = td4_fit_const(tc, reqs[r].fixed ? reqs[r].fixed : m->fixed_ls.data());
      order[r] = r;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return reqs[a].arrival_s < reqs[c].arrival_s; });
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    wait_caller(b, stream);
    reserve_part(b, n);
    // every slot idle; a slot's matrix is built when a request is admitted to it
    std::vector<int> slot_req(F, -1), free_slots;
    for (int f = F - 1; f >= 0; --f) free_slots.push_back(f);
    for (int f = 0; f < F; ++f) b->h_stat[f] = kFitIdle;
    hip_check(hipMemcpyAsync(b->stat.ptr, b->h_stat, sizeof(int) * F, hipMemcpyHostToDevice, b->stream),
              "hipMemcpyAsync");
    b->M_valid = false;  // the matrices no longer follow fn_vbatch_set_fixed
    const int stride = (int)(sizeof(VState) / sizeof(double));
    const auto t0 = std::chrono::steady_clock::now();
    auto now = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    std::vector<double> t_admit(n_req, -1.0);
    VState done_state;
    int next = 0, n_running = 0;
    std::vector<int> fin;
    while (true) {
      // admission at a step boundary: arrivals visible now, in arrival order, into free slots
      const double t = now();
      int n_adm = 0;
      for (int f = 0; f < F; ++f) b->h_sel[f] = 0;
      while (next < n_req && !free_slots.empty() && reqs[order[next]].arrival_s <= t) {
        const int r = order[next++];
        const int f = free_slots.back();
        free_slots.pop_back();
        b->h_fc[f] = fcs[r];
        VState& st = b->h_st[f];
        std::memset(&st, 0, sizeof(st));
        for (int i = 0; i < P; ++i) {
          st.xt[i] = reqs[r].theta0[i];
          st.mask[i] = free_mask ? (free_mask[i] != 0) : 1;
        }
        st.status = kFitRunning;
        st.phase = kPhaseStart;
        b->h_stat[f] = kFitRunning;
        b->h_sel[f] = 1;
        slot_req[f] = r;
        t_admit[r] = t;
        ++n_adm;
        ++n_running;
        hip_check(hipMemcpyAsync((Td4FitConst*)b->fc.ptr + f, &b->h_fc[f], sizeof(Td4FitConst),
                                 hipMemcpyHostToDevice, b->stream), "hipMemcpyAsync");
        hip_check(hipMemcpyAsync((VState*)b->st.ptr + f, &b->h_st[f], sizeof(VState), hipMemcpyHostToDevice,
                                 b->stream), "hipMemcpyAsync");
        hip_check(hipMemcpyAsync((int*)b->stat.ptr + f, &b->h_stat[f], sizeof(int), hipMemcpyHostToDevice,
                                 b->stream), "hipMemcpyAsync");
      }
      if (n_adm > 0) {
        // the admitted fits' tables (their lineshape constants) and normalization matrices
        hip_check(hipMemcpyAsync(b->sel.ptr, b->h_sel, sizeof(int) * F, hipMemcpyHostToDevice, b->stream),
                  "hipMemcpyAsync");
        const int* sel = (const int*)b->sel.ptr;
        td4_launch_prologue(tc, nullptr, (const double*)b->st.ptr, stride, (const Td4FitConst*)b->fc.ptr, sel, F,
                            (Td4Table*)b->tabs.ptr, b->stream);
        const int mchunk = 1024;
        const int64_t rows = (m->n_mc + mchunk - 1) / mchunk;
        b->mpart.reserve(sizeof(double) * (size_t)rows * F * 2 * td4_row_block(tc.K) * td4_kmax(tc.K));
        td4_launch_mmatrix(*m->td4_jit, tc, (const Td4Table*)b->tabs.ptr, F, (const double*)m->d_mc.ptr, m->n_mc,
                           m->n_mc, mchunk, (double*)b->mpart.ptr, (double*)b->Mc.ptr, b->stream, sel);
        hip_check(hipGetLastError(), "kernel launch");
        // the pinned staging of this round must not change before the copies ran
        hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
      }
      if (n_running == 0) {
        if (next >= n_req) break;
        const double wait = reqs[order[next]].arrival_s - now();
        if (wait > 0) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 1e-3)));
        continue;
      }
      for (int i = 0; i < poll_every; ++i) step(b, true, ev, n, ld, tol, max_iter);
      hip_check(hipMemcpyAsync(b->h_stat, b->stat.ptr, sizeof(int) * F, hipMemcpyDeviceToHost, b->stream),
                "hipMemcpyAsync");
      hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
      fin.clear();
      for (int f = 0; f < F; ++f)
        if (slot_req[f] >= 0 && (b->h_stat[f] == kFitConverged || b->h_stat[f] == kFitFailed)) fin.push_back(f);
      if (fin.empty()) continue;
      const double td = now();
      for (int f : fin) {
        hip_check(hipMemcpyAsync(&done_state, (VState*)b->st.ptr + f, sizeof(VState), hipMemcpyDeviceToHost,
                                 b->stream), "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
        const int r = slot_req[f];
        const VState& st = done_state;
        if (status_out) status_out[r] = st.status;
        if (nll_out) nll_out[r] = st.f;
        if (iters_out) iters_out[r] = st.iter;
        if (n_evals_out) n_evals_out[r] = st.n_eval;
        for (int i = 0; i < P; ++i) {
          if (theta_out) theta_out[(size_t)r * P + i] = st.x[i];
          if (err_out) err_out[(size_t)r * P + i] = st.mask[i] ? std::sqrt(std::fabs(st.H[i * kVbMaxP + i])) : 0.0;
        }
        if (t_admit_out) t_admit_out[r] = t_admit[r];
        if (t_done_out) t_done_out[r] = td;
        slot_req[f] = -1;
        free_slots.push_back(f);
        --n_running;
      }
    }
  });
}

}  // extern "C"
