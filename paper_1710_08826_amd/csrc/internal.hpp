// Host-side internals of libfitnll: error type, device buffers, the context
// and model objects behind the opaque C handles.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fitnll.h"
#include "kernels.hpp"
#include "model.hpp"
#include "td4.hpp"
#include "tddp.hpp"

namespace fn {

struct Error : std::runtime_error {
  fn_status code;
  Error(fn_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char* what);
void set_error(const std::string& s);
fn_status guard(const std::function<void()>& body);

// Grow-only device allocation.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  void reserve(size_t nbytes);
  void release();
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
};

enum ModelKind : int { kKindMix1d = 1, kKindDalitz3 = 2, kKindTd4 = 3, kKindTddp3 = 4 };

}  // namespace fn

struct fn_ctx {
  int device = 0;
  double* scratch = nullptr;  // this device's copy of the library's static scratch array
};

struct fn_model {
  fn_ctx* ctx = nullptr;
  int device = 0;
  int kind = 0;
  int P = 0;
  int n_obs = 0;
  int chunk = 1024;       // events per workgroup (defines the summation tree)
  int grid_chunk = 1024;  // grid cells per workgroup
  fn::Mix1dConst mix;
  fn::DalitzConst dal;
  fn::Td4Const td4;
  std::shared_ptr<fn::DalitzJit> dal_jit;  // structure-specialized passes
  int ept = 1;                              // dalitz3 events passes: events per thread and iteration
  std::shared_ptr<fn::DalitzJit> dal_jit2;  // their two-event form (built when first chosen)
  std::shared_ptr<fn::Td4Jit> td4_jit;
  std::shared_ptr<fn::TddpJit> tddp_jit;  // time-dependent Dalitz passes
  fn::TddpTime tdt;                        // its decay-time constants
  std::vector<double> fixed_ls;  // (m0, Gamma0) per resonance when not free; td4: fixed-constant vector
  int64_t n_mc = 0;              // td4 normalization sample size (0 = not set)
  int64_t mc_gen = 0;            // bumped whenever the sample is replaced
  bool M_valid = false;          // cached normalization matrix is current
  bool table_ready = false;      // fixed lineshapes: the table's lineshape constants are built
  fn::DevBuf d_table, d_part, d_npart, d_out, d_fixed, d_M, d_count, d_mc, d_gen;
  fn::DevBuf d_cells;            // dalitz3, free lineshapes: the grid cells inside the region (GridCell)
  int64_t n_inside = 0;          // their number
  double box[4] = {0.0, 0.0, 0.0, 0.0};  // Dalitz: kinematic box (s12 lo, hi, s13 lo, hi)
  fn::DevBuf d_theta;                    // tddp3: theta on the device for host-theta calls
  double* h_out = nullptr;       // pinned
  long long stats_calls = 0;
  int timing = 0;                // time every timing-th event-pass launch with HIP events (0 = off,
                                 // -1: in-kernel spans of every Dalitz event-pass launch into d_span)
  fn::DevBuf d_span;             // span record (sum of spans, launches), then two stamps per workgroup
  double span_khz = 0.0;         // device wall-clock rate
  int64_t timing_count = 0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
  hipEvent_t take_event();
  // Whether this event-pass launch is one of the timed ones.
  bool timed_launch() { return timing > 0 && timing_count++ % timing == 0; }
  // Issues an event-pass launch, launch(t0, t1): when it is one of the timed
  // ones, t0 and t1 are events that the dispatch fills with the kernel's own
  // start and end times (queued for fn_model_kernel_time once the launch has
  // been issued, back to the pool if it throws); otherwise both are null.
  template <class F>
  void timed(bool launches, F&& launch) {
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (launches && timed_launch()) {
      t0 = take_event();
      t1 = take_event();
    }
    try {
      launch(t0, t1);
    } catch (...) {
      if (t0) {
        ev_pool.push_back(t0);
        ev_pool.push_back(t1);
      }
      throw;
    }
    if (t0) ev_pending.emplace_back(t0, t1);
  }

  fn::Mix1dTable* table_mix() { return (fn::Mix1dTable*)d_table.ptr; }
  fn::DalitzTable* table_dal() { return (fn::DalitzTable*)d_table.ptr; }
  fn::Td4Table* table_td4() { return (fn::Td4Table*)d_table.ptr; }
  double* part() { return (double*)d_part.ptr; }
  double* npart() { return (double*)d_npart.ptr; }
  double* out() { return (double*)d_out.ptr; }
  double* fixed() { return (double*)d_fixed.ptr; }
  double* Mc() { return (double*)d_M.ptr; }
  ~fn_model();
};

namespace fn {
// A caller-provided device region for the partial rows of one NLL call
// (sizes in doubles): the events pass takes its rows from the front, the
// normalization from the back; a request that does not fit throws.
struct Workspace {
  double* base = nullptr;
  size_t cap = 0;
  size_t front = 0, back = 0;
  double* take_front(size_t count);
  double* take_back(size_t count);
};
void run_nll(fn_model* m, const ParamBlock* pb, const double* theta_dev, const double* ev, int64_t n, int64_t ld,
             bool grad, double* out_user, hipStream_t s, Workspace* ws = nullptr);
void nll_host(fn_model* m, const double* theta_host, const double* ev, int64_t n, int64_t ld, double* nll,
              double* grad, hipStream_t s);
void check_events_args(fn_model* m, const double* ev, int64_t n, int64_t ld);
// Binned data of a mix1d model: counts of nb uniform bins on [lo, hi] (device),
// statistic 0 Poisson NLL, 1 chi^2.
struct BinnedData {
  const double* counts;
  int64_t nb;
  int stat;
};
void nll_binned_host(fn_model* m, const double* theta_host, const BinnedData& bd, double* value, double* grad,
                     hipStream_t s);
// td4 fixed-constant vector ((m0, Gamma0) of every r12 entry, then of every
// r34 entry, then sigma_t) -> per-fit constants; throws on invalid values.
Td4FitConst td4_fit_const(const Td4Const& tc, const double* fixed);
int td4_n_fixed(const Td4Const& tc);
}  // namespace fn
