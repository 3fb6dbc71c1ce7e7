// Host-side launchers of the device kernels (defined next to the kernels).
#pragma once
#include <memory>
#include <string>

#include "model.hpp"

namespace fn {

struct DevBuf;

// mix1d
int mix1d_kmax(int K);
// Type signature a mixture's per-event passes are compiled for (mix_sig_K):
// 1..20 for one or two components, 0 (generic passes) for more.
int mix1d_sig(const Mix1dConst& mc);
// X(sig) for every signature of one or two components.
#define FN_MIX_SIGS(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20)
int mix1d_nv(int kmax, bool grad);
void mix1d_launch_prologue(const Mix1dConst& mc, const ParamBlock& pb, const double* theta_dev, int n_fits,
                           int theta_stride, Mix1dTable* tab, hipStream_t s);
// Events pass (one row of partial sums per chunk) and the level-2 step.
// start/stop (optional): events the dispatch records its start and end times into.
void mix1d_launch_events(const Mix1dConst& mc, const Mix1dTable* tab, const double* x, int64_t n, int chunk,
                         int64_t nchunks, bool grad, double* part, hipStream_t s, hipEvent_t start = nullptr,
                         hipEvent_t stop = nullptr);
void mix1d_launch_finalize(const Mix1dConst& mc, const Mix1dTable* tab, const double* part, int64_t nrows,
                           bool grad, double n_events, double* out, double* out_user, hipStream_t s);
// Binned data (counts of nb uniform bins on [lo, hi]): bins pass (one row per
// chunk of bins) and level-2 step; stat 0 Poisson NLL, 1 chi^2; out = [F, grad(P)].
int mix1d_nv_binned(int kmax, bool grad);
// nbuf: one device double of scratch (the total count for chi^2 without a yield).
void mix1d_launch_binned(const Mix1dConst& mc, const Mix1dTable* tab, const double* counts, int64_t nb, int chunk,
                         int64_t nchunks, int stat, bool grad, double* part, double* nbuf, double* out,
                         hipStream_t s);
void mix1d_launch_eval(const Mix1dConst& mc, const Mix1dTable* tab, const double* x, int64_t n, double* p,
                       hipStream_t s);
void mix1d_launch_check(const Mix1dConst& mc, const double* x, int64_t n, unsigned long long* bad, hipStream_t s);

// dalitz3
// Structure-specialized passes of one model (compiled at model creation).
struct JitProgram;
struct DalitzJit {
  std::shared_ptr<JitProgram> prog;
  hipFunction_t ev[3] = {nullptr, nullptr, nullptr};  // by gradient level
  hipFunction_t gr[3] = {nullptr, nullptr, nullptr};
  hipFunction_t mrows = nullptr;
  hipFunction_t gmax = nullptr, gen = nullptr;  // toy generation: grid maximum, accept-reject
};
// ept: events per thread and loop iteration of the events passes (1, or 2
// for a module with the events passes alone).
std::string dalitz_jit_source(const DalitzConst& dc, int ept = 1);
std::shared_ptr<DalitzJit> dalitz_jit(const DalitzConst& dc, int ept = 1);
int dalitz_kmax(int K);
int dalitz_nv_events(int kmax, int grad);
int dalitz_nv_mrows(int kmax);
void dalitz_launch_prologue(const DalitzConst& dc, const ParamBlock& pb, const double* theta_dev,
                            const double* fixed_ls, int n_fits, int theta_stride, DalitzTable* tab, hipStream_t s);
// Events pass: one row of partial sums per chunk of events.
// coef: (Re c_k, Im c_k) in device memory (theta itself, or the table's copy).
// With the cached grid matrix Mc (fixed lineshapes) and the output buffer
// out = [NLL, grad, I, dI], the pass also writes I and dI into out.
void dalitz_launch_events(const DalitzJit& j, const DalitzConst& dc, const DalitzTable* tab, const double* coef,
                          const double* ev, int64_t ld, int64_t n, int chunk, int64_t nchunks, int grad, double* part,
                          hipStream_t s, const double* Mc = nullptr, double* out = nullptr,
                          hipEvent_t start = nullptr, hipEvent_t stop = nullptr,
                          unsigned long long* span = nullptr);
// Level-2 sum of the event rows and of the normalization (grid rows, or the
// cached M when npart is null), NLL assembly: out = [NLL, grad, I, dI].
// norm_ready: the events pass already wrote I and dI into out (cached M).
// When the two row sets hold more than kPresumMinBytes, workgroups of
// kPresumRows rows each pre-sum them first (the same for the single-fit
// time-dependent passes), into presum_blocks(...)
// rows that the caller leaves free after each set (evpart, npart: writable).
constexpr int kPresumRows = 16;
constexpr int64_t kPresumMinBytes = 262144;
int64_t presum_blocks(int64_t rows, int nv, int64_t other_rows, int other_nv);
// The pre-summation itself: s0 workgroups add set 0 (n0 rows of nv0 sums at
// p0) in groups of kPresumRows rows into s0 rows at o0, s1 workgroups set 1.
void launch_rows_presum(const double* p0, int64_t n0, int nv0, double* o0, int64_t s0, const double* p1, int64_t n1,
                        int nv1, double* o1, int64_t s1, hipStream_t s);
void dalitz_launch_finalize(const DalitzConst& dc, const DalitzTable* tab, const double* coef, double* evpart,
                            int64_t ev_rows, int grad, double* npart, int64_t n_rows, int n_nv,
                            const double* Mc, double n_events, double* out, double* out_user, hipStream_t s,
                            bool norm_ready = false, unsigned long long* span = nullptr);
// The list of the grid cells inside the region (column-major) into `cells`;
// returns their number.  Synchronous on s (at model creation).
int64_t dalitz_build_grid_cells(const DalitzConst& dc, DevBuf& cells, hipStream_t s);
// Grid pass of a model with free lineshapes over the n_inside listed cells
// (nchunks >= 1 rows of partial sums; a row of an empty chunk holds zeros).
void dalitz_launch_grid(const DalitzJit& j, const DalitzConst& dc, const DalitzTable* tab, const double* coef,
                        const GridCell* cells, int64_t n_inside, int chunk, int64_t nchunks, int grad, double* part,
                        hipStream_t s);
// Level-2 of a row-block pass of K x K matrices (rows i0..i0+3, 2 K doubles
// each per chunk row) into Mc, scaled by the cell area.
void dalitz_launch_mrows_finalize(const DalitzConst& dc, const double* part, int64_t nchunks, int i0, double* Mc,
                                  hipStream_t s);
void dalitz_launch_mrows(const DalitzJit& j, const DalitzConst& dc, const DalitzTable* tab, int chunk,
                         int64_t nchunks, int i0, double* part, double* Mc, hipStream_t s);
// Toy events: vmax (zeroed by the caller) receives the bits of the largest P~
// over the grid cells inside the region; the generator writes n events (SoA,
// leading dimension ld) by accept-reject under envelope W from the box
// box = {lo12, hi12, lo13, hi13}; bad[0] counts accepted points above W,
// bad[1] events left unresolved after max_attempts (zeroed by the caller).
void dalitz_launch_gridmax(const DalitzJit& j, const DalitzConst& dc, const DalitzTable* tab,
                           unsigned long long* vmax, hipStream_t s);
void dalitz_launch_gen(const DalitzJit& j, const DalitzConst& dc, const DalitzTable* tab, uint32_t k0, uint32_t k1,
                       int64_t n, double W, const double box[4], int max_attempts, double* ev, int64_t ld,
                       unsigned long long* bad, hipStream_t s);
void dalitz_launch_eval(const DalitzConst& dc, const DalitzTable* tab, const double* ev, int64_t ld, int64_t n,
                        const double* norm, double* p, hipStream_t s);
void dalitz_launch_check(const DalitzConst& dc, const double* ev, int64_t ld, int64_t n, unsigned long long* bad,
                         hipStream_t s);

}  // namespace fn
