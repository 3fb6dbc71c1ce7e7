// Time-dependent three-body Dalitz-plot model: host launchers.
#pragma once
#include <memory>
#include <string>

#include "model.hpp"
#include "tddp_device.hpp"

namespace fn {

struct JitProgram;
struct TddpJit {
  std::shared_ptr<JitProgram> prog;
  hipFunction_t ev[2] = {nullptr, nullptr};   // without, with the gradient
  hipFunction_t mrows[3] = {nullptr, nullptr, nullptr};  // MAA, MBB, MAB row blocks
};
std::string tddp_jit_source(const DalitzConst& dc);
std::shared_ptr<TddpJit> tddp_jit(const DalitzConst& dc);
int tddp_nv(int K, bool grad);
// The three normalization matrices (each K x K complex, dA included) into
// Mc, Mc + 2K^2 and Mc + 4K^2; part holds one chunk of rows.
void tddp_launch_mmatrices(const TddpJit& j, const DalitzConst& dc, const DalitzTable* tab, int grid_chunk,
                           double* part, double* Mc, hipStream_t s);
// Events pass: one row of partial sums per chunk.  coef: theta on the device.
void tddp_launch_events(const TddpJit& j, const DalitzConst& dc, const DalitzTable* tab, const TddpTime& tt,
                        const double* coef, const double* ev, int64_t ld, int64_t n, int chunk, int64_t nchunks,
                        bool grad, double* part, hipStream_t s);
// Level-2 and NLL assembly: out = [NLL, grad(P), I, dI(P)].
void tddp_launch_finalize(const DalitzConst& dc, const DalitzTable* tab, const TddpTime& tt, const double* coef,
                          const double* part, int64_t nrows, bool grad, const double* Mc, double n_events,
                          double* out, double* out_user, hipStream_t s);
// theta (P doubles) passed by value -> device copy.
void tddp_launch_copy_theta(const ParamBlock& pb, int P, double* dst, hipStream_t s);

}  // namespace fn
