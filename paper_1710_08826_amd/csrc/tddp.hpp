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
  hipFunction_t gmax = nullptr, gen = nullptr;            // toy generation
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
                        bool grad, double* part, hipStream_t s, hipEvent_t start = nullptr,
                        hipEvent_t stop = nullptr);
// Level-2 and NLL assembly: out = [NLL, grad(P), I, dI(P)].
void tddp_launch_finalize(const DalitzConst& dc, const DalitzTable* tab, const TddpTime& tt, const double* coef,
                          const double* part, int64_t nrows, bool grad, const double* Mc, double n_events,
                          double* out, double* out_user, hipStream_t s);
// Toy generation: vmax (zeroed by the caller) receives the bits of the largest
// (|A| + |Abar|)^2 over the grid; the generator writes n events (3 rows,
// leading dimension ld), bad[0] / bad[1] as for the three-body generator.
void tddp_launch_gridmax(const TddpJit& j, const DalitzConst& dc, const DalitzTable* tab, const double* coef,
                         unsigned long long* vmax, hipStream_t s);
void tddp_launch_gen(const TddpJit& j, const DalitzConst& dc, const DalitzTable* tab, const double* coef,
                     const TddpTime& tt, uint32_t k0, uint32_t k1, int64_t n, double W, const double box[4],
                     int max_attempts, double* ev, int64_t ld, unsigned long long* bad, hipStream_t s);
// theta (P doubles) passed by value -> device copy.
void tddp_launch_copy_theta(const ParamBlock& pb, int P, double* dst, hipStream_t s);

}  // namespace fn
