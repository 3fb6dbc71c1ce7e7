// Time-dependent four-body model: host launchers (types in td4_types.hpp).
#pragma once
#include <memory>
#include <string>

#include "model.hpp"
#include "td4_types.hpp"

namespace fn {

// Shape-specialized passes of one model (compiled at model creation).
struct JitProgram;
struct Td4Jit {
  std::shared_ptr<JitProgram> prog;
  hipFunction_t ev[2] = {nullptr, nullptr};  // without, with the gradient
  hipFunction_t mrows = nullptr;
  hipFunction_t envmax = nullptr, gen = nullptr;  // toy generation
};
std::string td4_jit_source(const Td4Const& tc);
std::shared_ptr<Td4Jit> td4_jit(const Td4Const& tc);
int td4_kmax(int K);
int td4_nv(const Td4Const& tc, bool grad);  // doubles per events-pass partial row: NLL, then the gradient in theta order
void td4_weideman_coefficients(double* a, double* L);
// Bound of the phase-space weight used by the generators (host).
double td4_ps_wmax(const Td4Const& tc);
// n unweighted phase-space points (5 rows of leading dimension ld) from key
// (k0, k1) and first stream s0; bad counts points left NaN.
void td4_launch_phase_space(const Td4Const& tc, uint32_t k0, uint32_t k1, uint32_t s0, int max_attempts, int64_t n,
                            double* out, int64_t ld, unsigned long long* bad, hipStream_t s);
// Toy events of the model (6 rows): vmax (zeroed by the caller) receives the
// largest w (|A| + |Abar|)^2 / (q12 q34) over a phase-space sample (w the
// phase-space weight, q the pair proposals' densities); bad[0] / bad[1] as
// for the three-body generator.
// The toy generator's pair-mass proposals for the fit constants fc: half
// uniform and half split equally over the resonant entries of the pair,
// scale half the width (m0 +- s is the half-maximum of the peak).
Td4Proposal td4_proposal(const Td4Const& tc, const Td4FitConst& fc);
void td4_launch_envmax(const Td4Jit& j, const Td4Const& tc, const Td4Table* tab, const Td4Proposal& pr,
                       const double* mc, int64_t ld, int64_t n, unsigned long long* vmax, hipStream_t s);
void td4_launch_gen(const Td4Jit& j, const Td4Const& tc, const Td4Table* tab, const Td4Proposal& pr, uint32_t k0,
                    uint32_t k1, int64_t n, double W, int max_attempts, double* ev, int64_t ld,
                    unsigned long long* bad, hipStream_t s);
// theta: n_fits rows of theta_stride doubles on the device, or (pb != null,
// n_fits == 1) the parameter block passed by value.
void td4_launch_prologue(const Td4Const& tc, const ParamBlock* pb, const double* theta, int theta_stride,
                         const Td4FitConst* fc, const int* status, int n_fits, Td4Table* tabs, hipStream_t s);
// Normalization matrices M_f[i][j] = mean over the phase-space sample of
// B_i conj(B_j), for fits [0, n_fits) (constants fc), into Mc (n_fits x K x K complex).
// Normalization matrices of n_fits fits (only those with sel[f] != 0 when
// sel, a device array, is not null).
void td4_launch_mmatrix(const Td4Jit& j, const Td4Const& tc, const Td4Table* tabs, int n_fits, const double* mc,
                        int64_t ld_mc, int64_t n_mc, int chunk, double* part, double* Mc, hipStream_t s,
                        const int* sel = nullptr);
// Events pass for n_fits fits sharing one event sample (fit-major items); a
// fit whose status entry is not running is skipped (status may be null).
void td4_launch_events(const Td4Jit& j, const Td4Const& tc, const Td4Table* tabs, const int* status, int n_fits,
                       const double* ev, int64_t ld, int64_t n, int chunk, bool grad, double* part, hipStream_t s,
                       hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
// Level-2 and NLL assembly per fit: out + f * out_stride = [NLL, grad(P), I, dI(P)].
void td4_launch_finalize(const Td4Const& tc, const Td4Table* tabs, const int* status, int n_fits, const double* part,
                         int64_t rows_per_fit, bool grad, const double* Mc, double n_events, double* out,
                         int out_stride, double* out_user, hipStream_t s);
void td4_launch_check(const Td4Const& tc, const double* ev, int64_t ld, int64_t n, unsigned long long* bad,
                      hipStream_t s);
void td4_launch_eval(const Td4Const& tc, const Td4Table* tab, const double* ev, int64_t ld, int64_t n,
                     const double* norm, double* p, hipStream_t s);

}  // namespace fn
