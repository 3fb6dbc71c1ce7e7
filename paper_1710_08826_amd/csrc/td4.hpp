// Time-dependent four-body model: constants, per-fit tables, launchers.
#pragma once
#include "model.hpp"

namespace fn {

constexpr int kTd4MaxAmp = 12;   // basis amplitudes
constexpr int kTd4MaxRes = 4;    // resonances per pair
constexpr int kWeidN = 40;       // terms of the Faddeeva rational approximation

struct Td4Const {
  double M;                            // parent mass
  double m1s, m2s, m3s, m4s;           // squared daughter masses
  double sum12, dif12, sum34, dif34;   // (m1 +- m2)^2, (m3 +- m4)^2
  double r2;                           // squared barrier radius
  double gamma;                        // 1 / tau
  double wL;                           // Faddeeva approximation scale L
  double wa[kWeidN];                   // its polynomial coefficients a_1..a_N
  int K, n12, n34, n_params;
  int L12[kTd4MaxRes], L34[kTd4MaxRes];
  int nr12[kTd4MaxRes], nr34[kTd4MaxRes];  // 1 = non-resonant (flat) entry
  int amp1[kTd4MaxAmp], amp2[kTd4MaxAmp], atype[kTd4MaxAmp];
};

// Fixed constants of one fit (systematic variations change them per fit).
struct Td4FitConst {
  double m0_12[kTd4MaxRes], w0_12[kTd4MaxRes], m0_34[kTd4MaxRes], w0_34[kTd4MaxRes];
  double sigma;
};

// Per-fit table (prologue output).
struct Td4Table {
  double r12[kTd4MaxRes][3];  // m0^2, Kw, Ka  (resonant entries)
  double r34[kTd4MaxRes][3];
  double c[kTd4MaxAmp][2], cb[kTd4MaxAmp][2];
  double x, y, sigma;
  double valid;
};

int td4_kmax(int K);
int td4_nv(int kmax, bool grad);
void td4_weideman_coefficients(double* a, double* L);
// theta: n_fits rows of theta_stride doubles on the device, or (pb != null,
// n_fits == 1) the parameter block passed by value.
void td4_launch_prologue(const Td4Const& tc, const ParamBlock* pb, const double* theta, int theta_stride,
                         const Td4FitConst* fc, const int* status, int n_fits, Td4Table* tabs, hipStream_t s);
// Normalization matrices M_f[i][j] = mean over the phase-space sample of
// B_i conj(B_j), for fits [0, n_fits) (constants fc), into Mc (n_fits x K x K complex).
void td4_launch_mmatrix(const Td4Const& tc, const Td4Table* tabs, int n_fits, const double* mc, int64_t ld_mc,
                        int64_t n_mc, int chunk, double* part, double* Mc, hipStream_t s);
// Events pass for n_fits fits sharing one event sample (fit-major items); a
// fit whose status entry is not running is skipped (status may be null).
void td4_launch_events(const Td4Const& tc, const Td4Table* tabs, const int* status, int n_fits, const double* ev,
                       int64_t ld, int64_t n, int chunk, bool grad, double* part, hipStream_t s);
// Level-2 and NLL assembly per fit: out + f * out_stride = [NLL, grad(P), I, dI(P)].
void td4_launch_finalize(const Td4Const& tc, const Td4Table* tabs, const int* status, int n_fits, const double* part,
                         int64_t rows_per_fit, bool grad, const double* Mc, double n_events, double* out,
                         int out_stride, double* out_user, hipStream_t s);
void td4_launch_check(const Td4Const& tc, const double* ev, int64_t ld, int64_t n, unsigned long long* bad,
                      hipStream_t s);
void td4_launch_eval(const Td4Const& tc, const Td4Table* tab, const double* ev, int64_t ld, int64_t n,
                     const double* norm, double* p, hipStream_t s);

}  // namespace fn
