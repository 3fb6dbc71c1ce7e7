// Time-dependent four-body model: constants and per-fit tables shared by the
// host, the library's kernels and the kernels compiled at run time.
#pragma once
#include "model.hpp"

namespace fn {

constexpr int kTd4MaxAmp = 20;   // basis amplitudes
constexpr int kTd4MaxRes = 6;    // resonances per pair
constexpr int kWeidN = 40;       // terms of the Faddeeva rational approximation

// Rows of the normalization matrix accumulated per pass over the phase-space
// sample (2 x rows x K doubles per thread).
__host__ __device__ constexpr int td4_row_block(int K) { return K > 12 ? 2 : 4; }

struct Td4Const {
  double M;                            // parent mass
  double m1s, m2s, m3s, m4s;           // squared daughter masses
  double sum12, dif12, sum34, dif34;   // (m1 +- m2)^2, (m3 +- m4)^2
  double r2;                           // squared barrier radius
  double m1, m2, m3, m4;               // daughter masses
  double ps_wmax;                      // phase-space weight bound of the generators
  double gamma;                        // 1 / tau
  double wL;                           // Faddeeva approximation scale L
  double wa[kWeidN];                   // its polynomial coefficients a_1..a_N
  int K, n12, n34, n_params;
  int L12[kTd4MaxRes], L34[kTd4MaxRes];
  int nr12[kTd4MaxRes], nr34[kTd4MaxRes];  // 1 = non-resonant (flat) entry
  int amp1[kTd4MaxAmp], amp2[kTd4MaxAmp], atype[kTd4MaxAmp];
  // theta index of Re c_k (in A) and of Re cbar_k (in Abar); -1 when the
  // basis function is not a member of that sum
  int pa[kTd4MaxAmp], pb[kTd4MaxAmp];
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

}  // namespace fn
