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

// Proposal density of one pair mass in the toy generator: with probability
// wu uniform on [lo, hi]; otherwise resonance r (probability (1 - wu)/n each)
// through a Student-t density of two degrees of freedom, g(x) = (1 + x^2)^(-3/2)
// / 2, x = (m - m_r)/s_r, truncated to [lo, hi].  Its distribution function is
// (1 + v)/2 with v = x / sqrt(1 + x^2), so a truncated draw is v uniform in
// [vlo_r, vhi_r] and x = v / sqrt(1 - v^2): additions, products, quotients and
// square roots only, which the host reference reproduces bit for bit.  Its
// tails fall as |x|^-3, past the |x|^-2 of a Breit-Wigner intensity, so the
// uniform part carries the proposal away from the peaks.
struct Td4PairProposal {
  int n;                               // resonant entries (0: uniform only)
  double lo, hi, wu;
  double m[kTd4MaxRes], s[kTd4MaxRes], vlo[kTd4MaxRes], vhi[kTd4MaxRes];
};
struct Td4Proposal {
  Td4PairProposal p12, p34;
};

// Draw from the pair proposal with the component selector usel and the
// position upos (both uniform in [0, 1)).
__host__ __device__ inline double td4_prop_draw(const Td4PairProposal& p, double usel, double upos) {
#pragma clang fp contract(off)
  if (p.n == 0 || usel < p.wu) return p.lo + upos * (p.hi - p.lo);
  int r = (int)((usel - p.wu) / (1.0 - p.wu) * p.n);
  r = r < p.n ? r : p.n - 1;
  const double v = p.vlo[r] + upos * (p.vhi[r] - p.vlo[r]);
  return p.m[r] + p.s[r] * (v / sqrt(1.0 - v * v));
}

// The pair proposal's density at m (on [lo, hi]).
__host__ __device__ inline double td4_prop_density(const Td4PairProposal& p, double m) {
#pragma clang fp contract(off)
  double q = (p.n == 0 ? 1.0 : p.wu) / (p.hi - p.lo);
  const double wr = p.n == 0 ? 0.0 : (1.0 - p.wu) / p.n;
  for (int r = 0; r < p.n; ++r) {
    const double x = (m - p.m[r]) / p.s[r];
    const double t = 1.0 + x * x;
    q = q + wr / ((p.s[r] * (p.vhi[r] - p.vlo[r])) * (t * sqrt(t)));
  }
  return q;
}

// Per-fit table (prologue output).
struct Td4Table {
  double r12[kTd4MaxRes][3];  // m0^2, Kw, Ka  (resonant entries)
  double r34[kTd4MaxRes][3];
  double c[kTd4MaxAmp][2], cb[kTd4MaxAmp][2];
  double x, y, sigma;
  double valid;
};

}  // namespace fn
