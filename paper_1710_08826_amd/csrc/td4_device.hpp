// Device code of the time-dependent four-body model (the paper's four-body
// time-dependent amplitude analyses, Abstract and Sec. 5).  The per-event and
// normalization-matrix passes are compiled at run time for each model shape
// (which pair entries are resonant and with which spin, which entries and
// angular factor every basis amplitude takes) as compile-time constants; the
// time functions are shared with the library's own kernels.
//
// Per event (m12, m34, c12, c34, phi, t) and fit:
//   a12[r], a34[r]   pair lineshapes: 1 (non-resonant) or Ka F_L(q r) T with
//                    T = (a + i b)/(a^2 + b^2), a = m0^2 - s, b = Kw G_L(s),
//                    G_L = q^(2L+1) F_L(q r)^2 / sqrt(s) (as in the three-body kernel)
//   B_k = a12[r1_k] a34[r2_k] Omega_k(c12, c34, phi), A = sum c_k B_k, Abar = sum cbar_k B_k
//   R = 1/2 [(|A|^2+|Abar|^2) Hc + (|A|^2-|Abar|^2) Hcos - 2 Re(A* Abar) Hs - 2 Im(A* Abar) Hsin]
// with Hc, Hs = (h(G(1-y)) +- h(G(1+y)))/2 and Hcos + i Hsin = h(G(1 - i x)), where
// h(a; t) = exp(a^2 s^2/2 - a t) erfc((a s^2 - t)/(s sqrt2)) / 2 is the exponential
// convolved with the Gaussian resolution of width s, evaluated through the
// Faddeeva function w (Weideman, SIAM J. Numer. Anal. 31 (1994) 1497:
// w(z) = [2 p(Z)/(L - i z) + 1/sqrt(pi)] / (L - i z), Z = (L + i z)/(L - i z),
// p a polynomial of degree N-1 whose coefficients are the Fourier
// coefficients of exp(-t^2)(L^2 + t^2), t = L tan(theta/2); N = 40, L = sqrt(N/sqrt 2)).
// dh/da = (a s^2 - t) h - s/sqrt(2 pi) exp(-t^2/(2 s^2)) gives the x, y derivatives.
// I is the phase-space average of the t-integrated rate, a quadratic form in the
// coefficients through the per-fit matrix M_ij = <B_i conj(B_j)>.
#pragma once
#include "device_common.hpp"
#include "fastmath.hpp"
#include "philox.hpp"
#include "td4_types.hpp"

namespace fn {

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// c + a b as four chained FMAs
__device__ __forceinline__ cplx cfma(cplx a, cplx b, cplx c) {
  return {__builtin_fma(a.re, b.re, __builtin_fma(-a.im, b.im, c.re)),
          __builtin_fma(a.re, b.im, __builtin_fma(a.im, b.re, c.im))};
}
// (gr, gi) += (Re(l b), -Im(l b)): a gradient pair d/dRe, d/dIm from l b
__device__ __forceinline__ void grad_acc(cplx l, cplx b, double& gr, double& gi) {
  gr = __builtin_fma(l.re, b.re, __builtin_fma(-l.im, b.im, gr));
  gi = __builtin_fma(-l.re, b.im, __builtin_fma(-l.im, b.re, gi));
}
__device__ __forceinline__ cplx crcp(cplx a) {
  const double d = rcp_fast(__builtin_fma(a.re, a.re, a.im * a.im));
  return {a.re * d, -a.im * d};
}

constexpr double kInvSqrtPi = 0.56418958354775628695;
constexpr double kInvSqrt2Pi = 0.39894228040143267794;
constexpr double kInvSqrt2 = 0.70710678118654752440;

// The rational approximation: scale L and coefficients wa[0..N-1] = a_1..a_N.

// w(z) for Im z >= 0.
__device__ inline cplx faddeeva(const double* __restrict__ wa, double L, cplx z) {
  const cplx d = {L + z.im, -z.re};           // L - i z
  const cplx id = crcp(d);
  const cplx Z = cmul({L - z.im, z.re}, id);  // (L + i z)/(L - i z)
  cplx p = {wa[kWeidN - 1], 0.0};
#pragma unroll
  for (int n = kWeidN - 2; n >= 0; --n)
    p = {__builtin_fma(p.re, Z.re, __builtin_fma(-p.im, Z.im, wa[n])), __builtin_fma(p.re, Z.im, p.im * Z.re)};
  const cplx t = cmul({2.0 * p.re, 2.0 * p.im}, id);
  return cmul({t.re + kInvSqrtPi, t.im}, id);
}

// w(i y), y >= 0 (real on the imaginary axis): Z = (L - y)/(L + y).
__device__ inline double faddeeva_imag(const double* __restrict__ wa, double L, double y) {
  const double id = rcp_fast(L + y);
  const double Z = (L - y) * id;
  double p = wa[kWeidN - 1];
#pragma unroll
  for (int n = kWeidN - 2; n >= 0; --n) p = __builtin_fma(p, Z, wa[n]);
  return __builtin_fma(2.0 * p, id, kInvSqrtPi) * id;
}

// h(a; t) and dh/da for real a.  g = exp(-t^2/(2 s^2)).
__device__ inline void h_real(const double* __restrict__ wa, double L, double a, double t, double s, double s2,
                              double g, double& h, double& dh) {
  const double u = a * s2 - t;
  const double z = u * (kInvSqrt2 / s);
  const double w = faddeeva_imag(wa, L, fabs(z));
  h = z >= 0.0 ? 0.5 * g * w : exp(0.5 * a * a * s2 - a * t) - 0.5 * g * w;
  dh = u * h - s * kInvSqrt2Pi * g;
}

// h(a; t) and dh/da for complex a.
__device__ inline void h_cplx(const double* __restrict__ wa, double L, cplx a, double t, double s, double s2, double g,
                              cplx& h, cplx& dh) {
  const cplx u = {a.re * s2 - t, a.im * s2};
  const cplx z = {u.re * (kInvSqrt2 / s), u.im * (kInvSqrt2 / s)};
  const bool up = z.re >= 0.0;
  const cplx arg = up ? cplx{-z.im, z.re} : cplx{z.im, -z.re};  // i z or -i z, Im >= 0
  const cplx w = faddeeva(wa, L, arg);
  if (up) {
    h = {0.5 * g * w.re, 0.5 * g * w.im};
  } else {
    const double er = 0.5 * (a.re * a.re - a.im * a.im) * s2 - a.re * t;
    const double ei = a.re * a.im * s2 - a.im * t;
    double sn, cs;
    sincos(ei, &sn, &cs);
    const double e = exp(er);
    h = {e * cs - 0.5 * g * w.re, e * sn - 0.5 * g * w.im};
  }
  const cplx uh = cmul(u, h);
  dh = {uh.re - s * kInvSqrt2Pi * g, uh.im};
}

// ------------------------------------------------------- shape-specialized
// A shape S gives, as compile-time constants: K, N12, N34, L12[], NR12[],
// L34[], NR34[] (NR = 1 marks a flat entry), A1[], A2[] (pair entries of
// every basis amplitude) and T[] (angular factor).

template <int N>
__device__ __host__ constexpr bool any_l1(const int (&L)[N], const int (&NR)[N]) {
  bool u = false;
  for (int r = 0; r < N; ++r) u = u || (L[r] == 1 && !NR[r]);
  return u;
}

// Lineshapes of one pair from its invariant mass m (rt: the fit's m0^2, Kw, Ka).
template <int N, const int (&L)[N], const int (&NR)[N]>
__device__ __forceinline__ void pair_amps_s(double m, double sum2, double dif2, double r2,
                                            const double (*__restrict__ rt)[3], cplx (&amp)[N]) {
  const double s = m * m;
  const double im = rcp_fast(m);
  const double lq = fmax((s - sum2) * (s - dif2), 0.0);
  const double q2 = 0.25 * lq * im * im;
  const double G0 = sqrt_fast(q2) * im;
  double F1 = 1.0, G1 = 0.0;
  if (any_l1<N>(L, NR)) {
    F1 = rsqrt_fast(1.0 + q2 * r2);
    G1 = G0 * q2 * F1 * F1;
  }
#pragma unroll
  for (int r = 0; r < N; ++r) {
    amp[r] = {1.0, 0.0};
    if (!NR[r]) {
      const double G = L[r] == 1 ? G1 : G0;
      const double a = rt[r][0] - s;
      const double b = rt[r][1] * G;
      const double d = rcp_fast(__builtin_fma(a, a, b * b));
      const double k = (L[r] == 1 ? rt[r][2] * F1 : rt[r][2]) * d;
      amp[r] = {k * a, k * b};
    }
  }
}

// One kinematic point under one fit's lineshapes: the lineshapes of both
// pairs and the angular values every basis function is formed from.
template <class S>
struct Td4Point {
  cplx a12[S::N12], a34[S::N34];
  double c12, c34;
  double ssc, sss;  // 1/2 sin theta12 sin theta34 (cos phi, sin phi)
};

template <class S>
__device__ __forceinline__ void td4_point_s(const Td4Const& tc, const Td4Table& tb, double m12, double m34, double c12,
                                            double c34, double phi, Td4Point<S>& p) {
  pair_amps_s<S::N12, S::L12, S::NR12>(m12, tc.sum12, tc.dif12, tc.r2, tb.r12, p.a12);
  pair_amps_s<S::N34, S::L34, S::NR34>(m34, tc.sum34, tc.dif34, tc.r2, tb.r34, p.a34);
  constexpr bool has_sc = [] {
    bool u = false;
    for (int k = 0; k < S::K; ++k) u = u || S::T[k] >= 4;
    return u;
  }();
  p.c12 = c12;
  p.c34 = c34;
  p.ssc = 0.0;
  p.sss = 0.0;
  if (has_sc) {
    const double ss = 0.5 * sqrt_fast(fmax(1.0 - c12 * c12, 0.0)) * sqrt_fast(fmax(1.0 - c34 * c34, 0.0));
    double sp, cp;
    sincos(phi, &sp, &cp);
    p.ssc = ss * cp;
    p.sss = ss * sp;
  }
}

// Basis function B_k of a point (k a constant after unrolling); products
// with flat entries and real angular factors are formed as such.
template <class S>
__device__ __forceinline__ cplx td4_bk(const Td4Point<S>& p, int k) {
  const int r1 = S::A1[k], r2 = S::A2[k];
  cplx xy;
  if (S::NR12[r1] && S::NR34[r2]) xy = {1.0, 0.0};
  else if (S::NR12[r1]) xy = p.a34[r2];
  else if (S::NR34[r2]) xy = p.a12[r1];
  else xy = cmul(p.a12[r1], p.a34[r2]);
  switch (S::T[k]) {
    case 0: return xy;
    case 1: return {xy.re * p.c34, xy.im * p.c34};
    case 2: return {xy.re * p.c12, xy.im * p.c12};
    case 3: { const double cc = p.c12 * p.c34; return {xy.re * cc, xy.im * cc}; }
    case 4: return cmul(xy, {p.ssc, p.sss});
    default: return cmul(xy, {p.ssc, -p.sss});
  }
}

// Makes the compiler treat a point's values as new ones, so that basis
// functions formed after it are recomputed from the lineshapes instead of
// being kept in registers from an earlier loop.
template <class S>
__device__ __forceinline__ void td4_opaque(Td4Point<S>& p) {
#pragma unroll
  for (int r = 0; r < S::N12; ++r) asm volatile("" : "+v"(p.a12[r].re), "+v"(p.a12[r].im));
#pragma unroll
  for (int r = 0; r < S::N34; ++r) asm volatile("" : "+v"(p.a34[r].re), "+v"(p.a34[r].im));
  asm volatile("" : "+v"(p.c12), "+v"(p.c34), "+v"(p.ssc), "+v"(p.sss));
}

// All basis amplitudes B_k of one kinematic point under one fit's lineshapes.
template <class S>
__device__ __forceinline__ void td4_basis_s(const Td4Const& tc, const Td4Table& tb, double m12, double m34, double c12,
                                            double c34, double phi, cplx (&B)[S::K]) {
  Td4Point<S> p;
  td4_point_s<S>(tc, tb, m12, m34, c12, c34, phi, p);
#pragma unroll
  for (int k = 0; k < S::K; ++k) B[k] = td4_bk<S>(p, k);
}

// Workgroup -> (chunk, fit) of a pass over a sample shared by n_fits fits.
// Workgroups are handed to the eight XCDs round robin by index, and each XCD
// has its own L2: the n_fits workgroups of one chunk are given indices that
// are equal modulo 8, so that the chunk is fetched into one L2 only.  The
// launch has td4_blocks(nch, n_fits) workgroups; false for padding ones.
constexpr int kXcds = 8;
__host__ __device__ inline int64_t td4_blocks(int64_t nch, int n_fits) {
  return n_fits == 1 ? nch : (nch + kXcds - 1) / kXcds * kXcds * n_fits;
}
__device__ __forceinline__ bool td4_block_item(int64_t nch, int n_fits, int64_t& ch, int& f) {
  const int64_t b = blockIdx.x;
  if (n_fits == 1) {
    ch = b;
    f = 0;
    return true;
  }
  const int64_t x = b % kXcds, j = b / kXcds;
  f = (int)(j % n_fits);
  ch = (j / n_fits) * kXcds + x;
  return ch < nch;
}

// Events pass for n_fits fits sharing one sample: one workgroup per (chunk,
// fit), the fits of a chunk on one XCD so that they share it through its L2;
// a fit whose status entry is not running is skipped (status may be null).
template <class S, bool GRAD>
__device__ inline void td4_events_body(const Td4Const& tc, const Td4Table* __restrict__ tabs,
                                       const int* __restrict__ status, const double* __restrict__ ev, int64_t ld,
                                       int64_t n, int chunk, int64_t nch, int n_fits, double* __restrict__ part) {
  constexpr int K = S::K;
  constexpr int P = S::P;
  // partial row: NLL, then the gradient in theta order (A's coefficients,
  // Abar's, x, y)
  constexpr int NV = GRAD ? 1 + P : 1;
  __shared__ double lds[block_sum_lds(NV)];
  int64_t ch;
  int f;
  if (!td4_block_item(nch, n_fits, ch, f)) return;
  if (status && status[f] != 1) return;
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const double s = tabs[f].sigma, s2 = s * s, inv2s2 = 0.5 / s2;
  const double G = tc.gamma;
  const double ap = G * (1.0 - tabs[f].y), am = G * (1.0 + tabs[f].y);
  const cplx ac = {G, -G * tabs[f].x};
  const int64_t base = ch * chunk;
  const int64_t end = base + chunk < n ? base + chunk : n;
  LogProd lp;  // -sum ln R enters acc[0] once per thread, at the end
  for (int64_t i = base + threadIdx.x; i < end; i += kBlock) {
    // the fit's constants are re-read through the scalar cache on every event
    // (an opaque zero offset keeps them from being hoisted into SGPRs that
    // would overflow into VGPR lanes)
    int zero = 0;
    asm volatile("" : "+s"(zero));
    const Td4Table& tb = tabs[f + zero];
    // time functions first: the lineshapes are not live across the three
    // rational-approximation evaluations
    const double t = ev[5 * ld + i];
    const double g = exp(-t * t * inv2s2);
    double hp, dhp, hm, dhm;
    cplx hc, dhc;
    const double* wa = tc.wa + zero;  // re-read per event, like the table
    h_real(wa, tc.wL, ap, t, s, s2, g, hp, dhp);
    h_real(wa, tc.wL, am, t, s, s2, g, hm, dhm);
    h_cplx(wa, tc.wL, ac, t, s, s2, g, hc, dhc);
    Td4Point<S> pt;
    td4_point_s<S>(tc, tb, ev[i], ev[ld + i], ev[2 * ld + i], ev[3 * ld + i], ev[4 * ld + i], pt);
    cplx A = {0.0, 0.0}, Ab = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const cplx b = td4_bk<S>(pt, k);
      if (S::PA[k] >= 0) A = cfma({tb.c[k][0], tb.c[k][1]}, b, A);
      if (S::PB[k] >= 0) Ab = cfma({tb.cb[k][0], tb.cb[k][1]}, b, Ab);
    }
    const double Hc = 0.5 * (hp + hm), Hs = 0.5 * (hp - hm);
    const double a2 = A.re * A.re + A.im * A.im, b2 = Ab.re * Ab.re + Ab.im * Ab.im;
    const double zr = A.re * Ab.re + A.im * Ab.im, zi = A.re * Ab.im - A.im * Ab.re;  // conj(A) Abar
    const double R = 0.5 * ((a2 + b2) * Hc + (a2 - b2) * hc.re - 2.0 * zr * Hs - 2.0 * zi * hc.im);
    lp.mul(R);
    if (GRAD) {
      const double w = -rcp_fast(R);
      const double hpc = Hc + hc.re, hmc = Hc - hc.re;
      // dR/dRe c_k - i dR/dIm c_k = lc B_k and the same for cbar with lb, where
      // lc = hpc conj(A) - (Hs + i Hsin) conj(Abar), lb = hmc conj(Abar) - (Hs - i Hsin) conj(A)
      // (the event's factor w = -1/R included)
      const cplx lc = {w * (hpc * A.re - Hs * Ab.re - hc.im * Ab.im), w * (-hpc * A.im + Hs * Ab.im - hc.im * Ab.re)};
      const cplx lb = {w * (hmc * Ab.re - Hs * A.re + hc.im * A.im), w * (-hmc * Ab.im + Hs * A.im + hc.im * A.re)};
      // the basis functions again, formed from the lineshapes
      td4_opaque<S>(pt);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const cplx b = td4_bk<S>(pt, k);
        if (S::PA[k] >= 0) grad_acc(lc, b, acc[1 + S::PA[k]], acc[2 + S::PA[k]]);
        if (S::PB[k] >= 0) grad_acc(lb, b, acc[1 + S::PB[k]], acc[2 + S::PB[k]]);
      }
      // x: d hc/dx = -i G dh(ac);  y: d hp/dy = -G dh(ap), d hm/dy = +G dh(am)
      const double dcos = G * dhc.im, dsin = -G * dhc.re;
      acc[P - 1] += w * 0.5 * ((a2 - b2) * dcos - 2.0 * zi * dsin);
      const double dHc = 0.5 * G * (dhm - dhp), dHs = -0.5 * G * (dhp + dhm);
      acc[P] += w * 0.5 * ((a2 + b2) * dHc - 2.0 * zr * dHs);
    }
  }
  acc[0] = -lp.log();
  block_sum_row<NV>(acc, lds, part + ((int64_t)f * nch + ch) * NV);
}

// ------------------------------------------------------ four-body phase space
// Two-body momentum q(m; ma, mb) and the phase-space weight of (m12, m34)
// with the angles uniform: q(M; m12, m34) q(m12; m1, m2) q(m34; m3, m4).
// Contraction is off: the weight decides accept-reject draws and is the same
// plain IEEE evaluation on the host and the device.
__host__ __device__ inline double td4_q(double m, double ma, double mb) {
#pragma clang fp contract(off)
  const double l = (m * m - (ma + mb) * (ma + mb)) * (m * m - (ma - mb) * (ma - mb));
  return sqrt(l > 0.0 ? l : 0.0) / (2.0 * m);
}
__host__ __device__ inline double td4_ps_weight(const Td4Const& tc, double m12, double m34) {
#pragma clang fp contract(off)
  return td4_q(tc.M, m12, m34) * td4_q(m12, tc.m1, tc.m2) * td4_q(m34, tc.m3, tc.m4);
}

// Unweighted phase-space point i (m12, m34, cos theta12, cos theta34, phi):
// attempt a takes (u1, u2) from counter (i, s0 + 3a, 2), (u3, u4) from
// (i, s0 + 3a + 1, 2) and (u5, u6) from (i, s0 + 3a + 2, 2); (m12, m34)
// uniform in [m1 + m2, M - m3 - m4] x [m3 + m4, M - m1 - m2] is kept when
// m12 + m34 < M and u3 wmax < weight; then c12 = 2 u4 - 1, c34 = 2 u5 - 1,
// phi = (2 u6 - 1) pi.  false when no attempt is kept.
__device__ inline bool td4_ps_point(const Td4Const& tc, int64_t i, uint32_t k0, uint32_t k1, uint32_t s0,
                                    int max_attempts, double (&x)[5]) {
#pragma clang fp contract(off)
  const double lo12 = tc.m1 + tc.m2, hi12 = tc.M - tc.m3 - tc.m4;
  const double lo34 = tc.m3 + tc.m4, hi34 = tc.M - tc.m1 - tc.m2;
  for (int a = 0; a < max_attempts; ++a) {
    double u1, u2, u3, u4, u5, u6;
    philox_uniforms((uint64_t)i, s0 + 3u * a, 2u, k0, k1, u1, u2);
    philox_uniforms((uint64_t)i, s0 + 3u * a + 1u, 2u, k0, k1, u3, u4);
    philox_uniforms((uint64_t)i, s0 + 3u * a + 2u, 2u, k0, k1, u5, u6);
    const double m12 = lo12 + u1 * (hi12 - lo12);
    const double m34 = lo34 + u2 * (hi34 - lo34);
    if (m12 + m34 < tc.M && u3 * tc.ps_wmax < td4_ps_weight(tc, m12, m34)) {
      x[0] = m12;
      x[1] = m34;
      x[2] = 2.0 * u4 - 1.0;
      x[3] = 2.0 * u5 - 1.0;
      x[4] = (2.0 * u6 - 1.0) * 3.14159265358979323846;
      return true;
    }
  }
  return false;
}

// (|A| + |Abar|)^2 at one point of the model (the bound of the rate at t = 0).
template <class S>
__device__ inline double td4_env(const Td4Const& tc, const Td4Table& tb, double m12, double m34, double c12,
                                 double c34, double phi) {
  constexpr int K = S::K;
  cplx B[K];
  td4_basis_s<S>(tc, tb, m12, m34, c12, c34, phi, B);
  cplx A = {0.0, 0.0}, Ab = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const cplx p = cmul({tb.c[k][0], tb.c[k][1]}, B[k]);
    const cplx q = cmul({tb.cb[k][0], tb.cb[k][1]}, B[k]);
    A = {A.re + p.re, A.im + p.im};
    Ab = {Ab.re + q.re, Ab.im + q.im};
  }
  const double e = sqrt(A.re * A.re + A.im * A.im) + sqrt(Ab.re * Ab.re + Ab.im * Ab.im);
  return e * e;
}

// Toy events of the model by accept-reject with importance sampling of the
// pair masses: event i, attempt a takes (u1, u2) ... (u9, u10) from Philox
// counters (i, 5a + j, word 4), j = 0..4, key (k0, k1): m12 from the r12
// proposal with selector u1 and position u3, m34 from the r34 proposal with
// u2 and u4 (Td4Proposal), c12 = 2 u5 - 1, c34 = 2 u6 - 1, phi = (2 u7 - 1) pi,
// t = -ln(1 - u8)/lam with lam = G (1 - |y|); kept when
// u9 W q12(m12) q34(m34) e^{-lam t} < w(m12, m34) R, w the phase-space weight
// and R the unconvolved rate (at most e^{-lam t} (|A| + |Abar|)^2), so W
// must bound w (|A| + |Abar|)^2 / (q12 q34).  The measured time adds sigma
// times a Box-Muller normal from counter (i, 0, 5).  bad[0] counts kept
// events above the bound, bad[1] events left NaN.
template <class S>
__device__ inline void td4_gen_body(const Td4Const& tc, const Td4Table* __restrict__ tab, const Td4Proposal& pr,
                                    uint32_t k0, uint32_t k1, int64_t n, double W, int max_attempts,
                                    double* __restrict__ ev, int64_t ld, unsigned long long* __restrict__ bad) {
#pragma clang fp contract(off)
  constexpr int K = S::K;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const Td4Table& tb = *tab;
  const double G = tc.gamma, x = tb.x, y = tb.y;
  const double lam = G * (1.0 - fabs(y));
  double out[6];
  for (int j = 0; j < 6; ++j) out[j] = __builtin_nan("");
  double ratio = 0.0;
  for (int a = 0; a < max_attempts; ++a) {
    double u1, u2, u3, u4, u5, u6, u7, u8, u9, u10;
    philox_uniforms((uint64_t)i, 5u * a, 4u, k0, k1, u1, u2);
    philox_uniforms((uint64_t)i, 5u * a + 1u, 4u, k0, k1, u3, u4);
    philox_uniforms((uint64_t)i, 5u * a + 2u, 4u, k0, k1, u5, u6);
    philox_uniforms((uint64_t)i, 5u * a + 3u, 4u, k0, k1, u7, u8);
    philox_uniforms((uint64_t)i, 5u * a + 4u, 4u, k0, k1, u9, u10);
    const double m12 = td4_prop_draw(pr.p12, u1, u3);
    const double m34 = td4_prop_draw(pr.p34, u2, u4);
    if (!(m12 + m34 < tc.M)) continue;
    const double w = td4_ps_weight(tc, m12, m34);
    if (!(w > 0.0)) continue;
    const double c12 = 2.0 * u5 - 1.0, c34 = 2.0 * u6 - 1.0, phi = (2.0 * u7 - 1.0) * 3.14159265358979323846;
    const double t = -log1p(-u8) / lam;
    cplx B[K];
    td4_basis_s<S>(tc, tb, m12, m34, c12, c34, phi, B);
    cplx A = {0.0, 0.0}, Ab = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const cplx p = cmul({tb.c[k][0], tb.c[k][1]}, B[k]);
      const cplx q = cmul({tb.cb[k][0], tb.cb[k][1]}, B[k]);
      A = {A.re + p.re, A.im + p.im};
      Ab = {Ab.re + q.re, Ab.im + q.im};
    }
    const double a2 = A.re * A.re + A.im * A.im, b2 = Ab.re * Ab.re + Ab.im * Ab.im;
    const double zr = A.re * Ab.re + A.im * Ab.im, zi = A.re * Ab.im - A.im * Ab.re;
    const double gt = G * t;
    const double ep = exp(y * gt), em = exp(-y * gt);
    double sx, cx;
    sincos(x * gt, &sx, &cx);
    const double R = 0.5 * exp(-gt) *
                     ((a2 + b2) * (0.5 * (ep + em)) + (a2 - b2) * cx - 2.0 * zr * (0.5 * (ep - em)) - 2.0 * zi * sx);
    const double q12 = td4_prop_density(pr.p12, m12), q34 = td4_prop_density(pr.p34, m34);
    if (u9 * W * q12 * q34 * exp(-lam * t) < w * R) {
      out[0] = m12; out[1] = m34; out[2] = c12; out[3] = c34; out[4] = phi; out[5] = t;
      const double e = sqrt(a2) + sqrt(b2);
      ratio = w * (e * e) / (q12 * q34);
      break;
    }
  }
  double v1, v2;
  philox_uniforms((uint64_t)i, 0u, 5u, k0, k1, v1, v2);
  out[5] = out[5] + tb.sigma * (sqrt(-2.0 * log1p(-v1)) * cos(2.0 * 3.14159265358979323846 * v2));
  for (int j = 0; j < 6; ++j) ev[j * ld + i] = out[j];
  if (ratio > W) atomicAdd(bad, 1ull);
  if (out[0] != out[0]) atomicAdd(bad + 1, 1ull);
}

// Largest w (|A| + |Abar|)^2 / (q12 q34) over the points of a phase-space
// sample (the generator's bound; bits of a non-negative double) in *vmax.
template <class S>
__device__ inline void td4_envmax_body(const Td4Const& tc, const Td4Table* __restrict__ tab, const Td4Proposal& pr,
                                       const double* __restrict__ mc, int64_t ld, int64_t n,
                                       unsigned long long* __restrict__ vmax) {
  __shared__ double lds[kBlock];
  const Td4Table& tb = *tab;
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const double m12 = mc[i], m34 = mc[ld + i];
    const double e = td4_env<S>(tc, tb, m12, m34, mc[2 * ld + i], mc[3 * ld + i], mc[4 * ld + i]);
    const double r = td4_ps_weight(tc, m12, m34) * e / (td4_prop_density(pr.p12, m12) * td4_prop_density(pr.p34, m34));
    m = fmax(m, r);
  }
  lds[threadIdx.x] = m;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(vmax, (unsigned long long)__double_as_longlong(lds[0]));
}

// Rows i0..i0+RB-1 of M = sum over the phase-space sample of B_i conj(B_j)
// (per fit; fits with sel[f] == 0 are skipped, sel may be null).
template <class S>
__device__ inline void td4_mrows_body(const Td4Const& tc, const Td4Table* __restrict__ tabs,
                                      const int* __restrict__ sel, const double* __restrict__ mc, int64_t ld,
                                      int64_t n, int chunk, int64_t nch, int n_fits, int i0,
                                      double* __restrict__ part) {
  constexpr int K = S::K;
  constexpr int RB = td4_row_block(K);
  constexpr int NV = 2 * RB * K;
  __shared__ double lds[block_sum_lds(NV)];
  int64_t ch;
  int f;
  if (!td4_block_item(nch, n_fits, ch, f)) return;
  if (sel && !sel[f]) return;
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const int64_t base = ch * chunk;
  const int64_t end = base + chunk < n ? base + chunk : n;
  for (int64_t i = base + threadIdx.x; i < end; i += kBlock) {
    int zero = 0;
    asm volatile("" : "+s"(zero));
    const Td4Table& tb = tabs[f + zero];
    Td4Point<S> pt;
    td4_point_s<S>(tc, tb, mc[i], mc[ld + i], mc[2 * ld + i], mc[3 * ld + i], mc[4 * ld + i], pt);
    cplx bi[RB];
#pragma unroll
    for (int ib = 0; ib < RB; ++ib) {
      bi[ib] = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (k == i0 + ib) bi[ib] = td4_bk<S>(pt, k);
    }
    td4_opaque<S>(pt);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const cplx bj = td4_bk<S>(pt, j);
#pragma unroll
      for (int ib = 0; ib < RB; ++ib) {
        acc[2 * (ib * K + j)] = __builtin_fma(bi[ib].re, bj.re, __builtin_fma(bi[ib].im, bj.im, acc[2 * (ib * K + j)]));
        acc[2 * (ib * K + j) + 1] =
            __builtin_fma(bi[ib].im, bj.re, __builtin_fma(-bi[ib].re, bj.im, acc[2 * (ib * K + j) + 1]));
      }
    }
  }
  block_sum_row<NV>(acc, lds, part + ((int64_t)f * nch + ch) * NV);
}

}  // namespace fn

// Kernels for shape S (used by the generated source).
#define FN_TD4_EVENTS(NAME, S, GRAD)                                                                           \
  extern "C" __global__ __launch_bounds__(fn::kBlock) __attribute__((amdgpu_waves_per_eu(2))) void NAME(        \
      fn::Td4Const tc, const fn::Td4Table* __restrict__ tabs, const int* __restrict__ status,                  \
      const double* __restrict__ ev, int64_t ld, int64_t n, int chunk, int64_t nch, int n_fits,                \
      double* __restrict__ part) {                                                                              \
    fn::td4_events_body<S, GRAD>(tc, tabs, status, ev, ld, n, chunk, nch, n_fits, part);                       \
  }
#define FN_TD4_MROWS(NAME, S)                                                                                  \
  extern "C" __global__ __launch_bounds__(fn::kBlock) void NAME(                                                \
      fn::Td4Const tc, const fn::Td4Table* __restrict__ tabs, const int* __restrict__ sel,                     \
      const double* __restrict__ mc, int64_t ld, int64_t n, int chunk, int64_t nch, int n_fits, int i0,        \
      double* __restrict__ part) {                                                                              \
    fn::td4_mrows_body<S>(tc, tabs, sel, mc, ld, n, chunk, nch, n_fits, i0, part);                              \
  }
#define FN_TD4_GEN(ENVMAX, GEN, S)                                                                             \
  extern "C" __global__ __launch_bounds__(fn::kBlock) void ENVMAX(                                             \
      fn::Td4Const tc, const fn::Td4Table* __restrict__ tab, fn::Td4Proposal pr, const double* __restrict__ mc, \
      int64_t ld, int64_t n, unsigned long long* __restrict__ vmax) {                                          \
    fn::td4_envmax_body<S>(tc, tab, pr, mc, ld, n, vmax);                                                      \
  }                                                                                                            \
  extern "C" __global__ __launch_bounds__(fn::kBlock) void GEN(                                                \
      fn::Td4Const tc, const fn::Td4Table* __restrict__ tab, fn::Td4Proposal pr, uint32_t k0, uint32_t k1,     \
      int64_t n, double W, int max_attempts, double* __restrict__ ev, int64_t ld,                              \
      unsigned long long* __restrict__ bad) {                                                                  \
    fn::td4_gen_body<S>(tc, tab, pr, k0, k1, n, W, max_attempts, ev, ld, bad);                                 \
  }
