// Time-dependent four-body amplitude model (the paper's four-body
// time-dependent amplitude analyses, Abstract and Sec. 5).
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
#include <cmath>
#include <vector>

#include "device_common.hpp"
#include "fastmath.hpp"
#include "td4.hpp"

namespace fn {

namespace {

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx crcp(cplx a) {
  const double d = rcp_nr(__builtin_fma(a.re, a.re, a.im * a.im));
  return {a.re * d, -a.im * d};
}

constexpr double kInvSqrtPi = 0.56418958354775628695;
constexpr double kInvSqrt2Pi = 0.39894228040143267794;
constexpr double kInvSqrt2 = 0.70710678118654752440;

}  // namespace

// w(z) for Im z >= 0.
__device__ inline cplx faddeeva(const Td4Const& tc, cplx z) {
  const cplx d = {tc.wL + z.im, -z.re};      // L - i z
  const cplx id = crcp(d);
  const cplx Z = cmul({tc.wL - z.im, z.re}, id);  // (L + i z)/(L - i z)
  cplx p = {tc.wa[kWeidN - 1], 0.0};
#pragma unroll
  for (int n = kWeidN - 2; n >= 0; --n) {
    const cplx q = cmul(p, Z);
    p = {q.re + tc.wa[n], q.im};
  }
  const cplx t = cmul({2.0 * p.re, 2.0 * p.im}, id);
  return cmul({t.re + kInvSqrtPi, t.im}, id);
}

// w(i y), y >= 0 (real on the imaginary axis): Z = (L - y)/(L + y).
__device__ inline double faddeeva_imag(const Td4Const& tc, double y) {
  const double id = rcp_nr(tc.wL + y);
  const double Z = (tc.wL - y) * id;
  double p = tc.wa[kWeidN - 1];
#pragma unroll
  for (int n = kWeidN - 2; n >= 0; --n) p = __builtin_fma(p, Z, tc.wa[n]);
  return __builtin_fma(2.0 * p, id, kInvSqrtPi) * id;
}

// h(a; t) and dh/da for real a.  g = exp(-t^2/(2 s^2)).
__device__ inline void h_real(const Td4Const& tc, double a, double t, double s, double s2, double g, double& h,
                              double& dh) {
  const double u = a * s2 - t;
  const double z = u * (kInvSqrt2 / s);
  const double w = faddeeva_imag(tc, fabs(z));
  h = z >= 0.0 ? 0.5 * g * w : exp(0.5 * a * a * s2 - a * t) - 0.5 * g * w;
  dh = u * h - s * kInvSqrt2Pi * g;
}

// h(a; t) and dh/da for complex a.
__device__ inline void h_cplx(const Td4Const& tc, cplx a, double t, double s, double s2, double g, cplx& h, cplx& dh) {
  const cplx u = {a.re * s2 - t, a.im * s2};
  const cplx z = {u.re * (kInvSqrt2 / s), u.im * (kInvSqrt2 / s)};
  const bool up = z.re >= 0.0;
  const cplx arg = up ? cplx{-z.im, z.re} : cplx{z.im, -z.re};  // i z or -i z, Im >= 0
  const cplx w = faddeeva(tc, arg);
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

// Lineshapes of one pair from its invariant mass m: amp[r] for every resonance of the pair.
template <int NR>
__device__ __forceinline__ void pair_amps(double m, double sum2, double dif2, double r2, const int* L, const int* nr,
                                          int n, const double (*rt)[3], cplx (&amp)[NR]) {
  const double s = m * m;
  const double im = rcp_nr(m);
  const double lq = fmax((s - sum2) * (s - dif2), 0.0);
  const double q2 = 0.25 * lq * im * im;
  const double q = sqrt_nr(q2);
  const double G0 = q * im;
  const double z = q2 * r2;
  const double F1 = rsqrt_nr(1.0 + z);
  const double G1 = G0 * q2 * F1 * F1;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    amp[r] = {1.0, 0.0};
    if (r < n && !nr[r]) {
      const bool l1 = L[r] == 1;
      const double G = l1 ? G1 : G0;
      const double F = l1 ? F1 : 1.0;
      const double a = rt[r][0] - s;
      const double b = rt[r][1] * G;
      const double d = rcp_nr(__builtin_fma(a, a, b * b));
      const double k = rt[r][2] * F * d;
      amp[r] = {k * a, k * b};
    }
  }
}

// Basis amplitudes B_k of one kinematic point under one fit's lineshapes.
template <int KMAX>
__device__ __forceinline__ void td4_basis(const Td4Const& tc, const Td4Table& tb, double m12, double m34, double c12,
                                          double c34, double phi, cplx (&B)[KMAX]) {
  cplx a12[kTd4MaxRes], a34[kTd4MaxRes];
  pair_amps<kTd4MaxRes>(m12, tc.sum12, tc.dif12, tc.r2, tc.L12, tc.nr12, tc.n12, tb.r12, a12);
  pair_amps<kTd4MaxRes>(m34, tc.sum34, tc.dif34, tc.r2, tc.L34, tc.nr34, tc.n34, tb.r34, a34);
  const double ss = 0.5 * sqrt_nr(fmax(1.0 - c12 * c12, 0.0)) * sqrt_nr(fmax(1.0 - c34 * c34, 0.0));
  double sp, cp;
  sincos(phi, &sp, &cp);
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    B[k] = {0.0, 0.0};
    if (k < tc.K) {
      cplx x = a12[0], y = a34[0];
#pragma unroll
      for (int r = 1; r < kTd4MaxRes; ++r) {
        if (tc.amp1[k] == r) x = a12[r];
        if (tc.amp2[k] == r) y = a34[r];
      }
      const cplx xy = cmul(x, y);
      cplx om;
      switch (tc.atype[k]) {
        case 0: om = {1.0, 0.0}; break;
        case 1: om = {c34, 0.0}; break;
        case 2: om = {c12, 0.0}; break;
        case 3: om = {c12 * c34, 0.0}; break;
        case 4: om = {ss * cp, ss * sp}; break;
        default: om = {ss * cp, -ss * sp}; break;
      }
      B[k] = cmul(xy, om);
    }
  }
}

// --------------------------------------------------------------- prologue
__global__ void td4_prologue(Td4Const tc, ParamBlock pb, const double* __restrict__ theta, int theta_stride,
                             const Td4FitConst* __restrict__ fcs, const int* __restrict__ status, int n_fits,
                             Td4Table* __restrict__ tabs) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_fits || (status && status[f] != 1)) return;
  const double* th = theta ? theta + (int64_t)f * theta_stride : pb.v;
  const Td4FitConst& fc = fcs[f];
  Td4Table t;
  bool ok = fc.sigma > 0.0;
  auto lineshape = [&](double m0, double w0, int L, double sum2, double dif2, double* out) {
    const double x = m0 * m0;
    const double lam = (x - sum2) * (x - dif2);
    const double q02 = 0.25 * lam / x;
    double poly = L == 1 ? 1.0 + q02 * tc.r2 : 1.0;
    double q0pow = sqrt(q02);
    if (L == 1) q0pow *= q02;
    out[0] = x;
    out[1] = w0 * x * poly / q0pow;
    out[2] = sqrt(poly);
    if (!(m0 > 0.0) || !(w0 > 0.0) || !(lam > 0.0)) ok = false;
  };
  for (int r = 0; r < kTd4MaxRes; ++r) {
    t.r12[r][0] = t.r12[r][1] = t.r12[r][2] = 0.0;
    t.r34[r][0] = t.r34[r][1] = t.r34[r][2] = 0.0;
    if (r < tc.n12 && !tc.nr12[r]) lineshape(fc.m0_12[r], fc.w0_12[r], tc.L12[r], tc.sum12, tc.dif12, t.r12[r]);
    if (r < tc.n34 && !tc.nr34[r]) lineshape(fc.m0_34[r], fc.w0_34[r], tc.L34[r], tc.sum34, tc.dif34, t.r34[r]);
  }
  for (int k = 0; k < kTd4MaxAmp; ++k) {
    const bool in = k < tc.K;
    t.c[k][0] = in ? th[2 * k] : 0.0;
    t.c[k][1] = in ? th[2 * k + 1] : 0.0;
    t.cb[k][0] = in ? th[2 * tc.K + 2 * k] : 0.0;
    t.cb[k][1] = in ? th[2 * tc.K + 2 * k + 1] : 0.0;
  }
  t.x = th[4 * tc.K];
  t.y = th[4 * tc.K + 1];
  t.sigma = fc.sigma;
  if (!(fabs(t.y) < 1.0) || !isfinite(t.x)) ok = false;
  t.valid = ok ? 1.0 : 0.0;
  tabs[f] = t;
}

// ----------------------------------------------------------- events pass
template <bool GRAD, int KMAX>
__global__ __launch_bounds__(kBlock) void td4_events(Td4Const tc, const Td4Table* __restrict__ tabs,
                                                     const int* __restrict__ status, const double* __restrict__ ev,
                                                     int64_t ld, int64_t n, int chunk, int64_t nch, int n_fits,
                                                     double* __restrict__ part) {
  constexpr int NV = GRAD ? 3 + 4 * KMAX : 1;
  __shared__ double lds[block_sum_lds(NV)];
  // fits vary fastest: the workgroups of one event chunk run together and share it through L2
  const int64_t ch = blockIdx.x / n_fits;
  const int f = (int)(blockIdx.x - ch * n_fits);
  if (status && status[f] != 1) return;
  const Td4Table& tb = tabs[f];
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const double s = tb.sigma, s2 = s * s, inv2s2 = 0.5 / s2;
  const double G = tc.gamma;
  const double ap = G * (1.0 - tb.y), am = G * (1.0 + tb.y);
  const cplx ac = {G, -G * tb.x};
  const int64_t base = ch * chunk;
  const int64_t end = base + chunk < n ? base + chunk : n;
  for (int64_t i = base + threadIdx.x; i < end; i += kBlock) {
    cplx B[KMAX];
    td4_basis<KMAX>(tc, tb, ev[i], ev[ld + i], ev[2 * ld + i], ev[3 * ld + i], ev[4 * ld + i], B);
    const double t = ev[5 * ld + i];
    cplx A = {0.0, 0.0}, Ab = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      if (k < tc.K) {
        const cplx x = cmul({tb.c[k][0], tb.c[k][1]}, B[k]);
        const cplx y = cmul({tb.cb[k][0], tb.cb[k][1]}, B[k]);
        A = {A.re + x.re, A.im + x.im};
        Ab = {Ab.re + y.re, Ab.im + y.im};
      }
    }
    const double g = exp(-t * t * inv2s2);
    double hp, dhp, hm, dhm;
    cplx hc, dhc;
    h_real(tc, ap, t, s, s2, g, hp, dhp);
    h_real(tc, am, t, s, s2, g, hm, dhm);
    h_cplx(tc, ac, t, s, s2, g, hc, dhc);
    const double Hc = 0.5 * (hp + hm), Hs = 0.5 * (hp - hm);
    const double a2 = A.re * A.re + A.im * A.im, b2 = Ab.re * Ab.re + Ab.im * Ab.im;
    const double zr = A.re * Ab.re + A.im * Ab.im, zi = A.re * Ab.im - A.im * Ab.re;  // conj(A) Abar
    const double R = 0.5 * ((a2 + b2) * Hc + (a2 - b2) * hc.re - 2.0 * zr * Hs - 2.0 * zi * hc.im);
    acc[0] -= log_fast(R);
    if (GRAD) {
      const double w = -rcp_nr(R);
      const double hpc = Hc + hc.re, hmc = Hc - hc.re;
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < tc.K) {
          // u = conj(A) B_k, v = conj(Abar) B_k
          const cplx u = {A.re * B[k].re + A.im * B[k].im, A.re * B[k].im - A.im * B[k].re};
          const cplx v = {Ab.re * B[k].re + Ab.im * B[k].im, Ab.re * B[k].im - Ab.im * B[k].re};
          acc[1 + 2 * k] += w * (hpc * u.re - Hs * v.re + hc.im * v.im);
          acc[2 + 2 * k] += w * (-hpc * u.im + Hs * v.im + hc.im * v.re);
          acc[1 + 2 * KMAX + 2 * k] += w * (hmc * v.re - Hs * u.re - hc.im * u.im);
          acc[2 + 2 * KMAX + 2 * k] += w * (-hmc * v.im + Hs * u.im - hc.im * u.re);
        }
      }
      // x: d hc/dx = -i G dh(ac);  y: d hp/dy = -G dh(ap), d hm/dy = +G dh(am)
      const double dcos = G * dhc.im, dsin = -G * dhc.re;
      acc[1 + 4 * KMAX] += w * 0.5 * ((a2 - b2) * dcos - 2.0 * zi * dsin);
      const double dHc = 0.5 * G * (dhm - dhp), dHs = -0.5 * G * (dhp + dhm);
      acc[2 + 4 * KMAX] += w * 0.5 * ((a2 + b2) * dHc - 2.0 * zr * dHs);
    }
  }
  block_sum_row<NV>(acc, lds, part + ((int64_t)f * nch + ch) * NV);
}

// ---------------------------------------------------- normalization matrix
constexpr int kTd4RowBlock = 4;

template <int KMAX>
__global__ __launch_bounds__(kBlock) void td4_mrows(Td4Const tc, const Td4Table* __restrict__ tabs,
                                                    const double* __restrict__ mc, int64_t ld, int64_t n, int chunk,
                                                    int64_t nch, int n_fits, int i0, double* __restrict__ part) {
  constexpr int NV = 2 * kTd4RowBlock * KMAX;
  __shared__ double lds[block_sum_lds(NV)];
  const int64_t ch = blockIdx.x / n_fits;
  const int f = (int)(blockIdx.x - ch * n_fits);
  const Td4Table& tb = tabs[f];
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const int64_t base = ch * chunk;
  const int64_t end = base + chunk < n ? base + chunk : n;
  for (int64_t i = base + threadIdx.x; i < end; i += kBlock) {
    cplx B[KMAX];
    td4_basis<KMAX>(tc, tb, mc[i], mc[ld + i], mc[2 * ld + i], mc[3 * ld + i], mc[4 * ld + i], B);
#pragma unroll
    for (int ib = 0; ib < kTd4RowBlock; ++ib) {
      cplx bi = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < KMAX; ++k)
        if (k == i0 + ib) bi = B[k];
#pragma unroll
      for (int j = 0; j < KMAX; ++j) {
        acc[2 * (ib * KMAX + j)] += bi.re * B[j].re + bi.im * B[j].im;
        acc[2 * (ib * KMAX + j) + 1] += bi.im * B[j].re - bi.re * B[j].im;
      }
    }
  }
  block_sum_row<NV>(acc, lds, part + ((int64_t)f * nch + ch) * NV);
}

__global__ __launch_bounds__(kFinalBlock) void td4_mrows_finalize(Td4Const tc, const double* __restrict__ part,
                                                                  int64_t nch, int nv, int kmax, int i0,
                                                                  double inv_n, double* __restrict__ Mc) {
  __shared__ double scratch[kFinalBlock];
  __shared__ double res[kBlock];
  const int f = blockIdx.x;
  sum_rows_t<kFinalBlock>(part + (int64_t)f * nch * nv, nch, nv, scratch, res);
  const int K = tc.K;
  double* M = Mc + (int64_t)f * 2 * kTd4MaxAmp * kTd4MaxAmp;
  for (int t = threadIdx.x; t < kTd4RowBlock * kmax; t += kFinalBlock) {
    const int ib = t / kmax, j = t - ib * kmax;
    const int i = i0 + ib;
    if (i < K && j < K) {
      M[2 * (i * kTd4MaxAmp + j)] = inv_n * res[2 * t];
      M[2 * (i * kTd4MaxAmp + j) + 1] = inv_n * res[2 * t + 1];
    }
  }
}

// ---------------------------------------------------------------- finalize
// I = 1/2 [(a+b) cy + (a-b) cx - 2 Re(z) y cy - 2 Im(z) x cx], a = c^H M c form for A,
// b for Abar, z = <conj(A) Abar> = sum_kl conj(c_k) cb_l M_lk; cy = 1/(G(1-y^2)),
// cx = 1/(G(1+x^2)).  X_k = sum_j M_kj conj(c_j), Y_k = sum_j M_kj conj(cb_j),
// U_k = sum_l cb_l M_lk, V_l = sum_k conj(c_k) M_lk.
__global__ __launch_bounds__(kFinalBlock) void td4_finalize(Td4Const tc, const Td4Table* __restrict__ tabs,
                                                       const int* __restrict__ status, const double* __restrict__ part,
                                                       int64_t rows, int nv, int kmax, int with_grad,
                                                       const double* __restrict__ Mc, double n_events,
                                                       double* __restrict__ out, int out_stride,
                                                       double* __restrict__ out_user) {
  __shared__ double scratch[kFinalBlock];
  __shared__ double res[kBlock];
  __shared__ double M[2 * kTd4MaxAmp * kTd4MaxAmp];
  __shared__ double gI[4 * kTd4MaxAmp + 2];
  __shared__ double Ish;
  const int f = blockIdx.x;
  if (status && status[f] != 1) return;
  const Td4Table& tb = tabs[f];
  const int K = tc.K, P = tc.n_params;
  const int t = threadIdx.x;
  sum_rows_t<kFinalBlock>(part + (int64_t)f * rows * nv, rows, nv, scratch, res);
  for (int i = t; i < 2 * kTd4MaxAmp * kTd4MaxAmp; i += kFinalBlock)
    M[i] = Mc[(int64_t)f * 2 * kTd4MaxAmp * kTd4MaxAmp + i];
  __syncthreads();
  if (t == 0) {
    const double G = tc.gamma, x = tb.x, y = tb.y;
    const double cy = 1.0 / (G * (1.0 - y * y)), cx = 1.0 / (G * (1.0 + x * x));
    auto m = [&](int i, int j) { return cplx{M[2 * (i * kTd4MaxAmp + j)], M[2 * (i * kTd4MaxAmp + j) + 1]}; };
    double a = 0.0, b = 0.0, zr = 0.0, zi = 0.0;
    double Xr[kTd4MaxAmp], Xi[kTd4MaxAmp], Yr[kTd4MaxAmp], Yi[kTd4MaxAmp];
    double Ur[kTd4MaxAmp], Ui[kTd4MaxAmp], Vr[kTd4MaxAmp], Vi[kTd4MaxAmp];
    for (int k = 0; k < K; ++k) {
      Xr[k] = Xi[k] = Yr[k] = Yi[k] = Ur[k] = Ui[k] = Vr[k] = Vi[k] = 0.0;
      for (int j = 0; j < K; ++j) {
        const cplx mkj = m(k, j), mjk = m(j, k);
        const double cjr = tb.c[j][0], cji = tb.c[j][1], bjr = tb.cb[j][0], bji = tb.cb[j][1];
        // X_k += M_kj conj(c_j), Y_k += M_kj conj(cb_j)
        Xr[k] += mkj.re * cjr + mkj.im * cji;
        Xi[k] += mkj.im * cjr - mkj.re * cji;
        Yr[k] += mkj.re * bjr + mkj.im * bji;
        Yi[k] += mkj.im * bjr - mkj.re * bji;
        // U_k += cb_j M_jk, V_k += conj(c_j) M_kj
        Ur[k] += bjr * mjk.re - bji * mjk.im;
        Ui[k] += bjr * mjk.im + bji * mjk.re;
        Vr[k] += cjr * mkj.re + cji * mkj.im;
        Vi[k] += cjr * mkj.im - cji * mkj.re;
      }
      a += tb.c[k][0] * Xr[k] - tb.c[k][1] * Xi[k];
      b += tb.cb[k][0] * Yr[k] - tb.cb[k][1] * Yi[k];
      // z = sum_k conj(c_k) U_k
      zr += tb.c[k][0] * Ur[k] + tb.c[k][1] * Ui[k];
      zi += tb.c[k][0] * Ui[k] - tb.c[k][1] * Ur[k];
    }
    const double I = 0.5 * ((a + b) * cy + (a - b) * cx - 2.0 * zr * y * cy - 2.0 * zi * x * cx);
    Ish = I;
    for (int k = 0; k < K; ++k) {
      gI[2 * k] = 0.5 * ((cy + cx) * 2.0 * Xr[k] - 2.0 * y * cy * Ur[k] - 2.0 * x * cx * Ui[k]);
      gI[2 * k + 1] = 0.5 * (-2.0 * (cy + cx) * Xi[k] - 2.0 * y * cy * Ui[k] + 2.0 * x * cx * Ur[k]);
      gI[2 * K + 2 * k] = 0.5 * ((cy - cx) * 2.0 * Yr[k] - 2.0 * y * cy * Vr[k] - 2.0 * x * cx * Vi[k]);
      gI[2 * K + 2 * k + 1] = 0.5 * (-2.0 * (cy - cx) * Yi[k] + 2.0 * y * cy * Vi[k] - 2.0 * x * cx * Vr[k]);
    }
    const double dcx = -2.0 * x * G * cx * cx, dcy = 2.0 * y * G * cy * cy;
    gI[4 * K] = 0.5 * ((a - b) * dcx - 2.0 * zi * (cx + x * dcx));
    gI[4 * K + 1] = 0.5 * ((a + b) * dcy - 2.0 * zr * (cy + y * dcy));
  }
  __syncthreads();
  const double I = Ish;
  const bool ok = tb.valid != 0.0 && I > 0.0 && isfinite(I);
  double* o = out + (int64_t)f * out_stride;
  if (t == 0) {
    o[0] = ok ? res[0] + n_events * log(I) : INFINITY;
    o[1 + P] = I;
    if (out_user) out_user[0] = o[0];
  }
  if (t < P) {
    o[2 + P + t] = gI[t];
    if (with_grad) {
      // event slots: c at 1 + t, cb at 1 + 2 kmax + (t - 2K), x and y at 1 + 4 kmax
      int slot;
      if (t < 2 * K) slot = 1 + t;
      else if (t < 4 * K) slot = 1 + 2 * kmax + (t - 2 * K);
      else slot = 1 + 4 * kmax + (t - 4 * K);
      const double g = ok ? res[slot] + n_events * gI[t] / I : NAN;
      o[1 + t] = g;
      if (out_user) out_user[1 + t] = g;
    }
  }
}

// Events outside the observable domain: m12 >= m1 + m2, m34 >= m3 + m4,
// m12 + m34 <= M, |cos| <= 1, |phi| <= pi, t finite (relative slack 1e-9).
__global__ void td4_check(Td4Const tc, const double* __restrict__ ev, int64_t ld, int64_t n,
                          unsigned long long* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool b = false;
  if (i < n) {
    const double tol = 1e-9;
    const double m12 = ev[i], m34 = ev[ld + i], c12 = ev[2 * ld + i], c34 = ev[3 * ld + i];
    const double phi = ev[4 * ld + i], t = ev[5 * ld + i];
    const double lo12 = sqrt(tc.sum12), lo34 = sqrt(tc.sum34);
    b = !(m12 >= lo12 * (1 - tol) && m34 >= lo34 * (1 - tol) && m12 + m34 <= tc.M * (1 + tol) &&
          fabs(c12) <= 1.0 && fabs(c34) <= 1.0 && fabs(phi) <= M_PI * (1 + tol) && isfinite(t));
  }
  const unsigned long long cnt = __ballot(b);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(bad, (unsigned long long)__popcll(cnt));
}

// R(x_i, t_i) / I per event (I read from the finalize output).
__global__ void td4_eval(Td4Const tc, const Td4Table* __restrict__ tab, const double* __restrict__ ev, int64_t ld,
                         int64_t n, const double* __restrict__ norm, double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Td4Table& tb = *tab;
  cplx B[kTd4MaxAmp];
  td4_basis<kTd4MaxAmp>(tc, tb, ev[i], ev[ld + i], ev[2 * ld + i], ev[3 * ld + i], ev[4 * ld + i], B);
  cplx A = {0.0, 0.0}, Ab = {0.0, 0.0};
  for (int k = 0; k < tc.K; ++k) {
    const cplx x = cmul({tb.c[k][0], tb.c[k][1]}, B[k]);
    const cplx y = cmul({tb.cb[k][0], tb.cb[k][1]}, B[k]);
    A = {A.re + x.re, A.im + x.im};
    Ab = {Ab.re + y.re, Ab.im + y.im};
  }
  const double t = ev[5 * ld + i], s = tb.sigma, s2 = s * s;
  const double g = exp(-t * t * 0.5 / s2), G = tc.gamma;
  double hp, dhp, hm, dhm;
  cplx hc, dhc;
  h_real(tc, G * (1.0 - tb.y), t, s, s2, g, hp, dhp);
  h_real(tc, G * (1.0 + tb.y), t, s, s2, g, hm, dhm);
  h_cplx(tc, {G, -G * tb.x}, t, s, s2, g, hc, dhc);
  const double a2 = A.re * A.re + A.im * A.im, b2 = Ab.re * Ab.re + Ab.im * Ab.im;
  const double zr = A.re * Ab.re + A.im * Ab.im, zi = A.re * Ab.im - A.im * Ab.re;
  const double R = 0.5 * ((a2 + b2) * 0.5 * (hp + hm) + (a2 - b2) * hc.re - 2.0 * zr * 0.5 * (hp - hm) -
                          2.0 * zi * hc.im);
  p[i] = R / *norm;
}

// ---------------------------------------------------------------- launchers
int td4_kmax(int K) { return K <= 10 ? 10 : 12; }
int td4_nv(int kmax, bool grad) { return grad ? 3 + 4 * kmax : 1; }

// Fourier coefficients a_n (n = 1..N) of f(theta) = exp(-t^2)(L^2 + t^2),
// t = L tan(theta/2), by the trapezoidal rule on 2M - 1 interior points of
// (-pi, pi) with M = 2N (f vanishes at the end points), L = sqrt(N/sqrt 2).
void td4_weideman_coefficients(double* a, double* L_out) {
  const int N = kWeidN, M = 2 * N;
  const double L = std::sqrt(N / std::sqrt(2.0));
  std::vector<double> th, fv;
  for (int k = -M + 1; k <= M - 1; ++k) {
    const double t = k * M_PI / M;
    const double u = L * std::tan(0.5 * t);
    th.push_back(t);
    fv.push_back(std::exp(-u * u) * (L * L + u * u));
  }
  for (int n = 1; n <= N; ++n) {
    long double s = 0.0L;
    for (size_t j = 0; j < th.size(); ++j) s += (long double)fv[j] * std::cos((long double)n * th[j]);
    a[n - 1] = (double)(s / (2.0L * M));
  }
  *L_out = L;
}

void td4_launch_prologue(const Td4Const& tc, const ParamBlock* pb, const double* theta, int theta_stride,
                         const Td4FitConst* fc, const int* status, int n_fits, Td4Table* tabs, hipStream_t s) {
  ParamBlock zero;
  hipLaunchKernelGGL(td4_prologue, dim3((n_fits + 63) / 64), dim3(64), 0, s, tc, pb ? *pb : zero,
                     pb ? nullptr : theta, theta_stride, fc, status, n_fits, tabs);
}

void td4_launch_check(const Td4Const& tc, const double* ev, int64_t ld, int64_t n, unsigned long long* bad,
                      hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(td4_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tc, ev, ld, n, bad);
}

void td4_launch_mmatrix(const Td4Const& tc, const Td4Table* tabs, int n_fits, const double* mc, int64_t ld_mc,
                        int64_t n_mc, int chunk, double* part, double* Mc, hipStream_t s) {
  const int kmax = td4_kmax(tc.K);
  const int64_t nch = (n_mc + chunk - 1) / chunk;
  const int nv = 2 * kTd4RowBlock * kmax;
  for (int i0 = 0; i0 < tc.K; i0 += kTd4RowBlock) {
    const dim3 g((unsigned)(nch * n_fits)), b(kBlock);
    if (kmax == 10)
      hipLaunchKernelGGL((td4_mrows<10>), g, b, 0, s, tc, tabs, mc, ld_mc, n_mc, chunk, nch, n_fits, i0, part);
    else
      hipLaunchKernelGGL((td4_mrows<12>), g, b, 0, s, tc, tabs, mc, ld_mc, n_mc, chunk, nch, n_fits, i0, part);
    hipLaunchKernelGGL(td4_mrows_finalize, dim3(n_fits), dim3(kFinalBlock), 0, s, tc, part, nch, nv, kmax, i0,
                       1.0 / (double)n_mc, Mc);
  }
}

void td4_launch_events(const Td4Const& tc, const Td4Table* tabs, const int* status, int n_fits, const double* ev,
                       int64_t ld, int64_t n, int chunk, bool grad, double* part, hipStream_t s) {
  const int64_t nch = (n + chunk - 1) / chunk;
  if (nch == 0) return;
  const int kmax = td4_kmax(tc.K);
  const dim3 g((unsigned)(nch * n_fits)), b(kBlock);
#define FN_TD4(G, K) \
  hipLaunchKernelGGL((td4_events<G, K>), g, b, 0, s, tc, tabs, status, ev, ld, n, chunk, nch, n_fits, part)
  if (kmax == 10) {
    if (grad) FN_TD4(true, 10); else FN_TD4(false, 10);
  } else {
    if (grad) FN_TD4(true, 12); else FN_TD4(false, 12);
  }
#undef FN_TD4
}

void td4_launch_finalize(const Td4Const& tc, const Td4Table* tabs, const int* status, int n_fits, const double* part,
                         int64_t rows_per_fit, bool grad, const double* Mc, double n_events, double* out,
                         int out_stride, double* out_user, hipStream_t s) {
  const int kmax = td4_kmax(tc.K);
  hipLaunchKernelGGL(td4_finalize, dim3(n_fits), dim3(kFinalBlock), 0, s, tc, tabs, status, part, rows_per_fit,
                     td4_nv(kmax, grad), kmax, grad ? 1 : 0, Mc, n_events, out, out_stride, out_user);
}

void td4_launch_eval(const Td4Const& tc, const Td4Table* tab, const double* ev, int64_t ld, int64_t n,
                     const double* norm, double* p, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(td4_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tc, tab, ev, ld, n, norm, p);
}

}  // namespace fn
