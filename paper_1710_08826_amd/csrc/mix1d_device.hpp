// Device code of the one-observable mixture shared by the single-fit kernels
// (mix1d.hip) and the batched ones (batch.hip): the prologue table, the
// component shapes, the per-chunk evaluation and the level-2 step.
#pragma once
#include <cmath>

#include "device_common.hpp"
#include "fastmath.hpp"

namespace fn {

// Lower incomplete gamma function gamma(a, y), y >= 0, for a = 3/2 and 5/2.
// Series y^a e^-y sum_n y^n / (a (a+1) ... (a+n)) below y = 1, closed forms
// through erf above (gamma(3/2,y) = sqrt(pi)/2 erf(sqrt y) - sqrt(y) e^-y and
// gamma(5/2,y) = 3/2 gamma(3/2,y) - y^(3/2) e^-y).
__device__ inline double lower_gamma_half(int twice_a, double y) {
  const double a = 0.5 * twice_a;
  if (y <= 0.0) return 0.0;
  if (y < 1.0) {
    double term = 1.0 / a, sum = term;
    for (int n = 1; n < 60; ++n) {
      term *= y / (a + n);
      sum += term;
      if (term < 1e-18 * sum) break;
    }
    return pow(y, a) * exp(-y) * sum;
  }
  const double ry = sqrt(y);
  const double g32 = 0.88622692545275801365 * erf(ry) - ry * exp(-y);
  if (twice_a == 3) return g32;
  return 1.5 * g32 - y * ry * exp(-y);
}

// theta -> component k of the per-fit table: its fraction, 1/N_k and
// d ln N_k / d(its parameters) from its closed-form integral on [lo, hi], and
// its shape constants (written in place).  Returns false when the parameters
// do not define a density.
__device__ inline bool mix1d_component(const Mix1dConst& mc, const double* __restrict__ th, int k, Mix1dTable& t) {
  bool ok = true;
  const double lo = mc.lo, hi = mc.hi;
  t.a[k] = 0.0; t.b[k] = 0.0; t.c[k] = 0.0;
  if (k < mc.K - 1) {
    t.frac[k] = th[mc.fidx[k]];
  } else {
    // the last component takes 1 - sum of the others, subtracted in order
    double rest = 1.0;
    for (int j = 0; j < mc.K - 1; ++j) rest -= th[mc.fidx[j]];
    t.frac[k] = rest;
  }
  const double p0 = th[mc.pidx[k][0]];
  const double p1 = mc.npar[k] > 1 ? th[mc.pidx[k][1]] : 0.0;
  double N = 0.0, d0 = 0.0, d1 = 0.0;
  switch (mc.type[k]) {
    case kGauss: {
      const double mu = p0, sg = p1;
      if (!(sg > 0.0)) { ok = false; break; }
      const double s2 = sg * 1.41421356237309504880;
      const double A = (lo - mu) / s2, B = (hi - mu) / s2;
      double D;
      if (A > 0.0) D = erfc(A) - erfc(B);
      else if (B < 0.0) D = erfc(-B) - erfc(-A);
      else D = erf(B) - erf(A);
      N = sg * 1.25331413731550025121 * D;  // sqrt(pi/2)
      const double eA = exp(-A * A), eB = exp(-B * B);
      d0 = (eA - eB) / N;
      d1 = 1.0 / sg + 1.41421356237309504880 * (A * eA - B * eB) / N;
      t.a[k] = mu; t.b[k] = 1.0 / sg;
      break;
    }
    case kExp: {
      const double tau = p0, D = hi - lo;
      if (fabs(tau) < 1e-12) N = D * (1.0 + 0.5 * tau * (hi + lo));
      else N = exp(tau * lo) * expm1(tau * D) / tau;
      const double td = tau * D;
      if (fabs(td) < 1e-3) d0 = 0.5 * (hi + lo) + tau * D * D / 12.0 - td * td * td * D / 720.0;
      else d0 = lo + D / (-expm1(-td)) - 1.0 / tau;
      t.a[k] = tau;
      break;
    }
    case kArgus: {
      const double m0 = p0, c = p1;
      if (!(m0 > 0.0) || !(c < 0.0)) { ok = false; break; }
      const double kk = -c, im2 = 1.0 / (m0 * m0);
      const double wlo = fmax(0.0, 1.0 - lo * lo * im2), whi = fmax(0.0, 1.0 - hi * hi * im2);
      const double k32 = pow(kk, -1.5), k52 = pow(kk, -2.5), h = 0.5 * m0 * m0;
      N = h * k32 * (lower_gamma_half(3, kk * wlo) - lower_gamma_half(3, kk * whi));
      const double dNc = h * k52 * (lower_gamma_half(5, kk * wlo) - lower_gamma_half(5, kk * whi));
      const double im3 = im2 / m0;
      const double flo = wlo > 0.0 ? sqrt(wlo) * exp(-kk * wlo) * 2.0 * lo * lo * im3 : 0.0;
      const double fhi = whi > 0.0 ? sqrt(whi) * exp(-kk * whi) * 2.0 * hi * hi * im3 : 0.0;
      const double dNm = 2.0 * N / m0 + h * (flo - fhi);
      d0 = dNm / N;
      d1 = dNc / N;
      t.a[k] = im2; t.b[k] = c; t.c[k] = 1.0 / m0;
      break;
    }
    case kBW: {
      const double m0 = p0, g = p1;
      if (!(g > 0.0)) { ok = false; break; }
      const double hg = 0.5 * g, uh = (hi - m0) / hg, ul = (lo - m0) / hg;
      N = (atan(uh) - atan(ul)) / hg;
      const double ih = 1.0 / (1.0 + uh * uh), il = 1.0 / (1.0 + ul * ul);
      const double dNm = (il - ih) / (hg * hg);
      const double dNg = -N / g + (-uh * ih + ul * il) / (g * hg);
      d0 = dNm / N;
      d1 = dNg / N;
      t.a[k] = m0; t.b[k] = hg * hg; t.c[k] = g;
      break;
    }
    default:
      ok = false;
  }
  if (!(N > 0.0) || !isfinite(N)) ok = false;
  t.invN[k] = 1.0 / N;
  t.dlnN[k][0] = d0;
  t.dlnN[k][1] = d1;
  return ok;
}

// The table entries past the components, the yield (extended likelihood) and
// the validity flag; ok: every component's check.
__device__ inline void mix1d_table_rest(const Mix1dConst& mc, const double* __restrict__ th, bool ok, Mix1dTable& t) {
  for (int k = mc.K; k < kMixMaxComp; ++k) {
    t.frac[k] = 0.0; t.invN[k] = 0.0; t.a[k] = 0.0; t.b[k] = 0.0; t.c[k] = 0.0;
    t.dlnN[k][0] = 0.0; t.dlnN[k][1] = 0.0;
  }
  t.yield = mc.yidx >= 0 ? th[mc.yidx] : 0.0;
  if (mc.yidx >= 0 && !(t.yield > 0.0 && isfinite(t.yield))) ok = false;
  t.valid = ok ? 1.0 : 0.0;
}

// theta -> per-fit table, the components one after the other (one thread per
// fit; the single-fit prologue gives each component its own thread).
__device__ inline void mix1d_table(const Mix1dConst& mc, const double* __restrict__ th, Mix1dTable& out) {
  bool ok = true;
  for (int k = 0; k < mc.K; ++k) ok = mix1d_component(mc, th, k, out) && ok;
  mix1d_table_rest(mc, th, ok, out);
}

// Component shape s(x) and d ln s / d(its parameters).
template <bool GRAD>
__device__ inline double mix_shape(int type, const Mix1dTable& t, int k, double x,
                                   double& dl0, double& dl1) {
  switch (type) {
    case kGauss: {
      const double z = (x - t.a[k]) * t.b[k];
      if (GRAD) { dl0 = z * t.b[k]; dl1 = z * z * t.b[k]; }
      return exp(-0.5 * z * z);
    }
    case kExp: {
      if (GRAD) { dl0 = x; dl1 = 0.0; }
      return exp(t.a[k] * x);
    }
    case kArgus: {
      const double w = 1.0 - x * x * t.a[k];
      if (!(w > 0.0)) { if (GRAD) { dl0 = 0.0; dl1 = 0.0; } return 0.0; }
      if (GRAD) { dl0 = (0.5 / w + t.b[k]) * 2.0 * x * x * t.a[k] * t.c[k]; dl1 = w; }
      return x * sqrt(w) * exp(t.b[k] * w);
    }
    default: {  // kBW
      const double d = x - t.a[k];
      const double s = rcp_fast(__builtin_fma(d, d, t.b[k]));
      if (GRAD) { dl0 = 2.0 * d * s; dl1 = -0.5 * t.c[k] * s; }
      return s;
    }
  }
}

// Type signature of a mixture compiled for its component types: 0 for the
// generic passes (types read at run time), 1 + t0 for one component of type
// t0, 5 + 4 t0 + t1 for two (types in MixType order).  The per-event passes of
// mixtures of one or two components are instantiated for each signature, so
// that each component's shape code is selected at compile time.
constexpr int kMixSigCount = 21;
__host__ __device__ constexpr int mix_sig_K(int sig) { return sig == 0 ? 0 : (sig < 5 ? 1 : 2); }
__host__ __device__ constexpr int mix_sig_type(int sig, int k) {
  return sig < 5 ? sig - 1 : (k == 0 ? (sig - 5) / 4 : (sig - 5) % 4);
}

// slot[s] += w * dP/d(slot s) at one point: shape parameters of component k at
// 2k, 2k + 1 (dP = f_k u_k (d ln s_k - d ln N_k)), fraction k < K-1 at
// 2 KMAX + k (dP = u_k - u_{K-1}, the last component taking 1 - sum f).
template <int KMAX>
__device__ __forceinline__ void mix1d_add_dp(int K, const Mix1dTable& t, const double (&u)[KMAX],
                                             const double (&dl)[KMAX][2], double w, double* slot) {
  double ul = 0.0;
#pragma unroll
  for (int k = 0; k < KMAX; ++k)
    if (k == K - 1) ul = u[k];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < K) {
      const double wu = w * t.frac[k] * u[k];
      slot[2 * k] += wu * (dl[k][0] - t.dlnN[k][0]);
      slot[2 * k + 1] += wu * (dl[k][1] - t.dlnN[k][1]);
      if (k < K - 1) slot[2 * KMAX + k] += w * (u[k] - ul);
    }
  }
}

// One chunk of events -> one partial row (shared by the single-fit and the
// batched launches so that both produce the same bits).  SIG: the type
// signature the code is compiled for (0: generic, KMAX components at most).
template <bool GRAD, int KMAX, int SIG = 0>
__device__ inline void mix1d_chunk(const Mix1dConst& mc, const Mix1dTable* __restrict__ tabp,
                                   const double* __restrict__ x, int64_t n, int64_t chunk_idx,
                                   int chunk, double* __restrict__ out_row, double* lds) {
  static_assert(SIG == 0 || KMAX == 2, "typed passes hold two components");
  constexpr int NV = GRAD ? mix_nv(KMAX) : 1;
  const int K = SIG ? mix_sig_K(SIG) : mc.K;
  const Mix1dTable& t = *tabp;
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const int64_t base = chunk_idx * chunk;
  const int64_t end = base + chunk < n ? base + chunk : n;
  LogProd lp;  // -sum ln P enters acc[0] once per thread, at the end
  for (int64_t i = base + threadIdx.x; i < end; i += kBlock) {
    const double xv = x[i];
    double u[KMAX], dl[KMAX][2];
    double P = 0.0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      u[k] = 0.0; dl[k][0] = 0.0; dl[k][1] = 0.0;
      if (k < K) {
        const int type = SIG ? mix_sig_type(SIG, k) : mc.type[k];
        u[k] = mix_shape<GRAD>(type, t, k, xv, dl[k][0], dl[k][1]) * t.invN[k];
        P += t.frac[k] * u[k];
      }
    }
    lp.mul(P);
    if (GRAD) mix1d_add_dp<KMAX>(K, t, u, dl, -rcp_fast(P), acc + 1);
  }
  acc[0] = -lp.log();
  block_sum_row<NV>(acc, lds, out_row);
}

// Binned data: bin b of nb uniform bins on [lo, hi] holds n_b events, and the
// density at its centre x_b = lo + (b + 1/2) Delta gives the expected count
// nu_b = N Delta P(x_b).  One chunk of bins -> one partial row:
//   STAT 0 (Poisson): [W, X, Y, dX slots, dY slots], W = sum n_b,
//                     X = sum_b P_b, Y = sum_b n_b ln P_b (N enters at the end)
//   STAT 1 (chi^2 over the bins with n_b > 0, N = *nptr):
//                     [W, C, D, dC slots], C = sum (n_b - nu_b)^2 / n_b,
//                     D = dC/dN = -2 Delta sum (n_b - nu_b) P_b / n_b
//   STAT 2:           [W] (the total count, when N = W for chi^2)
template <int KMAX, int STAT, bool GRAD>
__host__ __device__ constexpr int mix1d_binned_nv() {
  return STAT == 2 ? 1 : (GRAD ? 3 + (STAT == 0 ? 2 : 1) * (mix_nv(KMAX) - 1) : 3);
}

template <bool GRAD, int KMAX, int STAT>
__device__ inline void mix1d_binned_chunk(const Mix1dConst& mc, const Mix1dTable* __restrict__ tabp,
                                          const double* __restrict__ counts, int64_t nb, const double* nptr,
                                          int64_t chunk_idx, int chunk, double* __restrict__ out_row, double* lds) {
  constexpr int G = mix_nv(KMAX) - 1;
  constexpr int NV = mix1d_binned_nv<KMAX, STAT, GRAD>();
  const Mix1dTable& t = *tabp;
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const double delta = (mc.hi - mc.lo) / (double)nb;
  const double N = STAT == 1 ? (nptr ? *nptr : t.yield) : 0.0;
  const int64_t base = chunk_idx * chunk;
  const int64_t end = base + chunk < nb ? base + chunk : nb;
  for (int64_t b = base + threadIdx.x; b < end; b += kBlock) {
    const double n = counts[b];
    acc[0] += n;
    if (STAT == 2) continue;
    const double xv = mc.lo + ((double)b + 0.5) * delta;
    double u[KMAX], dl[KMAX][2];
    double P = 0.0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      u[k] = 0.0; dl[k][0] = 0.0; dl[k][1] = 0.0;
      if (k < mc.K) {
        u[k] = mix_shape<GRAD>(mc.type[k], t, k, xv, dl[k][0], dl[k][1]) * t.invN[k];
        P += t.frac[k] * u[k];
      }
    }
    if (STAT == 0) {
      acc[1] += P;
      const double cy = n != 0.0 ? n * rcp_fast(P) : 0.0;
      if (n != 0.0) acc[2] += n * log_fast(P);
      if (GRAD) {
        mix1d_add_dp<KMAX>(mc.K, t, u, dl, 1.0, acc + 3);
        mix1d_add_dp<KMAX>(mc.K, t, u, dl, cy, acc + 3 + G);
      }
    } else if (n > 0.0) {
      const double in = 1.0 / n;
      const double r = n - N * delta * P;  // n_b - nu_b
      acc[1] += r * r * in;
      acc[2] -= 2.0 * delta * r * P * in;
      if (GRAD) mix1d_add_dp<KMAX>(mc.K, t, u, dl, -2.0 * N * delta * r * in, acc + 3);
    }
  }
  block_sum_row<NV>(acc, lds, out_row);
}

// Gradient of parameter p from gradient slots (slots sharing a parameter are
// added in slot order).
__device__ inline double mix1d_param_grad(const Mix1dConst& mc, int kmax, const double* slots, int p) {
  double g = 0.0;
  for (int k = 0; k < mc.K; ++k) {
    for (int j = 0; j < mc.npar[k]; ++j)
      if (mc.pidx[k][j] == p) g += slots[2 * k + j];
    if (k < mc.K - 1 && mc.fidx[k] == p) g += slots[2 * kmax + k];
  }
  return g;
}

// Level 2 and the slot -> parameter map; with an expected yield nu (extended
// likelihood) NLL gains nu - N ln nu and d/dnu = 1 - N/nu.
// out: [NLL, grad(P), I = 1, dI = 0]; out_user: [NLL, grad(P)].
__device__ inline void mix1d_finalize_one(const Mix1dConst& mc, const Mix1dTable& t,
                                          const double* part, int64_t nrows, int nv, int kmax,
                                          int with_grad, double n_events, double* out, double* out_user,
                                          double* scratch, double* res) {
  // the validity flag and the yield as vector loads issued before the row
  // sums (a lane-varying zero offset: scalar loads would be waited for with
  // the first kernel argument, before the rows are requested)
  int zero = 0;
  asm volatile("" : "+v"(zero));
  const double valid = (&t.valid)[zero], yield = (&t.yield)[zero];
  sum_rows(part, nrows, nv, scratch, res);
  const int P = mc.n_params;
  const int p = threadIdx.x;
  const bool ok = valid != 0.0;
  const bool ext = mc.yidx >= 0;
  if (p == 0) {
    double v = res[0];
    if (ext) v += yield - n_events * log(yield);
    out[0] = ok ? v : INFINITY;
    out[1 + P] = 1.0;
    if (out_user) out_user[0] = out[0];
  }
  if (p < P) {
    out[2 + P + p] = 0.0;
    if (with_grad) {
      double g = mix1d_param_grad(mc, kmax, res + 1, p);
      if (ext && p == mc.yidx) g += 1.0 - n_events / yield;
      if (!ok) g = NAN;
      out[1 + p] = g;
      if (out_user) out_user[1 + p] = g;
    }
  }
}

// Level 2 of binned data and the statistic, N the yield parameter (extended)
// or the total count W:
//   Poisson  F = sum_b (nu_b - n_b ln nu_b) = N Delta X - W ln(N Delta) - Y
//   chi^2    F = C
// out: [F, grad(P)].
__device__ inline void mix1d_binned_finalize_one(const Mix1dConst& mc, const Mix1dTable& t, const double* part,
                                                 int64_t nrows, int nv, int kmax, int stat, int64_t nb,
                                                 int with_grad, double* out, double* scratch, double* res) {
  sum_rows(part, nrows, nv, scratch, res);
  const int P = mc.n_params;
  const int G = 3 * kmax;
  const int p = threadIdx.x;
  const bool ok = t.valid != 0.0;
  const bool ext = mc.yidx >= 0;
  const double W = res[0];
  const double delta = (mc.hi - mc.lo) / (double)nb;
  const double N = ext ? t.yield : W;
  const double nd = N * delta;
  if (p == 0) {
    const double v = stat == 0 ? nd * res[1] - W * log(nd) - res[2] : res[1];
    out[0] = ok ? v : INFINITY;
  }
  if (with_grad && p < P) {
    double g;
    if (stat == 0) {
      g = nd * mix1d_param_grad(mc, kmax, res + 3, p) - mix1d_param_grad(mc, kmax, res + 3 + G, p);
      if (ext && p == mc.yidx) g += delta * res[1] - W / N;
    } else {
      g = mix1d_param_grad(mc, kmax, res + 3, p);
      if (ext && p == mc.yidx) g += res[2];
    }
    out[1 + p] = ok ? g : NAN;
  }
}

// Total of the rows' first entries into *total (one workgroup).
__device__ inline void mix1d_binned_total_one(const double* part, int64_t nrows, double* total, double* scratch,
                                              double* res) {
  sum_rows(part, nrows, 1, scratch, res);
  if (threadIdx.x == 0) *total = res[0];
}

}  // namespace fn
