// One-observable mixture models: components added with fractions into one
// density (the paper's basic and combination PDFs, Sec. 1 and Fig. 1).
//
//   P(x) = sum_k w_k s_k(x) / N_k,   w_k = f_k (k < K-1),  w_{K-1} = 1 - sum f
//
// s_k is a component shape (Gaussian, exponential, Argus with power 1/2,
// non-relativistic Breit-Wigner) and N_k its integral over [lo, hi] in closed
// form, so the overall normalization is 1 and NLL = -sum_i ln P(x_i).
//
// Kernels:
//   mix1d_prologue  theta -> per-fit table (1/N_k, d ln N_k, shape constants)
//   mix1d_events    one workgroup per chunk of events: -ln P and its
//                   gradient slots, reduced to one row per chunk
//   mix1d_finalize  rows -> NLL, gradient mapped from slots to parameters
//   mix1d_eval      P(x_i) per event;  mix1d_check  out-of-range count
// HBM traffic per event is 8 bytes (x); the work is FP64 exp/log and a few
// FMAs, so the events kernel is bound by FP64 VALU issue, not by HBM.
#include <cmath>

#include "device_common.hpp"
#include "fastmath.hpp"
#include "kernels.hpp"

namespace fn {

// Lower incomplete gamma function gamma(a, y), y >= 0, for a = 3/2 and 5/2.
// Series y^a e^-y sum_n y^n / (a (a+1) ... (a+n)) below y = 1, closed forms
// through erf above (gamma(3/2,y) = sqrt(pi)/2 erf(sqrt y) - sqrt(y) e^-y and
// gamma(5/2,y) = 3/2 gamma(3/2,y) - y^(3/2) e^-y).
__device__ static double lower_gamma_half(int twice_a, double y) {
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

__global__ void mix1d_prologue(Mix1dConst mc, ParamBlock pb, const double* __restrict__ theta_dev,
                               int n_fits, int theta_stride, Mix1dTable* __restrict__ tab) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_fits) return;
  const double* th = theta_dev ? theta_dev + (int64_t)f * theta_stride : pb.v;
  Mix1dTable t;
  bool ok = true;
  const double lo = mc.lo, hi = mc.hi;
  double rest = 1.0;
  for (int k = 0; k < kMixMaxComp; ++k) {
    t.frac[k] = 0.0; t.invN[k] = 0.0; t.a[k] = 0.0; t.b[k] = 0.0; t.c[k] = 0.0;
    t.dlnN[k][0] = 0.0; t.dlnN[k][1] = 0.0;
  }
  for (int k = 0; k < mc.K; ++k) {
    if (k < mc.K - 1) {
      t.frac[k] = th[mc.fidx[k]];
      rest -= t.frac[k];
    } else {
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
  }
  t.valid = ok ? 1.0 : 0.0;
  tab[f] = t;
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
      const double s = rcp_nr(__builtin_fma(d, d, t.b[k]));
      if (GRAD) { dl0 = 2.0 * d * s; dl1 = -0.5 * t.c[k] * s; }
      return s;
    }
  }
}

// One chunk of events -> one partial row (shared by the single-fit and the
// batched launches so that both produce the same bits).
template <bool GRAD, int KMAX>
__device__ inline void mix1d_chunk(const Mix1dConst& mc, const Mix1dTable* __restrict__ tabp,
                                   const double* __restrict__ x, int64_t n, int64_t chunk_idx,
                                   int chunk, double* __restrict__ out_row, double* lds) {
  constexpr int NV = GRAD ? mix_nv(KMAX) : 1;
  const Mix1dTable& t = *tabp;
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const int64_t base = chunk_idx * chunk;
  const int64_t end = base + chunk < n ? base + chunk : n;
  for (int64_t i = base + threadIdx.x; i < end; i += kBlock) {
    const double xv = x[i];
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
    acc[0] -= log_fast(P);
    if (GRAD) {
      const double w = -rcp_nr(P);
      double ul = 0.0;  // density of the last component (it takes 1 - sum f)
#pragma unroll
      for (int k = 0; k < KMAX; ++k)
        if (k == mc.K - 1) ul = u[k];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < mc.K) {
          const double wu = w * t.frac[k] * u[k];
          acc[1 + 2 * k] += wu * (dl[k][0] - t.dlnN[k][0]);
          acc[2 + 2 * k] += wu * (dl[k][1] - t.dlnN[k][1]);
          if (k < mc.K - 1) acc[1 + 2 * KMAX + k] += w * (u[k] - ul);
        }
      }
    }
  }
  block_sum_row<NV>(acc, lds, out_row);
}

// Level 2 and the slot -> parameter map (slots sharing a parameter are added
// in slot order).  out: [NLL, grad(P), I = 1, dI = 0]; out_user: [NLL, grad(P)].
__device__ inline void mix1d_finalize_one(const Mix1dConst& mc, const Mix1dTable& t,
                                          const double* part, int64_t nrows, int nv, int kmax,
                                          int with_grad, double* out, double* out_user, double* scratch,
                                          double* res) {
  sum_rows(part, nrows, nv, scratch, res);
  const int P = mc.n_params;
  const int p = threadIdx.x;
  const bool ok = t.valid != 0.0;
  if (p == 0) {
    out[0] = ok ? res[0] : INFINITY;
    out[1 + P] = 1.0;
    if (out_user) out_user[0] = out[0];
  }
  if (p < P) {
    out[2 + P + p] = 0.0;
    if (with_grad) {
      double g = 0.0;
      for (int k = 0; k < mc.K; ++k) {
        for (int j = 0; j < mc.npar[k]; ++j)
          if (mc.pidx[k][j] == p) g += res[1 + 2 * k + j];
        if (k < mc.K - 1 && mc.fidx[k] == p) g += res[1 + 2 * kmax + k];
      }
      if (!ok) g = NAN;
      out[1 + p] = g;
      if (out_user) out_user[1 + p] = g;
    }
  }
}

// Single fit: one workgroup per chunk of events, one row of partial sums each.
template <bool GRAD, int KMAX>
__global__ __launch_bounds__(kBlock) void mix1d_events(Mix1dConst mc, const Mix1dTable* __restrict__ tab,
                                                       const double* __restrict__ x, int64_t n, int chunk,
                                                       double* __restrict__ part) {
  constexpr int NV = GRAD ? mix_nv(KMAX) : 1;
  __shared__ double lds[kWaves * NV];
  mix1d_chunk<GRAD, KMAX>(mc, tab, x, n, blockIdx.x, chunk, part + (int64_t)blockIdx.x * NV, lds);
}

// Batched form: work item w = (fit, chunk) from a flat list; per-fit tables,
// event pointers, sizes and row bases come from device arrays.  The chunk
// routine is the one the single-fit kernel runs, so a fit's rows hold the same
// bits alone and in a batch.
template <bool GRAD, int KMAX>
__global__ __launch_bounds__(kBlock) void mix1d_events_batched(
    Mix1dConst mc, const Mix1dTable* __restrict__ tabs, const double* const* __restrict__ ev,
    const int64_t* __restrict__ n, const int32_t* __restrict__ item_fit,
    const int64_t* __restrict__ item_chunk, const int64_t* __restrict__ part_base, int chunk,
    double* __restrict__ part) {
  constexpr int NV = GRAD ? mix_nv(KMAX) : 1;
  __shared__ double lds[kWaves * NV];
  const int fit = item_fit[blockIdx.x];
  const int64_t ch = item_chunk[blockIdx.x];
  mix1d_chunk<GRAD, KMAX>(mc, tabs + fit, ev[fit], n[fit], ch, chunk, part + (part_base[fit] + ch) * NV, lds);
}

// Batched level-2: one workgroup per fit, output rows of stride out_stride.
__global__ __launch_bounds__(kBlock) void mix1d_finalize_batched(
    Mix1dConst mc, const Mix1dTable* __restrict__ tabs, const double* __restrict__ part,
    const int64_t* __restrict__ part_base, const int64_t* __restrict__ nrows, int nv, int kmax,
    int with_grad, double* __restrict__ out, int out_stride) {
  __shared__ double scratch[kBlock];
  __shared__ double res[kBlock];
  const int f = blockIdx.x;
  mix1d_finalize_one(mc, tabs[f], part + part_base[f] * nv, nrows[f], nv, kmax, with_grad,
                     out + (int64_t)f * out_stride, nullptr, scratch, res);
}

// Level-2 step of a single fit.
__global__ __launch_bounds__(kBlock) void mix1d_finalize(Mix1dConst mc, const Mix1dTable* __restrict__ tab,
                                                         const double* __restrict__ part, int64_t nrows,
                                                         int nv, int kmax, int with_grad,
                                                         double* __restrict__ out, double* __restrict__ out_user) {
  __shared__ double scratch[kBlock];
  __shared__ double res[kBlock];
  mix1d_finalize_one(mc, *tab, part, nrows, nv, kmax, with_grad, out, out_user, scratch, res);
}

__global__ void mix1d_eval(Mix1dConst mc, const Mix1dTable* __restrict__ tab, const double* __restrict__ x,
                           int64_t n, double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Mix1dTable& t = *tab;
  double P = 0.0, d0, d1;
  for (int k = 0; k < mc.K; ++k) P += t.frac[k] * mix_shape<false>(mc.type[k], t, k, x[i], d0, d1) * t.invN[k];
  p[i] = t.valid != 0.0 ? P : NAN;
}

__global__ void mix1d_check(Mix1dConst mc, const double* __restrict__ x, int64_t n,
                            unsigned long long* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool b = i < n && !(x[i] >= mc.lo && x[i] <= mc.hi);
  const unsigned long long cnt = __ballot(b);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(bad, (unsigned long long)__popcll(cnt));
}

// ---------------------------------------------------------------- launchers
int mix1d_kmax(int K) { return K <= 2 ? 2 : 8; }
int mix1d_nv(int kmax, bool grad) { return grad ? mix_nv(kmax) : 1; }

void mix1d_launch_prologue(const Mix1dConst& mc, const ParamBlock& pb, const double* theta_dev, int n_fits,
                           int theta_stride, Mix1dTable* tab, hipStream_t s) {
  hipLaunchKernelGGL(mix1d_prologue, dim3((n_fits + 63) / 64), dim3(64), 0, s, mc, pb, theta_dev, n_fits,
                     theta_stride, tab);
}

void mix1d_launch_events(const Mix1dConst& mc, const Mix1dTable* tab, const double* x, int64_t n, int chunk,
                         int64_t nchunks, bool grad, double* part, hipStream_t s) {
  if (nchunks == 0) return;
  const int kmax = mix1d_kmax(mc.K);
  const dim3 g((unsigned)nchunks), b(kBlock);
#define FN_MIX(G, K) hipLaunchKernelGGL((mix1d_events<G, K>), g, b, 0, s, mc, tab, x, n, chunk, part)
  if (kmax == 2) {
    if (grad) FN_MIX(true, 2); else FN_MIX(false, 2);
  } else {
    if (grad) FN_MIX(true, 8); else FN_MIX(false, 8);
  }
#undef FN_MIX
}

void mix1d_launch_finalize(const Mix1dConst& mc, const Mix1dTable* tab, const double* part, int64_t nrows,
                           bool grad, double* out, double* out_user, hipStream_t s) {
  const int kmax = mix1d_kmax(mc.K);
  hipLaunchKernelGGL(mix1d_finalize, dim3(1), dim3(kBlock), 0, s, mc, tab, part, nrows, mix1d_nv(kmax, grad),
                     kmax, grad ? 1 : 0, out, out_user);
}

void mix1d_launch_events_batched(const Mix1dConst& mc, const Mix1dTable* tabs, const double* const* ev,
                                 const int64_t* n, const int32_t* item_fit, const int64_t* item_chunk,
                                 const int64_t* part_base, int64_t n_items, int chunk, bool grad, double* part,
                                 hipStream_t s) {
  if (n_items == 0) return;
  const int kmax = mix1d_kmax(mc.K);
  const dim3 g((unsigned)n_items), b(kBlock);
#define FN_MIXB(G, K)                                                                                        \
  hipLaunchKernelGGL((mix1d_events_batched<G, K>), g, b, 0, s, mc, tabs, ev, n, item_fit, item_chunk, part_base, \
                     chunk, part)
  if (kmax == 2) {
    if (grad) FN_MIXB(true, 2); else FN_MIXB(false, 2);
  } else {
    if (grad) FN_MIXB(true, 8); else FN_MIXB(false, 8);
  }
#undef FN_MIXB
}

void mix1d_launch_finalize_batched(const Mix1dConst& mc, const Mix1dTable* tabs, const double* part,
                                   const int64_t* part_base, const int64_t* nrows, int n_fits, bool grad,
                                   double* out, int out_stride, hipStream_t s) {
  if (n_fits == 0) return;
  const int kmax = mix1d_kmax(mc.K);
  hipLaunchKernelGGL(mix1d_finalize_batched, dim3(n_fits), dim3(kBlock), 0, s, mc, tabs, part, part_base, nrows,
                     mix1d_nv(kmax, grad), kmax, grad ? 1 : 0, out, out_stride);
}

void mix1d_launch_eval(const Mix1dConst& mc, const Mix1dTable* tab, const double* x, int64_t n, double* p,
                       hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(mix1d_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, mc, tab, x, n, p);
}

void mix1d_launch_check(const Mix1dConst& mc, const double* x, int64_t n, unsigned long long* bad,
                        hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(mix1d_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, mc, x, n, bad);
}

}  // namespace fn
