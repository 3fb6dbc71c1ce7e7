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
#include <hip/hip_ext.h>
#include <cmath>

#include "kernels.hpp"
#include "mix1d_device.hpp"

namespace fn {

// One 64-thread workgroup per fit, component k computed by thread k (its
// theta loads and special functions run alongside the other components').
constexpr int kMixPrologueThreads = 64;
static_assert(kMixMaxComp <= kMixPrologueThreads, "one thread per component");
__global__ __launch_bounds__(kMixPrologueThreads) void mix1d_prologue(Mix1dConst mc, ParamBlock pb,
                                                                      const double* __restrict__ theta_dev,
                                                                      int n_fits, int theta_stride,
                                                                      Mix1dTable* __restrict__ tab) {
  const int f = blockIdx.x;
  if (f >= n_fits) return;
  const double* th = theta_dev ? theta_dev + (int64_t)f * theta_stride : pb.v;
  const int k = threadIdx.x;
  const bool ok = k < mc.K ? mix1d_component(mc, th, k, tab[f]) : true;
  const bool bad = __syncthreads_or(!ok);
  if (k == 0) mix1d_table_rest(mc, th, !bad, tab[f]);
}

// Single fit: one workgroup per chunk of events, one row of partial sums each
// (SIG: the type signature the pass is compiled for, 0 for the generic one).
template <bool GRAD, int KMAX, int SIG>
__global__ __launch_bounds__(kBlock) void mix1d_events(Mix1dConst mc, const Mix1dTable* __restrict__ tab,
                                                       const double* __restrict__ x, int64_t n, int chunk,
                                                       double* __restrict__ part) {
  constexpr int NV = GRAD ? mix_nv(KMAX) : 1;
  __shared__ double lds[block_sum_lds(NV)];
  mix1d_chunk<GRAD, KMAX, SIG>(mc, tab, x, n, blockIdx.x, chunk, part + (int64_t)blockIdx.x * NV, lds);
}

// Level-2 step of a single fit.
__global__ __launch_bounds__(kBlock) void mix1d_finalize(Mix1dConst mc, const Mix1dTable* __restrict__ tab,
                                                         const double* __restrict__ part, int64_t nrows,
                                                         int nv, int kmax, int with_grad, double n_events,
                                                         double* __restrict__ out, double* __restrict__ out_user) {
  __shared__ double scratch[kBlock];
  __shared__ double res[kBlock];
  mix1d_finalize_one(mc, *tab, part, nrows, nv, kmax, with_grad, n_events, out, out_user, scratch, res);
}

// Binned data: one workgroup per chunk of bins, then the level-2 step.
template <bool GRAD, int KMAX, int STAT>
__global__ __launch_bounds__(kBlock) void mix1d_binned(Mix1dConst mc, const Mix1dTable* __restrict__ tab,
                                                       const double* __restrict__ counts, int64_t nb,
                                                       const double* nptr, int chunk, double* __restrict__ part) {
  constexpr int NV = mix1d_binned_nv<KMAX, STAT, GRAD>();
  __shared__ double lds[block_sum_lds(NV)];
  mix1d_binned_chunk<GRAD, KMAX, STAT>(mc, tab, counts, nb, nptr, blockIdx.x, chunk,
                                       part + (int64_t)blockIdx.x * NV, lds);
}

__global__ __launch_bounds__(kBlock) void mix1d_binned_total(const double* __restrict__ part, int64_t nrows,
                                                             double* __restrict__ total) {
  __shared__ double scratch[kBlock];
  __shared__ double res[kBlock];
  mix1d_binned_total_one(part, nrows, total, scratch, res);
}

__global__ __launch_bounds__(kBlock) void mix1d_binned_finalize(Mix1dConst mc, const Mix1dTable* __restrict__ tab,
                                                                const double* __restrict__ part, int64_t nrows,
                                                                int nv, int kmax, int stat, int64_t nb,
                                                                int with_grad, double* __restrict__ out) {
  __shared__ double scratch[kBlock];
  __shared__ double res[kBlock];
  mix1d_binned_finalize_one(mc, *tab, part, nrows, nv, kmax, stat, nb, with_grad, out, scratch, res);
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
int mix1d_sig(const Mix1dConst& mc) {
  if (mc.K == 1) return 1 + mc.type[0];
  if (mc.K == 2) return 5 + 4 * mc.type[0] + mc.type[1];
  return 0;
}
int mix1d_nv(int kmax, bool grad) { return grad ? mix_nv(kmax) : 1; }

void mix1d_launch_prologue(const Mix1dConst& mc, const ParamBlock& pb, const double* theta_dev, int n_fits,
                           int theta_stride, Mix1dTable* tab, hipStream_t s) {
  if (n_fits <= 0) return;
  hipLaunchKernelGGL(mix1d_prologue, dim3(n_fits), dim3(kMixPrologueThreads), 0, s, mc, pb, theta_dev, n_fits,
                     theta_stride, tab);
}

void mix1d_launch_events(const Mix1dConst& mc, const Mix1dTable* tab, const double* x, int64_t n, int chunk,
                         int64_t nchunks, bool grad, double* part, hipStream_t s, hipEvent_t start,
                         hipEvent_t stop) {
  if (nchunks == 0) return;
  const int kmax = mix1d_kmax(mc.K);
  const dim3 g((unsigned)nchunks), b(kBlock);
#define FN_MIX(G, K, SIG) \
  hipExtLaunchKernelGGL((mix1d_events<G, K, SIG>), g, b, 0, s, start, stop, 0, mc, tab, x, n, chunk, part)
#define FN_MIX_SIG(SIG)                                  \
  case SIG:                                              \
    if (grad) FN_MIX(true, 2, SIG); else FN_MIX(false, 2, SIG); \
    break;
  switch (mix1d_sig(mc)) {
    FN_MIX_SIGS(FN_MIX_SIG)
    default:
      if (kmax == 2) {
        if (grad) FN_MIX(true, 2, 0); else FN_MIX(false, 2, 0);
      } else {
        if (grad) FN_MIX(true, 8, 0); else FN_MIX(false, 8, 0);
      }
  }
#undef FN_MIX_SIG
#undef FN_MIX
}

void mix1d_launch_finalize(const Mix1dConst& mc, const Mix1dTable* tab, const double* part, int64_t nrows,
                           bool grad, double n_events, double* out, double* out_user, hipStream_t s) {
  const int kmax = mix1d_kmax(mc.K);
  hipLaunchKernelGGL(mix1d_finalize, dim3(1), dim3(kBlock), 0, s, mc, tab, part, nrows, mix1d_nv(kmax, grad),
                     kmax, grad ? 1 : 0, n_events, out, out_user);
}

int mix1d_nv_binned(int kmax, bool grad) {
  // the largest row of the passes (Poisson: two gradient groups)
  return kmax == 2 ? mix1d_binned_nv<2, 0, true>() : mix1d_binned_nv<8, 0, true>();
}

void mix1d_launch_binned(const Mix1dConst& mc, const Mix1dTable* tab, const double* counts, int64_t nb, int chunk,
                         int64_t nchunks, int stat, bool grad, double* part, double* nbuf, double* out,
                         hipStream_t s) {
  const int kmax = mix1d_kmax(mc.K);
  const dim3 g((unsigned)nchunks), b(kBlock);
  const double* nptr = nullptr;
  if (stat == 1 && mc.yidx < 0) {
    // chi^2 with N = W: the total count first
    if (kmax == 2) hipLaunchKernelGGL((mix1d_binned<false, 2, 2>), g, b, 0, s, mc, tab, counts, nb, nullptr, chunk, part);
    else hipLaunchKernelGGL((mix1d_binned<false, 8, 2>), g, b, 0, s, mc, tab, counts, nb, nullptr, chunk, part);
    hipLaunchKernelGGL(mix1d_binned_total, dim3(1), dim3(kBlock), 0, s, part, nchunks, nbuf);
    nptr = nbuf;
  }
#define FN_BIN(G, K, S) \
  hipLaunchKernelGGL((mix1d_binned<G, K, S>), g, b, 0, s, mc, tab, counts, nb, nptr, chunk, part)
#define FN_BIN_K(G, S)            \
  if (kmax == 2) FN_BIN(G, 2, S); \
  else FN_BIN(G, 8, S)
  if (stat == 0) {
    if (grad) { FN_BIN_K(true, 0); } else { FN_BIN_K(false, 0); }
  } else {
    if (grad) { FN_BIN_K(true, 1); } else { FN_BIN_K(false, 1); }
  }
#undef FN_BIN_K
#undef FN_BIN
  const int nv = stat == 0 ? (kmax == 2 ? mix1d_binned_nv<2, 0, true>() : mix1d_binned_nv<8, 0, true>())
                           : (kmax == 2 ? mix1d_binned_nv<2, 1, true>() : mix1d_binned_nv<8, 1, true>());
  const int nv_used = grad ? nv : 3;
  hipLaunchKernelGGL(mix1d_binned_finalize, dim3(1), dim3(kBlock), 0, s, mc, tab, part, nchunks, nv_used, kmax,
                     stat, nb, grad ? 1 : 0, out);
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
