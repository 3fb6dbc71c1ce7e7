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

#include "kernels.hpp"
#include "mix1d_device.hpp"

namespace fn {

__global__ void mix1d_prologue(Mix1dConst mc, ParamBlock pb, const double* __restrict__ theta_dev,
                               int n_fits, int theta_stride, Mix1dTable* __restrict__ tab) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_fits) return;
  const double* th = theta_dev ? theta_dev + (int64_t)f * theta_stride : pb.v;
  mix1d_table(mc, th, tab[f]);
}

// Single fit: one workgroup per chunk of events, one row of partial sums each.
template <bool GRAD, int KMAX>
__global__ __launch_bounds__(kBlock) void mix1d_events(Mix1dConst mc, const Mix1dTable* __restrict__ tab,
                                                       const double* __restrict__ x, int64_t n, int chunk,
                                                       double* __restrict__ part) {
  constexpr int NV = GRAD ? mix_nv(KMAX) : 1;
  __shared__ double lds[block_sum_lds(NV)];
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
  __shared__ double lds[block_sum_lds(NV)];
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
