// Many fits of one mix1d model per launch, with a device-resident minimizer.
//
// One batch step = one NLL + gradient evaluation for every running fit at its
// trial point, followed by one state-machine step of BFGS with a strong-Wolfe
// line search (Nocedal & Wright, Alg. 3.5/3.6) per fit:
//
//   batch_prologue   per running fit: theta_trial -> mix1d table
//   batch_scan       exclusive scan of the running fits' chunk counts ->
//                    item bases, total item count, running-fit count
//   batch_eval       persistent kernel over (fit, chunk) items; each item runs
//                    the single-fit chunk routine, so rows are bitwise those of
//                    fn_nll for the same fit
//   batch_finalize   per running fit: fixed-order level-2 sum -> NLL, gradient
//   batch_bfgs       per running fit: accept/reject the trial, update H, pick
//                    the next trial point, or retire (converged / failed)
//
// No host synchronisation inside a step; the host polls the running-fit
// count between groups of steps.  Fits never interact, so a fit's trajectory
// (and result bits) is the same alone and inside any batch.
#include <cmath>

#include "batch.hpp"
#include "philox.hpp"

namespace fn {

// Toy events of the Gaussian + exponential mixture on [lo, hi] (theta_gen =
// mu, sigma, tau, f): component by a uniform draw, Gaussian by Box-Muller with
// redraws outside the range, exponential by the inverse CDF of the truncated
// exponential.  Event i, attempt a uses counters (i, 2a, word) and (i, 2a+1, word).
// NaN when no attempt lands in the range.
__device__ __forceinline__ double gen_mix1d_event(int64_t i, uint32_t k0, uint32_t k1, uint32_t word, double mu,
                                                  double sigma, double tau, double frac, double lo, double hi) {
  const double width = hi - lo;
  const double em = tau != 0.0 ? expm1(tau * width) : 0.0;
  for (int a = 0; a < kGenMaxAttempts; ++a) {
    double uc, u1, u2, unused;
    philox_uniforms((uint64_t)i, 2u * a, word, k0, k1, uc, u1);
    philox_uniforms((uint64_t)i, 2u * a + 1u, word, k0, k1, u2, unused);
    double t;
    if (uc < frac) {
      const double r = sqrt(-2.0 * log1p(-u1));
      t = mu + sigma * r * cos(2.0 * 3.14159265358979323846 * u2);
    } else {
      t = tau != 0.0 ? lo + log1p(u1 * em) / tau : lo + u1 * width;
      t = fmin(fmax(t, lo), hi);
    }
    if (t >= lo && t <= hi) return t;
  }
  return NAN;
}

__global__ void gen_mix1d_kernel(uint32_t k0, uint32_t k1, uint32_t word, int64_t n, double mu, double sigma,
                                 double tau, double frac, double lo, double hi, double* __restrict__ x,
                                 unsigned int* __restrict__ n_unresolved) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = gen_mix1d_event(i, k0, k1, word, mu, sigma, tau, frac, lo, hi);
  x[i] = v;
  if (v != v) atomicAdd(n_unresolved, 1u);
}

// ------------------------------------------------------------- admission
static_assert(sizeof(BfgsState) % sizeof(uint64_t) == 0, "state is cleared in 8-byte words");

__global__ __launch_bounds__(kBlock) void batch_admit(const AdmitRec* __restrict__ recs, int n_recs, int P,
                                                      double lo, double hi, BatchDev b,
                                                      unsigned int* __restrict__ n_unresolved) {
  const int64_t blk = blockIdx.x;
  if (blk < n_recs) {
    // a fresh fit: every field zero but the start point, the free mask, status and phase
    const AdmitRec& r = recs[blk];
    uint64_t* w = reinterpret_cast<uint64_t*>(b.st + r.slot);
    constexpr int kWords = (int)(sizeof(BfgsState) / sizeof(uint64_t));
    for (int i = threadIdx.x; i < kWords; i += blockDim.x) w[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
      BfgsState& st = b.st[r.slot];
      for (int i = 0; i < P; ++i) {
        st.xt[i] = r.theta0[i];
        st.mask[i] = 1;
      }
      st.status = kFitRunning;
      st.phase = kPhaseStart;
      b.stat[r.slot] = kFitRunning;
      b.ev[r.slot] = r.ev;
      b.nev[r.slot] = r.n;
    }
    return;
  }
  // generation workgroup g: the last record with block0 <= g owns it (records
  // without generation own no workgroups, so a later record with the same
  // block0 is the owner)
  const int64_t g = blk - n_recs;
  int a = 0, c = n_recs - 1;
  while (a < c) {
    const int mid = (a + c + 1) / 2;
    if (recs[mid].block0 <= g) a = mid;
    else c = mid - 1;
  }
  const AdmitRec& r = recs[a];
  const int64_t i = (g - r.block0) * kBlock + threadIdx.x;
  if (!r.generate || i >= r.n) return;
  const double v = gen_mix1d_event(i, r.seed, r.fit, 0u, r.theta_gen[0], r.theta_gen[1], r.theta_gen[2],
                                   r.theta_gen[3], lo, hi);
  r.ev[i] = v;
  if (v != v) atomicAdd(n_unresolved, 1u);
}

// fn_batch_set: workgroup f resets slot f -- a fresh fit at theta0[f] (all
// parameters free) for f < n_fits, idle beyond; event pointers and counts are
// copied separately.
__global__ __launch_bounds__(kBlock) void batch_set_kernel(const double* __restrict__ theta0, int n_fits, int P,
                                                           BatchDev b) {
  const int f = blockIdx.x;
  uint64_t* w = reinterpret_cast<uint64_t*>(b.st + f);
  constexpr int kWords = (int)(sizeof(BfgsState) / sizeof(uint64_t));
  for (int i = threadIdx.x; i < kWords; i += blockDim.x) w[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    if (f < n_fits) {
      BfgsState& st = b.st[f];
      for (int i = 0; i < P; ++i) {
        st.xt[i] = theta0[(int64_t)f * P + i];
        st.mask[i] = 1;
      }
      st.status = kFitRunning;
      st.phase = kPhaseStart;
    }
    b.stat[f] = f < n_fits ? kFitRunning : kFitIdle;
  }
}

void batch_launch_set(const BatchDev& b, const double* theta0, int n_fits, int max_fits, int P, hipStream_t s) {
  hipLaunchKernelGGL(batch_set_kernel, dim3((unsigned)max_fits), dim3(kBlock), 0, s, theta0, n_fits, P, b);
}

__global__ void batch_gather_rows(const double* __restrict__ rres, const int* __restrict__ slots, int n, int w,
                                  double* __restrict__ rows) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * w) return;
  const int i = (int)(t / w), j = (int)(t - (int64_t)i * w);
  rows[t] = rres[(int64_t)slots[i] * w + j];
}

// ------------------------------------------------------------------ steps
__global__ void batch_prologue(Mix1dConst mc, const BfgsState* __restrict__ st, const int* __restrict__ stat,
                               int n_fits, Mix1dTable* __restrict__ tabs) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_fits || stat[f] != kFitRunning) return;
  mix1d_table(mc, st[f].xt, tabs[f]);
}

// Single workgroup: item_base[f] = sum of chunk counts of running fits < f;
// item_base[n_fits] = total; *n_running = number of running fits.  Thread t
// takes a contiguous run of fits; the exclusive scan of the per-thread sums
// (thread order) is a shuffle scan within each wave plus the totals of the
// preceding waves: exact integer sums, the same as a serial loop.
__global__ __launch_bounds__(kBlock) void batch_scan(const int* __restrict__ stat, const int64_t* __restrict__ nev,
                                                     int n_fits, int chunk, int64_t* __restrict__ item_base,
                                                     int* __restrict__ n_running) {
  constexpr int kWaves = kBlock / 64;
  __shared__ int64_t wsum[kWaves];
  __shared__ int wcnt[kWaves];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int per = (n_fits + kBlock - 1) / kBlock;
  const int f0 = min(t * per, n_fits), f1 = min(f0 + per, n_fits);
  int64_t s = 0;
  int c = 0;
#pragma unroll 4
  for (int f = f0; f < f1; ++f) {
    if (stat[f] == kFitRunning) {
      s += (nev[f] + chunk - 1) / chunk;
      ++c;
    }
  }
  int64_t x = s;
  int cx = c;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t y = __shfl_up(x, d, 64);
    const int cy = __shfl_up(cx, d, 64);
    if (lane >= d) {
      x += y;
      cx += cy;
    }
  }
  if (lane == 63) {
    wsum[w] = x;
    wcnt[w] = cx;
  }
  __syncthreads();
  int64_t before = 0;
  for (int u = 0; u < w; ++u) before += wsum[u];
  if (t == kBlock - 1) {
    int total = 0;
    for (int u = 0; u < kWaves; ++u) total += wcnt[u];
    item_base[n_fits] = before + x;
    *n_running = total;
  }
  int64_t b = before + x - s;
#pragma unroll 4
  for (int f = f0; f < f1; ++f) {
    item_base[f] = b;
    if (stat[f] == kFitRunning) b += (nev[f] + chunk - 1) / chunk;
  }
}

template <bool GRAD, int KMAX, int SIG>
__global__ __launch_bounds__(kBlock) void batch_eval(Mix1dConst mc, const Mix1dTable* __restrict__ tabs,
                                                     const double* const* __restrict__ ev,
                                                     const int64_t* __restrict__ nev,
                                                     const int64_t* __restrict__ item_base,
                                                     const int64_t* __restrict__ part_base, int n_fits, int chunk,
                                                     double* __restrict__ part) {
  constexpr int NV = GRAD ? mix_nv(KMAX) : 1;
  __shared__ double lds[block_sum_lds(NV)];
  const int64_t total = item_base[n_fits];
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    // fit f with item_base[f] <= it < item_base[f+1] (non-running fits have
    // empty ranges, so the search lands on a running fit)
    int lo = 0, hi = n_fits;  // invariant: item_base[lo] <= it < item_base[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (item_base[mid] <= it) lo = mid;
      else hi = mid;
    }
    const int f = lo;
    const int64_t ch = it - item_base[f];
    mix1d_chunk<GRAD, KMAX, SIG>(mc, tabs + f, ev[f], nev[f], ch, chunk, part + (part_base[f] + ch) * NV, lds);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void batch_finalize(Mix1dConst mc, const Mix1dTable* __restrict__ tabs,
                                                         const int* __restrict__ stat,
                                                         const int64_t* __restrict__ nev,
                                                         const int64_t* __restrict__ part_base, const double* part,
                                                         int chunk, int nv, int kmax, double* __restrict__ out,
                                                         int out_stride) {
  __shared__ double scratch[kBlock];
  __shared__ double res[kBlock];
  const int f = blockIdx.x;
  if (stat[f] != kFitRunning) return;
  const int64_t rows = (nev[f] + chunk - 1) / chunk;
  mix1d_finalize_one(mc, tabs[f], part + part_base[f] * nv, rows, nv, kmax, 1, (double)nev[f],
                     out + (int64_t)f * out_stride,
                     nullptr, scratch, res);
}

// ---------------------------------------------------------------- launchers
void batch_launch_gen_mix1d(uint32_t k0, uint32_t k1, uint32_t word, int64_t n, const double* theta_gen, double lo,
                            double hi, double* x, unsigned int* n_unresolved, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(gen_mix1d_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, k0, k1, word, n,
                     theta_gen[0], theta_gen[1], theta_gen[2], theta_gen[3], lo, hi, x, n_unresolved);
}

void batch_launch_admit(const BatchDev& b, const AdmitRec* recs, int n_recs, int64_t gen_blocks, int P, double lo,
                        double hi, unsigned int* n_unresolved, hipStream_t s) {
  if (n_recs == 0) return;
  hipLaunchKernelGGL(batch_admit, dim3((unsigned)(n_recs + gen_blocks)), dim3(kBlock), 0, s, recs, n_recs, P, lo, hi,
                     b, n_unresolved);
}

void batch_launch_gather_rows(const BatchDev& b, const int* slots, int n, int P, double* rows_out, hipStream_t s) {
  if (n == 0) return;
  const int w = 3 + 2 * P;
  const int64_t total = (int64_t)n * w;
  hipLaunchKernelGGL(batch_gather_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, b.rres, slots, n, w,
                     rows_out);
}

void batch_launch_step(const BatchDev& b, const Mix1dConst& mc, int n_fits, int P, int chunk, int eval_grid,
                       double tol, int max_iter, hipStream_t s) {
  const int kmax = mix1d_kmax(mc.K);
  const int nv = mix1d_nv(kmax, true);
  const dim3 fg((n_fits + 63) / 64), fb(64);
  hipLaunchKernelGGL(batch_prologue, fg, fb, 0, s, mc, b.st, b.stat, n_fits, b.tabs);
  hipLaunchKernelGGL(batch_scan, dim3(1), dim3(kBlock), 0, s, b.stat, b.nev, n_fits, chunk, b.item_base,
                     b.n_running);
#define FN_EVAL(K, SIG)                                                                               \
  hipLaunchKernelGGL((batch_eval<true, K, SIG>), dim3(eval_grid), dim3(kBlock), 0, s, mc, b.tabs, b.ev, b.nev, \
                     b.item_base, b.part_base, n_fits, chunk, b.part)
#define FN_EVAL_SIG(SIG) \
  case SIG:              \
    FN_EVAL(2, SIG);     \
    break;
  switch (mix1d_sig(mc)) {
    FN_MIX_SIGS(FN_EVAL_SIG)
    default:
      if (kmax == 2) FN_EVAL(2, 0);
      else FN_EVAL(8, 0);
  }
#undef FN_EVAL_SIG
#undef FN_EVAL
  hipLaunchKernelGGL(batch_finalize, dim3(n_fits), dim3(kBlock), 0, s, mc, b.tabs, b.stat, b.nev, b.part_base, b.part,
                     chunk, nv, kmax, b.out, 2 + 2 * P);
  bfgs_launch<kBatchMaxP>(b.st, b.out, 2 + 2 * P, n_fits, P, tol, max_iter, b.stat, b.rres, s);
}

int batch_eval_blocks_per_cu(const Mix1dConst& mc) {
  int nb = 0;
#define FN_OCC_SIG(SIG)                                                                     \
  case SIG:                                                                                 \
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_eval<true, 2, SIG>, kBlock, 0); \
    break;
  switch (mix1d_sig(mc)) {
    FN_MIX_SIGS(FN_OCC_SIG)
    default:
      if (mix1d_kmax(mc.K) == 2)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_eval<true, 2, 0>, kBlock, 0);
      else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_eval<true, 8, 0>, kBlock, 0);
  }
#undef FN_OCC_SIG
  return nb > 0 ? nb : 1;
}

}  // namespace fn
