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

namespace fn {

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications with the published multipliers and Weyl key
// increments.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Two uniforms in [0, 1) from counter (i, stream, word): 53-bit mantissas of
// the 64-bit words (w0:w1) and (w2:w3).
__device__ __forceinline__ void philox_uniforms(uint64_t i, uint32_t stream, uint32_t word, uint32_t k0,
                                                uint32_t k1, double& ua, double& ub) {
  uint32_t c[4] = {(uint32_t)i, (uint32_t)(i >> 32), stream, word};
  philox4x32_10(c, k0, k1);
  const uint64_t a = (((uint64_t)c[0] << 32) | c[1]) >> 11;
  const uint64_t b = (((uint64_t)c[2] << 32) | c[3]) >> 11;
  ua = (double)a * 0x1.0p-53;
  ub = (double)b * 0x1.0p-53;
}

// Toy events of the Gaussian + exponential mixture on [lo, hi] (theta_gen =
// mu, sigma, tau, f): component by a uniform draw, Gaussian by Box-Muller with
// redraws outside the range, exponential by the inverse CDF of the truncated
// exponential.  Event i, attempt a uses counters (i, 2a, word) and (i, 2a+1, word).
__global__ void gen_mix1d_kernel(uint32_t k0, uint32_t k1, uint32_t word, int64_t n, double mu, double sigma,
                                 double tau, double frac, double lo, double hi, double* __restrict__ x,
                                 unsigned int* __restrict__ n_unresolved) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double width = hi - lo;
  const double em = tau != 0.0 ? expm1(tau * width) : 0.0;
  double v = NAN;
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
    if (t >= lo && t <= hi) {
      v = t;
      break;
    }
  }
  x[i] = v;
  if (v != v) atomicAdd(n_unresolved, 1u);
}

// ------------------------------------------------------------------ steps
__global__ void batch_prologue(Mix1dConst mc, BfgsState* __restrict__ st, int n_fits, Mix1dTable* __restrict__ tabs) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_fits || st[f].status != kFitRunning) return;
  mix1d_table(mc, st[f].xt, tabs[f]);
}

// Single workgroup: item_base[f] = sum of chunk counts of running fits < f;
// item_base[n_fits] = total; *n_running = number of running fits.
__global__ __launch_bounds__(kBlock) void batch_scan(const BfgsState* __restrict__ st, const int64_t* __restrict__ nev,
                                                     int n_fits, int chunk, int64_t* __restrict__ item_base,
                                                     int* __restrict__ n_running) {
  __shared__ int64_t sums[kBlock];
  __shared__ int counts[kBlock];
  const int t = threadIdx.x;
  const int per = (n_fits + kBlock - 1) / kBlock;
  const int f0 = t * per, f1 = min(f0 + per, n_fits);
  int64_t s = 0;
  int c = 0;
  for (int f = f0; f < f1; ++f) {
    if (st[f].status == kFitRunning) {
      s += (nev[f] + chunk - 1) / chunk;
      ++c;
    }
  }
  sums[t] = s;
  counts[t] = c;
  __syncthreads();
  if (t == 0) {
    int64_t acc = 0;
    int cacc = 0;
    for (int u = 0; u < kBlock; ++u) {
      const int64_t v = sums[u];
      sums[u] = acc;
      acc += v;
      cacc += counts[u];
    }
    item_base[n_fits] = acc;
    *n_running = cacc;
  }
  __syncthreads();
  int64_t b = sums[t];
  for (int f = f0; f < f1; ++f) {
    item_base[f] = b;
    if (st[f].status == kFitRunning) b += (nev[f] + chunk - 1) / chunk;
  }
}

template <bool GRAD, int KMAX>
__global__ __launch_bounds__(kBlock) void batch_eval(Mix1dConst mc, const Mix1dTable* __restrict__ tabs,
                                                     const double* const* __restrict__ ev,
                                                     const int64_t* __restrict__ nev,
                                                     const int64_t* __restrict__ item_base,
                                                     const int64_t* __restrict__ part_base, int n_fits, int chunk,
                                                     double* __restrict__ part) {
  constexpr int NV = GRAD ? mix_nv(KMAX) : 1;
  __shared__ double lds[kWaves * NV];
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
    mix1d_chunk<GRAD, KMAX>(mc, tabs + f, ev[f], nev[f], ch, chunk, part + (part_base[f] + ch) * NV, lds);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void batch_finalize(Mix1dConst mc, const Mix1dTable* __restrict__ tabs,
                                                         const BfgsState* __restrict__ st,
                                                         const int64_t* __restrict__ nev,
                                                         const int64_t* __restrict__ part_base, const double* part,
                                                         int chunk, int nv, int kmax, double* __restrict__ out,
                                                         int out_stride) {
  __shared__ double scratch[kBlock];
  __shared__ double res[kBlock];
  const int f = blockIdx.x;
  if (st[f].status != kFitRunning) return;
  const int64_t rows = (nev[f] + chunk - 1) / chunk;
  mix1d_finalize_one(mc, tabs[f], part + part_base[f] * nv, rows, nv, kmax, 1, out + (int64_t)f * out_stride,
                     nullptr, scratch, res);
}

// --------------------------------------------------------------- BFGS step
__device__ inline double dotp(const double* a, const double* b, int P) {
  double s = 0.0;
  for (int i = 0; i < P; ++i) s += a[i] * b[i];
  return s;
}

// Direction p = -H g (fixed parameters have zero rows/columns in H).
__device__ inline void new_direction(BfgsState& s, int P) {
  for (int i = 0; i < P; ++i) {
    double v = 0.0;
    for (int j = 0; j < P; ++j) v += s.H[i * kBatchMaxP + j] * s.g[j];
    s.p[i] = -v;
  }
  s.d0 = dotp(s.g, s.p, P);
}

__device__ inline void set_trial(BfgsState& s, int P, double a) {
  s.alpha = a;
  for (int i = 0; i < P; ++i) s.xt[i] = s.x[i] + a * s.p[i];
}

// Start the next iteration from the accepted point (x, f, g) in s.
__device__ inline void begin_iteration(BfgsState& s, int P, double tol, int max_iter) {
  // estimated distance to the minimum
  double edm = 0.0;
  for (int i = 0; i < P; ++i) {
    double v = 0.0;
    for (int j = 0; j < P; ++j) v += s.H[i * kBatchMaxP + j] * s.g[j];
    edm += s.g[i] * v;
  }
  edm *= 0.5;
  s.edm = edm;
  if (edm >= 0.0 && edm < tol) {
    s.status = kFitConverged;
    return;
  }
  if (s.iter >= max_iter) {
    s.status = kFitFailed;
    return;
  }
  new_direction(s, P);
  if (!(s.d0 < 0.0)) {
    // not a descent direction: restart from a scaled identity
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j) s.H[i * kBatchMaxP + j] = (i == j && s.mask[i]) ? s.h0 : 0.0;
    new_direction(s, P);
    if (!(s.d0 < 0.0)) {
      s.status = kFitFailed;
      return;
    }
  }
  s.phase = kPhaseBracket;
  s.ls_it = 0;
  s.a_prev = 0.0;
  s.f_prev = s.f;
  s.d_prev = s.d0;
  set_trial(s, P, 1.0);
}

__device__ inline void accept_trial(BfgsState& s, int P, const double* gt, double ft, double tol, int max_iter) {
  double sv[kBatchMaxP], yv[kBatchMaxP], Hy[kBatchMaxP];
  for (int i = 0; i < P; ++i) {
    sv[i] = s.xt[i] - s.x[i];
    yv[i] = gt[i] - s.g[i];
  }
  const double sy = dotp(sv, yv, P);
  if (sy > 0.0) {
    if (s.iter == 0) {
      // Nocedal & Wright Eq. 6.20: rescale the initial matrix before the first update
      const double sc = sy / dotp(yv, yv, P);
      for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) s.H[i * kBatchMaxP + j] = (i == j && s.mask[i]) ? sc : 0.0;
      s.h0 = sc;
    }
    const double rho = 1.0 / sy;
    for (int i = 0; i < P; ++i) {
      double v = 0.0;
      for (int j = 0; j < P; ++j) v += s.H[i * kBatchMaxP + j] * yv[j];
      Hy[i] = v;
    }
    const double yHy = dotp(yv, Hy, P);
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j)
        s.H[i * kBatchMaxP + j] += rho * ((1.0 + rho * yHy) * sv[i] * sv[j] - Hy[i] * sv[j] - sv[i] * Hy[j]);
  }
  for (int i = 0; i < P; ++i) {
    s.x[i] = s.xt[i];
    s.g[i] = gt[i];
  }
  s.f = ft;
  s.iter += 1;
  begin_iteration(s, P, tol, max_iter);
}

// Safeguarded quadratic interpolation in [lo, hi] from (lo, f_lo, d_lo), (hi, f_hi).
__device__ inline double zoom_trial(const BfgsState& s) {
  const double lo = s.a_lo, hi = s.a_hi, dh = hi - lo;
  double a;
  const double den = 2.0 * (s.f_hi - s.f_lo - s.d_lo * dh);
  if (isfinite(s.f_hi) && den > 0.0) a = lo - s.d_lo * dh * dh / den;
  else a = lo + 0.5 * dh;
  const double b0 = fmin(lo, hi) + 0.1 * fabs(dh), b1 = fmax(lo, hi) - 0.1 * fabs(dh);
  if (!(a >= b0 && a <= b1)) a = lo + 0.5 * dh;
  return a;
}

__device__ void bfgs_update(BfgsState& s, const double* __restrict__ o, int P, double tol, int max_iter) {
  double ft = o[0];
  double gt[kBatchMaxP];
  bool ok = isfinite(ft);
  for (int i = 0; i < P; ++i) {
    gt[i] = s.mask[i] ? o[1 + i] : 0.0;
    ok = ok && isfinite(gt[i]);
  }
  if (!ok) ft = INFINITY;
  s.n_eval += 1;
  const double c1 = 1e-4, c2 = 0.9;
  if (s.phase == kPhaseStart) {
    if (!ok) {
      s.status = kFitFailed;
      return;
    }
    for (int i = 0; i < P; ++i) {
      s.x[i] = s.xt[i];
      s.g[i] = gt[i];
    }
    s.f = ft;
    // starting inverse Hessian: first step moves the largest gradient component by 1e-3 of its scale
    double gmax = 0.0;
    for (int i = 0; i < P; ++i) gmax = fmax(gmax, fabs(gt[i]));
    s.h0 = gmax > 0.0 ? 1e-3 / gmax : 1.0;
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j) s.H[i * kBatchMaxP + j] = (i == j && s.mask[i]) ? s.h0 : 0.0;
    s.iter = 0;
    begin_iteration(s, P, tol, max_iter);
    return;
  }
  const double dt = ok ? dotp(gt, s.p, P) : NAN;
  const double a = s.alpha;
  s.ls_it += 1;
  if (s.ls_it > kMaxLineSearch) {
    // give up on this line: accept the best sufficient-decrease point if any
    if (s.phase == kPhaseZoom && s.a_lo > 0.0 && s.f_lo < s.f) {
      set_trial(s, P, s.a_lo);
      s.phase = kPhaseAcceptLo;
      return;
    }
    s.status = kFitFailed;
    return;
  }
  if (s.phase == kPhaseAcceptLo) {
    if (!ok) {
      s.status = kFitFailed;
      return;
    }
    accept_trial(s, P, gt, ft, tol, max_iter);
    return;
  }
  if (s.phase == kPhaseBracket) {
    if (!ok || ft > s.f + c1 * a * s.d0 || (s.a_prev > 0.0 && ft >= s.f_prev)) {
      s.a_lo = s.a_prev; s.f_lo = s.f_prev; s.d_lo = s.d_prev;
      s.a_hi = a; s.f_hi = ft;
      s.phase = kPhaseZoom;
      set_trial(s, P, zoom_trial(s));
      return;
    }
    if (fabs(dt) <= -c2 * s.d0) {
      accept_trial(s, P, gt, ft, tol, max_iter);
      return;
    }
    if (dt >= 0.0) {
      s.a_lo = a; s.f_lo = ft; s.d_lo = dt;
      s.a_hi = s.a_prev; s.f_hi = s.f_prev;
      s.phase = kPhaseZoom;
      set_trial(s, P, zoom_trial(s));
      return;
    }
    s.a_prev = a; s.f_prev = ft; s.d_prev = dt;
    set_trial(s, P, 2.0 * a);
    return;
  }
  // zoom
  if (!ok || ft > s.f + c1 * a * s.d0 || ft >= s.f_lo) {
    s.a_hi = a;
    s.f_hi = ft;
  } else {
    if (fabs(dt) <= -c2 * s.d0) {
      accept_trial(s, P, gt, ft, tol, max_iter);
      return;
    }
    if (dt * (s.a_hi - s.a_lo) >= 0.0) {
      s.a_hi = s.a_lo;
      s.f_hi = s.f_lo;
    }
    s.a_lo = a; s.f_lo = ft; s.d_lo = dt;
  }
  if (fabs(s.a_hi - s.a_lo) < 1e-15 * fmax(1.0, fabs(s.a_lo))) {
    if (s.a_lo > 0.0 && s.f_lo < s.f) {
      set_trial(s, P, s.a_lo);
      s.phase = kPhaseAcceptLo;
      return;
    }
    s.status = kFitFailed;
    return;
  }
  set_trial(s, P, zoom_trial(s));
}

// One minimizer step per running fit; every slot's status is mirrored into
// stat[], and a fit that retires in this step writes its result row
// [NLL, iterations, evaluations, theta(P), sqrt|H_ii|(P)] into rres.
__global__ void batch_bfgs(BfgsState* __restrict__ st, const double* __restrict__ out, int out_stride, int n_fits,
                           int P, double tol, int max_iter, int* __restrict__ stat, double* __restrict__ rres) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_fits) return;
  BfgsState& s = st[f];
  if (s.status == kFitRunning) {
    bfgs_update(s, out + (int64_t)f * out_stride, P, tol, max_iter);
    if (s.status != kFitRunning) {
      double* r = rres + (int64_t)f * (3 + 2 * P);
      r[0] = s.f;
      r[1] = s.iter;
      r[2] = s.n_eval;
      for (int i = 0; i < P; ++i) {
        r[3 + i] = s.x[i];
        r[3 + P + i] = s.mask[i] ? sqrt(fabs(s.H[i * kBatchMaxP + i])) : 0.0;
      }
    }
  }
  stat[f] = s.status;
}

// ---------------------------------------------------------------- launchers
void batch_launch_gen_mix1d(uint32_t k0, uint32_t k1, uint32_t word, int64_t n, const double* theta_gen, double lo,
                            double hi, double* x, unsigned int* n_unresolved, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(gen_mix1d_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, k0, k1, word, n,
                     theta_gen[0], theta_gen[1], theta_gen[2], theta_gen[3], lo, hi, x, n_unresolved);
}

void batch_launch_step(const BatchDev& b, const Mix1dConst& mc, int n_fits, int P, int chunk, int eval_grid,
                       double tol, int max_iter, hipStream_t s) {
  const int kmax = mix1d_kmax(mc.K);
  const int nv = mix1d_nv(kmax, true);
  const dim3 fg((n_fits + 63) / 64), fb(64);
  hipLaunchKernelGGL(batch_prologue, fg, fb, 0, s, mc, b.st, n_fits, b.tabs);
  hipLaunchKernelGGL(batch_scan, dim3(1), dim3(kBlock), 0, s, b.st, b.nev, n_fits, chunk, b.item_base, b.n_running);
  if (kmax == 2)
    hipLaunchKernelGGL((batch_eval<true, 2>), dim3(eval_grid), dim3(kBlock), 0, s, mc, b.tabs, b.ev, b.nev,
                       b.item_base, b.part_base, n_fits, chunk, b.part);
  else
    hipLaunchKernelGGL((batch_eval<true, 8>), dim3(eval_grid), dim3(kBlock), 0, s, mc, b.tabs, b.ev, b.nev,
                       b.item_base, b.part_base, n_fits, chunk, b.part);
  hipLaunchKernelGGL(batch_finalize, dim3(n_fits), dim3(kBlock), 0, s, mc, b.tabs, b.st, b.nev, b.part_base, b.part,
                     chunk, nv, kmax, b.out, 2 + 2 * P);
  hipLaunchKernelGGL(batch_bfgs, fg, fb, 0, s, b.st, b.out, 2 + 2 * P, n_fits, P, tol, max_iter, b.stat, b.rres);
}

int batch_eval_blocks_per_cu(const Mix1dConst& mc) {
  int nb = 0;
  if (mix1d_kmax(mc.K) == 2)
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_eval<true, 2>, kBlock, 0);
  else
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_eval<true, 8>, kBlock, 0);
  return nb > 0 ? nb : 1;
}

}  // namespace fn
