// Device-resident quasi-Newton minimizer shared by the batched fit paths:
// BFGS with a strong-Wolfe line search (Nocedal & Wright, Alg. 3.5/3.6, the
// initial-matrix rescale of Eq. 6.20), written as a state machine that
// consumes one NLL + gradient evaluation per step.  PM is the largest
// parameter count a state holds.  When the estimated distance to the minimum
// EDM = g^T H g / 2 drops below the tolerance with the BFGS matrix, the
// minimizer checks it the way Minuit's MIGRAD does after HESSE: it builds a
// numerical Hessian from central differences of the gradient (2 evaluations
// per free parameter), inverts it, and re-tests the EDM with that matrix,
// continuing the iterations from it when the test fails.  A fit that converges
// this way reports errors from the numerical Hessian.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace fn {

constexpr int kMaxLineSearch = 40;  // evaluations per line search before giving up
constexpr int kMaxHessian = 3;      // numerical-Hessian checks per fit

enum FitStatus : int { kFitIdle = 0, kFitRunning = 1, kFitConverged = 2, kFitFailed = 3 };
enum FitPhase : int {
  kPhaseStart = 0,
  kPhaseBracket = 1,
  kPhaseZoom = 2,
  kPhaseAcceptLo = 3,
  kPhaseHessPlus = 4,   // gradient at x + h e_col
  kPhaseHessMinus = 5   // gradient at x - h e_col
};

// One fit's BFGS + line-search state (device memory, one thread per fit).
// xt comes first so that a state array doubles as a strided array of trial points.
template <int PM>
struct BfgsStateT {
  double xt[PM];       // trial point: the next evaluation happens here
  double x[PM];        // accepted point
  double g[PM];        // gradient at x
  double p[PM];        // search direction
  double H[PM * PM];   // inverse Hessian approximation
  double Hn[PM * PM];  // numerical Hessian under construction (then its Cholesky factor)
  double gp[PM];       // gradient at x + h e_col
  double f, d0, alpha, h0, edm, hstep;
  double a_prev, f_prev, d_prev, a_lo, f_lo, d_lo, a_hi, f_hi;
  int mask[PM];        // 1 = free parameter
  int status, phase, iter, ls_it, n_eval, hcol, n_hess, fresh;  // fresh: H is the numerical inverse
};

// --------------------------------------------------------------- BFGS step
__device__ inline double dotp(const double* a, const double* b, int P) {
  double s = 0.0;
  for (int i = 0; i < P; ++i) s += a[i] * b[i];
  return s;
}

// Direction p = -H g (fixed parameters have zero rows/columns in H).
template <int PM>
__device__ inline void new_direction(BfgsStateT<PM>& s, int P) {
  for (int i = 0; i < P; ++i) {
    double v = 0.0;
    for (int j = 0; j < P; ++j) v += s.H[i * PM + j] * s.g[j];
    s.p[i] = -v;
  }
  s.d0 = dotp(s.g, s.p, P);
}

template <int PM>
__device__ inline void set_trial(BfgsStateT<PM>& s, int P, double a) {
  s.alpha = a;
  for (int i = 0; i < P; ++i) s.xt[i] = s.x[i] + a * s.p[i];
}

// Step of the numerical-Hessian column for parameter i: 1e-4 of the error
// the current matrix implies, with a floor relative to the parameter.
template <int PM>
__device__ inline double hess_step(const BfgsStateT<PM>& s, int i) {
  const double v = fabs(s.H[i * PM + i]);
  return fmax(1e-4 * sqrt(v), 1e-9 * fmax(fabs(s.x[i]), 1.0));
}

template <int PM>
__device__ inline bool start_hessian_column(BfgsStateT<PM>& s, int P, int from) {
  for (int i = from; i < P; ++i) {
    if (!s.mask[i]) continue;
    s.hcol = i;
    s.hstep = hess_step(s, i);
    for (int j = 0; j < P; ++j) s.xt[j] = s.x[j];
    s.xt[i] = s.x[i] + s.hstep;
    s.phase = kPhaseHessPlus;
    return true;
  }
  return false;
}

template <int PM>
__device__ inline bool start_hessian(BfgsStateT<PM>& s, int P) {
  for (int i = 0; i < PM * PM; ++i) s.Hn[i] = 0.0;
  return start_hessian_column(s, P, 0);
}

// Inverse of the symmetric positive definite matrix Hn restricted to the free
// parameters (Cholesky factor in place, then inverse of the factor in place,
// then H = L^-T L^-1); false if Hn is not positive definite.
template <int PM>
__device__ inline bool hessian_inverse(BfgsStateT<PM>& s, int P) {
  int idx[PM];
  int D = 0;
  for (int i = 0; i < P; ++i)
    if (s.mask[i]) idx[D++] = i;
  auto A = [&](int i, int j) -> double& { return s.Hn[idx[i] * PM + idx[j]]; };
  for (int j = 0; j < D; ++j) {
    double d = A(j, j);
    for (int k = 0; k < j; ++k) d -= A(j, k) * A(j, k);
    if (!(d > 0.0) || !isfinite(d)) return false;
    const double l = sqrt(d);
    A(j, j) = l;
    for (int i = j + 1; i < D; ++i) {
      double v = A(i, j);
      for (int k = 0; k < j; ++k) v -= A(i, k) * A(j, k);
      A(i, j) = v / l;
    }
  }
  for (int i = 0; i < D; ++i) {
    for (int j = 0; j < i; ++j) {
      double v = 0.0;
      for (int k = j; k < i; ++k) v += A(i, k) * A(k, j);
      A(i, j) = -v / A(i, i);
    }
    A(i, i) = 1.0 / A(i, i);
  }
  for (int i = 0; i < P * PM; ++i) s.H[i] = 0.0;
  for (int a = 0; a < D; ++a)
    for (int b = 0; b <= a; ++b) {
      double v = 0.0;
      for (int k = a; k < D; ++k) v += A(k, a) * A(k, b);
      s.H[idx[a] * PM + idx[b]] = v;
      s.H[idx[b] * PM + idx[a]] = v;
    }
  return true;
}

template <int PM>
__device__ inline void begin_iteration(BfgsStateT<PM>& s, int P, double tol, int max_iter);

// One gradient of the numerical Hessian has arrived (phase HessPlus or HessMinus).
template <int PM>
__device__ inline void hessian_step(BfgsStateT<PM>& s, int P, const double* gt, bool ok, double tol, int max_iter) {
  const int c = s.hcol;
  if (!ok) {
    // a neighbour of the minimum is not finite: keep the BFGS matrix
    for (int j = 0; j < P; ++j) s.xt[j] = s.x[j];
    s.status = kFitConverged;
    return;
  }
  if (s.phase == kPhaseHessPlus) {
    for (int i = 0; i < P; ++i) s.gp[i] = gt[i];
    s.xt[c] = s.x[c] - s.hstep;
    s.phase = kPhaseHessMinus;
    return;
  }
  const double den = (s.x[c] + s.hstep) - (s.x[c] - s.hstep);
  for (int i = 0; i < P; ++i) s.Hn[i * PM + c] = s.mask[i] ? (s.gp[i] - gt[i]) / den : 0.0;
  if (start_hessian_column(s, P, c + 1)) return;
  for (int j = 0; j < P; ++j) s.xt[j] = s.x[j];
  for (int i = 0; i < P; ++i)
    for (int j = 0; j < i; ++j) {
      const double v = 0.5 * (s.Hn[i * PM + j] + s.Hn[j * PM + i]);
      s.Hn[i * PM + j] = s.Hn[j * PM + i] = v;
    }
  s.n_hess += 1;
  if (!hessian_inverse(s, P)) {
    // not positive definite: keep the BFGS matrix and its verdict
    s.status = kFitConverged;
    return;
  }
  s.fresh = 1;
  begin_iteration(s, P, tol, max_iter);
}

// Start the next iteration from the accepted point (x, f, g) in s.
template <int PM>
__device__ inline void begin_iteration(BfgsStateT<PM>& s, int P, double tol, int max_iter) {
  // estimated distance to the minimum
  double edm = 0.0;
  for (int i = 0; i < P; ++i) {
    double v = 0.0;
    for (int j = 0; j < P; ++j) v += s.H[i * PM + j] * s.g[j];
    edm += s.g[i] * v;
  }
  edm *= 0.5;
  s.edm = edm;
  if (edm >= 0.0 && edm < tol) {
    if (s.fresh || s.n_hess >= kMaxHessian || !start_hessian(s, P)) s.status = kFitConverged;
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
      for (int j = 0; j < P; ++j) s.H[i * PM + j] = (i == j && s.mask[i]) ? s.h0 : 0.0;
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

template <int PM>
__device__ inline void accept_trial(BfgsStateT<PM>& s, int P, const double* gt, double ft, double tol, int max_iter) {
  double sv[PM], yv[PM], Hy[PM];
  for (int i = 0; i < P; ++i) {
    sv[i] = s.xt[i] - s.x[i];
    yv[i] = gt[i] - s.g[i];
  }
  const double sy = dotp(sv, yv, P);
  if (sy > 0.0) {
    if (s.iter == 0 && s.n_hess == 0) {
      // Nocedal & Wright Eq. 6.20: rescale the initial matrix before the first update
      const double sc = sy / dotp(yv, yv, P);
      for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) s.H[i * PM + j] = (i == j && s.mask[i]) ? sc : 0.0;
      s.h0 = sc;
    }
    const double rho = 1.0 / sy;
    for (int i = 0; i < P; ++i) {
      double v = 0.0;
      for (int j = 0; j < P; ++j) v += s.H[i * PM + j] * yv[j];
      Hy[i] = v;
    }
    const double yHy = dotp(yv, Hy, P);
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j)
        s.H[i * PM + j] += rho * ((1.0 + rho * yHy) * sv[i] * sv[j] - Hy[i] * sv[j] - sv[i] * Hy[j]);
  }
  for (int i = 0; i < P; ++i) {
    s.x[i] = s.xt[i];
    s.g[i] = gt[i];
  }
  s.f = ft;
  s.iter += 1;
  s.fresh = 0;
  begin_iteration(s, P, tol, max_iter);
}

// Safeguarded quadratic interpolation in [lo, hi] from (lo, f_lo, d_lo), (hi, f_hi).
template <int PM>
__device__ inline double zoom_trial(const BfgsStateT<PM>& s) {
  const double lo = s.a_lo, hi = s.a_hi, dh = hi - lo;
  double a;
  const double den = 2.0 * (s.f_hi - s.f_lo - s.d_lo * dh);
  if (isfinite(s.f_hi) && den > 0.0) a = lo - s.d_lo * dh * dh / den;
  else a = lo + 0.5 * dh;
  const double b0 = fmin(lo, hi) + 0.1 * fabs(dh), b1 = fmax(lo, hi) - 0.1 * fabs(dh);
  if (!(a >= b0 && a <= b1)) a = lo + 0.5 * dh;
  return a;
}

template <int PM>
__device__ void bfgs_update(BfgsStateT<PM>& s, const double* __restrict__ o, int P, double tol, int max_iter) {
  double ft = o[0];
  double gt[PM];
  bool ok = isfinite(ft);
  for (int i = 0; i < P; ++i) {
    gt[i] = s.mask[i] ? o[1 + i] : 0.0;
    ok = ok && isfinite(gt[i]);
  }
  if (!ok) ft = INFINITY;
  s.n_eval += 1;
  if (s.phase == kPhaseHessPlus || s.phase == kPhaseHessMinus) {
    hessian_step(s, P, gt, ok, tol, max_iter);
    return;
  }
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
      for (int j = 0; j < P; ++j) s.H[i * PM + j] = (i == j && s.mask[i]) ? s.h0 : 0.0;
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
template <int PM>
__global__ void bfgs_step(BfgsStateT<PM>* __restrict__ st, const double* __restrict__ out, int out_stride, int n_fits,
                           int P, double tol, int max_iter, int* __restrict__ stat, double* __restrict__ rres) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_fits) return;
  BfgsStateT<PM>& s = st[f];
  if (s.status == kFitRunning) {
    bfgs_update(s, out + (int64_t)f * out_stride, P, tol, max_iter);
    if (s.status != kFitRunning) {
      double* r = rres + (int64_t)f * (3 + 2 * P);
      r[0] = s.f;
      r[1] = s.iter;
      r[2] = s.n_eval;
      for (int i = 0; i < P; ++i) {
        r[3 + i] = s.x[i];
        r[3 + P + i] = s.mask[i] ? sqrt(fabs(s.H[i * PM + i])) : 0.0;
      }
    }
  }
  stat[f] = s.status;
}

}  // namespace fn
