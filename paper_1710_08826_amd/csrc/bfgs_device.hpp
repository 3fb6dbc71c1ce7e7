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

  static constexpr int kCap = PM;
  static constexpr bool kFull = true;  // can run the numerical-Hessian phases
  __device__ double& Hm(int i, int j) { return H[i * PM + j]; }
  __device__ double Hm(int i, int j) const { return H[i * PM + j]; }
  __device__ double& Hnm(int i, int j) { return Hn[i * PM + j]; }
  __device__ double& gpv(int i) { return gp[i]; }
};

// The same state for a fit with exactly PC parameters, held in registers for
// one step (loaded from and stored back to the device-memory state, whose
// numerical-Hessian work space it keeps using in place).
template <int PC, int PM>
struct BfgsLocal {
  double xt[PC], x[PC], g[PC], p[PC], H[PC * PC];
  double f, d0, alpha, h0, edm, hstep;
  double a_prev, f_prev, d_prev, a_lo, f_lo, d_lo, a_hi, f_hi;
  int mask[PC];
  int status, phase, iter, ls_it, n_eval, hcol, n_hess, fresh;
  BfgsStateT<PM>* mem;

  static constexpr int kCap = PC;
  static constexpr bool kFull = false;
  __device__ double& Hm(int i, int j) { return H[i * PC + j]; }
  __device__ double Hm(int i, int j) const { return H[i * PC + j]; }
  __device__ double& Hnm(int i, int j) { return mem->Hn[i * PM + j]; }
  __device__ double& gpv(int i) { return mem->gp[i]; }

  __device__ void load(BfgsStateT<PM>& m) {
    mem = &m;
#pragma unroll
    for (int i = 0; i < PC; ++i) {
      xt[i] = m.xt[i]; x[i] = m.x[i]; g[i] = m.g[i]; p[i] = m.p[i]; mask[i] = m.mask[i];
#pragma unroll
      for (int j = 0; j < PC; ++j) H[i * PC + j] = m.H[i * PM + j];
    }
    f = m.f; d0 = m.d0; alpha = m.alpha; h0 = m.h0; edm = m.edm; hstep = m.hstep;
    a_prev = m.a_prev; f_prev = m.f_prev; d_prev = m.d_prev;
    a_lo = m.a_lo; f_lo = m.f_lo; d_lo = m.d_lo; a_hi = m.a_hi; f_hi = m.f_hi;
    status = m.status; phase = m.phase; iter = m.iter; ls_it = m.ls_it; n_eval = m.n_eval;
    hcol = m.hcol; n_hess = m.n_hess; fresh = m.fresh;
  }
  __device__ void store(BfgsStateT<PM>& m) const {
#pragma unroll
    for (int i = 0; i < PC; ++i) {
      m.xt[i] = xt[i]; m.x[i] = x[i]; m.g[i] = g[i]; m.p[i] = p[i]; m.mask[i] = mask[i];
#pragma unroll
      for (int j = 0; j < PC; ++j) m.H[i * PM + j] = H[i * PC + j];
    }
    m.f = f; m.d0 = d0; m.alpha = alpha; m.h0 = h0; m.edm = edm; m.hstep = hstep;
    m.a_prev = a_prev; m.f_prev = f_prev; m.d_prev = d_prev;
    m.a_lo = a_lo; m.f_lo = f_lo; m.d_lo = d_lo; m.a_hi = a_hi; m.f_hi = f_hi;
    m.status = status; m.phase = phase; m.iter = iter; m.ls_it = ls_it; m.n_eval = n_eval;
    m.hcol = hcol; m.n_hess = n_hess; m.fresh = fresh;
  }
};

// --------------------------------------------------------------- BFGS step
__device__ __forceinline__ double dotp(const double* a, const double* b, int P) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < P; ++i) s += a[i] * b[i];
  return s;
}

// Direction p = -H g (fixed parameters have zero rows/columns in H).
template <class ST>
__device__ __forceinline__ void new_direction(ST& s, int P) {
#pragma unroll
  for (int i = 0; i < P; ++i) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) v += s.Hm(i, j) * s.g[j];
    s.p[i] = -v;
  }
  s.d0 = dotp(s.g, s.p, P);
}

template <class ST>
__device__ __forceinline__ void set_trial(ST& s, int P, double a) {
  s.alpha = a;
#pragma unroll
  for (int i = 0; i < P; ++i) s.xt[i] = s.x[i] + a * s.p[i];
}

// Start the numerical-Hessian column of the first free parameter c >= from:
// gradient at x + h e_c, with h 1e-4 of the error the current matrix implies
// and a floor relative to the parameter.  Selects instead of indexing by c
// keep a register copy of the state addressable.
template <class ST>
__device__ __forceinline__ bool start_hessian_column(ST& s, int P, int from) {
  int c = -1;
#pragma unroll
  for (int i = P - 1; i >= from; --i)
    if (s.mask[i]) c = i;
  if (c < 0) return false;
  double hd = 0.0, xc = 0.0;
#pragma unroll
  for (int i = 0; i < P; ++i)
    if (i == c) {
      hd = s.Hm(i, i);
      xc = s.x[i];
    }
  s.hcol = c;
  s.hstep = fmax(1e-4 * sqrt(fabs(hd)), 1e-9 * fmax(fabs(xc), 1.0));
#pragma unroll
  for (int j = 0; j < P; ++j) s.xt[j] = j == c ? s.x[j] + s.hstep : s.x[j];
  s.phase = kPhaseHessPlus;
  return true;
}

template <class ST>
__device__ __forceinline__ bool start_hessian(ST& s, int P) {
#pragma unroll
  for (int i = 0; i < P; ++i)
#pragma unroll
    for (int j = 0; j < P; ++j) s.Hnm(i, j) = 0.0;
  return start_hessian_column(s, P, 0);
}

// Inverse of the symmetric positive definite matrix Hn restricted to the free
// parameters (Cholesky factor in place, then inverse of the factor in place,
// then H = L^-T L^-1); false if Hn is not positive definite.
template <class ST>
__device__ __forceinline__ bool hessian_inverse(ST& s, int P) {
  int idx[ST::kCap];
  int D = 0;
  for (int i = 0; i < P; ++i)
    if (s.mask[i]) idx[D++] = i;
  auto A = [&](int i, int j) -> double& { return s.Hnm(idx[i], idx[j]); };
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
  for (int i = 0; i < P; ++i)
    for (int j = 0; j < P; ++j) s.Hm(i, j) = 0.0;
  for (int a = 0; a < D; ++a)
    for (int b = 0; b <= a; ++b) {
      double v = 0.0;
      for (int k = a; k < D; ++k) v += A(k, a) * A(k, b);
      s.Hm(idx[a], idx[b]) = v;
      s.Hm(idx[b], idx[a]) = v;
    }
  return true;
}

template <class ST>
__device__ __forceinline__ void begin_iteration(ST& s, int P, double tol, int max_iter);

// One gradient of the numerical Hessian has arrived (phase HessPlus or HessMinus).
template <class ST>
__device__ __forceinline__ void hessian_step(ST& s, int P, const double* gt, bool ok, double tol, int max_iter) {
  const int c = s.hcol;
  if (!ok) {
    // a neighbour of the minimum is not finite: keep the BFGS matrix
    for (int j = 0; j < P; ++j) s.xt[j] = s.x[j];
    s.status = kFitConverged;
    return;
  }
  if (s.phase == kPhaseHessPlus) {
    for (int i = 0; i < P; ++i) s.gpv(i) = gt[i];
    s.xt[c] = s.x[c] - s.hstep;
    s.phase = kPhaseHessMinus;
    return;
  }
  const double den = (s.x[c] + s.hstep) - (s.x[c] - s.hstep);
  for (int i = 0; i < P; ++i) s.Hnm(i, c) = s.mask[i] ? (s.gpv(i) - gt[i]) / den : 0.0;
  if (start_hessian_column(s, P, c + 1)) return;
  for (int j = 0; j < P; ++j) s.xt[j] = s.x[j];
  for (int i = 0; i < P; ++i)
    for (int j = 0; j < i; ++j) {
      const double v = 0.5 * (s.Hnm(i, j) + s.Hnm(j, i));
      s.Hnm(i, j) = s.Hnm(j, i) = v;
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
template <class ST>
__device__ __forceinline__ void begin_iteration(ST& s, int P, double tol, int max_iter) {
  // estimated distance to the minimum
  double edm = 0.0;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) v += s.Hm(i, j) * s.g[j];
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
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
      for (int j = 0; j < P; ++j) s.Hm(i, j) = (i == j && s.mask[i]) ? s.h0 : 0.0;
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

template <class ST>
__device__ __forceinline__ void accept_trial(ST& s, int P, const double* gt, double ft, double tol, int max_iter) {
  double sv[ST::kCap], yv[ST::kCap], Hy[ST::kCap];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    sv[i] = s.xt[i] - s.x[i];
    yv[i] = gt[i] - s.g[i];
  }
  const double sy = dotp(sv, yv, P);
  if (sy > 0.0) {
    if (s.iter == 0 && s.n_hess == 0) {
      // Nocedal & Wright Eq. 6.20: rescale the initial matrix before the first update
      const double sc = sy / dotp(yv, yv, P);
#pragma unroll
      for (int i = 0; i < P; ++i)
#pragma unroll
        for (int j = 0; j < P; ++j) s.Hm(i, j) = (i == j && s.mask[i]) ? sc : 0.0;
      s.h0 = sc;
    }
    const double rho = 1.0 / sy;
#pragma unroll
    for (int i = 0; i < P; ++i) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < P; ++j) v += s.Hm(i, j) * yv[j];
      Hy[i] = v;
    }
    const double yHy = dotp(yv, Hy, P);
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
      for (int j = 0; j < P; ++j)
        s.Hm(i, j) += rho * ((1.0 + rho * yHy) * sv[i] * sv[j] - Hy[i] * sv[j] - sv[i] * Hy[j]);
  }
#pragma unroll
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
template <class ST>
__device__ __forceinline__ double zoom_trial(const ST& s) {
  const double lo = s.a_lo, hi = s.a_hi, dh = hi - lo;
  double a;
  const double den = 2.0 * (s.f_hi - s.f_lo - s.d_lo * dh);
  if (isfinite(s.f_hi) && den > 0.0) a = lo - s.d_lo * dh * dh / den;
  else a = lo + 0.5 * dh;
  const double b0 = fmin(lo, hi) + 0.1 * fabs(dh), b1 = fmax(lo, hi) - 0.1 * fabs(dh);
  if (!(a >= b0 && a <= b1)) a = lo + 0.5 * dh;
  return a;
}

template <class ST>
__device__ __forceinline__ void bfgs_update(ST& s, const double* __restrict__ o, int P, double tol, int max_iter) {
  double ft = o[0];
  double gt[ST::kCap];
  bool ok = isfinite(ft);
#pragma unroll
  for (int i = 0; i < P; ++i) {
    gt[i] = s.mask[i] ? o[1 + i] : 0.0;
    ok = ok && isfinite(gt[i]);
  }
  if (!ok) ft = INFINITY;
  s.n_eval += 1;
  if (s.phase == kPhaseHessPlus || s.phase == kPhaseHessMinus) {
    if constexpr (ST::kFull) hessian_step(s, P, gt, ok, tol, max_iter);
    return;
  }
  const double c1 = 1e-4, c2 = 0.9;
  if (s.phase == kPhaseStart) {
    if (!ok) {
      s.status = kFitFailed;
      return;
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
      s.x[i] = s.xt[i];
      s.g[i] = gt[i];
    }
    s.f = ft;
    // starting inverse Hessian: first step moves the largest gradient component by 1e-3 of its scale
    double gmax = 0.0;
#pragma unroll
    for (int i = 0; i < P; ++i) gmax = fmax(gmax, fabs(gt[i]));
    s.h0 = gmax > 0.0 ? 1e-3 / gmax : 1.0;
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
      for (int j = 0; j < P; ++j) s.Hm(i, j) = (i == j && s.mask[i]) ? s.h0 : 0.0;
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

// Result row [NLL, iterations, evaluations, theta(P), sqrt|H_ii|(P)] of a fit
// that has just retired.
template <class ST>
__device__ __forceinline__ void write_result(const ST& s, int P, double* __restrict__ r) {
  r[0] = s.f;
  r[1] = s.iter;
  r[2] = s.n_eval;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    r[3 + i] = s.x[i];
    r[3 + P + i] = s.mask[i] ? sqrt(fabs(s.Hm(i, i))) : 0.0;
  }
}

// One minimizer step per running fit; every slot's status is mirrored into
// stat[], and a fit that retires in this step writes its result row into rres.
template <int PM>
__global__ __launch_bounds__(64) void bfgs_step(BfgsStateT<PM>* __restrict__ st, const double* __restrict__ out,
                                                int out_stride, int n_fits, int P, double tol, int max_iter,
                                                int* __restrict__ stat, double* __restrict__ rres) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_fits) return;
  BfgsStateT<PM>& s = st[f];
  if (s.status == kFitRunning) {
    bfgs_update(s, out + (int64_t)f * out_stride, P, tol, max_iter);
    if (s.status != kFitRunning) write_result(s, P, rres + (int64_t)f * (3 + 2 * P));
  }
  stat[f] = s.status;
}

// The same step for fits with exactly PC parameters, on a register copy of the
// state (one round of loads and one of stores instead of a chain of dependent
// device-memory accesses).  The numerical-Hessian phases, a few evaluations
// per fit, index the state at run time and stay on the device-memory copy.
template <int PM, int PC>
__global__ __launch_bounds__(64) void bfgs_step_small(BfgsStateT<PM>* __restrict__ st,
                                                      const double* __restrict__ out, int out_stride, int n_fits,
                                                      double tol, int max_iter, int* __restrict__ stat,
                                                      double* __restrict__ rres) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_fits) return;
  BfgsStateT<PM>& m = st[f];
  int status = m.status;
  if (status == kFitRunning) {
    const double* o = out + (int64_t)f * out_stride;
    double* r = rres + (int64_t)f * (3 + 2 * PC);
    if (m.phase == kPhaseHessPlus || m.phase == kPhaseHessMinus) {
      bfgs_update(m, o, PC, tol, max_iter);
      status = m.status;
      if (status != kFitRunning) write_result(m, PC, r);
    } else {
      BfgsLocal<PC, PM> s;
      s.load(m);
      bfgs_update(s, o, PC, tol, max_iter);
      s.store(m);
      status = s.status;
      if (status != kFitRunning) write_result(s, PC, r);
    }
  }
  stat[f] = status;
}

// Launch of one minimizer step for n_fits fits of P parameters (a register copy
// of the state for P <= 8).
template <int PM>
inline void bfgs_launch(BfgsStateT<PM>* st, const double* out, int out_stride, int n_fits, int P, double tol,
                        int max_iter, int* stat, double* rres, hipStream_t s) {
  const dim3 g((n_fits + 63) / 64), b(64);
#define FN_BFGS_SMALL(PC)                                                                                      \
  case PC:                                                                                                   \
    hipLaunchKernelGGL((bfgs_step_small<PM, PC>), g, b, 0, s, st, out, out_stride, n_fits, tol, max_iter,   \
                       stat, rres);                                                                          \
    return;
  switch (PM >= 8 ? P : 0) {
    FN_BFGS_SMALL(1)
    FN_BFGS_SMALL(2)
    FN_BFGS_SMALL(3)
    FN_BFGS_SMALL(4)
    FN_BFGS_SMALL(5)
    FN_BFGS_SMALL(6)
    FN_BFGS_SMALL(7)
    FN_BFGS_SMALL(8)
    default:
      break;
  }
#undef FN_BFGS_SMALL
  hipLaunchKernelGGL((bfgs_step<PM>), g, b, 0, s, st, out, out_stride, n_fits, P, tol, max_iter, stat, rres);
}

}  // namespace fn
