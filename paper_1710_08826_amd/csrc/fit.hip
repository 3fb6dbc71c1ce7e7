// Single-fit quasi-Newton minimizer on the host, driving the device NLL.
// This takes the place of the paper's FitManager + Minuit loop (Fig. 1,
// Sec. 4): BFGS on the inverse Hessian with a line search that satisfies the
// strong Wolfe conditions (Nocedal & Wright, Numerical Optimization, 2nd ed.,
// Algorithms 3.5/3.6 and Eq. 6.17), convergence on the estimated distance to
// the minimum EDM = g^T H g / 2, errors from the inverse of a numerical
// Hessian (error definition 1/2 for an NLL).  An EDM below the tolerance is
// re-tested with the inverse numerical Hessian before the fit is declared
// converged, and the iterations continue from that matrix when it fails.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace fn {
namespace {

constexpr int kMaxHessianChecks = 3;

struct Objective {
  fn_model* m;
  const double* ev;
  int64_t n, ld;
  hipStream_t s;
  int grad_mode;                // 0 adjoint, 1 central differences
  std::vector<int> free_idx;    // indices of free parameters
  std::vector<double> full;     // full theta (fixed entries stay)
  const BinnedData* binned = nullptr;  // binned data instead of events
  long long calls = 0;

  void value(const double* th, double* f, double* g) {
    if (binned) nll_binned_host(m, th, *binned, f, g, s);
    else nll_host(m, th, ev, n, ld, f, g, s);
  }

  int dim() const { return (int)free_idx.size(); }

  // f and (optionally) gradient w.r.t. free parameters; returns false when
  // the NLL is not finite.
  bool eval(const std::vector<double>& x, double& f, std::vector<double>* g) {
    for (int i = 0; i < dim(); ++i) full[free_idx[i]] = x[i];
    std::vector<double> gfull(m->P);
    if (!g || grad_mode == 1) {
      if (!nll_only(full, f)) return false;
      if (g) {
        g->assign(dim(), 0.0);
        for (int i = 0; i < dim(); ++i) {
          const int p = free_idx[i];
          const double h = 1e-6 * std::fmax(std::fabs(full[p]), 1.0);
          std::vector<double> tp = full, tm = full;
          tp[p] += h;
          tm[p] -= h;
          double fp, fm;
          if (!nll_only(tp, fp) || !nll_only(tm, fm)) return false;
          (*g)[i] = (fp - fm) / (tp[p] - tm[p]);
        }
      }
      return true;
    }
    calls += 1;
    try {
      value(full.data(), &f, gfull.data());
    } catch (const Error& e) {
      if (e.code == FN_E_NONFINITE) return false;
      throw;
    }
    g->resize(dim());
    for (int i = 0; i < dim(); ++i) (*g)[i] = gfull[free_idx[i]];
    return true;
  }

  bool nll_only(const std::vector<double>& th, double& f) {
    calls += 1;
    try {
      value(th.data(), &f, nullptr);
    } catch (const Error& e) {
      if (e.code == FN_E_NONFINITE) return false;
      throw;
    }
    return true;
  }
};

double dot(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

// Strong-Wolfe line search along p from x (f0, g0); returns step alpha and
// fills xn, fn_, gn; alpha = 0 when no acceptable point was found.
double line_search(Objective& obj, const std::vector<double>& x, double f0, const std::vector<double>& g0,
                   const std::vector<double>& p, std::vector<double>& xn, double& fnew, std::vector<double>& gn) {
  const double c1 = 1e-4, c2 = 0.9;
  const double d0 = dot(g0, p);
  if (!(d0 < 0.0)) return 0.0;
  const int D = (int)x.size();
  auto phi = [&](double a, double& fa, std::vector<double>& ga, double& da) {
    xn.resize(D);
    for (int i = 0; i < D; ++i) xn[i] = x[i] + a * p[i];
    if (!obj.eval(xn, fa, &ga)) {
      fa = INFINITY;
      da = NAN;
      return;
    }
    da = dot(ga, p);
  };
  double a_prev = 0.0, f_prev = f0, d_prev = d0;
  double a = 1.0;
  std::vector<double> ga;
  auto zoom = [&](double lo, double flo, double dlo, double hi, double fhi) -> double {
    for (int it = 0; it < 40; ++it) {
      // quadratic interpolation from (lo, flo, dlo) and (hi, fhi), safeguarded
      double aj;
      const double dh = hi - lo;
      const double den = 2.0 * (fhi - flo - dlo * dh);
      if (std::isfinite(fhi) && den > 0.0) aj = lo - dlo * dh * dh / den;
      else aj = lo + 0.5 * dh;
      const double lo_b = std::fmin(lo, hi) + 0.1 * std::fabs(dh);
      const double hi_b = std::fmax(lo, hi) - 0.1 * std::fabs(dh);
      if (!(aj >= lo_b && aj <= hi_b)) aj = lo + 0.5 * dh;
      double fj, dj;
      phi(aj, fj, ga, dj);
      if (!(fj <= f0 + c1 * aj * d0) || fj >= flo) {
        hi = aj;
        fhi = fj;
      } else {
        if (std::fabs(dj) <= -c2 * d0) {
          fnew = fj;
          gn = ga;
          return aj;
        }
        if (dj * (hi - lo) >= 0.0) {
          hi = lo;
          fhi = flo;
        }
        lo = aj;
        flo = fj;
        dlo = dj;
      }
      if (std::fabs(hi - lo) < 1e-16 * std::fmax(1.0, std::fabs(lo))) break;
    }
    // fall back to the best sufficient-decrease point seen (lo), if any
    if (lo > 0.0) {
      double fl, dl;
      phi(lo, fl, ga, dl);
      if (std::isfinite(fl) && fl < f0) {
        fnew = fl;
        gn = ga;
        return lo;
      }
    }
    return 0.0;
  };
  for (int i = 0; i < 40; ++i) {
    double fa, da;
    phi(a, fa, ga, da);
    if (!(fa <= f0 + c1 * a * d0) || (i > 0 && fa >= f_prev)) return zoom(a_prev, f_prev, d_prev, a, fa);
    if (std::fabs(da) <= -c2 * d0) {
      fnew = fa;
      gn = ga;
      return a;
    }
    if (da >= 0.0) return zoom(a, fa, da, a_prev, f_prev);
    a_prev = a;
    f_prev = fa;
    d_prev = da;
    a *= 2.0;
  }
  return 0.0;
}

// Inverse of a symmetric positive definite matrix by Cholesky; false if not SPD.
bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> L(n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    if (!(s > 0.0)) return false;
    L[j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / L[j * n + j];
    }
  }
  // inverse of L, then A^-1 = L^-T L^-1
  std::vector<double> Li(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    Li[i * n + i] = 1.0 / L[i * n + i];
    for (int j = 0; j < i; ++j) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s -= L[i * n + k] * Li[k * n + j];
      Li[i * n + j] = s / L[i * n + i];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = std::max(i, j); k < n; ++k) s += Li[k * n + i] * Li[k * n + j];
      A[i * n + j] = s;
    }
  return true;
}

}  // namespace

// Inverse of the numerical Hessian at x (central differences of the gradient,
// step 1e-4 of the error the matrix H implies, floored relative to |x|);
// false if an evaluation fails or the Hessian is not positive definite.
bool numerical_inverse_hessian(Objective& obj, const std::vector<double>& x, const std::vector<double>& H,
                               std::vector<double>& Hn) {
  const int D = obj.dim();
  Hn.assign((size_t)D * D, 0.0);
  for (int i = 0; i < D; ++i) {
    const double d = std::fmax(1e-4 * std::sqrt(std::fabs(H[i * D + i])), 1e-9 * std::fmax(std::fabs(x[i]), 1.0));
    std::vector<double> xp = x, xm = x, gp, gm;
    xp[i] += d;
    xm[i] -= d;
    double fp, fm;
    if (!obj.eval(xp, fp, &gp) || !obj.eval(xm, fm, &gm)) return false;
    for (int j = 0; j < D; ++j) Hn[j * D + i] = (gp[j] - gm[j]) / (xp[i] - xm[i]);
  }
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < i; ++j) Hn[i * D + j] = Hn[j * D + i] = 0.5 * (Hn[i * D + j] + Hn[j * D + i]);
  return spd_inverse(Hn, D);
}

void fit_host(fn_model* m, const double* theta0, const int32_t* mask, const double* ev, int64_t n, int64_t ld,
              const BinnedData* binned, int grad_mode, double tol, int max_iter, double* theta_out, double* err_out,
              double* nll_out, int32_t* n_iter_out, int32_t* n_calls_out, hipStream_t s) {
  if (!theta0) throw Error(FN_E_INVALID, "theta0 is NULL");
  if (grad_mode != 0 && grad_mode != 1) throw Error(FN_E_INVALID, "grad_mode must be 0 or 1");
  if (!binned) check_events_args(m, ev, n, ld);
  Objective obj{m, ev, n, ld, s, grad_mode, {}, std::vector<double>(theta0, theta0 + m->P)};
  obj.binned = binned;
  for (int p = 0; p < m->P; ++p)
    if (!mask || mask[p]) obj.free_idx.push_back(p);
  const int D = obj.dim();
  if (tol <= 0.0) tol = 1e-7;
  if (max_iter <= 0) max_iter = 500;
  std::vector<double> x(D), g, xn, gn;
  for (int i = 0; i < D; ++i) x[i] = theta0[obj.free_idx[i]];
  double f;
  if (!obj.eval(x, f, &g)) throw Error(FN_E_NONFINITE, "NLL is not finite at the start point");
  // starting inverse Hessian: diagonal from second differences of the NLL
  std::vector<double> H(D * D, 0.0);
  for (int i = 0; i < D; ++i) {
    const double d = 1e-3 * std::fmax(std::fabs(x[i]), 0.1);
    std::vector<double> xp = x, xm = x;
    xp[i] += d;
    xm[i] -= d;
    double fp, fm;
    const bool ok = obj.eval(xp, fp, nullptr) && obj.eval(xm, fm, nullptr);
    const double h2 = ok ? (fp - 2.0 * f + fm) / (d * d) : -1.0;
    H[i * D + i] = (h2 > 0.0 && std::isfinite(h2)) ? 1.0 / h2 : d / std::fmax(std::fabs(g[i]), 1e-300);
  }
  int iter = 0;
  bool converged = false;
  bool fresh = false;  // H is the inverse of the numerical Hessian at x
  int n_hess = 0;
  std::vector<double> p(D);
  for (; iter < max_iter; ++iter) {
    double edm = 0.0;
    for (int i = 0; i < D; ++i) {
      double hi = 0.0;
      for (int j = 0; j < D; ++j) hi += H[i * D + j] * g[j];
      p[i] = -hi;
      edm += g[i] * hi;
    }
    edm *= 0.5;
    if (edm < tol && edm >= 0.0) {
      // check the BFGS estimate with the numerical Hessian (as Minuit's MIGRAD does after HESSE)
      std::vector<double> Hi;
      if (fresh || n_hess >= kMaxHessianChecks || !numerical_inverse_hessian(obj, x, H, Hi)) {
        converged = true;
        break;
      }
      n_hess += 1;
      H = Hi;
      fresh = true;
      --iter;  // re-test without consuming an iteration
      continue;
    }
    double fnew = f;
    double a = line_search(obj, x, f, g, p, xn, fnew, gn);
    if (a == 0.0) {
      // reset to steepest descent scaled by the diagonal once, then give up
      bool reset_ok = false;
      std::vector<double> Hd(D * D, 0.0);
      for (int i = 0; i < D; ++i) Hd[i * D + i] = std::fabs(H[i * D + i]) > 0 ? std::fabs(H[i * D + i]) : 1e-6;
      for (int i = 0; i < D; ++i) p[i] = -Hd[i * D + i] * g[i];
      a = line_search(obj, x, f, g, p, xn, fnew, gn);
      if (a != 0.0) {
        H = Hd;
        reset_ok = true;
      }
      if (!reset_ok) break;
    }
    std::vector<double> sv(D), yv(D);
    for (int i = 0; i < D; ++i) {
      sv[i] = xn[i] - x[i];
      yv[i] = gn[i] - g[i];
    }
    const double sy = dot(sv, yv);
    if (sy > 0.0) {
      if (iter == 0 && n_hess == 0) {
        // Nocedal & Wright Eq. 6.20 rescaling before the first update
        const double scale = sy / dot(yv, yv);
        for (int i = 0; i < D; ++i)
          for (int j = 0; j < D; ++j) H[i * D + j] = (i == j) ? scale : 0.0;
      }
      const double rho = 1.0 / sy;
      std::vector<double> Hy(D);
      for (int i = 0; i < D; ++i) {
        double t = 0.0;
        for (int j = 0; j < D; ++j) t += H[i * D + j] * yv[j];
        Hy[i] = t;
      }
      const double yHy = dot(yv, Hy);
      for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j)
          H[i * D + j] += rho * ((1.0 + rho * yHy) * sv[i] * sv[j] - Hy[i] * sv[j] - sv[i] * Hy[j]);
    }
    x = xn;
    f = fnew;
    g = gn;
    fresh = false;
  }
  for (int i = 0; i < D; ++i) obj.full[obj.free_idx[i]] = x[i];
  if (theta_out)
    for (int p2 = 0; p2 < m->P; ++p2) theta_out[p2] = obj.full[p2];
  if (nll_out) *nll_out = f;
  if (err_out) {
    for (int p2 = 0; p2 < m->P; ++p2) err_out[p2] = 0.0;
    std::vector<double> Hn;
    const std::vector<double>* C = &H;  // BFGS estimate as the fallback
    if (fresh) {
      C = &H;
    } else if (numerical_inverse_hessian(obj, x, H, Hn)) {
      C = &Hn;
    }
    // error definition: 1/2 for an NLL, 1 for chi^2 (covariance 2 H^-1)
    const double up2 = binned && binned->stat == 1 ? 2.0 : 1.0;
    for (int i = 0; i < D; ++i) err_out[obj.free_idx[i]] = std::sqrt(up2 * std::fabs((*C)[i * D + i]));
  }
  if (n_iter_out) *n_iter_out = iter;
  if (n_calls_out) *n_calls_out = (int32_t)obj.calls;
  if (!converged) throw Error(FN_E_INVALID, "fit did not converge in " + std::to_string(iter) + " iterations");
}

}  // namespace fn

extern "C" fn_status fn_fit(fn_model* m, const double* theta0_host, const int32_t* free_mask, const double* ev,
                            int64_t n, int64_t ld, int32_t grad_mode, double tol, int32_t max_iter,
                            double* theta_out, double* err_out, double* nll_out, int32_t* n_iter,
                            int32_t* n_calls, void* stream) {
  return fn::guard([&] {
    if (!m) throw fn::Error(FN_E_INVALID, "model is NULL");
    fn::hip_check(hipSetDevice(m->device), "hipSetDevice");
    fn::fit_host(m, theta0_host, free_mask, ev, n, ld, nullptr, grad_mode, tol, max_iter, theta_out, err_out,
                 nll_out, n_iter, n_calls, (hipStream_t)stream);
  });
}

extern "C" fn_status fn_fit_binned(fn_model* m, const double* theta0_host, const int32_t* free_mask,
                                   const double* counts_dev, int64_t n_bins, int32_t stat, int32_t grad_mode,
                                   double tol, int32_t max_iter, double* theta_out, double* err_out,
                                   double* value_out, int32_t* n_iter, int32_t* n_calls, void* stream) {
  return fn::guard([&] {
    if (!m) throw fn::Error(FN_E_INVALID, "model is NULL");
    if (m->kind != fn::kKindMix1d) throw fn::Error(FN_E_INVALID, "binned data: mix1d models only");
    if (n_bins < 1 || !counts_dev) throw fn::Error(FN_E_INVALID, "binned data: need n_bins >= 1 and counts");
    if (stat != 0 && stat != 1) throw fn::Error(FN_E_INVALID, "stat must be 0 (Poisson) or 1 (chi^2)");
    fn::hip_check(hipSetDevice(m->device), "hipSetDevice");
    const fn::BinnedData bd{counts_dev, n_bins, stat};
    fn::fit_host(m, theta0_host, free_mask, nullptr, 0, 0, &bd, grad_mode, tol, max_iter, theta_out, err_out,
                 value_out, n_iter, n_calls, (hipStream_t)stream);
  });
}
