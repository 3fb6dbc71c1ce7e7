// Time-dependent four-body amplitude model (the paper's four-body
// time-dependent amplitude analyses, Abstract and Sec. 5): host launchers and
// the kernels that do not depend on the model's shape (prologue, level-2
// finalize, per-event density, domain check).  The per-event and
// normalization-matrix passes live in td4_device.hpp and are compiled at model
// creation with the model's shape as compile-time constants (td4_jit below).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>
#include <vector>

#include "internal.hpp"
#include "jit.hpp"
#include "td4.hpp"
#include "td4_device.hpp"

namespace fn {

// Lineshapes of one pair from its invariant mass m: amp[r] for every resonance of the pair.
template <int NR>
__device__ __forceinline__ void pair_amps(double m, double sum2, double dif2, double r2, const int* L, const int* nr,
                                          int n, const double (*rt)[3], cplx (&amp)[NR]) {
  const double s = m * m;
  const double im = rcp_fast(m);
  const double lq = fmax((s - sum2) * (s - dif2), 0.0);
  const double q2 = 0.25 * lq * im * im;
  const double q = sqrt_fast(q2);
  const double G0 = q * im;
  const double z = q2 * r2;
  const double F1 = rsqrt_fast(1.0 + z);
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
      const double d = rcp_fast(__builtin_fma(a, a, b * b));
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
  const double ss = 0.5 * sqrt_fast(fmax(1.0 - c12 * c12, 0.0)) * sqrt_fast(fmax(1.0 - c34 * c34, 0.0));
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
// One 64-thread workgroup per fit, each table entry written by its own thread
// (so that the loads of theta and of the fixed constants are issued together,
// not one after the other): threads 0..5 the r12 lineshapes, 8..13 the r34
// ones, 16..35 the coefficients of basis function j - 16 in A and in Abar,
// 40 x, y, sigma; thread 0 writes the validity flag once all checks are in.
constexpr int kTd4PrologueThreads = 64;
static_assert(16 + kTd4MaxAmp <= 40 && kTd4MaxRes <= 8, "prologue thread map");
__global__ __launch_bounds__(kTd4PrologueThreads) void td4_prologue(Td4Const tc, ParamBlock pb,
                                                                    const double* __restrict__ theta, int theta_stride,
                                                                    const Td4FitConst* __restrict__ fcs,
                                                                    const int* __restrict__ status, int n_fits,
                                                                    Td4Table* __restrict__ tabs) {
  const int f = blockIdx.x;
  if (f >= n_fits || (status && status[f] != 1)) return;
  const int j = threadIdx.x;
  const double* th = theta ? theta + (int64_t)f * theta_stride : pb.v;
  const Td4FitConst& fc = fcs[f];
  Td4Table& t = tabs[f];
  bool ok = true;
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
  if (j < kTd4MaxRes) {
    const int r = j;
    t.r12[r][0] = t.r12[r][1] = t.r12[r][2] = 0.0;
    if (r < tc.n12 && !tc.nr12[r]) lineshape(fc.m0_12[r], fc.w0_12[r], tc.L12[r], tc.sum12, tc.dif12, t.r12[r]);
  } else if (j >= 8 && j < 8 + kTd4MaxRes) {
    const int r = j - 8;
    t.r34[r][0] = t.r34[r][1] = t.r34[r][2] = 0.0;
    if (r < tc.n34 && !tc.nr34[r]) lineshape(fc.m0_34[r], fc.w0_34[r], tc.L34[r], tc.sum34, tc.dif34, t.r34[r]);
  } else if (j >= 16 && j < 16 + kTd4MaxAmp) {
    // a basis function outside a sum has a zero coefficient there
    const int k = j - 16;
    const int ia = k < tc.K ? tc.pa[k] : -1, ib = k < tc.K ? tc.pb[k] : -1;
    t.c[k][0] = ia >= 0 ? th[ia] : 0.0;
    t.c[k][1] = ia >= 0 ? th[ia + 1] : 0.0;
    t.cb[k][0] = ib >= 0 ? th[ib] : 0.0;
    t.cb[k][1] = ib >= 0 ? th[ib + 1] : 0.0;
  } else if (j == 40) {
    t.x = th[tc.n_params - 2];
    t.y = th[tc.n_params - 1];
    t.sigma = fc.sigma;
    ok = fc.sigma > 0.0 && fabs(t.y) < 1.0 && isfinite(t.x);
  }
  const bool bad = __syncthreads_or(!ok);
  if (j == 0) t.valid = bad ? 0.0 : 1.0;
}

// ---------------------------------------------------- normalization matrix
__global__ __launch_bounds__(kFinalBlock) void td4_mrows_finalize(Td4Const tc, const int* __restrict__ sel,
                                                                  const double* __restrict__ part, int64_t nch,
                                                                  int nv, int kmax, int i0, int rb, double inv_n,
                                                                  double* __restrict__ Mc) {
  __shared__ double scratch[kFinalBlock];
  __shared__ double res[kBlock];
  const int f = blockIdx.x;
  if (sel && !sel[f]) return;
  sum_rows_t<kFinalBlock>(part + (int64_t)f * nch * nv, nch, nv, scratch, res);
  const int K = tc.K;
  double* M = Mc + (int64_t)f * 2 * kTd4MaxAmp * kTd4MaxAmp;
  for (int t = threadIdx.x; t < rb * kmax; t += kFinalBlock) {
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
  __shared__ double XYUV[8][kTd4MaxAmp];       // Re, Im of X, Y, U, V per amplitude
  __shared__ double gI[4 * kTd4MaxAmp + 2];    // dI/dtheta in theta order
  __shared__ double form[4];                   // a, b, Re z, Im z
  __shared__ double Ish;
  __shared__ double cc[4 * kTd4MaxAmp];        // c then cb, (Re, Im) per amplitude
  static_assert(2 * kTd4MaxAmp * kTd4MaxAmp <= kFinalBlock, "one entry of M per thread");
  const int f = blockIdx.x;
  if (status && status[f] != 1) return;
  const Td4Table& tb = tabs[f];
  const int K = tc.K, P = tc.n_params;
  const int t = threadIdx.x;
  // M, the coefficients, x, y and the validity flag are loaded first, by every
  // thread (clamped indices, values not needed discarded; lane-varying offsets
  // so that the uniform ones are vector loads too): no wait for them comes
  // before the rows are requested, and their latency overlaps the row sums
  int zero = 0;
  asm volatile("" : "+v"(zero));
  constexpr int nm = 2 * kTd4MaxAmp * kTd4MaxAmp;
  const double mv = Mc[(int64_t)f * nm + (t < nm ? t : 0)];
  static_assert(offsetof(Td4Table, cb) == offsetof(Td4Table, c) + 2 * kTd4MaxAmp * sizeof(double),
                "cb follows c");
  const double cv = reinterpret_cast<const double*>(&tb)[offsetof(Td4Table, c) / sizeof(double) +
                                                         (t < 4 * kTd4MaxAmp ? t : 0)];
  const double x = (&tb.x)[zero], y = (&tb.y)[zero], valid = (&tb.valid)[zero];
  sum_rows_t<kFinalBlock>(part + (int64_t)f * rows * nv, rows, nv, scratch, res);
  if (t < nm) M[t] = mv;
  if (t < 4 * kTd4MaxAmp) cc[t] = cv;
  __syncthreads();
  auto m = [&](int i, int j) { return cplx{M[2 * (i * kTd4MaxAmp + j)], M[2 * (i * kTd4MaxAmp + j) + 1]}; };
  const double* c = cc;
  const double* cb = cc + 2 * kTd4MaxAmp;
  // thread k < K: the k-th entries of the four matrix-vector products
  if (t < K) {
    const int k = t;
    double Xr = 0.0, Xi = 0.0, Yr = 0.0, Yi = 0.0, Ur = 0.0, Ui = 0.0, Vr = 0.0, Vi = 0.0;
    for (int j = 0; j < K; ++j) {
      const cplx mkj = m(k, j), mjk = m(j, k);
      const double cjr = c[2 * j], cji = c[2 * j + 1], bjr = cb[2 * j], bji = cb[2 * j + 1];
      // X_k += M_kj conj(c_j), Y_k += M_kj conj(cb_j)
      Xr += mkj.re * cjr + mkj.im * cji;
      Xi += mkj.im * cjr - mkj.re * cji;
      Yr += mkj.re * bjr + mkj.im * bji;
      Yi += mkj.im * bjr - mkj.re * bji;
      // U_k += cb_j M_jk, V_k += conj(c_j) M_kj
      Ur += bjr * mjk.re - bji * mjk.im;
      Ui += bjr * mjk.im + bji * mjk.re;
      Vr += cjr * mkj.re + cji * mkj.im;
      Vi += cjr * mkj.im - cji * mkj.re;
    }
    XYUV[0][k] = Xr; XYUV[1][k] = Xi; XYUV[2][k] = Yr; XYUV[3][k] = Yi;
    XYUV[4][k] = Ur; XYUV[5][k] = Ui; XYUV[6][k] = Vr; XYUV[7][k] = Vi;
  }
  __syncthreads();
  const double G = tc.gamma;
  const double cy = 1.0 / (G * (1.0 - y * y)), cx = 1.0 / (G * (1.0 + x * x));
  if (t == 0) {
    // the quadratic forms, summed over k in order
    double a = 0.0, b = 0.0, zr = 0.0, zi = 0.0;
    for (int k = 0; k < K; ++k) {
      a += c[2 * k] * XYUV[0][k] - c[2 * k + 1] * XYUV[1][k];
      b += cb[2 * k] * XYUV[2][k] - cb[2 * k + 1] * XYUV[3][k];
      // z = sum_k conj(c_k) U_k
      zr += c[2 * k] * XYUV[4][k] + c[2 * k + 1] * XYUV[5][k];
      zi += c[2 * k] * XYUV[5][k] - c[2 * k + 1] * XYUV[4][k];
    }
    form[0] = a;
    form[1] = b;
    form[2] = zr;
    form[3] = zi;
    Ish = 0.5 * ((a + b) * cy + (a - b) * cx - 2.0 * zr * y * cy - 2.0 * zi * x * cx);
  }
  if (t < K) {
    const int k = t, ia = tc.pa[k], ib = tc.pb[k];
    const double Xr = XYUV[0][k], Xi = XYUV[1][k], Yr = XYUV[2][k], Yi = XYUV[3][k];
    const double Ur = XYUV[4][k], Ui = XYUV[5][k], Vr = XYUV[6][k], Vi = XYUV[7][k];
    if (ia >= 0) {
      gI[ia] = 0.5 * ((cy + cx) * 2.0 * Xr - 2.0 * y * cy * Ur - 2.0 * x * cx * Ui);
      gI[ia + 1] = 0.5 * (-2.0 * (cy + cx) * Xi - 2.0 * y * cy * Ui + 2.0 * x * cx * Ur);
    }
    if (ib >= 0) {
      gI[ib] = 0.5 * ((cy - cx) * 2.0 * Yr - 2.0 * y * cy * Vr - 2.0 * x * cx * Vi);
      gI[ib + 1] = 0.5 * (-2.0 * (cy - cx) * Yi + 2.0 * y * cy * Vi - 2.0 * x * cx * Vr);
    }
  }
  __syncthreads();
  if (t == 0) {
    const double a = form[0], b = form[1], zr = form[2], zi = form[3];
    const double dcx = -2.0 * x * G * cx * cx, dcy = 2.0 * y * G * cy * cy;
    gI[P - 2] = 0.5 * ((a - b) * dcx - 2.0 * zi * (cx + x * dcx));
    gI[P - 1] = 0.5 * ((a + b) * dcy - 2.0 * zr * (cy + y * dcy));
  }
  __syncthreads();
  const double I = Ish;
  const bool ok = valid != 0.0 && I > 0.0 && isfinite(I);
  double* o = out + (int64_t)f * out_stride;
  if (t == 0) {
    o[0] = ok ? res[0] + n_events * log(I) : INFINITY;
    o[1 + P] = I;
    if (out_user) out_user[0] = o[0];
  }
  if (t < P) {
    o[2 + P + t] = gI[t];
    if (with_grad) {
      // event slot of theta entry t: 1 + t
      const double g = ok ? res[1 + t] + n_events * gI[t] / I : NAN;
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
  h_real(tc.wa, tc.wL, G * (1.0 - tb.y), t, s, s2, g, hp, dhp);
  h_real(tc.wa, tc.wL, G * (1.0 + tb.y), t, s, s2, g, hm, dhm);
  h_cplx(tc.wa, tc.wL, {G, -G * tb.x}, t, s, s2, g, hc, dhc);
  const double a2 = A.re * A.re + A.im * A.im, b2 = Ab.re * Ab.re + Ab.im * Ab.im;
  const double zr = A.re * Ab.re + A.im * Ab.im, zi = A.re * Ab.im - A.im * Ab.re;
  const double R = 0.5 * ((a2 + b2) * 0.5 * (hp + hm) + (a2 - b2) * hc.re - 2.0 * zr * 0.5 * (hp - hm) -
                          2.0 * zi * hc.im);
  p[i] = R / *norm;
}

// ---------------------------------------------------------------- launchers
int td4_kmax(int K) { return K; }  // partial rows hold exactly the model's amplitudes
int td4_nv(const Td4Const& tc, bool grad) { return grad ? 1 + tc.n_params : 1; }

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
  if (n_fits <= 0) return;
  hipLaunchKernelGGL(td4_prologue, dim3(n_fits), dim3(kTd4PrologueThreads), 0, s, tc, pb ? *pb : zero,
                     pb ? nullptr : theta, theta_stride, fc, status, n_fits, tabs);
}

void td4_launch_check(const Td4Const& tc, const double* ev, int64_t ld, int64_t n, unsigned long long* bad,
                      hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(td4_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tc, ev, ld, n, bad);
}

// Source of the shape-specialized passes of a model: the pair entries (spin,
// flat or resonant) and every amplitude's entries and angular factor as
// compile-time constants, then the events pass without and with the gradient
// and the M rows.
std::string td4_jit_source(const Td4Const& tc) {
  std::ostringstream o;
  auto arr = [&](const char* name, const int* v, int n) {
    o << "  static constexpr int " << name << "[" << n << "] = {";
    for (int i = 0; i < n; ++i) o << (i ? ", " : "") << v[i];
    o << "};\n";
  };
  o << "#include \"td4_device.hpp\"\n";
  o << "struct fn_td4_shape {\n  static constexpr int K = " << tc.K
    << ";\n  static constexpr int N12 = " << tc.n12 << ";\n  static constexpr int N34 = " << tc.n34 << ";\n";
  arr("L12", tc.L12, tc.n12);
  arr("NR12", tc.nr12, tc.n12);
  arr("L34", tc.L34, tc.n34);
  arr("NR34", tc.nr34, tc.n34);
  arr("A1", tc.amp1, tc.K);
  arr("A2", tc.amp2, tc.K);
  arr("T", tc.atype, tc.K);
  arr("PA", tc.pa, tc.K);
  arr("PB", tc.pb, tc.K);
  o << "  static constexpr int P = " << tc.n_params << ";\n";
  o << "};\n"
       "FN_TD4_EVENTS(fn_td4_ev0, fn_td4_shape, false)\n"
       "FN_TD4_EVENTS(fn_td4_ev1, fn_td4_shape, true)\n"
       "FN_TD4_MROWS(fn_td4_mrows, fn_td4_shape)\n"
       "FN_TD4_GEN(fn_td4_envmax, fn_td4_gen, fn_td4_shape)\n";
  return o.str();
}

std::shared_ptr<Td4Jit> td4_jit(const Td4Const& tc) {
  auto j = std::make_shared<Td4Jit>();
  j->prog = jit_load(td4_jit_source(tc), {"fn_td4_ev0", "fn_td4_ev1", "fn_td4_mrows", "fn_td4_envmax", "fn_td4_gen"});
  j->ev[0] = j->prog->fns[0];
  j->ev[1] = j->prog->fns[1];
  j->mrows = j->prog->fns[2];
  j->envmax = j->prog->fns[3];
  j->gen = j->prog->fns[4];
  return j;
}

void td4_launch_mmatrix(const Td4Jit& j, const Td4Const& tc, const Td4Table* tabs, int n_fits, const double* mc,
                        int64_t ld_mc, int64_t n_mc, int chunk, double* part, double* Mc, hipStream_t s,
                        const int* sel) {
  const int kmax = td4_kmax(tc.K);
  const int64_t nch = (n_mc + chunk - 1) / chunk;
  const int rb = td4_row_block(tc.K);
  const int nv = 2 * rb * kmax;
  for (int i0 = 0; i0 < tc.K; i0 += rb) {
    Td4Const c = tc;
    const Td4Table* t = tabs;
    const int* se = sel;
    const double* m = mc;
    int64_t l = ld_mc, nn = n_mc, nc = nch;
    int ck = chunk, nf = n_fits, ii = i0;
    double* p = part;
    void* args[] = {&c, &t, &se, &m, &l, &nn, &ck, &nc, &nf, &ii, &p};
    jit_launch(j.mrows, (unsigned)td4_blocks(nch, n_fits), kBlock, s, args);
    hipLaunchKernelGGL(td4_mrows_finalize, dim3(n_fits), dim3(kFinalBlock), 0, s, tc, sel, part, nch, nv, kmax, i0,
                       rb, 1.0 / (double)n_mc, Mc);
  }
}

void td4_launch_events(const Td4Jit& j, const Td4Const& tc, const Td4Table* tabs, const int* status, int n_fits,
                       const double* ev, int64_t ld, int64_t n, int chunk, bool grad, double* part, hipStream_t s,
                       hipEvent_t start, hipEvent_t stop) {
  const int64_t nch = (n + chunk - 1) / chunk;
  if (nch == 0) return;
  Td4Const c = tc;
  const Td4Table* t = tabs;
  const int* st = status;
  const double* e = ev;
  int64_t l = ld, nn = n, nc = nch;
  int ck = chunk, nf = n_fits;
  double* p = part;
  void* args[] = {&c, &t, &st, &e, &l, &nn, &ck, &nc, &nf, &p};
  const int64_t blocks = td4_blocks(nch, n_fits);
  if (blocks > 0x7fffffff) throw Error(FN_E_INVALID, "td4: too many workgroups (chunks x fits)");
  jit_launch(j.ev[grad ? 1 : 0], (unsigned)blocks, kBlock, s, args, start, stop);
}

void td4_launch_finalize(const Td4Const& tc, const Td4Table* tabs, const int* status, int n_fits, const double* part,
                         int64_t rows_per_fit, bool grad, const double* Mc, double n_events, double* out,
                         int out_stride, double* out_user, hipStream_t s) {
  const int kmax = td4_kmax(tc.K);
  hipLaunchKernelGGL(td4_finalize, dim3(n_fits), dim3(kFinalBlock), 0, s, tc, tabs, status, part, rows_per_fit,
                     td4_nv(tc, grad), kmax, grad ? 1 : 0, Mc, n_events, out, out_stride, out_user);
}

void td4_launch_eval(const Td4Const& tc, const Td4Table* tab, const double* ev, int64_t ld, int64_t n,
                     const double* norm, double* p, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(td4_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tc, tab, ev, ld, n, norm, p);
}

// ------------------------------------------------------- phase-space sample
// 1.05 x the largest phase-space weight on a 801 x 801 grid of (m12, m34)
// over the box, points spaced like a linear grid whose last point is the
// upper edge, zero weight where m12 + m34 >= M.
double td4_ps_wmax(const Td4Const& tc) {
#pragma clang fp contract(off)
  const int n = 801;
  const double lo12 = tc.m1 + tc.m2, hi12 = tc.M - tc.m3 - tc.m4;
  const double lo34 = tc.m3 + tc.m4, hi34 = tc.M - tc.m1 - tc.m2;
  const double d12 = (hi12 - lo12) / (n - 1), d34 = (hi34 - lo34) / (n - 1);
  double w = 0.0;
  for (int i = 0; i < n; ++i) {
    const double a = i == n - 1 ? hi12 : (double)i * d12 + lo12;
    for (int j = 0; j < n; ++j) {
      const double b = j == n - 1 ? hi34 : (double)j * d34 + lo34;
      if (a + b < tc.M) w = std::max(w, td4_ps_weight(tc, a, b));
    }
  }
  return 1.05 * w;
}

__global__ void td4_phase_space_kernel(Td4Const tc, uint32_t k0, uint32_t k1, uint32_t s0, int max_attempts,
                                       int64_t n, double* __restrict__ out, int64_t ld,
                                       unsigned long long* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x[5];
  if (!td4_ps_point(tc, i, k0, k1, s0, max_attempts, x)) {
    for (int j = 0; j < 5; ++j) x[j] = __builtin_nan("");
    atomicAdd(bad, 1ull);
  }
  for (int j = 0; j < 5; ++j) out[j * ld + i] = x[j];
}

void td4_launch_phase_space(const Td4Const& tc, uint32_t k0, uint32_t k1, uint32_t s0, int max_attempts, int64_t n,
                            double* out, int64_t ld, unsigned long long* bad, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(td4_phase_space_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tc, k0, k1, s0,
                     max_attempts, n, out, ld, bad);
}

static Td4PairProposal pair_proposal(double lo, double hi, int n, const int* nr, const double* m0,
                                     const double* w0) {
#pragma clang fp contract(off)
  Td4PairProposal p;
  std::memset(&p, 0, sizeof(p));
  p.lo = lo;
  p.hi = hi;
  for (int r = 0; r < n; ++r) {
    if (nr[r]) continue;
    const int k = p.n++;
    p.m[k] = m0[r];
    p.s[k] = 0.5 * w0[r];
    const double xlo = (lo - p.m[k]) / p.s[k], xhi = (hi - p.m[k]) / p.s[k];
    p.vlo[k] = xlo / std::sqrt(1.0 + xlo * xlo);
    p.vhi[k] = xhi / std::sqrt(1.0 + xhi * xhi);
  }
  p.wu = p.n ? 0.5 : 1.0;
  return p;
}

Td4Proposal td4_proposal(const Td4Const& tc, const Td4FitConst& fc) {
  Td4Proposal pr;
  pr.p12 = pair_proposal(tc.m1 + tc.m2, tc.M - tc.m3 - tc.m4, tc.n12, tc.nr12, fc.m0_12, fc.w0_12);
  pr.p34 = pair_proposal(tc.m3 + tc.m4, tc.M - tc.m1 - tc.m2, tc.n34, tc.nr34, fc.m0_34, fc.w0_34);
  return pr;
}

void td4_launch_envmax(const Td4Jit& j, const Td4Const& tc, const Td4Table* tab, const Td4Proposal& pr,
                       const double* mc, int64_t ld, int64_t n, unsigned long long* vmax, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
  Td4Const c = tc;
  const Td4Table* t = tab;
  Td4Proposal q = pr;
  const double* p = mc;
  int64_t l = ld, nn = n;
  unsigned long long* v = vmax;
  void* args[] = {&c, &t, &q, &p, &l, &nn, &v};
  jit_launch(j.envmax, (unsigned)blocks, kBlock, s, args);
}

void td4_launch_gen(const Td4Jit& j, const Td4Const& tc, const Td4Table* tab, const Td4Proposal& pr, uint32_t k0,
                    uint32_t k1, int64_t n, double W, int max_attempts, double* ev, int64_t ld,
                    unsigned long long* bad, hipStream_t s) {
  if (n == 0) return;
  Td4Const c = tc;
  const Td4Table* t = tab;
  Td4Proposal q = pr;
  uint32_t a0 = k0, a1 = k1;
  int64_t nn = n, l = ld;
  double w = W;
  int ma = max_attempts;
  double* e = ev;
  unsigned long long* b = bad;
  void* args[] = {&c, &t, &q, &a0, &a1, &nn, &w, &ma, &e, &l, &b};
  jit_launch(j.gen, (unsigned)((n + kBlock - 1) / kBlock), kBlock, s, args);
}

}  // namespace fn
