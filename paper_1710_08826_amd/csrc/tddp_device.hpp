// Device code of the time-dependent three-body Dalitz-plot model with mixing
// (the paper's pi+ pi- pi0 time-dependent amplitude fit, Sec. 1 Table 2 and
// Fig. 2), compiled at run time for each model structure like the
// time-integrated three-body passes.
//
// Daughters 2 and 3 are charge conjugates (m2 = m3), so the Dbar0 amplitude
// at (s12, s13) is the D0 one at (s13, s12):
//   A = sum_k c_k A_k(s12, s13),  Abar = sum_k cbar_k A_k(s13, s12),
// with A_k the isobar amplitudes of dalitz_device.hpp (fixed lineshapes), and
// the rate is the mixing and resolution form of td4_device.hpp:
//   R = 1/2 [(|A|^2+|Abar|^2) Hc + (|A|^2-|Abar|^2) Hcos - 2 Re(A* Abar) Hs - 2 Im(A* Abar) Hsin].
// The normalization is the grid integral of the t-integrated rate, a
// quadratic form in (c, cbar) through three K x K matrices of grid sums,
//   MAA_ij = dA sum A_i conj(A_j),  MBB_ij = dA sum B_i conj(B_j),
//   MAB_ij = dA sum conj(A_i) B_j,  B_k(s12, s13) = A_k(s13, s12),
// built once per model (the lineshapes are fixed).
#pragma once
#include "dalitz_device.hpp"
#include "td4_device.hpp"

namespace fn {

// Decay-time constants of a model: 1/tau, the resolution width and the
// Faddeeva approximation of the resolution functions.
struct TddpTime {
  double gamma;
  double sigma;
  double wL;
  double wa[kWeidN];
};

// Both amplitude sets at one point: A_k(s12, s13) and B_k = A_k(s13, s12).
// With m2 = m3 (the model requires it) the pair terms at the mirrored point
// are those at (s12, s13) with pairs "12" and "13" exchanged, and for pair
// "23" only the spin-1 angular factor changes, by its sign (Z_1 = s_ac - s_bc
// with s_ac and s_bc exchanged; its mass term vanishes for equal masses), so
// each pair's terms are formed once per point.
template <class S>
__device__ __forceinline__ void tddp_basis2(const DalitzConst& dc, const double* __restrict__ r, double s12,
                                            double s13, double (&are)[S::K], double (&aim)[S::K],
                                            double (&bre)[S::K], double (&bim)[S::K]) {
  constexpr int K = S::K;
  constexpr bool u1_01 = shape_uses<S>(0, 1) || shape_uses<S>(1, 1);
  constexpr bool u2_01 = shape_uses<S>(0, 2) || shape_uses<S>(1, 2);
  constexpr bool any01 = u1_01 || u2_01 || shape_uses<S>(0, 0) || shape_uses<S>(1, 0);
  constexpr bool any2 = shape_uses<S>(2, 0) || shape_uses<S>(2, 1) || shape_uses<S>(2, 2);
  const double s23 = dc.msum - s12 - s13;
  PairTerms p0, p1, p2;
  if (any01) {
    pair_terms_t<u1_01, u2_01>(dc.ch[0], s12, s13, s23, dc.r2, dc.rD2, p0);
    pair_terms_t<u1_01, u2_01>(dc.ch[1], s13, s12, s23, dc.r2, dc.rD2, p1);
  }
  if (any2) pair_terms_t<shape_uses<S>(2, 1), shape_uses<S>(2, 2)>(dc.ch[2], s23, s12, s13, dc.r2, dc.rD2, p2);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int C = S::chan[k], L = S::L[k];
    const PairTerms& pa = C == 0 ? p0 : (C == 1 ? p1 : p2);
    const PairTerms& pb = C == 0 ? p1 : (C == 1 ? p0 : p2);
    const double hb = (C == 2 && L == 1) ? -pb.H[L] : pb.H[L];
    const double* rk = r + k * kDalFields;
    double a, b, d;
    dalitz_bw(rk, pa.s, pa.G[L], pa.H[L], are[k], aim[k], a, b, d);
    dalitz_bw(rk, pb.s, pb.G[L], hb, bre[k], bim[k], a, b, d);
  }
}

// Events pass: one workgroup per chunk of events (s12, s13, t rows at
// ev, ev + ld, ev + 2 ld), one row of partial sums each:
// [-sum ln R, d/dRe c_k, d/dIm c_k (k), d/dRe cbar_k, d/dIm cbar_k (k), d/dx, d/dy].
// coef: theta on the device, (c, cbar, x, y).
template <class S, bool GRAD>
__device__ inline void tddp_events_body(const DalitzConst& dc, const DalitzTable* __restrict__ tab,
                                        const TddpTime& tt, const double* __restrict__ coef0,
                                        const double* __restrict__ ev, int64_t ld, int64_t n, int chunk,
                                        double* __restrict__ part) {
  constexpr int K = S::K;
  constexpr int NV = GRAD ? 3 + 4 * K : 1;
  __shared__ double lds[block_sum_lds(NV)];
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const double s = tt.sigma, s2 = s * s, inv2s2 = 0.5 / s2;
  const double G = tt.gamma;
  const double x = coef0[4 * K], y = coef0[4 * K + 1];
  const double ap = G * (1.0 - y), am = G * (1.0 + y);
  const cplx ac = {G, -G * x};
  const int64_t base = (int64_t)blockIdx.x * chunk;
  const int64_t end = base + chunk < n ? base + chunk : n;
  const double* const r0 = &tab->r[0][0];
  LogProd lp;  // -sum ln R enters acc[0] once per thread, at the end
  for (int64_t i = base + threadIdx.x; i < end; i += kBlock) {
    // constants re-read through the scalar cache per event (an opaque zero
    // offset keeps them out of SGPRs that would overflow into VGPR lanes)
    int zero = 0;
    asm volatile("" : "+s"(zero));
    const double* r = r0 + zero;
    const double* coef = coef0 + zero;
    const double* wa = tt.wa + zero;
    const double t = ev[2 * ld + i];
    const double g = exp(-t * t * inv2s2);
    double hp, dhp, hm, dhm;
    cplx hc, dhc;
    h_real(wa, tt.wL, ap, t, s, s2, g, hp, dhp);
    h_real(wa, tt.wL, am, t, s, s2, g, hm, dhm);
    h_cplx(wa, tt.wL, ac, t, s, s2, g, hc, dhc);
    const double s12 = ev[i], s13 = ev[ld + i];
    double Are[K], Aim[K], Bre[K], Bim[K];
    tddp_basis2<S>(dc, r, s12, s13, Are, Aim, Bre, Bim);
    cplx A = {0.0, 0.0}, Ab = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double cr = coef[2 * k], ci = coef[2 * k + 1];
      const double br = coef[2 * K + 2 * k], bi = coef[2 * K + 2 * k + 1];
      A = cfma({cr, ci}, {Are[k], Aim[k]}, A);
      Ab = cfma({br, bi}, {Bre[k], Bim[k]}, Ab);
    }
    const double Hc = 0.5 * (hp + hm), Hs = 0.5 * (hp - hm);
    const double a2 = A.re * A.re + A.im * A.im, b2 = Ab.re * Ab.re + Ab.im * Ab.im;
    const double zr = A.re * Ab.re + A.im * Ab.im, zi = A.re * Ab.im - A.im * Ab.re;  // conj(A) Abar
    const double R = 0.5 * ((a2 + b2) * Hc + (a2 - b2) * hc.re - 2.0 * zr * Hs - 2.0 * zi * hc.im);
    lp.mul(R);
    if (GRAD) {
      const double w = -rcp_fast(R);
      const double hpc = Hc + hc.re, hmc = Hc - hc.re;
      // dR/dRe c_k - i dR/dIm c_k = lc A_k, and with lb and B_k for cbar:
      // lc = hpc conj(A) - (Hs + i Hsin) conj(Abar), lb = hmc conj(Abar) - (Hs - i Hsin) conj(A)
      // (the event's factor w = -1/R included)
      const cplx lc = {w * (hpc * A.re - Hs * Ab.re - hc.im * Ab.im), w * (-hpc * A.im + Hs * Ab.im - hc.im * Ab.re)};
      const cplx lb = {w * (hmc * Ab.re - Hs * A.re + hc.im * A.im), w * (-hmc * Ab.im + Hs * A.im + hc.im * A.re)};
#pragma unroll
      for (int k = 0; k < K; ++k) {
        grad_acc(lc, {Are[k], Aim[k]}, acc[1 + 2 * k], acc[2 + 2 * k]);
        grad_acc(lb, {Bre[k], Bim[k]}, acc[1 + 2 * K + 2 * k], acc[2 + 2 * K + 2 * k]);
      }
      // x: d hc/dx = -i G dh(ac);  y: d hp/dy = -G dh(ap), d hm/dy = +G dh(am)
      const double dcos = G * dhc.im, dsin = -G * dhc.re;
      acc[1 + 4 * K] += w * 0.5 * ((a2 - b2) * dcos - 2.0 * zi * dsin);
      const double dHc = 0.5 * G * (dhm - dhp), dHs = -0.5 * G * (dhp + dhm);
      acc[2 + 4 * K] += w * 0.5 * ((a2 + b2) * dHc - 2.0 * zr * dHs);
    }
  }
  acc[0] = -lp.log();
  block_sum_row<NV>(acc, lds, part + (int64_t)blockIdx.x * NV);
}

// Rows i0..i0+3 of one normalization matrix over one chunk of grid cells:
// WHICH 0: A_i conj(A_j), 1: B_i conj(B_j), 2: conj(A_i) B_j (re, im pairs).
template <class S, int WHICH>
__device__ inline void tddp_mrows_body(const DalitzConst& dc, const DalitzTable* __restrict__ tab, int chunk,
                                       int i0, double* __restrict__ part) {
  constexpr int K = S::K;
  constexpr int NV = 2 * kMRowBlock * K;
  __shared__ double lds[block_sum_lds(NV)];
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const int64_t ncell = (int64_t)dc.nx * dc.ny;
  const int64_t base = (int64_t)blockIdx.x * chunk;
  const int64_t end = base + chunk < ncell ? base + chunk : ncell;
  const double* const r0 = &tab->r[0][0];
  for (int64_t c = base + threadIdx.x; c < end; c += kBlock) {
    int zero = 0;
    asm volatile("" : "+s"(zero));
    const double* r = r0 + zero;
    const int64_t ix = c / dc.ny, iy = c - ix * dc.ny;
    const double s12 = grid_centre(dc.a12, ix, dc.d12);
    const double s13 = grid_centre(dc.a13, iy, dc.d13);
    if (!dalitz_inside(dc, s12, s13)) continue;
    double Are[K], Aim[K], Bre[K], Bim[K], Lre[K], Lim[K], Rre[K], Rim[K];
    tddp_basis2<S>(dc, r, s12, s13, Are, Aim, Bre, Bim);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      Lre[k] = WHICH == 1 ? Bre[k] : Are[k];
      Lim[k] = WHICH == 1 ? Bim[k] : Aim[k];
      Rre[k] = WHICH == 0 ? Are[k] : Bre[k];
      Rim[k] = WHICH == 0 ? Aim[k] : Bim[k];
    }
#pragma unroll
    for (int ib = 0; ib < kMRowBlock; ++ib) {
      double xr = 0.0, xi = 0.0;  // left factor i = i0 + ib, selected with uniform guards
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (k == i0 + ib) {
          xr = Lre[k];
          xi = WHICH == 2 ? -Lim[k] : Lim[k];
        }
#pragma unroll
      for (int j = 0; j < K; ++j) {
        // (xr + i xi) times conj(R_j) for WHICH 0/1, times R_j for WHICH 2
        const double rr = Rre[j], ri = WHICH == 2 ? Rim[j] : -Rim[j];
        acc[2 * (ib * K + j)] = __builtin_fma(xr, rr, __builtin_fma(-xi, ri, acc[2 * (ib * K + j)]));
        acc[2 * (ib * K + j) + 1] = __builtin_fma(xr, ri, __builtin_fma(xi, rr, acc[2 * (ib * K + j) + 1]));
      }
    }
  }
  block_sum_row<NV>(acc, lds, part + (int64_t)blockIdx.x * NV);
}

// ---------------------------------------------------------------- toy events
// A and Abar at one point.
template <class S>
__device__ __forceinline__ void tddp_amps(const DalitzConst& dc, const double* __restrict__ r,
                                          const double* __restrict__ coef, double s12, double s13, cplx& A,
                                          cplx& Ab) {
  constexpr int K = S::K;
  double Are[K], Aim[K], Bre[K], Bim[K];
  tddp_basis2<S>(dc, r, s12, s13, Are, Aim, Bre, Bim);
  A = {0.0, 0.0};
  Ab = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double cr = coef[2 * k], ci = coef[2 * k + 1];
    const double br = coef[2 * K + 2 * k], bi = coef[2 * K + 2 * k + 1];
    A = {A.re + cr * Are[k] - ci * Aim[k], A.im + cr * Aim[k] + ci * Are[k]};
    Ab = {Ab.re + br * Bre[k] - bi * Bim[k], Ab.im + br * Bim[k] + bi * Bre[k]};
  }
}

// Largest (|A| + |Abar|)^2 over the grid-cell centres inside the region (bits
// of a non-negative double, ordered like the value) in *vmax.
template <class S>
__device__ inline void tddp_gridmax_body(const DalitzConst& dc, const DalitzTable* __restrict__ tab,
                                         const double* __restrict__ coef, unsigned long long* __restrict__ vmax) {
  __shared__ double lds[kBlock];
  const int64_t ncell = (int64_t)dc.nx * dc.ny;
  const double* r = &tab->r[0][0];
  double m = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * kBlock) {
    const int64_t ix = c / dc.ny, iy = c - ix * dc.ny;
    const double s12 = grid_centre(dc.a12, ix, dc.d12);
    const double s13 = grid_centre(dc.a13, iy, dc.d13);
    if (!dalitz_inside(dc, s12, s13)) continue;
    cplx A, Ab;
    tddp_amps<S>(dc, r, coef, s12, s13, A, Ab);
    const double e = sqrt(A.re * A.re + A.im * A.im) + sqrt(Ab.re * Ab.re + Ab.im * Ab.im);
    m = fmax(m, e * e);
  }
  lds[threadIdx.x] = m;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(vmax, (unsigned long long)__double_as_longlong(lds[0]));
}

// Accept-reject toy events: R(s12, s13, t) <= e^{-lam t} (|A| + |Abar|)^2 with
// lam = G (1 - |y|), so event i, attempt a takes (u1, u2) from counter
// (i, 2a, 2) and (u3, u4) from (i, 2a + 1, 2) under key (k0, k1): the
// candidate (lo12 + u1 (hi12 - lo12), lo13 + u2 (hi13 - lo13), t = -ln(1 - u3)/lam)
// is kept when it lies in the region and u4 W e^{-lam t} < R; the measured
// time adds sigma_t times a Box-Muller normal from counter (i, 0, 3).  bad[0]
// counts kept events with (|A| + |Abar|)^2 > W, bad[1] events left NaN after
// max_attempts.
template <class S>
__device__ inline void tddp_gen_body(const DalitzConst& dc, const DalitzTable* __restrict__ tab,
                                     const double* __restrict__ coef, const TddpTime& tt, uint32_t k0, uint32_t k1,
                                     int64_t n, double W, double lo12, double hi12, double lo13, double hi13,
                                     int max_attempts, double* __restrict__ ev, int64_t ld,
                                     unsigned long long* __restrict__ bad) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double* r = &tab->r[0][0];
  constexpr int K = S::K;
  const double x = coef[4 * K], y = coef[4 * K + 1];
  const double G = tt.gamma;
  const double lam = G * (1.0 - fabs(y));
  const double w12 = hi12 - lo12, w13 = hi13 - lo13;
  double o12 = __builtin_nan(""), o13 = __builtin_nan(""), ot = __builtin_nan(""), env = 0.0;
  for (int a = 0; a < max_attempts; ++a) {
    double u1, u2, u3, u4;
    philox_uniforms((uint64_t)i, 2u * a, 2u, k0, k1, u1, u2);
    philox_uniforms((uint64_t)i, 2u * a + 1u, 2u, k0, k1, u3, u4);
    const double s12 = lo12 + u1 * w12;
    const double s13 = lo13 + u2 * w13;
    if (!dalitz_inside(dc, s12, s13)) continue;
    const double t = -log1p(-u3) / lam;
    cplx A, Ab;
    tddp_amps<S>(dc, r, coef, s12, s13, A, Ab);
    const double a2 = A.re * A.re + A.im * A.im, b2 = Ab.re * Ab.re + Ab.im * Ab.im;
    const double zr = A.re * Ab.re + A.im * Ab.im, zi = A.re * Ab.im - A.im * Ab.re;
    const double gt = G * t;
    const double ep = exp(y * gt), em = exp(-y * gt);
    double sx, cx;
    sincos(x * gt, &sx, &cx);
    const double R = 0.5 * exp(-gt) *
                     ((a2 + b2) * (0.5 * (ep + em)) + (a2 - b2) * cx - 2.0 * zr * (0.5 * (ep - em)) - 2.0 * zi * sx);
    if (u4 * W * exp(-lam * t) < R) {
      o12 = s12;
      o13 = s13;
      ot = t;
      const double e = sqrt(a2) + sqrt(b2);
      env = e * e;
      break;
    }
  }
  double v1, v2;
  philox_uniforms((uint64_t)i, 0u, 3u, k0, k1, v1, v2);
  ot = ot + tt.sigma * (sqrt(-2.0 * log1p(-v1)) * cos(2.0 * 3.14159265358979323846 * v2));
  ev[i] = o12;
  ev[ld + i] = o13;
  ev[2 * ld + i] = ot;
  if (env > W) atomicAdd(bad, 1ull);
  if (o12 != o12) atomicAdd(bad + 1, 1ull);
}

}  // namespace fn

// Kernels for shape S (used by the generated source).
#define FN_TDDP_EVENTS(NAME, S, GRAD)                                                                          \
  extern "C" __global__ __launch_bounds__(fn::kBlock) void NAME(                                               \
      fn::DalitzConst dc, const fn::DalitzTable* __restrict__ tab, fn::TddpTime tt,                            \
      const double* __restrict__ coef, const double* __restrict__ ev, int64_t ld, int64_t n, int chunk,       \
      double* __restrict__ part) {                                                                             \
    fn::tddp_events_body<S, GRAD>(dc, tab, tt, coef, ev, ld, n, chunk, part);                                 \
  }
#define FN_TDDP_MROWS(NAME, S, WHICH)                                                                          \
  extern "C" __global__ __launch_bounds__(fn::kBlock) void NAME(                                               \
      fn::DalitzConst dc, const fn::DalitzTable* __restrict__ tab, int chunk, int i0,                          \
      double* __restrict__ part) {                                                                             \
    fn::tddp_mrows_body<S, WHICH>(dc, tab, chunk, i0, part);                                                   \
  }
#define FN_TDDP_GEN(GRIDMAX, GEN, S)                                                                           \
  extern "C" __global__ __launch_bounds__(fn::kBlock) void GRIDMAX(                                            \
      fn::DalitzConst dc, const fn::DalitzTable* __restrict__ tab, const double* __restrict__ coef,            \
      unsigned long long* __restrict__ vmax) {                                                                 \
    fn::tddp_gridmax_body<S>(dc, tab, coef, vmax);                                                             \
  }                                                                                                            \
  extern "C" __global__ __launch_bounds__(fn::kBlock) void GEN(                                                \
      fn::DalitzConst dc, const fn::DalitzTable* __restrict__ tab, const double* __restrict__ coef,            \
      fn::TddpTime tt, uint32_t k0, uint32_t k1, int64_t n, double W, double lo12, double hi12, double lo13,   \
      double hi13, int max_attempts, double* __restrict__ ev, int64_t ld, unsigned long long* __restrict__ bad) { \
    fn::tddp_gen_body<S>(dc, tab, coef, tt, k0, k1, n, W, lo12, hi12, lo13, hi13, max_attempts, ev, ld, bad);  \
  }
