// Device code of the three-body Dalitz-plot model, compiled at run time for
// each model structure (the resonances' pairs and spins become compile-time
// constants; see jit.hpp) and, for the structure-generic helpers, into the
// library.
//
//   P~(s12, s13) = |sum_k c_k A_k|^2,
//   A_k = [F_L(q r)/F_L(q0 r)] F_L(p r_D) Z_L(s) T_k(s_AB)
//   T_k = 1 / (m0^2 - s_AB - i m0 Gamma_k(s_AB))
//   Gamma_k(s) = Gamma0 (q/q0)^(2L+1) (m0/sqrt s) [F_L(q r)/F_L(q0 r)]^2
//
// with Blatt-Weisskopf factors F_0 = 1, F_1 = (1+z)^-1/2,
// F_2 = (z^2+3z+9)^-1/2 (z = (q r)^2) and Zemach spin factors Z_0 = 1,
// Z_1 = s_AC - s_BC + (M^2 - mC^2)(mB^2 - mA^2)/s_AB, Z_2 = Z_1^2 - X Y / 3,
// X = lambda(s_AB, M^2, mC^2)/s_AB, Y = lambda(s_AB, mA^2, mB^2)/s_AB.
//
// Per event, all in registers:
//  * every quantity that depends only on the pair (s_AB, q, p, the barrier
//    polynomials, Zemach factors) is computed once per pair and shared by all
//    resonances of that pair;
//  * per resonance the lineshape reduces to T = (a + i b)/(a^2 + b^2) with
//    a = m0^2 - s and b = m0 Gamma(s) = Kw * G_{pair,L}(s), where
//    G = q^(2L+1) F_L(q r)^2 / sqrt(s) is per pair and
//    Kw = Gamma0 m0^2 / (q0^(2L+1) F_L(q0 r)^2) comes from the prologue;
//  * the amplitude is A = Ka * H_{pair,L} * T with H = F_L(q r) F_L(p r_D) Z_L
//    per pair and Ka = 1/F_L(q0 r) per resonance.
//
// Modes of the chunk routine:
//   kEvents  -ln P~ over an event chunk (+ adjoint gradient)          -> NLL
//   kGrid    P~ over a chunk of grid cells inside the region (+ dP~)  -> I
//   kMRows   rows i0..i0+3 of sum_cells A_i conj(A_j)                 -> cached M
#pragma once
#include "device_common.hpp"
#include "fastmath.hpp"
#include "model.hpp"
#include "philox.hpp"

namespace fn {

enum DalMode : int { kEvents = 0, kGrid = 1, kMRows = 2 };
constexpr int kMRowBlock = 4;

__host__ __device__ constexpr int dal_nv(int mode, int grad, int k) {
  return mode == kMRows ? 2 * kMRowBlock * k : 1 + (grad == 0 ? 0 : (grad == 1 ? 2 * k : 4 * k));
}

struct PairTerms {
  double s;         // s_AB
  double G[3];      // q^(2L+1) F_L(q r)^2 / sqrt(s)
  double H[3];      // F_L(q r) F_L(p r_D) Z_L
};

// G and H of one pair from (s_AB, s_AC, s_BC), for the spins U1 (L = 1) and
// U2 (L = 2) the pair needs (L = 0 is always formed):
//   q/sqrt(s) = sqrt(lambda_q) / (2 s),  q^2 = lambda_q / (4 s),  p^2 = lambda_p / (4 s)
//   G_1 = (q/sqrt s) q^2 / (1 + z_q),          H_1 = Z_1 / sqrt((1 + z_q)(1 + z_p))
//   G_2 = (q/sqrt s) q^4 / (z_q^2 + 3 z_q + 9), H_2 = Z_2 / sqrt(poly(z_q) poly(z_p))
template <bool U1, bool U2>
__device__ __forceinline__ void pair_terms_is(const DalitzChan& ch, double s_ab, double is, double s_ac, double s_bc,
                                              double r2, double rD2, PairTerms& o) {
  const double lq = fmax((s_ab - ch.sum2) * (s_ab - ch.dif2), 0.0);
  const double q2 = 0.25 * lq * is;
  const double qirs = 0.5 * sqrt_fast(lq) * is;
  o.s = s_ab;
  o.G[0] = qirs;
  o.H[0] = 1.0;
  o.G[1] = o.G[2] = o.H[1] = o.H[2] = 0.0;
  if (U1 || U2) {
    const double lp = fmax((s_ab - ch.Psum2) * (s_ab - ch.Pdif2), 0.0);
    const double p2 = 0.25 * lp * is;
    const double zq = q2 * r2, zp = p2 * rD2;
    const double z1 = __builtin_fma(ch.zc, is, s_ac - s_bc);
    // 1/u_q = (1/sqrt(u_q u_p))^2 u_p: one reciprocal square root serves both
    if (U1) {
      const double uq = 1.0 + zq, up = 1.0 + zp;
      const double r = rsqrt_fast(uq * up);
      o.G[1] = qirs * q2 * (r * r * up);
      o.H[1] = z1 * r;
    }
    if (U2) {
      const double vq = __builtin_fma(zq, zq + 3.0, 9.0), vp = __builtin_fma(zp, zp + 3.0, 9.0);
      const double r = rsqrt_fast(vq * vp);
      o.G[2] = qirs * q2 * q2 * (r * r * vp);
      const double z2 = z1 * z1 - (lp * is) * (lq * is) * (1.0 / 3.0);
      o.H[2] = z2 * r;
    }
  }
}

// The same, forming 1/s_AB itself.
template <bool U1, bool U2>
__device__ __forceinline__ void pair_terms_t(const DalitzChan& ch, double s_ab, double s_ac, double s_bc, double r2,
                                             double rD2, PairTerms& o) {
  pair_terms_is<U1, U2>(ch, s_ab, rcp_fast(s_ab), s_ac, s_bc, r2, rD2, o);
}

// The same with the spins used by the pair given at run time.
__device__ __forceinline__ void pair_terms(const DalitzChan& ch, double s_ab, double s_ac, double s_bc, double r2,
                                           double rD2, PairTerms& o) {
  if (ch.useL[2]) {
    if (ch.useL[1]) pair_terms_t<true, true>(ch, s_ab, s_ac, s_bc, r2, rD2, o);
    else pair_terms_t<false, true>(ch, s_ab, s_ac, s_bc, r2, rD2, o);
  } else {
    if (ch.useL[1]) pair_terms_t<true, false>(ch, s_ab, s_ac, s_bc, r2, rD2, o);
    else pair_terms_t<false, false>(ch, s_ab, s_ac, s_bc, r2, rD2, o);
  }
}

// Centre of cell i along a grid axis that starts at a with cells of size d,
// as the plain IEEE evaluation (no contraction), so that every pass and the
// cell list see the same bits.
__device__ inline double grid_centre(double a, int64_t i, double d) {
#pragma clang fp contract(off)
  return a + (i + 0.5) * d;
}

// Physical-region bounds of the grid row at s12: s23 between lo and hi, from
// the energies of daughters 2 and 3 in the (12) rest frame.  Contraction is
// off so that the decision is the plain IEEE evaluation.
__device__ inline void dalitz_row_bounds(const DalitzConst& dc, double s12, double& lo, double& hi) {
#pragma clang fp contract(off)
  const double rs = sqrt(s12);
  const double e2 = (s12 - dc.m1s + dc.m2s) / (2.0 * rs);
  const double e3 = (dc.M2 - s12 - dc.m3s) / (2.0 * rs);
  const double p2 = sqrt(fmax(e2 * e2 - dc.m2s, 0.0));
  const double p3 = sqrt(fmax(e3 * e3 - dc.m3s, 0.0));
  const double es = e2 + e3;
  lo = es * es - (p2 + p3) * (p2 + p3);
  hi = es * es - (p2 - p3) * (p2 - p3);
}

// Physical-region predicate at a grid-cell centre, given its row's bounds.
__device__ inline bool dalitz_in_row(const DalitzConst& dc, double s12, double s13, double lo, double hi) {
#pragma clang fp contract(off)
  const double s23 = dc.msum - s12 - s13;
  return s23 >= lo && s23 <= hi;
}

__device__ inline bool dalitz_inside(const DalitzConst& dc, double s12, double s13) {
  double lo, hi;
  dalitz_row_bounds(dc, s12, lo, hi);
  return dalitz_in_row(dc, s12, s13, lo, hi);
}

// Compile-time structure queries on a shape S (S::K, S::chan[], S::L[]).
template <class S>
__host__ __device__ constexpr bool shape_uses(int c, int l) {
  bool u = false;
  for (int k = 0; k < S::K; ++k) u = u || (S::chan[k] == c && S::L[k] == l);
  return u;
}

// One resonance's amplitude from its pair's terms: A_k = Ka H T with
// T = 1 / (a - i b) = (a + i b) d, a = m0^2 - s, b = Kw G, d = 1 / (a^2 + b^2)
// (rk: the resonance's row of the table), in two steps so that the
// reciprocals of several resonances can be formed together (rcp_group).
__device__ __forceinline__ void bw_denominator(const double* __restrict__ rk, double s, double G, double& a,
                                               double& b, double& D) {
  a = rk[dM0SQ] - s;
  b = rk[dKW] * G;
  D = __builtin_fma(a, a, b * b);
}

__device__ __forceinline__ void bw_amplitude(const double* __restrict__ rk, double H, double a, double b, double d,
                                             double& ar, double& ai) {
  const double u = (rk[dKA] * H) * d;
  ar = u * a;
  ai = u * b;
}

__device__ __forceinline__ void dalitz_bw(const double* __restrict__ rk, double s, double G, double H, double& ar,
                                          double& ai, double& a, double& b, double& d) {
  double D;
  bw_denominator(rk, s, G, a, b, D);
  d = rcp_fast(D);
  bw_amplitude(rk, H, a, b, d, ar, ai);
}

template <class S, int C>
__host__ __device__ constexpr bool pair_used() {
  return shape_uses<S>(C, 0) || shape_uses<S>(C, 1) || shape_uses<S>(C, 2);
}

// Pair terms of pair C (compile-time) at a point, when the shape uses it
// (is: 1/s_AB).
template <class S, int C>
__device__ __forceinline__ void dalitz_pair_terms(const DalitzConst& dc, double s12, double s13, double s23,
                                                  double is, PairTerms& pt) {
  if (!pair_used<S, C>()) return;
  // pair "12": (A,B,C) = (1,2,3); "13": (1,3,2); "23": (2,3,1)
  const double s_ab = C == 0 ? s12 : (C == 1 ? s13 : s23);
  const double s_ac = C == 0 ? s13 : s12;
  const double s_bc = C == 2 ? s13 : s23;
  pair_terms_is<shape_uses<S>(C, 1), shape_uses<S>(C, 2)>(dc.ch[C], s_ab, is, s_ac, s_bc, dc.r2, dc.rD2, pt);
}

// Amplitudes of all resonances (in model order, four at a time for the
// reciprocals), added to the coherent sum S = sum_k c_k A_k.
template <class S, int MODE, bool KEEP_A, bool KEEP_T>
__device__ __forceinline__ void dalitz_amps(const DalitzConst& dc, const double* __restrict__ r,
                                            const double* __restrict__ coef, double s12, double s13, double s23,
                                            double (&Are)[S::K], double (&Aim)[S::K], double (&Tre)[S::K],
                                            double (&Tim)[S::K], double (&Gk)[S::K], double& Sre, double& Sim) {
  constexpr int K = S::K;
  // 1/s of the pairs in use from one reciprocal (an unused pair's 1 drops out)
  double is[4] = {pair_used<S, 0>() ? s12 : 1.0, pair_used<S, 1>() ? s13 : 1.0, pair_used<S, 2>() ? s23 : 1.0, 1.0};
  rcp_group(is, 3);
  PairTerms pt0, pt1, pt2;
  dalitz_pair_terms<S, 0>(dc, s12, s13, s23, is[0], pt0);
  dalitz_pair_terms<S, 1>(dc, s12, s13, s23, is[1], pt1);
  dalitz_pair_terms<S, 2>(dc, s12, s13, s23, is[2], pt2);
#pragma unroll
  for (int g = 0; g < K; g += 4) {
    const int n = K - g < 4 ? K - g : 4;
    double a[4], b[4], D[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j < n) {
        const int k = g + j;
        const PairTerms& pt = S::chan[k] == 0 ? pt0 : (S::chan[k] == 1 ? pt1 : pt2);
        bw_denominator(r + k * kDalFields, pt.s, pt.G[S::L[k]], a[j], b[j], D[j]);
      }
    }
    rcp_group(D, n);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j < n) {
        const int k = g + j;
        const int L = S::L[k];
        const PairTerms& pt = S::chan[k] == 0 ? pt0 : (S::chan[k] == 1 ? pt1 : pt2);
        const double* rk = r + k * kDalFields;
        double ar, ai;
        bw_amplitude(rk, pt.H[L], a[j], b[j], D[j], ar, ai);
        if (KEEP_A) { Are[k] = ar; Aim[k] = ai; }
        if (KEEP_T) { Tre[k] = a[j] * D[j]; Tim[k] = b[j] * D[j]; Gk[k] = pt.G[L]; }
        if (MODE != kMRows) {
          // S += c_k A_k as four chained FMAs
          const double cr = coef[2 * k], ci = coef[2 * k + 1];
          Sre = __builtin_fma(cr, ar, __builtin_fma(-ci, ai, Sre));
          Sim = __builtin_fma(cr, ai, __builtin_fma(ci, ar, Sim));
        }
      }
    }
  }
}

// One event or grid cell: its terms added to acc when `valid` (otherwise it
// contributes exact zeros, so the sum is unchanged).
template <class S, int MODE, int GRAD>
__device__ __forceinline__ void dalitz_point(const DalitzConst& dc, const double* __restrict__ r,
                                             const double* __restrict__ coef, double s12, double s13, bool valid,
                                             int i0, double (&acc)[dal_nv(MODE, GRAD, S::K)], LogProd& lp) {
  constexpr int K = S::K;
  constexpr bool KEEP_A = (GRAD >= 1) || MODE == kMRows;
  constexpr bool KEEP_T = GRAD == 2;
  const double s23 = dc.msum - s12 - s13;
  double Are[K], Aim[K], Tre[K], Tim[K], Gk[K];
  double Sre = 0.0, Sim = 0.0;
  dalitz_amps<S, MODE, KEEP_A, KEEP_T>(dc, r, coef, s12, s13, s23, Are, Aim, Tre, Tim, Gk, Sre, Sim);
  auto add = [&](int idx, double v) { acc[idx] += valid ? v : 0.0; };
  // acc[idx] += x1 y1 + x2 y2 as two chained FMAs
  auto add2 = [&](int idx, double x1, double y1, double x2, double y2) {
    const double t = __builtin_fma(x2, y2, __builtin_fma(x1, y1, acc[idx]));
    acc[idx] = valid ? t : acc[idx];
  };
  if (MODE == kMRows) {
#pragma unroll
    for (int ib = 0; ib < kMRowBlock; ++ib) {
      // A_i for i = i0 + ib, selected from registers with uniform guards
      double xr = 0.0, xi = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (k == i0 + ib) { xr = Are[k]; xi = Aim[k]; }
#pragma unroll
      for (int j = 0; j < K; ++j) {
        add2(2 * (ib * K + j), xr, Are[j], xi, Aim[j]);
        add2(2 * (ib * K + j) + 1, xi, Are[j], -xr, Aim[j]);
      }
    }
    return;
  }
  const double Pt = __builtin_fma(Sre, Sre, Sim * Sim);
  double w;  // multiplies dP~/dtheta
  if (MODE == kEvents) {
    lp.mul(valid ? Pt : 1.0);  // -ln P~ enters acc[0] once per thread, at the end
    if (GRAD >= 1) w = -rcp_fast(Pt);
  } else {
    add(0, Pt);
    w = 1.0;
  }
  if (GRAD >= 1) {
    const double w2 = 2.0 * w;
    const double ur = w2 * Sre, ui = w2 * Sim;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      // dP~/dRe c = 2 Re(conj(S) A), dP~/dIm c = 2 (Sim Are - Sre Aim)
      add2(1 + 2 * k, ur, Are[k], ui, Aim[k]);
      add2(2 + 2 * k, ui, Are[k], -ur, Aim[k]);
    }
  }
  if (GRAD == 2) {
    // (ur, ui) = 2 w S from the coefficient terms above
    const double ur = 2.0 * w * Sre, ui = 2.0 * w * Sim;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double* rk = r + k * kDalFields;
      const double cr = coef[2 * k], ci = coef[2 * k + 1];
      // E = 2 w conj(S) c A
      const double car = cr * Are[k] - ci * Aim[k], cai = cr * Aim[k] + ci * Are[k];
      const double er = __builtin_fma(ur, car, ui * cai), ei = __builtin_fma(ur, cai, -(ui * car));
      // dA/dm0 = A (dlnKa - X), X = T (2 m0 - i G dKw/dm0);  dP~ = 2 Re(E (dlnKa - X))
      const double gd = Gk[k] * rk[dDKW_DM0], tm = rk[dTWOM0];
      const double xr = __builtin_fma(tm, Tre[k], Tim[k] * gd);
      const double xi = __builtin_fma(tm, Tim[k], -(Tre[k] * gd));
      add2(1 + 2 * K + 2 * k, er, rk[dDLNKA] - xr, ei, xi);
      // dA/dGamma0 = i A T gw with gw = G Kw/Gamma0, so dP~ (times 2w) = Re(E i T) gw
      // = -gw (er Tim + ei Tre)
      const double gw = Gk[k] * rk[dKW_W0];
      const double q = __builtin_fma(er, Tim[k], ei * Tre[k]);
      const double t = __builtin_fma(-gw, q, acc[2 + 2 * K + 2 * k]);
      acc[2 + 2 * K + 2 * k] = valid ? t : acc[2 + 2 * K + 2 * k];
    }
  }
}

// One fixed chunk of events or grid cells -> one row of partial sums.
// GRAD: 0 none, 1 coefficients only, 2 coefficients + masses and widths.
// EPT events per thread and loop iteration (independent work for the
// scheduler to interleave); each thread still adds its points in index order.
// Two per iteration measured slower than one for the eight-resonance model on
// MI355X (more VGPRs); the events passes come in both forms and the
// autotuner times them, the grid and matrix-row passes use one.
template <class S, int MODE, int GRAD, int EPT = 1>
__device__ inline void dalitz_chunk(const DalitzConst& dc, const DalitzTable* __restrict__ tab,
                                    const double* __restrict__ coef0, const double* __restrict__ ev, int64_t ld,
                                    int64_t n, int64_t chunk_idx, int chunk, int i0, double* __restrict__ out_row,
                                    double* lds) {
  constexpr int NV = dal_nv(MODE, GRAD, S::K);
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const int64_t base = chunk_idx * chunk;
  const int64_t end = base + chunk < n ? base + chunk : n;
  const double* const r0 = &tab->r[0][0];
  LogProd lp;
  // matrix-row passes over the whole grid, one cell per thread and
  // iteration: the cell's (ix, iy) advanced by kBlock cells per iteration
  // instead of a 64-bit division, and the region's bounds computed once per
  // grid column
  int64_t gx = 0, gy = 0, row_ix = -1;
  double row_lo = 0.0, row_hi = 0.0;
  if (MODE == kMRows && EPT == 1) {
    gx = (base + threadIdx.x) / dc.ny;
    gy = (base + threadIdx.x) - gx * dc.ny;
  }
  for (int64_t i = base + threadIdx.x; i < end; i += EPT * kBlock) {
    // The per-resonance constants are read through the scalar cache on every
    // event: an empty asm makes a zero offset opaque to the loop so that the
    // compiler does not keep the whole table resident in SGPRs, which
    // overflows them into VGPR lanes (a v_readlane per use); the pointer keeps
    // its provenance, so the reads stay scalar loads.
    int zero = 0;
    asm volatile("" : "+s"(zero));
    const double* r = r0 + zero;
    const double* coef = coef0 + zero;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int64_t j = i + e * kBlock;
      bool valid = e == 0 || j < end;
      const int64_t jj = valid ? j : i;  // a valid index; its terms are masked out
      double s12, s13;
      if (MODE == kEvents) {
        s12 = ev[jj];
        s13 = ev[ld + jj];
      } else if (MODE == kGrid) {
        // grid passes walk the list of the cells inside the region (ev)
        const GridCell g = reinterpret_cast<const GridCell*>(ev)[jj];
        s12 = grid_centre(dc.a12, g.ix, dc.d12);
        s13 = grid_centre(dc.a13, g.iy, dc.d13);
      } else if (EPT == 1) {
        const int64_t ix = gx, iy = gy;
        gy += kBlock;
        while (gy >= dc.ny) {
          gy -= dc.ny;
          ++gx;
        }
        s12 = grid_centre(dc.a12, ix, dc.d12);
        s13 = grid_centre(dc.a13, iy, dc.d13);
        if (ix != row_ix) {
          dalitz_row_bounds(dc, s12, row_lo, row_hi);
          row_ix = ix;
        }
        if (!dalitz_in_row(dc, s12, s13, row_lo, row_hi)) continue;
      } else {
        const int64_t ix = jj / dc.ny;
        const int64_t iy = jj - ix * dc.ny;
        s12 = grid_centre(dc.a12, ix, dc.d12);
        s13 = grid_centre(dc.a13, iy, dc.d13);
        valid = valid && dalitz_inside(dc, s12, s13);
      }
      dalitz_point<S, MODE, GRAD>(dc, r, coef, s12, s13, valid, i0, acc, lp);
    }
  }
  if (MODE == kEvents) acc[0] = -lp.log();
  block_sum_row<NV>(acc, lds, out_row);
}

// Normalization of a model with fixed lineshapes from the cached grid matrix
// M (K x K complex, M_kj = dA sum over cells of A_k conj(A_j)): I = c^H M c =
// sum_k Re(c_k X_k) with X_k = sum_j M_kj conj(c_j), dI/dRe c_k = 2 Re X_k,
// dI/dIm c_k = -2 Im X_k.  Writes out[0] = I and out[1 + 2k], out[2 + 2k];
// all threads of the workgroup call it.
template <class S>
__device__ inline void dalitz_cached_norm(const double* __restrict__ M, const double* __restrict__ coef,
                                          double* __restrict__ out) {
  constexpr int K = S::K;
  __shared__ double ip[K];
  const int t = threadIdx.x;
  if (t < K) {
    double xr = 0.0, xi = 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const double mr = M[2 * (t * K + j)], mi = M[2 * (t * K + j) + 1];
      const double cr = coef[2 * j], ci = coef[2 * j + 1];
      xr = __builtin_fma(mr, cr, __builtin_fma(mi, ci, xr));
      xi = __builtin_fma(mi, cr, __builtin_fma(-mr, ci, xi));
    }
    ip[t] = __builtin_fma(coef[2 * t], xr, -(coef[2 * t + 1] * xi));
    out[1 + 2 * t] = 2.0 * xr;
    out[2 + 2 * t] = -2.0 * xi;
  }
  __syncthreads();
  if (t == 0) {
    double I = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) I += ip[k];
    out[0] = I;
  }
}

// One workgroup per chunk, one row of NV partial sums each.
// coef: (Re c_k, Im c_k) of the resonances (theta's first 2K entries, or the
// table's copy of them); unused by kMRows.  Events pass with a cached grid
// matrix (M not null): the last workgroup, whose chunk is the shortest,
// also evaluates the normalization into norm_out (dalitz_cached_norm), so
// that the level-2 step only sums rows.  span: the launch's span record
// (span_begin / span_end), null when the launch is not measured.
template <class S, int MODE, int GRAD, int EPT = 1>
__device__ inline void dalitz_pass_body(const DalitzConst& dc, const DalitzTable* __restrict__ tab,
                                        const double* __restrict__ coef, const double* __restrict__ ev, int64_t ld,
                                        int64_t n, int chunk, int i0, double* __restrict__ part,
                                        const double* __restrict__ M, double* __restrict__ norm_out,
                                        unsigned long long* __restrict__ span) {
  constexpr int NV = dal_nv(MODE, GRAD, S::K);
  __shared__ double lds[block_sum_lds(NV)];
  if (span) span_begin(span);
  dalitz_chunk<S, MODE, GRAD, EPT>(dc, tab, coef, ev, ld, n, blockIdx.x, chunk, i0,
                                   part + (int64_t)blockIdx.x * NV, lds);
  if (MODE == kEvents && M && blockIdx.x == gridDim.x - 1) dalitz_cached_norm<S>(M, coef, norm_out);
  if (span) span_end(span);
}

// ---------------------------------------------------------------- toy events
// P~(s12, s13) = |sum_k c_k A_k|^2 at one point.
template <class S>
__device__ __forceinline__ double dalitz_value(const DalitzConst& dc, const double* __restrict__ r,
                                               const double* __restrict__ coef, double s12, double s13) {
  constexpr int K = S::K;
  const double s23 = dc.msum - s12 - s13;
  double Are[K], Aim[K], Tre[K], Tim[K], Gk[K];
  double Sre = 0.0, Sim = 0.0;
  dalitz_amps<S, kGrid, false, false>(dc, r, coef, s12, s13, s23, Are, Aim, Tre, Tim, Gk, Sre, Sim);
  return __builtin_fma(Sre, Sre, Sim * Sim);
}

// Largest P~ over the centres of the grid cells inside the region, as the
// bit pattern of a non-negative double (ordered like the value) in *vmax.
template <class S>
__device__ inline void dalitz_gridmax_body(const DalitzConst& dc, const DalitzTable* __restrict__ tab,
                                           unsigned long long* __restrict__ vmax) {
  __shared__ double lds[kBlock];
  const int64_t ncell = (int64_t)dc.nx * dc.ny;
  const double* r = &tab->r[0][0];
  double m = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * kBlock) {
    const int64_t ix = c / dc.ny, iy = c - ix * dc.ny;
    const double s12 = grid_centre(dc.a12, ix, dc.d12);
    const double s13 = grid_centre(dc.a13, iy, dc.d13);
    if (!dalitz_inside(dc, s12, s13)) continue;
    m = fmax(m, dalitz_value<S>(dc, r, tab->coef, s12, s13));
  }
  lds[threadIdx.x] = m;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(vmax, (unsigned long long)__double_as_longlong(lds[0]));
}

// Events distributed as P~ by accept-reject from the bounding box
// [box12] x [box13] (the box of the kinematic limits, as the host computes
// it): event i, attempt a takes (u1, u2) from counter (i, 2a, 1) and u3 from
// counter (i, 2a + 1, 1) under key (k0, k1); the candidate
// (box12.lo + u1 (box12.hi - box12.lo), box13.lo + u2 (...)) is kept when it
// lies in the region and u3 W < P~.  An event whose accepted P~ exceeds W
// (the envelope was too low there) counts in bad[0]; an event not accepted
// within max_attempts is NaN and counts in bad[1].
template <class S>
__device__ inline void dalitz_gen_body(const DalitzConst& dc, const DalitzTable* __restrict__ tab, uint32_t k0,
                                       uint32_t k1, int64_t n, double W, double lo12, double hi12, double lo13,
                                       double hi13, int max_attempts, double* __restrict__ ev, int64_t ld,
                                       unsigned long long* __restrict__ bad) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double* r = &tab->r[0][0];
  const double w12 = hi12 - lo12, w13 = hi13 - lo13;
  double x12 = __builtin_nan(""), x13 = __builtin_nan(""), px = 0.0;
  for (int a = 0; a < max_attempts; ++a) {
    double u1, u2, u3, unused;
    philox_uniforms((uint64_t)i, 2u * a, 1u, k0, k1, u1, u2);
    philox_uniforms((uint64_t)i, 2u * a + 1u, 1u, k0, k1, u3, unused);
    const double s12 = lo12 + u1 * w12;
    const double s13 = lo13 + u2 * w13;
    if (!dalitz_inside(dc, s12, s13)) continue;
    const double p = dalitz_value<S>(dc, r, tab->coef, s12, s13);
    if (u3 * W < p) {
      x12 = s12;
      x13 = s13;
      px = p;
      break;
    }
  }
  ev[i] = x12;
  ev[ld + i] = x13;
  if (px > W) atomicAdd(bad, 1ull);
  if (x12 != x12) atomicAdd(bad + 1, 1ull);
}

}  // namespace fn

// Kernel NAME for shape S, mode, gradient level and events per thread and
// iteration (used by the generated source).
#define FN_DALITZ_KERNEL(NAME, S, MODE, GRAD, EPT)                                                           \
  extern "C" __global__ __launch_bounds__(fn::kBlock) void NAME(                                               \
      fn::DalitzConst dc, const fn::DalitzTable* __restrict__ tab, const double* __restrict__ coef,           \
      const double* __restrict__ ev, int64_t ld, int64_t n, int chunk, int i0, double* __restrict__ part,     \
      const double* __restrict__ M, double* __restrict__ norm_out, unsigned long long* __restrict__ span) {    \
    fn::dalitz_pass_body<S, MODE, GRAD, EPT>(dc, tab, coef, ev, ld, n, chunk, i0, part, M, norm_out, span);    \
  }

// Grid maximum and accept-reject generator for shape S.
#define FN_DALITZ_GEN(GRIDMAX, GEN, S)                                                                        \
  extern "C" __global__ __launch_bounds__(fn::kBlock) void GRIDMAX(                                            \
      fn::DalitzConst dc, const fn::DalitzTable* __restrict__ tab, unsigned long long* __restrict__ vmax) {   \
    fn::dalitz_gridmax_body<S>(dc, tab, vmax);                                                                 \
  }                                                                                                            \
  extern "C" __global__ __launch_bounds__(fn::kBlock) void GEN(                                                \
      fn::DalitzConst dc, const fn::DalitzTable* __restrict__ tab, uint32_t k0, uint32_t k1, int64_t n,        \
      double W, double lo12, double hi12, double lo13, double hi13, int max_attempts,                          \
      double* __restrict__ ev, int64_t ld, unsigned long long* __restrict__ bad) {                             \
    fn::dalitz_gen_body<S>(dc, tab, k0, k1, n, W, lo12, hi12, lo13, hi13, max_attempts, ev, ld, bad);         \
  }
