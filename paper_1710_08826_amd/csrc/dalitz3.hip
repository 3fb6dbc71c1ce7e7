// Three-body Dalitz-plot amplitude model (the paper's amplitude analyses of
// three-body decays, Sec. 1 and 5):  P~(s12, s13) = |sum_k c_k A_k|^2,
//
//   A_k = [F_L(q r)/F_L(q0 r)] F_L(p r_D) Z_L(s) T_k(s_AB)
//   T_k = 1 / (m0^2 - s_AB - i m0 Gamma_k(s_AB))
//   Gamma_k(s) = Gamma0 (q/q0)^(2L+1) (m0/sqrt s) [F_L(q r)/F_L(q0 r)]^2
//
// with Blatt-Weisskopf factors F_0 = 1, F_1 = (1+z)^-1/2,
// F_2 = (z^2+3z+9)^-1/2 (z = (q r)^2) and Zemach spin factors Z_0 = 1,
// Z_1 = s_AC - s_BC + (M^2 - mC^2)(mB^2 - mA^2)/s_AB, Z_2 = Z_1^2 - X Y / 3,
// X = lambda(s_AB, M^2, mC^2)/s_AB, Y = lambda(s_AB, mA^2, mB^2)/s_AB.
//
// GPU organisation (per event, all in registers):
//  * every quantity that depends only on the pair (s_AB, q, p, the barrier
//    polynomials, Zemach factors) is computed once per pair and shared by all
//    resonances of that pair: the model has three pairs and eight resonances,
//    so this removes most of the square roots and divisions;
//  * per resonance the lineshape reduces to T = (a + i b)/(a^2 + b^2) with
//    a = m0^2 - s and b = m0 Gamma(s) = Kw * G_{pair,L}(s), where
//    G = q^(2L+1) F_L(q r)^2 / sqrt(s) is per pair and
//    Kw = Gamma0 m0^2 / (q0^(2L+1) F_L(q0 r)^2) comes from the prologue;
//  * the amplitude is A = Ka * H_{pair,L} * T with H = F_L(q r) F_L(p r_D) Z_L
//    per pair and Ka = 1/F_L(q0 r) per resonance.
// The resonance loop is unrolled to a compile-time maximum with uniform
// guards, so amplitudes and gradient accumulators stay in VGPRs.
//
// Modes of the shared chunk routine:
//   kEvents  -ln P~ over an event chunk (+ adjoint gradient)          -> NLL
//   kGrid    P~ over a chunk of grid cells inside the region (+ dP~)  -> I
//   kMRows   rows i0..i0+3 of sum_cells A_i conj(A_j)                 -> cached M
#include <cmath>

#include "device_common.hpp"
#include "fastmath.hpp"
#include "kernels.hpp"

namespace fn {

enum DalMode : int { kEvents = 0, kGrid = 1, kMRows = 2 };
constexpr int kMRowBlock = 4;

__host__ __device__ constexpr int dal_nv(int mode, int grad, int kmax) {
  return mode == kMRows ? 2 * kMRowBlock * kmax : 1 + (grad == 0 ? 0 : (grad == 1 ? 2 * kmax : 4 * kmax));
}

// ---------------------------------------------------------------- prologue
// Per resonance: Kw, Ka and (for lineshape gradients) their derivatives.
__global__ void dalitz_prologue(DalitzConst dc, ParamBlock pb, const double* __restrict__ theta_dev,
                                const double* __restrict__ fixed_ls, int n_fits, int theta_stride,
                                DalitzTable* __restrict__ tab) {
  const int f = blockIdx.x;
  const int k = threadIdx.x;
  const double* th = theta_dev ? theta_dev + (int64_t)f * theta_stride : pb.v;
  __shared__ int bad;
  if (k == 0) bad = 0;
  __syncthreads();
  if (k < dc.K) {
    const DalitzChan& ch = dc.ch[dc.chan[k]];
    const int L = dc.L[k];
    const double m0 = dc.free_ls ? th[2 * dc.K + 2 * k] : fixed_ls[2 * k];
    const double w0 = dc.free_ls ? th[2 * dc.K + 2 * k + 1] : fixed_ls[2 * k + 1];
    const double x = m0 * m0;
    const double lam = (x - ch.sum2) * (x - ch.dif2);
    const double q02 = 0.25 * lam / x;
    // d(q0^2)/dm0 = 2 m0 d(q0^2)/dx, d(q0^2)/dx = (lam' x - lam) / (4 x^2)
    const double dlam = 2.0 * x - ch.sum2 - ch.dif2;
    const double dq02 = 2.0 * m0 * (dlam * x - lam) / (4.0 * x * x);
    const double z0 = q02 * dc.r2, dz0 = dq02 * dc.r2;
    double poly = 1.0, dpoly = 0.0;  // 1/F_L(q0 r)^2 and its z-derivative
    if (L == 1) { poly = 1.0 + z0; dpoly = 1.0; }
    if (L == 2) { poly = z0 * z0 + 3.0 * z0 + 9.0; dpoly = 2.0 * z0 + 3.0; }
    const double ka = sqrt(poly);
    const double dlnka = 0.5 * dpoly * dz0 / poly;
    const double q0 = sqrt(q02);
    double q0pow = q0;  // q0^(2L+1)
    for (int l = 0; l < L; ++l) q0pow *= q02;
    const double kw = w0 * x * poly / q0pow;
    // d ln Kw / dm0 = 2/m0 + 2 d ln Ka/dm0 - (2L+1) d ln q0/dm0
    const double dlnkw = 2.0 / m0 + 2.0 * dlnka - (2.0 * L + 1.0) * 0.5 * dq02 / q02;
    double* r = tab[f].r[k];
    r[dM0SQ] = x;
    r[dKW] = kw;
    r[dKA] = ka;
    r[dCRE] = th[2 * k];
    r[dCIM] = th[2 * k + 1];
    r[dDLNKA] = dlnka;
    r[dDKW_DM0] = kw * dlnkw;
    r[dKW_W0] = x * poly / q0pow;
    r[dTWOM0] = 2.0 * m0;
    if (!(m0 > 0.0) || !(w0 > 0.0) || !(lam > 0.0) || !isfinite(kw)) atomicOr(&bad, 1);
  }
  __syncthreads();
  if (k == 0) tab[f].valid = bad ? 0.0 : 1.0;
}

// ------------------------------------------------------------- pair terms
struct PairTerms {
  double s;         // s_AB
  double G[3];      // q^(2L+1) F_L(q r)^2 / sqrt(s)
  double H[3];      // F_L(q r) F_L(p r_D) Z_L
};

// G and H of one pair from (s_AB, s_AC, s_BC):
//   q/sqrt(s) = sqrt(lambda_q) / (2 s),  q^2 = lambda_q / (4 s),  p^2 = lambda_p / (4 s)
//   G_1 = (q/sqrt s) q^2 / (1 + z_q),          H_1 = Z_1 / sqrt((1 + z_q)(1 + z_p))
//   G_2 = (q/sqrt s) q^4 / (z_q^2 + 3 z_q + 9), H_2 = Z_2 / sqrt(poly(z_q) poly(z_p))
__device__ __forceinline__ void pair_terms(const DalitzChan& ch, double s_ab, double s_ac, double s_bc, double r2,
                                           double rD2, PairTerms& o) {
  const double irs = rsqrt_nr(s_ab);
  const double is = irs * irs;
  const double lq = fmax((s_ab - ch.sum2) * (s_ab - ch.dif2), 0.0);
  const double lp = fmax((s_ab - ch.Psum2) * (s_ab - ch.Pdif2), 0.0);
  const double q2 = 0.25 * lq * is;
  const double qirs = 0.5 * sqrt_nr(lq) * is;
  o.s = s_ab;
  o.G[0] = qirs;
  o.H[0] = 1.0;
  o.G[1] = o.G[2] = o.H[1] = o.H[2] = 0.0;
  if (ch.useL[1] | ch.useL[2]) {
    const double p2 = 0.25 * lp * is;
    const double zq = q2 * r2, zp = p2 * rD2;
    const double z1 = __builtin_fma(ch.zc, is, s_ac - s_bc);
    if (ch.useL[1]) {
      const double uq = 1.0 + zq, up = 1.0 + zp;
      o.G[1] = qirs * q2 * rcp_nr(uq);
      o.H[1] = z1 * rsqrt_nr(uq * up);
    }
    if (ch.useL[2]) {
      const double vq = __builtin_fma(zq, zq + 3.0, 9.0), vp = __builtin_fma(zp, zp + 3.0, 9.0);
      o.G[2] = qirs * q2 * q2 * rcp_nr(vq);
      const double z2 = z1 * z1 - (lp * is) * (lq * is) * (1.0 / 3.0);
      o.H[2] = z2 * rsqrt_nr(vq * vp);
    }
  }
}

// Physical-region predicate at a grid-cell centre: s23 between its limits at
// this s12, from the energies of daughters 2 and 3 in the (12) rest frame.
// Contraction is off so that the decision is the plain IEEE evaluation.
__device__ inline bool dalitz_inside(const DalitzConst& dc, double s12, double s13) {
#pragma clang fp contract(off)
  const double rs = sqrt(s12);
  const double e2 = (s12 - dc.m1s + dc.m2s) / (2.0 * rs);
  const double e3 = (dc.M2 - s12 - dc.m3s) / (2.0 * rs);
  const double p2 = sqrt(fmax(e2 * e2 - dc.m2s, 0.0));
  const double p3 = sqrt(fmax(e3 * e3 - dc.m3s, 0.0));
  const double es = e2 + e3;
  const double lo = es * es - (p2 + p3) * (p2 + p3);
  const double hi = es * es - (p2 - p3) * (p2 - p3);
  const double s23 = dc.msum - s12 - s13;
  return s23 >= lo && s23 <= hi;
}

// ------------------------------------------------------------ chunk routine
// GRAD: 0 none, 1 coefficients only, 2 coefficients + masses and widths.
// Pairs are visited one at a time (only one pair's G/H are live) and each
// resonance of the pair adds c_k A_k to the coherent sum.
template <int MODE, int GRAD, int KMAX>
__device__ inline void dalitz_chunk(const DalitzConst& dc, const DalitzTable* __restrict__ tab,
                                    const double* __restrict__ ev, int64_t ld, int64_t n, int64_t chunk_idx,
                                    int chunk, int i0, double* __restrict__ out_row, double* lds) {
  constexpr int NV = dal_nv(MODE, GRAD, KMAX);
  constexpr bool KEEP_A = (GRAD >= 1) || MODE == kMRows;
  constexpr bool KEEP_T = GRAD == 2;
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const int64_t base = chunk_idx * chunk;
  const int64_t end = base + chunk < n ? base + chunk : n;
  const double* r = &tab->r[0][0];
  for (int64_t i = base + threadIdx.x; i < end; i += kBlock) {
    double s12, s13;
    if (MODE == kEvents) {
      s12 = ev[i];
      s13 = ev[ld + i];
    } else {
      const int64_t ix = i / dc.ny;
      const int64_t iy = i - ix * dc.ny;
      s12 = dc.a12 + (ix + 0.5) * dc.d12;
      s13 = dc.a13 + (iy + 0.5) * dc.d13;
      if (!dalitz_inside(dc, s12, s13)) continue;
    }
    const double s23 = dc.msum - s12 - s13;
    double Are[KMAX], Aim[KMAX], Tre[KMAX], Tim[KMAX], Gk[KMAX];
    double Sre = 0.0, Sim = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const DalitzChan& ch = dc.ch[c];
      if (!(ch.useL[0] | ch.useL[1] | ch.useL[2])) continue;
      // pair "12": (A,B,C) = (1,2,3); "13": (1,3,2); "23": (2,3,1)
      const double s_ab = c == 0 ? s12 : (c == 1 ? s13 : s23);
      const double s_ac = c == 0 ? s13 : s12;
      const double s_bc = c == 2 ? s13 : s23;
      PairTerms pt;
      pair_terms(ch, s_ab, s_ac, s_bc, dc.r2, dc.rD2, pt);
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < dc.K && dc.chan[k] == c) {
          const int L = dc.L[k];
          const double* rk = r + k * kDalFields;
          const double G = L == 0 ? pt.G[0] : (L == 1 ? pt.G[1] : pt.G[2]);
          const double H = L == 0 ? pt.H[0] : (L == 1 ? pt.H[1] : pt.H[2]);
          const double a = rk[dM0SQ] - pt.s;
          const double b = rk[dKW] * G;
          const double d = rcp_nr(__builtin_fma(a, a, b * b));
          const double tr = a * d, ti = b * d;
          const double kh = rk[dKA] * H;
          const double ar = kh * tr, ai = kh * ti;
          if (KEEP_A) { Are[k] = ar; Aim[k] = ai; }
          if (KEEP_T) { Tre[k] = tr; Tim[k] = ti; Gk[k] = G; }
          if (MODE != kMRows) {
            const double cr = rk[dCRE], ci = rk[dCIM];
            Sre += cr * ar - ci * ai;
            Sim += cr * ai + ci * ar;
          }
        }
      }
    }
    if (MODE == kMRows) {
#pragma unroll
      for (int ib = 0; ib < kMRowBlock; ++ib) {
        // A_i for i = i0 + ib, selected from registers with uniform guards
        double xr = 0.0, xi = 0.0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
          if (k == i0 + ib) { xr = Are[k]; xi = Aim[k]; }
#pragma unroll
        for (int j = 0; j < KMAX; ++j) {
          if (j < dc.K) {
            acc[2 * (ib * KMAX + j)] += xr * Are[j] + xi * Aim[j];
            acc[2 * (ib * KMAX + j) + 1] += xi * Are[j] - xr * Aim[j];
          }
        }
      }
      continue;
    }
    const double Pt = __builtin_fma(Sre, Sre, Sim * Sim);
    double w;  // multiplies dP~/dtheta
    if (MODE == kEvents) {
      acc[0] -= log_fast(Pt);
      w = -rcp_nr(Pt);
    } else {
      acc[0] += Pt;
      w = 1.0;
    }
    if (GRAD >= 1) {
      const double w2 = 2.0 * w;
      const double ur = w2 * Sre, ui = w2 * Sim;
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < dc.K) {
          // dP~/dRe c = 2 Re(conj(S) A), dP~/dIm c = 2 (Sim Are - Sre Aim)
          acc[1 + 2 * k] += ur * Are[k] + ui * Aim[k];
          acc[2 + 2 * k] += ui * Are[k] - ur * Aim[k];
        }
      }
    }
    if (GRAD == 2) {
      const double w2 = 2.0 * w;
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < dc.K) {
          const double* rk = r + k * kDalFields;
          const double cr = rk[dCRE], ci = rk[dCIM];
          // E = conj(S) c A
          const double car = cr * Are[k] - ci * Aim[k], cai = cr * Aim[k] + ci * Are[k];
          const double er = Sre * car + Sim * cai, ei = Sre * cai - Sim * car;
          // dA/dm0 = A (dlnKa - T (2 m0 - i G dKw/dm0));  dP~ = 2 Re(E * (...))
          const double gd = Gk[k] * rk[dDKW_DM0], tm = rk[dTWOM0];
          const double xr = tm * Tre[k] + Tim[k] * gd;
          const double xi = tm * Tim[k] - Tre[k] * gd;
          const double yr = rk[dDLNKA] - xr, yi = -xi;
          acc[1 + 2 * KMAX + 2 * k] += w2 * (er * yr - ei * yi);
          // dA/dGamma0 = i A T G Kw/Gamma0
          const double gw = Gk[k] * rk[dKW_W0];
          acc[2 + 2 * KMAX + 2 * k] += w2 * gw * (-er * Tim[k] - ei * Tre[k]);
        }
      }
    }
  }
  block_sum_row<NV>(acc, lds, out_row);
}

// FN_DALITZ_WAVES > 0 asks the register allocator for that many waves per
// SIMD (a tuning knob; 0 leaves the choice to the compiler).
#ifndef FN_DALITZ_WAVES
#define FN_DALITZ_WAVES 0
#endif
#if FN_DALITZ_WAVES > 0
#define FN_DALITZ_WAVES_ATTR __attribute__((amdgpu_waves_per_eu(FN_DALITZ_WAVES, 8)))
#else
#define FN_DALITZ_WAVES_ATTR
#endif

// ------------------------------------------------------------- finalize
// Arguments of the level-2 + NLL assembly step.
struct DalFinal {
  const double* npart;       // grid rows (free lineshapes) or nullptr (cached M)
  int64_t n_rows;
  int n_nv;
  const double* Mc;          // cached M (K x K complex) when npart == nullptr
  double n_events;
  int with_grad;
  double* out;               // [NLL, grad(P), I, dI(P)]
  double* out_user;          // optional [NLL, grad(P)]
};

struct DalFinalLds {
  double scratch[kBlock];
  double res[kBlock];
  double nres[kBlock];
  double cre[kDalMaxRes], cim[kDalMaxRes], ipart[kDalMaxRes];
  double dI[4 * kDalMaxRes];
  double I;
};

// Level-2 over the event rows and the normalization (grid rows or cached M),
// then NLL = -sum ln P~ + N ln I and its gradient, one thread per entry.
__device__ void dalitz_finalize_body(const DalitzConst& dc, const DalitzTable* __restrict__ tab,
                                     const double* __restrict__ evpart, int64_t ev_rows, int ev_nv, int kmax,
                                     const DalFinal& f, DalFinalLds& L) {
  const int K = dc.K;
  const int P = dc.free_ls ? 4 * K : 2 * K;
  const int t = threadIdx.x;
  sum_rows(evpart, ev_rows, ev_nv, L.scratch, L.res);
  if (f.npart) sum_rows(f.npart, f.n_rows, f.n_nv, L.scratch, L.nres);
  if (t < K) {
    L.cre[t] = tab->r[t][dCRE];
    L.cim[t] = tab->r[t][dCIM];
  }
  if (t < P) L.dI[t] = 0.0;
  __syncthreads();
  if (f.npart) {
    if (t < K && f.n_nv > 1) {
      L.dI[2 * t] = dc.dA * L.nres[1 + 2 * t];
      L.dI[2 * t + 1] = dc.dA * L.nres[2 + 2 * t];
      if (dc.free_ls && f.n_nv > 1 + 2 * kmax) {
        L.dI[2 * K + 2 * t] = dc.dA * L.nres[1 + 2 * kmax + 2 * t];
        L.dI[2 * K + 2 * t + 1] = dc.dA * L.nres[2 + 2 * kmax + 2 * t];
      }
    }
    if (t == 0) L.I = dc.dA * L.nres[0];
  } else if (t < K) {
    // I = sum_k Re(c_k X_k), X_k = sum_j M_kj conj(c_j);
    // dI/dRe c_k = 2 Re X_k, dI/dIm c_k = -2 Im X_k
    double xr = 0.0, xi = 0.0;
    for (int j = 0; j < K; ++j) {
      const double mr = f.Mc[2 * (t * K + j)], mi = f.Mc[2 * (t * K + j) + 1];
      xr += mr * L.cre[j] + mi * L.cim[j];
      xi += mi * L.cre[j] - mr * L.cim[j];
    }
    L.ipart[t] = L.cre[t] * xr - L.cim[t] * xi;
    L.dI[2 * t] = 2.0 * xr;
    L.dI[2 * t + 1] = -2.0 * xi;
  }
  __syncthreads();
  if (!f.npart && t == 0) {
    double I = 0.0;
    for (int k = 0; k < K; ++k) I += L.ipart[k];
    L.I = I;
  }
  __syncthreads();
  const double I = L.I;
  const bool okI = tab->valid != 0.0 && I > 0.0 && isfinite(I);
  if (t == 0) {
    const double v = okI ? L.res[0] + f.n_events * log(I) : INFINITY;
    f.out[0] = v;
    f.out[1 + P] = I;
    if (f.out_user) f.out_user[0] = v;
  }
  if (t < P) {
    f.out[2 + P + t] = L.dI[t];
    if (f.with_grad) {
      // event slot of parameter t: coefficients at 1 + t, lineshapes after 2 kmax
      const int slot = t < 2 * K ? 1 + t : 1 + 2 * kmax + (t - 2 * K);
      const double e = slot < ev_nv ? L.res[slot] : 0.0;
      const double g = okI ? e + f.n_events * L.dI[t] / I : NAN;
      f.out[1 + t] = g;
      if (f.out_user) f.out_user[1 + t] = g;
    }
  }
}

// Evaluation pass: one workgroup per chunk, one row of partial sums each.
// (Finishing the level-2 sum inside the last workgroup to retire, behind a
// device-scope fence per workgroup, measured 2.5x slower on MI355X than the
// separate level-2 launch below, so the two steps stay separate kernels.)
template <int MODE, int GRAD, int KMAX>
__global__ __launch_bounds__(kBlock) FN_DALITZ_WAVES_ATTR void dalitz_pass(DalitzConst dc, const DalitzTable* __restrict__ tab,
                                                      const double* __restrict__ ev, int64_t ld, int64_t n,
                                                      int chunk, int i0, double* __restrict__ part) {
  constexpr int NV = dal_nv(MODE, GRAD, KMAX);
  __shared__ double lds[kWaves * NV];
  dalitz_chunk<MODE, GRAD, KMAX>(dc, tab, ev, ld, n, blockIdx.x, chunk, i0, part + (int64_t)blockIdx.x * NV,
                                 lds);
}

// Level-2 step: one workgroup.
__global__ __launch_bounds__(kBlock) void dalitz_finalize(DalitzConst dc, const DalitzTable* __restrict__ tab,
                                                          const double* __restrict__ evpart, int64_t ev_rows,
                                                          int ev_nv, int kmax, DalFinal fin) {
  __shared__ DalFinalLds L;
  dalitz_finalize_body(dc, tab, evpart, ev_rows, ev_nv, kmax, fin, L);
}

// Level-2 of the M-row passes: rows i0..i0+3 of M (scaled by dA) into Mc.
__global__ __launch_bounds__(kBlock) void dalitz_mrows_finalize(DalitzConst dc, const double* __restrict__ part,
                                                                int64_t nrows, int nv, int kmax, int i0,
                                                                double* __restrict__ Mc) {
  __shared__ double scratch[kBlock];
  __shared__ double res[kBlock];
  sum_rows(part, nrows, nv, scratch, res);
  const int K = dc.K;
  for (int t = threadIdx.x; t < kMRowBlock * kmax; t += kBlock) {
    const int ib = t / kmax, j = t - ib * kmax;
    const int i = i0 + ib;
    if (i < K && j < K) {
      Mc[2 * (i * K + j)] = dc.dA * res[2 * t];
      Mc[2 * (i * K + j) + 1] = dc.dA * res[2 * t + 1];
    }
  }
}

// P~(x_i)/I per event (I read from the finalize output).
__global__ void dalitz_eval(DalitzConst dc, const DalitzTable* __restrict__ tab, const double* __restrict__ ev,
                            int64_t ld, int64_t n, const double* __restrict__ norm, double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s12 = ev[i], s13 = ev[ld + i];
  const double s23 = dc.msum - s12 - s13;
  PairTerms pt[3];
  pair_terms(dc.ch[0], s12, s13, s23, dc.r2, dc.rD2, pt[0]);
  pair_terms(dc.ch[1], s13, s12, s23, dc.r2, dc.rD2, pt[1]);
  pair_terms(dc.ch[2], s23, s12, s13, dc.r2, dc.rD2, pt[2]);
  double Sre = 0.0, Sim = 0.0;
  for (int k = 0; k < dc.K; ++k) {
    const PairTerms& q = pt[dc.chan[k]];
    const double* rk = tab->r[k];
    const double a = rk[dM0SQ] - q.s, b = rk[dKW] * q.G[dc.L[k]];
    const double d = 1.0 / (a * a + b * b);
    const double kh = rk[dKA] * q.H[dc.L[k]];
    const double ar = kh * a * d, ai = kh * b * d;
    Sre += rk[dCRE] * ar - rk[dCIM] * ai;
    Sim += rk[dCRE] * ai + rk[dCIM] * ar;
  }
  p[i] = (Sre * Sre + Sim * Sim) / *norm;
}

__global__ void dalitz_check(DalitzConst dc, const double* __restrict__ ev, int64_t ld, int64_t n,
                             unsigned long long* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool b = false;
  if (i < n) {
    const double s12 = ev[i], s13 = ev[ld + i];
    const double tol = 1e-9;
    const double b12 = dc.a12 + dc.nx * dc.d12, b13 = dc.a13 + dc.ny * dc.d13;
    b = !(s12 >= dc.a12 * (1 - tol) && s12 <= b12 * (1 + tol) && s13 >= dc.a13 * (1 - tol) &&
          s13 <= b13 * (1 + tol));
    if (!b) {
      const double rs = sqrt(s12);
      const double e2 = (s12 - dc.m1s + dc.m2s) / (2.0 * rs);
      const double e3 = (dc.M2 - s12 - dc.m3s) / (2.0 * rs);
      const double p2 = sqrt(fmax(e2 * e2 - dc.m2s, 0.0));
      const double p3 = sqrt(fmax(e3 * e3 - dc.m3s, 0.0));
      const double es = e2 + e3;
      const double lo = es * es - (p2 + p3) * (p2 + p3);
      const double hi = es * es - (p2 - p3) * (p2 - p3);
      const double s23 = dc.msum - s12 - s13;
      const double slack = tol * dc.msum;
      b = !(s23 >= lo - slack && s23 <= hi + slack);
    }
  }
  const unsigned long long cnt = __ballot(b);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(bad, (unsigned long long)__popcll(cnt));
}

// ---------------------------------------------------------------- launchers
int dalitz_kmax(int K) { return K <= 8 ? 8 : 16; }
int dalitz_nv_events(int kmax, int grad) { return dal_nv(kEvents, grad, kmax); }
int dalitz_nv_mrows(int kmax) { return dal_nv(kMRows, 0, kmax); }

void dalitz_launch_prologue(const DalitzConst& dc, const ParamBlock& pb, const double* theta_dev,
                            const double* fixed_ls, int n_fits, int theta_stride, DalitzTable* tab, hipStream_t s) {
  hipLaunchKernelGGL(dalitz_prologue, dim3(n_fits), dim3(64), 0, s, dc, pb, theta_dev, fixed_ls, n_fits,
                     theta_stride, tab);
}

template <int MODE, int GRAD>
static void launch_pass_k(const DalitzConst& dc, const DalitzTable* tab, const double* ev, int64_t ld, int64_t n,
                          int chunk, int64_t nchunks, int i0, double* part, hipStream_t s) {
  if (dalitz_kmax(dc.K) == 8)
    hipLaunchKernelGGL((dalitz_pass<MODE, GRAD, 8>), dim3((unsigned)nchunks), dim3(kBlock), 0, s, dc, tab, ev, ld,
                       n, chunk, i0, part);
  else
    hipLaunchKernelGGL((dalitz_pass<MODE, GRAD, 16>), dim3((unsigned)nchunks), dim3(kBlock), 0, s, dc, tab, ev,
                       ld, n, chunk, i0, part);
}

static DalFinal make_final(const double* npart, int64_t n_rows, int n_nv, const double* Mc, double n_events,
                           bool grad, double* out, double* out_user) {
  DalFinal f;
  f.npart = npart;
  f.n_rows = n_rows;
  f.n_nv = n_nv;
  f.Mc = Mc;
  f.n_events = n_events;
  f.with_grad = grad ? 1 : 0;
  f.out = out;
  f.out_user = out_user;
  return f;
}

void dalitz_launch_events(const DalitzConst& dc, const DalitzTable* tab, const double* ev, int64_t ld, int64_t n,
                          int chunk, int64_t nchunks, int grad, double* part, hipStream_t s) {
  if (nchunks == 0) return;
  if (grad == 0) launch_pass_k<kEvents, 0>(dc, tab, ev, ld, n, chunk, nchunks, 0, part, s);
  else if (grad == 1) launch_pass_k<kEvents, 1>(dc, tab, ev, ld, n, chunk, nchunks, 0, part, s);
  else launch_pass_k<kEvents, 2>(dc, tab, ev, ld, n, chunk, nchunks, 0, part, s);
}

void dalitz_launch_finalize(const DalitzConst& dc, const DalitzTable* tab, const double* evpart, int64_t ev_rows,
                            int grad, const double* npart, int64_t n_rows, int n_nv, const double* Mc,
                            double n_events, double* out, double* out_user, hipStream_t s) {
  const int kmax = dalitz_kmax(dc.K);
  const DalFinal fin = make_final(npart, n_rows, n_nv, Mc, n_events, grad != 0, out, out_user);
  hipLaunchKernelGGL(dalitz_finalize, dim3(1), dim3(kBlock), 0, s, dc, tab, evpart, ev_rows,
                     dal_nv(kEvents, grad, kmax), kmax, fin);
}

void dalitz_launch_grid(const DalitzConst& dc, const DalitzTable* tab, int chunk, int64_t nchunks, int grad,
                        double* part, hipStream_t s) {
  const int64_t ncell = (int64_t)dc.nx * dc.ny;
  if (grad == 0) launch_pass_k<kGrid, 0>(dc, tab, nullptr, 0, ncell, chunk, nchunks, 0, part, s);
  else if (grad == 1) launch_pass_k<kGrid, 1>(dc, tab, nullptr, 0, ncell, chunk, nchunks, 0, part, s);
  else launch_pass_k<kGrid, 2>(dc, tab, nullptr, 0, ncell, chunk, nchunks, 0, part, s);
}

void dalitz_launch_mrows(const DalitzConst& dc, const DalitzTable* tab, int chunk, int64_t nchunks, int i0,
                         double* part, double* Mc, hipStream_t s) {
  const int64_t ncell = (int64_t)dc.nx * dc.ny;
  launch_pass_k<kMRows, 0>(dc, tab, nullptr, 0, ncell, chunk, nchunks, i0, part, s);
  const int kmax = dalitz_kmax(dc.K);
  hipLaunchKernelGGL(dalitz_mrows_finalize, dim3(1), dim3(kBlock), 0, s, dc, part, nchunks,
                     dal_nv(kMRows, 0, kmax), kmax, i0, Mc);
}

void dalitz_launch_eval(const DalitzConst& dc, const DalitzTable* tab, const double* ev, int64_t ld, int64_t n,
                        const double* norm, double* p, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(dalitz_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dc, tab, ev, ld, n, norm, p);
}

void dalitz_launch_check(const DalitzConst& dc, const double* ev, int64_t ld, int64_t n, unsigned long long* bad,
                         hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(dalitz_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dc, ev, ld, n, bad);
}

}  // namespace fn
