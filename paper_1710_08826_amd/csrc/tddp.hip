// Time-dependent three-body Dalitz-plot model with D0 mixing (the paper's
// pi+ pi- pi0 time-dependent amplitude fit, Sec. 1 Table 2 and Fig. 2): host
// launchers and the kernels that do not depend on the model's structure (the
// level-2 step with the normalization quadratic form).  The per-event and
// normalization-matrix passes live in tddp_device.hpp and are compiled at
// model creation with the model's structure as compile-time constants.
#include <algorithm>
#include <sstream>

#include "internal.hpp"
#include "jit.hpp"
#include "kernels.hpp"
#include "tddp.hpp"

namespace fn {

int tddp_nv(int K, bool grad) { return grad ? 3 + 4 * K : 1; }

std::string tddp_jit_source(const DalitzConst& dc) {
  std::ostringstream o;
  o << "#include \"tddp_device.hpp\"\n";
  o << "struct fn_shape {\n  static constexpr int K = " << dc.K << ";\n  static constexpr int chan[" << dc.K
    << "] = {";
  for (int k = 0; k < dc.K; ++k) o << (k ? ", " : "") << dc.chan[k];
  o << "};\n  static constexpr int L[" << dc.K << "] = {";
  for (int k = 0; k < dc.K; ++k) o << (k ? ", " : "") << dc.L[k];
  o << "};\n};\n";
  o << "FN_TDDP_EVENTS(fn_tddp_ev0, fn_shape, false)\n"
       "FN_TDDP_EVENTS(fn_tddp_ev1, fn_shape, true)\n"
       "FN_TDDP_MROWS(fn_tddp_maa, fn_shape, 0)\n"
       "FN_TDDP_MROWS(fn_tddp_mbb, fn_shape, 1)\n"
       "FN_TDDP_MROWS(fn_tddp_mab, fn_shape, 2)\n"
       "FN_TDDP_GEN(fn_tddp_gmax, fn_tddp_gen, fn_shape)\n";
  return o.str();
}

std::shared_ptr<TddpJit> tddp_jit(const DalitzConst& dc) {
  auto j = std::make_shared<TddpJit>();
  j->prog = jit_load(tddp_jit_source(dc), {"fn_tddp_ev0", "fn_tddp_ev1", "fn_tddp_maa", "fn_tddp_mbb", "fn_tddp_mab",
                                           "fn_tddp_gmax", "fn_tddp_gen"});
  const auto& f = j->prog->fns;
  j->ev[0] = f[0];
  j->ev[1] = f[1];
  for (int w = 0; w < 3; ++w) j->mrows[w] = f[2 + w];
  j->gmax = f[5];
  j->gen = f[6];
  return j;
}

// ------------------------------------------------------------- kernels
__global__ void tddp_copy_theta(ParamBlock pb, int P, double* __restrict__ dst) {
  const int p = threadIdx.x;
  if (p < P) dst[p] = pb.v[p];
}

struct TddpFinalLds {
  double scratch[kFinalBlock];
  double M[6 * kDalMaxRes * kDalMaxRes];
  double res[kBlock];
  double cre[kDalMaxRes], cim[kDalMaxRes], bre[kDalMaxRes], bim[kDalMaxRes];
  double X[kDalMaxRes][2], Xb[kDalMaxRes][2], U[kDalMaxRes][2], V[kDalMaxRes][2];
  double Ia, Ib, Zr, Zi;
};

// Level 2 and the normalization
//   I = 1/2 [cy (Ia + Ib) + cx (Ia - Ib) - 2 y cy Re Z - 2 x cx Im Z],
//   Ia = sum c_i conj(c_j) MAA_ij, Ib = sum cbar_i conj(cbar_j) MBB_ij,
//   Z = sum conj(c_i) cbar_j MAB_ij, cy = tau/(1-y^2), cx = tau/(1+x^2),
// with X_k = sum_j MAA_kj conj(c_j), Xb_k = sum_j MBB_kj conj(cbar_j),
// U_i = sum_j MAB_ij cbar_j, V_j = sum_i conj(c_i) MAB_ij:
//   dIa/dRe c_k = 2 Re X_k, dIa/dIm c_k = -2 Im X_k (Ib, cbar and Xb alike),
//   dZ/dRe c_i = U_i, dZ/dIm c_i = -i U_i, dZ/dRe cbar_j = V_j, dZ/dIm cbar_j = i V_j.
// out = [NLL, grad(P), I, dI(P)].
__global__ __launch_bounds__(kFinalBlock) void tddp_finalize(DalitzConst dc, const DalitzTable* __restrict__ tab,
                                                             TddpTime tt, const double* __restrict__ coef,
                                                             const double* __restrict__ part, int64_t nrows, int nv,
                                                             int with_grad, const double* __restrict__ Mc,
                                                             double n_events, double* __restrict__ out,
                                                             double* __restrict__ out_user) {
  __shared__ TddpFinalLds L;
  const int K = dc.K;
  const int P = 4 * K + 2;
  const int t = threadIdx.x;
  // the three matrices and the coefficients are loaded first, by every thread
  // (clamped indices, values past the end discarded: no branch makes a wave
  // wait for them), so that their latency overlaps the row sums
  const int nm = 6 * K * K;
  double mv[(6 * kDalMaxRes * kDalMaxRes + kFinalBlock - 1) / kFinalBlock];
#pragma unroll
  for (int u = 0; u < (int)(sizeof(mv) / sizeof(mv[0])); ++u) {
    const int i = t + u * kFinalBlock;
    mv[u] = Mc[i < nm ? i : 0];
  }
  const int tc = t < K ? t : 0;
  const double c0 = coef[2 * tc], c1 = coef[2 * tc + 1], c2 = coef[2 * K + 2 * tc], c3 = coef[2 * K + 2 * tc + 1];
  // the same for the uniform values, as vector loads (a lane-varying zero
  // offset): scalar ones would be waited for before the rows are requested
  int zero = 0;
  asm volatile("" : "+v"(zero));
  const double x = coef[4 * K + zero], y = coef[4 * K + 1 + zero], valid = (&tab->valid)[zero];
  sum_rows_t<kFinalBlock>(part, nrows, nv, L.scratch, L.res);
#pragma unroll
  for (int u = 0; u < (int)(sizeof(mv) / sizeof(mv[0])); ++u) {
    const int i = t + u * kFinalBlock;
    if (i < nm) L.M[i] = mv[u];
  }
  if (t < K) {
    L.cre[t] = c0;
    L.cim[t] = c1;
    L.bre[t] = c2;
    L.bim[t] = c3;
  }
  __syncthreads();
  const double* MAA = L.M;
  const double* MBB = L.M + 2 * K * K;
  const double* MAB = L.M + 4 * K * K;
  if (t < K) {
    double xr = 0.0, xi = 0.0, br = 0.0, bi = 0.0, ur = 0.0, ui = 0.0, vr = 0.0, vi = 0.0;
    for (int j = 0; j < K; ++j) {
      // X_t = sum_j MAA_tj conj(c_j)
      const double mr = MAA[2 * (t * K + j)], mi = MAA[2 * (t * K + j) + 1];
      xr += mr * L.cre[j] + mi * L.cim[j];
      xi += mi * L.cre[j] - mr * L.cim[j];
      const double nr = MBB[2 * (t * K + j)], ni = MBB[2 * (t * K + j) + 1];
      br += nr * L.bre[j] + ni * L.bim[j];
      bi += ni * L.bre[j] - nr * L.bim[j];
      // U_t = sum_j MAB_tj cbar_j
      const double ar = MAB[2 * (t * K + j)], ai = MAB[2 * (t * K + j) + 1];
      ur += ar * L.bre[j] - ai * L.bim[j];
      ui += ar * L.bim[j] + ai * L.bre[j];
      // V_t = sum_i conj(c_i) MAB_it
      const double qr = MAB[2 * (j * K + t)], qi = MAB[2 * (j * K + t) + 1];
      vr += L.cre[j] * qr + L.cim[j] * qi;
      vi += L.cre[j] * qi - L.cim[j] * qr;
    }
    L.X[t][0] = xr; L.X[t][1] = xi;
    L.Xb[t][0] = br; L.Xb[t][1] = bi;
    L.U[t][0] = ur; L.U[t][1] = ui;
    L.V[t][0] = vr; L.V[t][1] = vi;
  }
  __syncthreads();
  if (t == 0) {
    double ia = 0.0, ib = 0.0, zr = 0.0, zi = 0.0;
    for (int k = 0; k < K; ++k) {
      ia += L.cre[k] * L.X[k][0] - L.cim[k] * L.X[k][1];   // Re(c_k X_k)
      ib += L.bre[k] * L.Xb[k][0] - L.bim[k] * L.Xb[k][1];
      zr += L.cre[k] * L.U[k][0] + L.cim[k] * L.U[k][1];   // conj(c_k) U_k
      zi += L.cre[k] * L.U[k][1] - L.cim[k] * L.U[k][0];
    }
    L.Ia = ia; L.Ib = ib; L.Zr = zr; L.Zi = zi;
  }
  __syncthreads();
  const double tau = 1.0 / tt.gamma;
  const double dy = 1.0 - y * y, dx = 1.0 + x * x;
  const double cy = tau / dy, cx = tau / dx;
  const double I = 0.5 * (cy * (L.Ia + L.Ib) + cx * (L.Ia - L.Ib) - 2.0 * y * cy * L.Zr - 2.0 * x * cx * L.Zi);
  const bool ok = valid != 0.0 && I > 0.0 && isfinite(I) && dy > 0.0;
  if (t == 0) {
    const double v = ok ? L.res[0] + n_events * log(I) : INFINITY;
    out[0] = v;
    out[1 + P] = I;
    if (out_user) out_user[0] = v;
  }
  if (t < P) {
    double dI;
    if (t < 2 * K) {
      const int k = t >> 1;
      dI = (t & 1) == 0 ? 0.5 * (2.0 * (cy + cx) * L.X[k][0] - 2.0 * y * cy * L.U[k][0] - 2.0 * x * cx * L.U[k][1])
                        : 0.5 * (-2.0 * (cy + cx) * L.X[k][1] - 2.0 * y * cy * L.U[k][1] + 2.0 * x * cx * L.U[k][0]);
    } else if (t < 4 * K) {
      const int k = (t - 2 * K) >> 1;
      dI = (t & 1) == 0 ? 0.5 * (2.0 * (cy - cx) * L.Xb[k][0] - 2.0 * y * cy * L.V[k][0] - 2.0 * x * cx * L.V[k][1])
                        : 0.5 * (-2.0 * (cy - cx) * L.Xb[k][1] + 2.0 * y * cy * L.V[k][1] - 2.0 * x * cx * L.V[k][0]);
    } else if (t == 4 * K) {
      const double dcx = -2.0 * x * tau / (dx * dx), dxcx = tau * (1.0 - x * x) / (dx * dx);
      dI = 0.5 * ((L.Ia - L.Ib) * dcx - 2.0 * L.Zi * dxcx);
    } else {
      const double dcy = 2.0 * y * tau / (dy * dy), dycy = tau * (1.0 + y * y) / (dy * dy);
      dI = 0.5 * ((L.Ia + L.Ib) * dcy - 2.0 * L.Zr * dycy);
    }
    out[2 + P + t] = dI;
    if (with_grad) {
      const double g = ok ? L.res[1 + t] + n_events * dI / I : NAN;
      out[1 + t] = g;
      if (out_user) out_user[1 + t] = g;
    }
  }
}

// ------------------------------------------------------------- launchers
void tddp_launch_copy_theta(const ParamBlock& pb, int P, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(tddp_copy_theta, dim3(1), dim3(kBlock), 0, s, pb, P, dst);
}

void tddp_launch_mmatrices(const TddpJit& j, const DalitzConst& dc, const DalitzTable* tab, int grid_chunk,
                           double* part, double* Mc, hipStream_t s) {
  const int64_t ncell = (int64_t)dc.nx * dc.ny;
  const int64_t nch = (ncell + grid_chunk - 1) / grid_chunk;
  const int K = dc.K;
  for (int w = 0; w < 3; ++w) {
    for (int i0 = 0; i0 < K; i0 += kMRowBlock) {
      DalitzConst c = dc;
      const DalitzTable* t = tab;
      int ch = grid_chunk, ii = i0;
      double* p = part;
      void* args[] = {&c, &t, &ch, &ii, &p};
      jit_launch(j.mrows[w], (unsigned)nch, kBlock, s, args);
      // the level-2 step of the three-body normalization matrix writes the
      // same layout (rows i0..i0+3, dA applied)
      dalitz_launch_mrows_finalize(dc, part, nch, i0, Mc + (int64_t)w * 2 * K * K, s);
    }
  }
}

void tddp_launch_gridmax(const TddpJit& j, const DalitzConst& dc, const DalitzTable* tab, const double* coef,
                         unsigned long long* vmax, hipStream_t s) {
  const int64_t ncell = (int64_t)dc.nx * dc.ny;
  const int64_t blocks = std::min<int64_t>((ncell + kBlock - 1) / kBlock, 4096);
  DalitzConst c = dc;
  const DalitzTable* t = tab;
  const double* cf = coef;
  unsigned long long* v = vmax;
  void* args[] = {&c, &t, &cf, &v};
  jit_launch(j.gmax, (unsigned)blocks, kBlock, s, args);
}

void tddp_launch_gen(const TddpJit& j, const DalitzConst& dc, const DalitzTable* tab, const double* coef,
                     const TddpTime& tt, uint32_t k0, uint32_t k1, int64_t n, double W, const double box[4],
                     int max_attempts, double* ev, int64_t ld, unsigned long long* bad, hipStream_t s) {
  if (n == 0) return;
  DalitzConst c = dc;
  const DalitzTable* t = tab;
  const double* cf = coef;
  TddpTime tm = tt;
  uint32_t a0 = k0, a1 = k1;
  int64_t nn = n, l = ld;
  double w = W, b0 = box[0], b1 = box[1], b2 = box[2], b3 = box[3];
  int ma = max_attempts;
  double* e = ev;
  unsigned long long* b = bad;
  void* args[] = {&c, &t, &cf, &tm, &a0, &a1, &nn, &w, &b0, &b1, &b2, &b3, &ma, &e, &l, &b};
  jit_launch(j.gen, (unsigned)((n + kBlock - 1) / kBlock), kBlock, s, args);
}

void tddp_launch_events(const TddpJit& j, const DalitzConst& dc, const DalitzTable* tab, const TddpTime& tt,
                        const double* coef, const double* ev, int64_t ld, int64_t n, int chunk, int64_t nchunks,
                        bool grad, double* part, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
  if (nchunks == 0) return;
  DalitzConst c = dc;
  const DalitzTable* t = tab;
  TddpTime tm = tt;
  const double* cf = coef;
  const double* e = ev;
  int64_t l = ld, nn = n;
  int ch = chunk;
  double* p = part;
  void* args[] = {&c, &t, &tm, &cf, &e, &l, &nn, &ch, &p};
  jit_launch(j.ev[grad ? 1 : 0], (unsigned)nchunks, kBlock, s, args, start, stop);
}

void tddp_launch_finalize(const DalitzConst& dc, const DalitzTable* tab, const TddpTime& tt, const double* coef,
                          const double* part, int64_t nrows, bool grad, const double* Mc, double n_events,
                          double* out, double* out_user, hipStream_t s) {
  hipLaunchKernelGGL(tddp_finalize, dim3(1), dim3(kFinalBlock), 0, s, dc, tab, tt, coef, part, nrows,
                     tddp_nv(dc.K, grad), grad ? 1 : 0, Mc, n_events, out, out_user);
}

}  // namespace fn
