// Three-body Dalitz-plot amplitude model (the paper's amplitude analyses of
// three-body decays, Sec. 1 and 5): host launchers, and the kernels that do
// not depend on the model's structure (prologue, level-2 finalize, per-event
// density, domain check).  The per-event, grid and normalization-matrix
// passes live in dalitz_device.hpp and are compiled at model creation with
// the model's structure as compile-time constants (dalitz_jit below).
#include <algorithm>
#include <cmath>
#include <sstream>
#include <vector>

#include "dalitz_device.hpp"
#include "internal.hpp"
#include "jit.hpp"
#include "kernels.hpp"

namespace fn {

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
    tab[f].coef[2 * k] = th[2 * k];
    tab[f].coef[2 * k + 1] = th[2 * k + 1];
    r[dDLNKA] = dlnka;
    r[dDKW_DM0] = kw * dlnkw;
    r[dKW_W0] = x * poly / q0pow;
    r[dTWOM0] = 2.0 * m0;
    if (!(m0 > 0.0) || !(w0 > 0.0) || !(lam > 0.0) || !isfinite(kw)) atomicOr(&bad, 1);
  }
  __syncthreads();
  if (k == 0) tab[f].valid = bad ? 0.0 : 1.0;
}

// ------------------------------------------------------------- finalize
// Arguments of the level-2 + NLL assembly step.
struct DalFinal {
  const double* npart;       // grid rows (free lineshapes) or nullptr (cached M)
  int64_t n_rows;
  int n_nv;
  const double* Mc;          // cached M (K x K complex) when npart == nullptr
  const double* coef;        // (Re c_k, Im c_k)
  double n_events;
  int with_grad;
  int norm_ready;            // the events pass wrote I and dI into out (cached M)
  double* out;               // [NLL, grad(P), I, dI(P)]
  double* out_user;          // optional [NLL, grad(P)]
  unsigned long long* span;  // span record of the measured events pass (or nullptr)
  int64_t span_blocks;       // workgroups of that pass
};

struct DalFinalLds {
  double scratch[kFinalBlock];
  double res[kBlock];
  double nres[kBlock];
  double cre[kDalMaxRes], cim[kDalMaxRes], ipart[kDalMaxRes];
  double dI[4 * kDalMaxRes];
  double M[2 * kDalMaxRes * kDalMaxRes];
  double I;
};
static_assert(2 * kDalMaxRes * kDalMaxRes <= kFinalBlock, "one entry of M per thread");

// Level-2 over the event rows and the normalization (grid rows or cached M),
// then NLL = -sum ln P~ + N ln I and its gradient, one thread per entry.
__device__ void dalitz_finalize_body(const DalitzConst& dc, const DalitzTable* __restrict__ tab,
                                     const double* __restrict__ evpart, int64_t ev_rows, int ev_nv, int kmax,
                                     const DalFinal& f, DalFinalLds& L) {
  const int K = dc.K;
  const int P = dc.free_ls ? 4 * K : 2 * K;
  const int t = threadIdx.x;
  // the small inputs are loaded first, so that their latency overlaps the row
  // sums, in forms that make no wave wait for them before the rows are
  // requested (a zero written before a load; I and dI loaded by every thread
  // at a clamped index and used only where t <= P)
  const bool own_norm = !f.npart && !f.norm_ready;
  double mv = 0.0, cv = 0.0;
  if (own_norm && t < 2 * K * K) mv = f.Mc[t];
  if (own_norm && t < 2 * K) cv = f.coef[t];
  const double nrm = f.out[1 + P + (t <= P ? t : P)];  // I, then dI
  // the validity flag as a vector load (lane-varying zero offset): a scalar
  // one would be waited for with the kernel arguments, before the rows
  int zero = 0;
  asm volatile("" : "+v"(zero));
  const double valid = (&tab->valid)[zero];
  sum_rows_t<kFinalBlock>(evpart, ev_rows, ev_nv, L.scratch, L.res);
  if (f.npart) sum_rows_t<kFinalBlock>(f.npart, f.n_rows, f.n_nv, L.scratch, L.nres);
  if (f.norm_ready) {
    // I and dI from the events pass
    if (t == 0) L.I = nrm;
    if (t >= 1 && t <= P) L.dI[t - 1] = nrm;
    __syncthreads();
  } else {
    if (t < 2 * K * K) L.M[t] = mv;
    if (t < 2 * K) (t & 1 ? L.cim : L.cre)[t >> 1] = cv;
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
        const double mr = L.M[2 * (t * K + j)], mi = L.M[2 * (t * K + j) + 1];
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
  }
  const double I = L.I;
  const bool okI = valid != 0.0 && I > 0.0 && isfinite(I);
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

// Level-2 step: one workgroup.
__global__ __launch_bounds__(kFinalBlock) void dalitz_finalize(DalitzConst dc, const DalitzTable* __restrict__ tab,
                                                          const double* __restrict__ evpart, int64_t ev_rows,
                                                          int ev_nv, int kmax, DalFinal fin) {
  __shared__ DalFinalLds L;
  unsigned long long lo = 0, hi = 0;
  if (fin.span) span_load<kFinalBlock>(fin.span, fin.span_blocks, lo, hi);
  dalitz_finalize_body(dc, tab, evpart, ev_rows, ev_nv, kmax, fin, L);
  if (fin.span) span_add<kFinalBlock>(fin.span, fin.span_blocks, lo, hi, L.scratch);
}

// Pre-summation of long row sets (before the level-2 step, which then reads
// one row per workgroup here instead of all of them through one compute
// unit): workgroup b < s0 adds rows [b R, (b+1) R) of set 0 in row order into
// row b of o0, the others the same for set 1.
__global__ __launch_bounds__(kBlock) void rows_presum(const double* __restrict__ p0, int64_t n0, int nv0,
                                                      double* __restrict__ o0, int64_t s0,
                                                      const double* __restrict__ p1, int64_t n1, int nv1,
                                                      double* __restrict__ o1, int rows_per_block) {
  __shared__ double scratch[kBlock];
  __shared__ double res[kBlock];
  const int64_t b = blockIdx.x;
  const bool first = b < s0;
  const int64_t bb = first ? b : b - s0;
  const double* p = first ? p0 : p1;
  const int64_t n = first ? n0 : n1;
  const int nv = first ? nv0 : nv1;
  const int64_t r0 = bb * rows_per_block;
  const int64_t rr = n - r0 < rows_per_block ? n - r0 : rows_per_block;
  sum_rows_t<kBlock>(p + r0 * nv, rr, nv, scratch, res);
  if ((int)threadIdx.x < nv) (first ? o0 : o1)[bb * nv + threadIdx.x] = res[threadIdx.x];
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

// The grid cells inside the region, per column ix (s12): counted, then
// listed in column-major order at the offsets of the counts' prefix sums;
// the same predicate and cell centres as every grid pass.
__global__ void dalitz_grid_count(DalitzConst dc, int32_t* __restrict__ cnt) {
  const int64_t ix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ix >= dc.nx) return;
  const double s12 = grid_centre(dc.a12, ix, dc.d12);
  double lo, hi;
  dalitz_row_bounds(dc, s12, lo, hi);
  int32_t c = 0;
  for (int64_t iy = 0; iy < dc.ny; ++iy) c += dalitz_in_row(dc, s12, grid_centre(dc.a13, iy, dc.d13), lo, hi);
  cnt[ix] = c;
}

__global__ void dalitz_grid_fill(DalitzConst dc, const int64_t* __restrict__ off, GridCell* __restrict__ cells) {
  const int64_t ix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ix >= dc.nx) return;
  const double s12 = grid_centre(dc.a12, ix, dc.d12);
  double lo, hi;
  dalitz_row_bounds(dc, s12, lo, hi);
  int64_t o = off[ix];
  const int64_t end = off[ix + 1];
  for (int64_t iy = 0; iy < dc.ny && o < end; ++iy)
    if (dalitz_in_row(dc, s12, grid_centre(dc.a13, iy, dc.d13), lo, hi)) cells[o++] = GridCell{(int32_t)ix, (int32_t)iy};
}

// ---------------------------------------------------------------- launchers
int64_t dalitz_build_grid_cells(const DalitzConst& dc, DevBuf& cells, hipStream_t s) {
  const int64_t nx = dc.nx;
  DevBuf d_cnt, d_off;
  d_cnt.reserve(sizeof(int32_t) * nx);
  d_off.reserve(sizeof(int64_t) * (nx + 1));
  const unsigned blocks = (unsigned)((nx + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(dalitz_grid_count, dim3(blocks), dim3(kBlock), 0, s, dc, (int32_t*)d_cnt.ptr);
  hip_check(hipGetLastError(), "dalitz_grid_count");
  std::vector<int32_t> cnt(nx);
  hip_check(hipMemcpyAsync(cnt.data(), d_cnt.ptr, sizeof(int32_t) * nx, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  std::vector<int64_t> off(nx + 1, 0);
  for (int64_t i = 0; i < nx; ++i) off[i + 1] = off[i] + cnt[i];
  const int64_t n_in = off[nx];
  cells.reserve(sizeof(GridCell) * (size_t)(n_in > 0 ? n_in : 1));
  if (n_in > 0) {
    hip_check(hipMemcpyAsync(d_off.ptr, off.data(), sizeof(int64_t) * (nx + 1), hipMemcpyHostToDevice, s),
              "hipMemcpyAsync");
    hipLaunchKernelGGL(dalitz_grid_fill, dim3(blocks), dim3(kBlock), 0, s, dc, (const int64_t*)d_off.ptr,
                       (GridCell*)cells.ptr);
    hip_check(hipGetLastError(), "dalitz_grid_fill");
  }
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  return n_in;
}

int dalitz_kmax(int K) { return K; }  // partial rows hold exactly the model's resonances
int dalitz_nv_events(int kmax, int grad) { return dal_nv(kEvents, grad, kmax); }
int dalitz_nv_mrows(int kmax) { return dal_nv(kMRows, 0, kmax); }

void dalitz_launch_prologue(const DalitzConst& dc, const ParamBlock& pb, const double* theta_dev,
                            const double* fixed_ls, int n_fits, int theta_stride, DalitzTable* tab, hipStream_t s) {
  hipLaunchKernelGGL(dalitz_prologue, dim3(n_fits), dim3(64), 0, s, dc, pb, theta_dev, fixed_ls, n_fits,
                     theta_stride, tab);
}

// Source of the structure-specialized passes of a model: the shape (K, pair
// and spin of every resonance) as compile-time constants, then the kernels the
// model uses (fixed lineshapes: events without and with the coefficient
// gradient, the M rows; free lineshapes: events and grid without and with the
// full gradient).  ept = 2: only the events passes, with two events per
// thread and loop iteration (each thread still adds its events in index
// order, so the sums are bitwise those of the one-event form).
std::string dalitz_jit_source(const DalitzConst& dc, int ept) {
  std::ostringstream o;
  o << "#include \"dalitz_device.hpp\"\n";
  o << "struct fn_shape {\n  static constexpr int K = " << dc.K << ";\n  static constexpr int chan[" << dc.K
    << "] = {";
  for (int k = 0; k < dc.K; ++k) o << (k ? ", " : "") << dc.chan[k];
  o << "};\n  static constexpr int L[" << dc.K << "] = {";
  for (int k = 0; k < dc.K; ++k) o << (k ? ", " : "") << dc.L[k];
  o << "};\n};\n";
  if (ept == 2) {
    o << "FN_DALITZ_KERNEL(fn_dal_ev0, fn_shape, fn::kEvents, 0, 2)\n";
    if (!dc.free_ls) o << "FN_DALITZ_KERNEL(fn_dal_ev1, fn_shape, fn::kEvents, 1, 2)\n";
    else o << "FN_DALITZ_KERNEL(fn_dal_ev2, fn_shape, fn::kEvents, 2, 2)\n";
    return o.str();
  }
  if (!dc.free_ls) {
    o << "FN_DALITZ_KERNEL(fn_dal_ev0, fn_shape, fn::kEvents, 0, 1)\n"
         "FN_DALITZ_KERNEL(fn_dal_ev1, fn_shape, fn::kEvents, 1, 1)\n"
         "FN_DALITZ_KERNEL(fn_dal_mrows, fn_shape, fn::kMRows, 0, 1)\n";
  } else {
    o << "FN_DALITZ_KERNEL(fn_dal_ev0, fn_shape, fn::kEvents, 0, 1)\n"
         "FN_DALITZ_KERNEL(fn_dal_ev2, fn_shape, fn::kEvents, 2, 1)\n"
         "FN_DALITZ_KERNEL(fn_dal_gr0, fn_shape, fn::kGrid, 0, 1)\n"
         "FN_DALITZ_KERNEL(fn_dal_gr2, fn_shape, fn::kGrid, 2, 1)\n";
  }
  o << "FN_DALITZ_GEN(fn_dal_gmax, fn_dal_gen, fn_shape)\n";
  return o.str();
}

std::shared_ptr<DalitzJit> dalitz_jit(const DalitzConst& dc, int ept) {
  auto j = std::make_shared<DalitzJit>();
  std::vector<std::string> names;
  if (ept == 2) {
    names = {"fn_dal_ev0", dc.free_ls ? "fn_dal_ev2" : "fn_dal_ev1"};
    j->prog = jit_load(dalitz_jit_source(dc, 2), names);
    j->ev[0] = j->prog->fns[0];
    j->ev[dc.free_ls ? 2 : 1] = j->prog->fns[1];
    return j;
  }
  if (!dc.free_ls) names = {"fn_dal_ev0", "fn_dal_ev1", "fn_dal_mrows"};
  else names = {"fn_dal_ev0", "fn_dal_ev2", "fn_dal_gr0", "fn_dal_gr2"};
  const size_t ngen = names.size();
  names.push_back("fn_dal_gmax");
  names.push_back("fn_dal_gen");
  j->prog = jit_load(dalitz_jit_source(dc, 1), names);
  const auto& f = j->prog->fns;
  if (!dc.free_ls) {
    j->ev[0] = f[0];
    j->ev[1] = f[1];
    j->mrows = f[2];
  } else {
    j->ev[0] = f[0];
    j->ev[2] = f[1];
    j->gr[0] = f[2];
    j->gr[2] = f[3];
  }
  j->gmax = f[ngen];
  j->gen = f[ngen + 1];
  return j;
}

static void launch_pass(hipFunction_t f, const DalitzConst& dc, const DalitzTable* tab, const double* coef,
                        const double* ev, int64_t ld, int64_t n, int chunk, int64_t nchunks, int i0, double* part,
                        hipStream_t s, const double* Mc = nullptr, double* norm_out = nullptr,
                        hipEvent_t start = nullptr, hipEvent_t stop = nullptr,
                        unsigned long long* span = nullptr) {
  if (!f) throw Error(FN_E_INVALID, "this model was not compiled with the requested pass");
  DalitzConst c = dc;
  const DalitzTable* t = tab;
  const double* cf = coef;
  const double* e = ev;
  int64_t l = ld, nn = n;
  int ch = chunk, ii = i0;
  double* p = part;
  const double* m = Mc;
  double* no = norm_out;
  unsigned long long* sp = span;
  void* args[] = {&c, &t, &cf, &e, &l, &nn, &ch, &ii, &p, &m, &no, &sp};
  jit_launch(f, (unsigned)nchunks, kBlock, s, args, start, stop);
}

static DalFinal make_final(const double* npart, int64_t n_rows, int n_nv, const double* Mc, const double* coef,
                           double n_events, bool grad, bool norm_ready, double* out, double* out_user) {
  DalFinal f;
  f.span = nullptr;
  f.span_blocks = 0;
  f.norm_ready = norm_ready ? 1 : 0;
  f.npart = npart;
  f.n_rows = n_rows;
  f.n_nv = n_nv;
  f.Mc = Mc;
  f.coef = coef;
  f.n_events = n_events;
  f.with_grad = grad ? 1 : 0;
  f.out = out;
  f.out_user = out_user;
  return f;
}

void dalitz_launch_events(const DalitzJit& j, const DalitzConst& dc, const DalitzTable* tab, const double* coef,
                          const double* ev, int64_t ld, int64_t n, int chunk, int64_t nchunks, int grad, double* part,
                          hipStream_t s, const double* Mc, double* out, hipEvent_t start, hipEvent_t stop,
                          unsigned long long* span) {
  if (nchunks == 0) return;
  const int P = dc.free_ls ? 4 * dc.K : 2 * dc.K;
  launch_pass(j.ev[grad], dc, tab, coef, ev, ld, n, chunk, nchunks, 0, part, s, Mc,
              Mc && out ? out + 1 + P : nullptr, start, stop, span);
}

int64_t presum_blocks(int64_t rows, int nv, int64_t other_rows, int other_nv) {
  const int64_t bytes = 8 * (rows * nv + other_rows * other_nv);
  return bytes > kPresumMinBytes ? (rows + kPresumRows - 1) / kPresumRows : 0;
}

void launch_rows_presum(const double* p0, int64_t n0, int nv0, double* o0, int64_t s0, const double* p1, int64_t n1,
                        int nv1, double* o1, int64_t s1, hipStream_t s) {
  if (s0 + s1 == 0) return;
  hipLaunchKernelGGL(rows_presum, dim3((unsigned)(s0 + s1)), dim3(kBlock), 0, s, p0, n0, nv0, o0, s0, p1, n1, nv1, o1,
                     kPresumRows);
}

void dalitz_launch_finalize(const DalitzConst& dc, const DalitzTable* tab, const double* coef, double* evpart,
                            int64_t ev_rows, int grad, double* npart, int64_t n_rows, int n_nv,
                            const double* Mc, double n_events, double* out, double* out_user, hipStream_t s,
                            bool norm_ready, unsigned long long* span) {
  const int kmax = dalitz_kmax(dc.K);
  const int ev_nv = dal_nv(kEvents, grad, kmax);
  const int64_t span_blocks = ev_rows;
  // long row sets: pre-summed by many workgroups into the room the caller
  // left after each set's rows
  const int64_t se = presum_blocks(ev_rows, ev_nv, npart ? n_rows : 0, n_nv);
  if (se > 0) {
    const int64_t sg = npart ? presum_blocks(n_rows, n_nv, ev_rows, ev_nv) : 0;
    double* ev_red = evpart + ev_rows * ev_nv;
    double* n_red = npart ? npart + n_rows * n_nv : nullptr;
    launch_rows_presum(evpart, ev_rows, ev_nv, ev_red, se, npart, n_rows, n_nv, n_red, sg, s);
    evpart = ev_red;
    ev_rows = se;
    if (npart) {
      npart = n_red;
      n_rows = sg;
    }
  }
  DalFinal fin = make_final(npart, n_rows, n_nv, Mc, coef, n_events, grad != 0, norm_ready && !npart, out,
                            out_user);
  fin.span = span;
  fin.span_blocks = span_blocks;
  hipLaunchKernelGGL(dalitz_finalize, dim3(1), dim3(kFinalBlock), 0, s, dc, tab, evpart, ev_rows, ev_nv, kmax,
                     fin);
}

void dalitz_launch_grid(const DalitzJit& j, const DalitzConst& dc, const DalitzTable* tab, const double* coef,
                        const GridCell* cells, int64_t n_inside, int chunk, int64_t nchunks, int grad, double* part,
                        hipStream_t s) {
  launch_pass(j.gr[grad], dc, tab, coef, reinterpret_cast<const double*>(cells), 0, n_inside, chunk, nchunks, 0,
              part, s);
}

void dalitz_launch_mrows(const DalitzJit& j, const DalitzConst& dc, const DalitzTable* tab, int chunk,
                         int64_t nchunks, int i0, double* part, double* Mc, hipStream_t s) {
  const int64_t ncell = (int64_t)dc.nx * dc.ny;
  launch_pass(j.mrows, dc, tab, nullptr, nullptr, 0, ncell, chunk, nchunks, i0, part, s);
  dalitz_launch_mrows_finalize(dc, part, nchunks, i0, Mc, s);
}

void dalitz_launch_mrows_finalize(const DalitzConst& dc, const double* part, int64_t nchunks, int i0, double* Mc,
                                  hipStream_t s) {
  const int kmax = dalitz_kmax(dc.K);
  hipLaunchKernelGGL(dalitz_mrows_finalize, dim3(1), dim3(kBlock), 0, s, dc, part, nchunks,
                     dal_nv(kMRows, 0, kmax), kmax, i0, Mc);
}

void dalitz_launch_gridmax(const DalitzJit& j, const DalitzConst& dc, const DalitzTable* tab,
                           unsigned long long* vmax, hipStream_t s) {
  const int64_t ncell = (int64_t)dc.nx * dc.ny;
  const int64_t blocks = std::min<int64_t>((ncell + kBlock - 1) / kBlock, 4096);
  DalitzConst c = dc;
  const DalitzTable* t = tab;
  unsigned long long* v = vmax;
  void* args[] = {&c, &t, &v};
  jit_launch(j.gmax, (unsigned)blocks, kBlock, s, args);
}

void dalitz_launch_gen(const DalitzJit& j, const DalitzConst& dc, const DalitzTable* tab, uint32_t k0, uint32_t k1,
                       int64_t n, double W, const double box[4], int max_attempts, double* ev, int64_t ld,
                       unsigned long long* bad, hipStream_t s) {
  if (n == 0) return;
  DalitzConst c = dc;
  const DalitzTable* t = tab;
  uint32_t a0 = k0, a1 = k1;
  int64_t nn = n, l = ld;
  double w = W, b0 = box[0], b1 = box[1], b2 = box[2], b3 = box[3];
  int ma = max_attempts;
  double* e = ev;
  unsigned long long* b = bad;
  void* args[] = {&c, &t, &a0, &a1, &nn, &w, &b0, &b1, &b2, &b3, &ma, &e, &l, &b};
  jit_launch(j.gen, (unsigned)((n + kBlock - 1) / kBlock), kBlock, s, args);
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
