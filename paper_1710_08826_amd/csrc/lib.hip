// C ABI of libfitnll: contexts, the model compiler (JSON description ->
// constant structs + device buffers), and the NLL pipeline
//   prologue (theta -> table) -> normalization -> events pass -> finalize.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fitnll.h"
#include "internal.hpp"
#include "jit.hpp"
#include "json.hpp"
#include "kernels.hpp"

namespace fn {

// Device toy generation by model: envelope = this factor x the largest density
// on the integration grid when the caller gives none; attempts per event.
constexpr double kGenEnvelopeFactor = 1.2;
constexpr int kGenMaxAttemptsModel = 4096;
constexpr int kGenMaxAttemptsTd4 = 65536;  // four-body model acceptance is near 1e-3 per attempt
// First counter stream of the four-body phase-space sample (the sample of
// fn_model_generate_norm_sample is that of the input sampler's default).
constexpr uint32_t kPhaseSpaceStream0 = 100;

// Chunk sizes (events per workgroup) tried by fn_model_autotune: the powers
// of two 256 .. 16384, then the chunks (multiples of 256) that give j times
// as many workgroups as the device has compute units, j = 1 .. 8 -- counts
// that fill the resident workgroup slots evenly, without a partly filled last
// round (a pass of 1221 workgroups at two per compute unit runs 2.4 rounds
// on 256 compute units) -- where they differ from the first ones.
constexpr int kTunePow2 = 7;
constexpr int kTuneMultiples = 8;
constexpr int kMaxChunk = 1 << 22;
static_assert(kTunePow2 + kTuneMultiples <= FN_TUNE_MAX, "candidate table");
constexpr double kTuneTie = 0.02;  // relative time difference treated as a tie

static int tune_candidates(int64_t n, int cus, int32_t* out) {
  int c = 0;
  for (int k = 0; k < kTunePow2; ++k) out[c++] = 256 << k;
  for (int j = 1; j <= kTuneMultiples; ++j) {
    const int64_t per = (n + (int64_t)j * cus - 1) / ((int64_t)j * cus);
    int64_t ch = (per + 255) / 256 * 256;
    ch = ch < 256 ? 256 : (ch > kMaxChunk ? kMaxChunk : ch);
    bool seen = false;
    for (int i = 0; i < c; ++i) seen = seen || out[i] == (int32_t)ch;
    if (!seen) out[c++] = (int32_t)ch;
  }
  return c;
}

// Scratch of the allocation-free NLL entry point (fn_nll_async_noalloc): the
// partial rows of one call, 2^21 doubles (16 MiB) on every device the library
// runs on, held until the process ends.  In host code `scratch` names a
// host-side stand-in; kernels get this device's address, taken once per
// device when its context is created.
constexpr size_t kScratchDoubles = size_t(1) << 21;
static __device__ __align__(256) double scratch[kScratchDoubles];

void hip_check(hipError_t e, const char* what);

// Device address of `scratch` on the current device (looked up on first use).
static double* scratch_address(int device) {
  static std::mutex mu;
  static std::vector<double*> addr;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= device) addr.resize((size_t)device + 1, nullptr);
  if (!addr[device]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) throw Error(FN_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    addr[device] = (double*)p;
  }
  return addr[device];
}

static thread_local std::string g_last_error;

void set_error(const std::string& s) { g_last_error = s; }
void clear_error() { g_last_error.clear(); }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(FN_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

fn_status guard(const std::function<void()>& body) {
  clear_error();
  try {
    body();
    return FN_OK;
  } catch (const Error& e) {
    set_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return FN_E_NOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return FN_E_INVALID;
  }
}

// ------------------------------------------------------------ device buffer
void DevBuf::reserve(size_t nbytes) {
  if (nbytes <= bytes) return;
  if (ptr) hip_check(hipFree(ptr), "hipFree");
  ptr = nullptr;
  bytes = 0;
  const size_t want = nbytes < 256 ? 256 : nbytes;
  if (hipMalloc(&ptr, want) != hipSuccess) {
    ptr = nullptr;
    (void)hipGetLastError();
    throw Error(FN_E_NOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  bytes = want;
}
void DevBuf::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

// ------------------------------------------------------------ model compiler

static void compile_mix1d(const json::Value& d, fn_model* m) {
  Mix1dConst& mc = m->mix;
  std::memset(&mc, 0, sizeof(mc));
  mc.lo = d.at("lo").number();
  mc.hi = d.at("hi").number();
  if (!(mc.hi > mc.lo)) throw Error(FN_E_INVALID, "mix1d: need hi > lo");
  const auto& comps = d.at("components").array();
  mc.K = (int)comps.size();
  if (mc.K < 1 || mc.K > kMixMaxComp) throw Error(FN_E_INVALID, "mix1d: 1..8 components");
  int maxidx = -1;
  for (int k = 0; k < mc.K; ++k) {
    const std::string& t = comps[k].at("type").string();
    const auto& ps = comps[k].at("params").array();
    int need;
    if (t == "gauss") { mc.type[k] = kGauss; need = 2; }
    else if (t == "exp") { mc.type[k] = kExp; need = 1; }
    else if (t == "argus") { mc.type[k] = kArgus; need = 2; }
    else if (t == "bw") { mc.type[k] = kBW; need = 2; }
    else throw Error(FN_E_INVALID, "mix1d: unknown component type \"" + t + "\"");
    if ((int)ps.size() != need) throw Error(FN_E_INVALID, "mix1d: wrong parameter count for " + t);
    if (mc.type[k] == kArgus && mc.lo < 0.0) throw Error(FN_E_INVALID, "mix1d: argus needs lo >= 0");
    mc.npar[k] = need;
    for (int j = 0; j < need; ++j) {
      const long idx = ps[j].integer();
      if (idx < 0 || idx >= kMaxParams) throw Error(FN_E_INVALID, "mix1d: parameter index out of range");
      mc.pidx[k][j] = (int)idx;
      if (idx > maxidx) maxidx = (int)idx;
    }
  }
  const auto& fr = d.has("fracs") ? d.at("fracs").array() : std::vector<json::Value>();
  if ((int)fr.size() != mc.K - 1) throw Error(FN_E_INVALID, "mix1d: need K-1 fractions");
  for (int k = 0; k < mc.K - 1; ++k) {
    const long idx = fr[k].integer();
    if (idx < 0 || idx >= kMaxParams) throw Error(FN_E_INVALID, "mix1d: fraction index out of range");
    mc.fidx[k] = (int)idx;
    if (idx > maxidx) maxidx = (int)idx;
  }
  int P = maxidx + 1;
  if (d.has("n_params")) {
    const long np = d.at("n_params").integer();
    if (np < P || np > kMaxParams) throw Error(FN_E_INVALID, "mix1d: n_params smaller than the indices used");
    P = (int)np;
  }
  mc.yidx = -1;
  if (d.has("yield")) {
    const long idx = d.at("yield").integer();
    if (idx < 0 || idx >= kMaxParams) throw Error(FN_E_INVALID, "mix1d: yield index out of range");
    mc.yidx = (int)idx;
    if (idx + 1 > P) P = (int)idx + 1;
    if (d.has("n_params") && d.at("n_params").integer() < idx + 1)
      throw Error(FN_E_INVALID, "mix1d: n_params smaller than the indices used");
  }
  mc.n_params = P;
  m->P = P;
  m->n_obs = 1;
  m->chunk = 1024;  // measured on MI355X for 1e5 events (512: +30%, 2048: same)
  m->d_table.reserve(sizeof(Mix1dTable));
}

static void compile_dalitz3(const json::Value& d, fn_model* m, bool device = true) {
  DalitzConst& dc = m->dal;
  std::memset(&dc, 0, sizeof(dc));
  const double M = d.at("M").number();
  const auto& ms = d.at("m").array();
  if (ms.size() != 3) throw Error(FN_E_INVALID, "dalitz3: need three daughter masses");
  const double mm[4] = {M, ms[0].number(), ms[1].number(), ms[2].number()};
  if (!(M > mm[1] + mm[2] + mm[3]) || !(mm[1] > 0) || !(mm[2] > 0) || !(mm[3] > 0))
    throw Error(FN_E_INVALID, "dalitz3: masses must be positive and M > m1 + m2 + m3");
  const double rr = d.has("r_res") ? d.at("r_res").number() : 1.5;
  const double rd = d.has("r_D") ? d.at("r_D").number() : 5.0;
  dc.M2 = M * M;
  dc.m1s = mm[1] * mm[1];
  dc.m2s = mm[2] * mm[2];
  dc.m3s = mm[3] * mm[3];
  dc.msum = M * M + mm[1] * mm[1] + mm[2] * mm[2] + mm[3] * mm[3];
  dc.r2 = rr * rr;
  dc.rD2 = rd * rd;
  long nx = 1024, ny = 1024;
  if (d.has("grid")) {
    const auto& g = d.at("grid").array();
    if (g.size() != 2) throw Error(FN_E_INVALID, "dalitz3: grid must be [nx, ny]");
    nx = g[0].integer();
    ny = g[1].integer();
  }
  if (nx < 1 || ny < 1 || nx * ny > (1L << 30)) throw Error(FN_E_INVALID, "dalitz3: bad grid size");
  dc.nx = (int)nx;
  dc.ny = (int)ny;
  dc.a12 = (mm[1] + mm[2]) * (mm[1] + mm[2]);
  dc.d12 = ((M - mm[3]) * (M - mm[3]) - dc.a12) / nx;
  dc.a13 = (mm[1] + mm[3]) * (mm[1] + mm[3]);
  dc.d13 = ((M - mm[2]) * (M - mm[2]) - dc.a13) / ny;
  dc.dA = dc.d12 * dc.d13;
  m->box[0] = dc.a12;
  m->box[1] = (M - mm[3]) * (M - mm[3]);
  m->box[2] = dc.a13;
  m->box[3] = (M - mm[2]) * (M - mm[2]);
  // pairs: 0 = "12" (A,B,C) = (1,2,3); 1 = "13" (1,3,2); 2 = "23" (2,3,1)
  const int who[3][3] = {{1, 2, 3}, {1, 3, 2}, {2, 3, 1}};
  for (int c = 0; c < 3; ++c) {
    DalitzChan& ch = dc.ch[c];
    const double mA = mm[who[c][0]], mB = mm[who[c][1]], mC = mm[who[c][2]];
    ch.mA2 = mA * mA;
    ch.mB2 = mB * mB;
    ch.mC2 = mC * mC;
    ch.sum2 = (mA + mB) * (mA + mB);
    ch.dif2 = (mA - mB) * (mA - mB);
    ch.Psum2 = (M + mC) * (M + mC);
    ch.Pdif2 = (M - mC) * (M - mC);
    ch.zc = (M * M - mC * mC) * (mB * mB - mA * mA);
  }
  dc.free_ls = d.has("free_lineshapes") ? (d.at("free_lineshapes").boolean() ? 1 : 0) : 0;
  const auto& res = d.at("resonances").array();
  dc.K = (int)res.size();
  if (dc.K < 1 || dc.K > kDalMaxRes) throw Error(FN_E_INVALID, "dalitz3: 1..16 resonances");
  m->fixed_ls.assign(2 * dc.K, 0.0);
  for (int k = 0; k < dc.K; ++k) {
    const std::string& p = res[k].at("pair").string();
    int c;
    if (p == "12") c = 0;
    else if (p == "13") c = 1;
    else if (p == "23") c = 2;
    else throw Error(FN_E_INVALID, "dalitz3: pair must be \"12\", \"13\" or \"23\"");
    const long L = res[k].at("L").integer();
    if (L < 0 || L > 2) throw Error(FN_E_INVALID, "dalitz3: L must be 0, 1 or 2");
    dc.chan[k] = c;
    dc.L[k] = (int)L;
    dc.ch[c].useL[L] = 1;
    m->fixed_ls[2 * k] = res[k].at("m0").number();
    m->fixed_ls[2 * k + 1] = res[k].at("w0").number();
  }
  m->P = dc.free_ls ? 4 * dc.K : 2 * dc.K;
  m->n_obs = 2;
  // measured on MI355X with the structure-specialized kernels: 2048 events per
  // workgroup is fastest for the coefficient gradient (17 sums per row) at 1M
  // events, 4096 amortises the 33-sum rows of free lineshapes
  m->chunk = dc.free_ls ? 4096 : 2048;
  m->grid_chunk = 1024;
  if (!device) return;
  m->dal_jit = dalitz_jit(dc);
  // free lineshapes: the grid passes walk the list of the inside cells
  if (dc.free_ls) m->n_inside = dalitz_build_grid_cells(dc, m->d_cells, nullptr);
  m->d_table.reserve(sizeof(DalitzTable));
  m->d_fixed.reserve(sizeof(double) * 2 * dc.K);
  hip_check(hipMemcpy(m->d_fixed.ptr, m->fixed_ls.data(), sizeof(double) * 2 * dc.K, hipMemcpyHostToDevice),
            "hipMemcpy");
  m->d_M.reserve(sizeof(double) * 2 * dc.K * dc.K);
}

static void compile_tddp3(const json::Value& d, fn_model* m, bool device = true) {
  if (d.has("free_lineshapes") && d.at("free_lineshapes").boolean())
    throw Error(FN_E_INVALID, "tddp3: the lineshapes are fixed");
  compile_dalitz3(d, m, false);  // kinematics, grid and resonances of the three-body model
  const auto& ms = d.at("m").array();
  if (ms[1].number() != ms[2].number())
    throw Error(FN_E_INVALID, "tddp3: daughters 2 and 3 must be charge conjugates (equal masses)");
  const DalitzConst& dc = m->dal;
  if (dc.nx != dc.ny) throw Error(FN_E_INVALID, "tddp3: the grid must be square (nx == ny)");
  const double tau = d.at("tau").number(), sig = d.at("sigma_t").number();
  if (!(tau > 0.0) || !(sig > 0.0)) throw Error(FN_E_INVALID, "tddp3: need tau > 0 and sigma_t > 0");
  m->tdt.gamma = 1.0 / tau;
  m->tdt.sigma = sig;
  td4_weideman_coefficients(m->tdt.wa, &m->tdt.wL);
  m->P = 4 * dc.K + 2;
  m->n_obs = 3;
  // the autotuner's choice on MI355X at 1M events (1024: 90.5 us, 2048: 83.9, 4096: 80.2, 8192: 130)
  m->chunk = 4096;
  if (!device) return;
  m->tddp_jit = tddp_jit(dc);
  m->d_table.reserve(sizeof(DalitzTable));
  m->d_fixed.reserve(sizeof(double) * 2 * dc.K);
  hip_check(hipMemcpy(m->d_fixed.ptr, m->fixed_ls.data(), sizeof(double) * 2 * dc.K, hipMemcpyHostToDevice),
            "hipMemcpy");
  m->d_M.reserve(sizeof(double) * 6 * dc.K * dc.K);
  m->d_theta.reserve(sizeof(double) * m->P);
}

int td4_n_fixed(const Td4Const& tc) { return 2 * (tc.n12 + tc.n34) + 1; }

Td4FitConst td4_fit_const(const Td4Const& tc, const double* fixed) {
  Td4FitConst fc;
  std::memset(&fc, 0, sizeof(fc));
  const double lo12 = std::sqrt(tc.sum12), lo34 = std::sqrt(tc.sum34);
  for (int r = 0; r < tc.n12; ++r) {
    fc.m0_12[r] = fixed[2 * r];
    fc.w0_12[r] = fixed[2 * r + 1];
    if (!tc.nr12[r] && !(fc.m0_12[r] > lo12 && fc.w0_12[r] > 0.0 && std::isfinite(fc.m0_12[r] + fc.w0_12[r])))
      throw Error(FN_E_INVALID, "td4: r12 resonance " + std::to_string(r) + " needs m0 > m1 + m2 and w0 > 0");
  }
  const double* f34 = fixed + 2 * tc.n12;
  for (int r = 0; r < tc.n34; ++r) {
    fc.m0_34[r] = f34[2 * r];
    fc.w0_34[r] = f34[2 * r + 1];
    if (!tc.nr34[r] && !(fc.m0_34[r] > lo34 && fc.w0_34[r] > 0.0 && std::isfinite(fc.m0_34[r] + fc.w0_34[r])))
      throw Error(FN_E_INVALID, "td4: r34 resonance " + std::to_string(r) + " needs m0 > m3 + m4 and w0 > 0");
  }
  fc.sigma = fixed[2 * (tc.n12 + tc.n34)];
  if (!(fc.sigma > 0.0) || !std::isfinite(fc.sigma)) throw Error(FN_E_INVALID, "td4: sigma_t must be > 0");
  return fc;
}

static void compile_td4(const json::Value& d, fn_model* m, bool device = true) {
  Td4Const& tc = m->td4;
  std::memset(&tc, 0, sizeof(tc));
  const double M = d.at("M").number();
  const auto& ms = d.at("m").array();
  if (ms.size() != 4) throw Error(FN_E_INVALID, "td4: need four daughter masses");
  double mm[4];
  for (int i = 0; i < 4; ++i) mm[i] = ms[i].number();
  if (!(mm[0] > 0 && mm[1] > 0 && mm[2] > 0 && mm[3] > 0) || !(M > mm[0] + mm[1] + mm[2] + mm[3]))
    throw Error(FN_E_INVALID, "td4: masses must be positive and M > m1 + m2 + m3 + m4");
  tc.M = M;
  tc.m1 = mm[0];
  tc.m2 = mm[1];
  tc.m3 = mm[2];
  tc.m4 = mm[3];
  tc.m1s = mm[0] * mm[0];
  tc.m2s = mm[1] * mm[1];
  tc.m3s = mm[2] * mm[2];
  tc.m4s = mm[3] * mm[3];
  tc.sum12 = (mm[0] + mm[1]) * (mm[0] + mm[1]);
  tc.dif12 = (mm[0] - mm[1]) * (mm[0] - mm[1]);
  tc.sum34 = (mm[2] + mm[3]) * (mm[2] + mm[3]);
  tc.dif34 = (mm[2] - mm[3]) * (mm[2] - mm[3]);
  const double rr = d.has("r_res") ? d.at("r_res").number() : 1.5;
  if (!(rr >= 0.0)) throw Error(FN_E_INVALID, "td4: r_res must be >= 0");
  tc.r2 = rr * rr;
  const double tau = d.at("tau").number();
  if (!(tau > 0.0)) throw Error(FN_E_INVALID, "td4: tau must be > 0");
  tc.gamma = 1.0 / tau;
  td4_weideman_coefficients(tc.wa, &tc.wL);
  tc.ps_wmax = td4_ps_wmax(tc);
  std::vector<double> fixed;
  auto pair = [&](const char* key, int* n, int* L, int* nr) {
    const auto& rs = d.at(key).array();
    *n = (int)rs.size();
    if (*n < 1 || *n > kTd4MaxRes)
      throw Error(FN_E_INVALID, std::string("td4: ") + key + " needs 1.." + std::to_string(kTd4MaxRes) + " entries");
    for (int r = 0; r < *n; ++r) {
      const long l = rs[r].at("L").integer();
      if (l < 0 || l > 1) throw Error(FN_E_INVALID, "td4: L must be 0 or 1");
      L[r] = (int)l;
      const double m0 = rs[r].at("m0").number(), w0 = rs[r].at("w0").number();
      nr[r] = m0 == 0.0 ? 1 : 0;
      fixed.push_back(m0);
      fixed.push_back(w0);
    }
  };
  pair("r12", &tc.n12, tc.L12, tc.nr12);
  pair("r34", &tc.n34, tc.L34, tc.nr34);
  fixed.push_back(d.at("sigma_t").number());
  const auto& amps = d.at("amps").array();
  tc.K = (int)amps.size();
  if (tc.K < 1 || tc.K > kTd4MaxAmp)
    throw Error(FN_E_INVALID, "td4: 1.." + std::to_string(kTd4MaxAmp) + " amplitudes");
  int side[kTd4MaxAmp];  // 0: in A and Abar, 1: A only, 2: Abar only
  for (int k = 0; k < tc.K; ++k) {
    const auto& a = amps[k].array();
    if (a.size() != 3 && a.size() != 4)
      throw Error(FN_E_INVALID, "td4: an amplitude is [r12 index, r34 index, angular type(, \"A\" | \"Abar\" | \"both\")]");
    const long r1 = a[0].integer(), r2 = a[1].integer(), ty = a[2].integer();
    if (r1 < 0 || r1 >= tc.n12 || r2 < 0 || r2 >= tc.n34 || ty < 0 || ty > 5)
      throw Error(FN_E_INVALID, "td4: amplitude index out of range");
    tc.amp1[k] = (int)r1;
    tc.amp2[k] = (int)r2;
    tc.atype[k] = (int)ty;
    side[k] = 0;
    if (a.size() == 4) {
      const std::string& sd = a[3].string();
      if (sd == "A") side[k] = 1;
      else if (sd == "Abar") side[k] = 2;
      else if (sd != "both") throw Error(FN_E_INVALID, "td4: an amplitude's sum is \"A\", \"Abar\" or \"both\"");
    }
  }
  // theta: A's members' coefficients, then Abar's, then x and y
  int p = 0;
  for (int k = 0; k < tc.K; ++k) {
    tc.pa[k] = side[k] != 2 ? p : -1;
    if (side[k] != 2) p += 2;
  }
  for (int k = 0; k < tc.K; ++k) {
    tc.pb[k] = side[k] != 1 ? p : -1;
    if (side[k] != 1) p += 2;
  }
  tc.n_params = p + 2;
  const Td4FitConst fc = td4_fit_const(tc, fixed.data());
  m->fixed_ls = fixed;
  m->P = tc.n_params;
  m->n_obs = 6;
  // events per workgroup: median NLL + gradient on 10M events measured 588 /
  // 550 / 532 / 538 us at 1024 / 2048 / 4096 / 8192 (fewer level-2 rows of
  // 43 sums); fn_model_autotune refines it for a given sample
  m->chunk = 4096;
  if (!device) return;
  m->td4_jit = td4_jit(tc);
  m->d_table.reserve(sizeof(Td4Table));
  m->d_fixed.reserve(sizeof(Td4FitConst));
  hip_check(hipMemcpy(m->d_fixed.ptr, &fc, sizeof(fc), hipMemcpyHostToDevice), "hipMemcpy");
  m->d_M.reserve(sizeof(double) * 2 * kTd4MaxAmp * kTd4MaxAmp);
}

// ------------------------------------------------------------ pipeline
static int64_t nchunks_for(int64_t n, int chunk) { return (n + chunk - 1) / chunk; }

double* Workspace::take_front(size_t count) {
  if (count > cap - front - back)
    throw Error(FN_E_INVALID, "the call needs " + std::to_string(front + back + count) +
                                  " doubles of scratch, more than the " + std::to_string(cap) + " available");
  double* p = base + front;
  front += count;
  return p;
}
double* Workspace::take_back(size_t count) {
  if (count > cap - front - back)
    throw Error(FN_E_INVALID, "the call needs " + std::to_string(front + back + count) +
                                  " doubles of scratch, more than the " + std::to_string(cap) + " available");
  back += count;
  return base + (cap - back);
}

void run_nll(fn_model* m, const ParamBlock* pb, const double* theta_dev, const double* ev, int64_t n, int64_t ld,
             bool grad, double* out_user, hipStream_t s, Workspace* ws) {
  const int64_t nch = nchunks_for(n, m->chunk);
  // level-1 partial rows of the events pass, and the normalization's partial
  // rows: model-owned buffers, or the front and the back of a workspace
  double* part = nullptr;
  double* npart = nullptr;
  auto events_rows = [&](size_t doubles) {
    if (ws) {
      part = ws->take_front(doubles);
    } else {
      m->d_part.reserve(sizeof(double) * doubles);
      part = m->part();
    }
  };
  auto norm_rows = [&](size_t doubles) {
    if (ws) {
      npart = ws->take_back(doubles);
    } else {
      m->d_npart.reserve(sizeof(double) * doubles);
      npart = m->npart();
    }
  };
  // workspace calls are never timed: timing takes HIP events from a pool
  const bool launches = nch > 0 && !ws;
  if (m->kind == kKindMix1d) {
    const Mix1dConst& mc = m->mix;
    const int kmax = mix1d_kmax(mc.K);
    const int nv = mix1d_nv(kmax, grad);
    events_rows((size_t)(nch > 0 ? nch : 1) * nv);
    ParamBlock zero;
    mix1d_launch_prologue(mc, pb ? *pb : zero, pb ? nullptr : theta_dev, 1, 0, m->table_mix(), s);
    m->timed(launches, [&](hipEvent_t t0, hipEvent_t t1) {
      mix1d_launch_events(mc, m->table_mix(), ev, n, m->chunk, nch, grad, part, s, t0, t1);
    });
    mix1d_launch_finalize(mc, m->table_mix(), part, nch, grad, (double)n, m->out(), out_user, s);
  } else if (m->kind == kKindTddp3) {
    const DalitzConst& dc = m->dal;
    const int nv = tddp_nv(dc.K, grad);
    const int64_t pre = presum_blocks(nch, nv, 0, 0);
    events_rows((size_t)((nch > 0 ? nch : 1) + pre) * nv);
    if (pb || !m->table_ready) {
      ParamBlock zero;
      dalitz_launch_prologue(dc, pb ? *pb : zero, pb ? nullptr : theta_dev, m->fixed(), 1, 0, m->table_dal(), s);
      m->table_ready = true;
    }
    const double* coef = theta_dev;
    if (pb) {
      tddp_launch_copy_theta(*pb, m->P, (double*)m->d_theta.ptr, s);
      coef = (const double*)m->d_theta.ptr;
    }
    if (!m->M_valid) {
      const int64_t ncell = (int64_t)dc.nx * dc.ny;
      const int64_t mrows = nchunks_for(ncell, m->grid_chunk);
      norm_rows((size_t)mrows * 2 * kMRowBlock * dc.K);
      tddp_launch_mmatrices(*m->tddp_jit, dc, m->table_dal(), m->grid_chunk, npart, m->Mc(), s);
      m->M_valid = true;
    }
    m->timed(launches, [&](hipEvent_t t0, hipEvent_t t1) {
      tddp_launch_events(*m->tddp_jit, dc, m->table_dal(), m->tdt, coef, ev, ld, n, m->chunk, nch, grad,
                         part, s, t0, t1);
    });
    // long row sets: pre-summed into the room after the rows
    launch_rows_presum(part, nch, nv, part + nch * nv, pre, nullptr, 0, 0, nullptr, 0, s);
    tddp_launch_finalize(dc, m->table_dal(), m->tdt, coef, pre ? part + nch * nv : part, pre ? pre : nch, grad,
                         m->Mc(), (double)n, m->out(), out_user, s);
  } else if (m->kind == kKindTd4) {
    const Td4Const& tc = m->td4;
    if (m->n_mc <= 0) throw Error(FN_E_INVALID, "td4: normalization sample not set (fn_model_set_norm_sample)");
    const int kmax = td4_kmax(tc.K);
    const int nv = td4_nv(tc, grad);
    const int64_t pre = presum_blocks(nch, nv, 0, 0);
    events_rows((size_t)((nch > 0 ? nch : 1) + pre) * nv);
    const Td4FitConst* fc = (const Td4FitConst*)m->d_fixed.ptr;
    td4_launch_prologue(tc, pb, theta_dev, m->P, fc, nullptr, 1, m->table_td4(), s);
    if (!m->M_valid) {
      const int mchunk = 1024;
      const int64_t mrows = nchunks_for(m->n_mc, mchunk);
      norm_rows((size_t)mrows * 2 * td4_row_block(tc.K) * kmax);
      td4_launch_mmatrix(*m->td4_jit, tc, m->table_td4(), 1, (const double*)m->d_mc.ptr, m->n_mc, m->n_mc, mchunk,
                         npart,
                         m->Mc(), s);
      m->M_valid = true;
    }
    m->timed(launches, [&](hipEvent_t t0, hipEvent_t t1) {
      td4_launch_events(*m->td4_jit, tc, m->table_td4(), nullptr, 1, ev, ld, n, m->chunk, grad, part, s, t0,
                        t1);
    });
    // long row sets: pre-summed into the room after the rows
    launch_rows_presum(part, nch, nv, part + nch * nv, pre, nullptr, 0, 0, nullptr, 0, s);
    td4_launch_finalize(tc, m->table_td4(), nullptr, 1, pre ? part + nch * nv : part, pre ? pre : nch, grad, m->Mc(),
                        (double)n, m->out(), 0, out_user, s);
  } else {
    const DalitzConst& dc = m->dal;
    const int kmax = dalitz_kmax(dc.K);
    const int g = grad ? (dc.free_ls ? 2 : 1) : 0;
    const int nv = dalitz_nv_events(kmax, g);
    // grid rows when the lineshapes are free; long row sets get room for
    // their pre-summed rows after them (see dalitz_launch_finalize)
    const int64_t grid_rows_n =
        dc.free_ls ? std::max<int64_t>(1, nchunks_for(m->n_inside, m->grid_chunk)) : 0;
    const int grid_nv = dc.free_ls ? dalitz_nv_events(kmax, g) : 0;
    const int64_t pre_e = presum_blocks(nch, nv, grid_rows_n, grid_nv);
    const int64_t pre_g = pre_e > 0 && dc.free_ls ? presum_blocks(grid_rows_n, grid_nv, nch, nv) : 0;
    events_rows((size_t)((nch > 0 ? nch : 1) + pre_e) * nv);
    // The table holds the lineshape constants (functions of theta only when the
    // lineshapes are free) and a copy of the coefficients; with fixed lineshapes
    // and theta on the device, the passes read the coefficients from theta and
    // the table is built once.
    if (dc.free_ls || pb || !m->table_ready) {
      ParamBlock zero;
      dalitz_launch_prologue(dc, pb ? *pb : zero, pb ? nullptr : theta_dev, m->fixed(), 1, 0, m->table_dal(), s);
      if (!dc.free_ls) m->table_ready = true;
    }
    const double* coef = theta_dev ? theta_dev : m->table_dal()->coef;
    double* grid_rows = nullptr;
    int64_t nrows = 0;
    int nnv = 0;
    if (dc.free_ls) {
      // lineshapes move: integrate P~ (and dP~) over the grid every call
      nrows = grid_rows_n;
      nnv = grid_nv;
      norm_rows((size_t)(nrows + pre_g) * nnv);
      dalitz_launch_grid(*m->dal_jit, dc, m->table_dal(), coef, (const GridCell*)m->d_cells.ptr, m->n_inside,
                         m->grid_chunk, nrows, g, npart, s);
      grid_rows = npart;
    } else if (!m->M_valid) {
      // fixed lineshapes: reduce the grid once to M_ij = dA sum A_i conj(A_j)
      const int64_t ncell = (int64_t)dc.nx * dc.ny;
      const int64_t mrows = nchunks_for(ncell, m->grid_chunk);
      norm_rows((size_t)mrows * dalitz_nv_mrows(kmax));
      for (int i0 = 0; i0 < dc.K; i0 += 4)
        dalitz_launch_mrows(*m->dal_jit, dc, m->table_dal(), m->grid_chunk, mrows, i0, npart, m->Mc(), s);
      m->M_valid = true;
    }
    // cached M: the events pass evaluates I = c^H M c in its last workgroup
    const bool norm_in_pass = !dc.free_ls && nch > 0;
    // span mode: the pass stamps its workgroups, the level-2 kernel adds the span
    unsigned long long* span = nullptr;
    if (m->timing < 0 && !ws && nch > 0) {
      const size_t need = sizeof(unsigned long long) * (size_t)(2 + 2 * nch);
      if (need > m->d_span.bytes) {
        // room for this launch's stamps; the record so far moves with it
        // (synchronous: the first launch of a larger sample must not be
        // captured into a graph)
        unsigned long long rec[2];
        hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
        hip_check(hipMemcpy(rec, m->d_span.ptr, sizeof(rec), hipMemcpyDeviceToHost), "hipMemcpy");
        m->d_span.reserve(need);
        hip_check(hipMemcpy(m->d_span.ptr, rec, sizeof(rec), hipMemcpyHostToDevice), "hipMemcpy");
      }
      span = (unsigned long long*)m->d_span.ptr;
    }
    m->timed(launches, [&](hipEvent_t t0, hipEvent_t t1) {
      dalitz_launch_events(m->ept == 2 ? *m->dal_jit2 : *m->dal_jit, dc, m->table_dal(), coef, ev, ld, n, m->chunk,
                           nch, g, part, s,
                           norm_in_pass ? m->Mc() : nullptr, norm_in_pass ? m->out() : nullptr, t0, t1, span);
    });
    dalitz_launch_finalize(dc, m->table_dal(), coef, part, nch, g, grid_rows, nrows, nnv, m->Mc(), (double)n,
                           m->out(), out_user, s, norm_in_pass, span);
  }
  hip_check(hipGetLastError(), "kernel launch");
}

void check_events_args(fn_model* m, const double* ev, int64_t n, int64_t ld) {
  if (n < 0) throw Error(FN_E_INVALID, "n must be >= 0");
  if (n > 0 && !ev) throw Error(FN_E_INVALID, "events pointer is NULL");
  if (m->n_obs > 1 && ld < n) throw Error(FN_E_INVALID, "ld must be >= n");
}

ParamBlock make_block(const fn_model* m, const double* theta_host) {
  if (!theta_host) throw Error(FN_E_INVALID, "theta is NULL");
  ParamBlock pb;
  std::memset(&pb, 0, sizeof(pb));
  for (int p = 0; p < m->P; ++p) pb.v[p] = theta_host[p];
  return pb;
}

void nll_host(fn_model* m, const double* theta_host, const double* ev, int64_t n, int64_t ld, double* nll,
              double* grad, hipStream_t s) {
  check_events_args(m, ev, n, ld);
  const ParamBlock pb = make_block(m, theta_host);
  const bool g = grad != nullptr;
  run_nll(m, &pb, nullptr, ev, n, ld, g, nullptr, s);
  const size_t cnt = (size_t)(g ? 1 + m->P : 1);
  hip_check(hipMemcpyAsync(m->h_out, m->out(), sizeof(double) * cnt, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  const double v = m->h_out[0];
  m->stats_calls += 1;
  if (grad)
    for (int p = 0; p < m->P; ++p) grad[p] = m->h_out[1 + p];
  if (!std::isfinite(v)) {
    if (nll) *nll = INFINITY;
    if (grad)
      for (int p = 0; p < m->P; ++p) grad[p] = NAN;
    throw Error(FN_E_NONFINITE, "NLL is not finite (P~ <= 0 at some event, invalid parameters, or I <= 0)");
  }
  bool gbad = false;
  if (grad)
    for (int p = 0; p < m->P; ++p) gbad |= !std::isfinite(grad[p]);
  if (nll) *nll = v;
  if (gbad) throw Error(FN_E_NONFINITE, "gradient is not finite");
}

void nll_binned_host(fn_model* m, const double* theta_host, const BinnedData& bd, double* value, double* grad,
                     hipStream_t s) {
  if (m->kind != kKindMix1d) throw Error(FN_E_INVALID, "binned data: mix1d models only");
  if (bd.nb < 1 || !bd.counts) throw Error(FN_E_INVALID, "binned data: need n_bins >= 1 and a counts pointer");
  if (bd.stat != 0 && bd.stat != 1) throw Error(FN_E_INVALID, "binned data: stat must be 0 (Poisson) or 1 (chi^2)");
  const ParamBlock pb = make_block(m, theta_host);
  const Mix1dConst& mc = m->mix;
  const bool g = grad != nullptr;
  mix1d_launch_prologue(mc, pb, nullptr, 1, 0, m->table_mix(), s);
  const int64_t nch = nchunks_for(bd.nb, m->chunk);
  m->d_part.reserve(sizeof(double) * (size_t)nch * mix1d_nv_binned(mix1d_kmax(mc.K), g));
  m->d_gen.reserve(3 * sizeof(unsigned long long));
  mix1d_launch_binned(mc, m->table_mix(), bd.counts, bd.nb, m->chunk, nch, bd.stat, g, m->part(),
                      (double*)m->d_gen.ptr, m->out(), s);
  hip_check(hipGetLastError(), "kernel launch");
  const size_t cnt = (size_t)(g ? 1 + m->P : 1);
  hip_check(hipMemcpyAsync(m->h_out, m->out(), sizeof(double) * cnt, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  m->stats_calls += 1;
  const double v = m->h_out[0];
  bool gbad = false;
  if (g)
    for (int p = 0; p < m->P; ++p) {
      grad[p] = m->h_out[1 + p];
      gbad |= !std::isfinite(grad[p]);
    }
  if (value) *value = std::isfinite(v) ? v : INFINITY;
  if (!std::isfinite(v))
    throw Error(FN_E_NONFINITE, "binned statistic is not finite (P <= 0 in a filled bin, invalid parameters, "
                                "or no events)");
  if (gbad) throw Error(FN_E_NONFINITE, "gradient is not finite");
}

void generate_td4(fn_model* m, const double* theta_host, uint32_t seed, uint32_t fit, int64_t n, double envelope,
                  double* ev_dev, int64_t ld, double* envelope_used, hipStream_t s) {
  if (n < 0 || (n > 0 && !ev_dev)) throw Error(FN_E_INVALID, "bad output");
  if (ld < n) throw Error(FN_E_INVALID, "ld must be >= n");
  if (!(envelope >= 0.0) || !std::isfinite(envelope)) throw Error(FN_E_INVALID, "envelope must be finite and >= 0");
  if (!(std::fabs(theta_host[m->P - 1]) < 1.0)) throw Error(FN_E_INVALID, "td4 generation needs |y| < 1");
  hip_check(hipSetDevice(m->device), "hipSetDevice");
  const Td4Const& tc = m->td4;
  const ParamBlock pb = make_block(m, theta_host);
  const Td4FitConst* fc = (const Td4FitConst*)m->d_fixed.ptr;
  td4_launch_prologue(tc, &pb, nullptr, m->P, fc, nullptr, 1, m->table_td4(), s);
  const Td4Proposal pr = td4_proposal(tc, td4_fit_const(tc, m->fixed_ls.data()));
  m->d_gen.reserve(3 * sizeof(unsigned long long));
  unsigned long long* g = (unsigned long long*)m->d_gen.ptr;
  hip_check(hipMemsetAsync(g, 0, 3 * sizeof(unsigned long long), s), "hipMemsetAsync");
  double W = envelope;
  if (W == 0.0) {
    if (m->n_mc <= 0)
      throw Error(FN_E_INVALID, "td4: the automatic envelope needs the normalization sample (or give an envelope)");
    td4_launch_envmax(*m->td4_jit, tc, m->table_td4(), pr, (const double*)m->d_mc.ptr, m->n_mc, m->n_mc, g, s);
    hip_check(hipGetLastError(), "kernel launch");
    unsigned long long bits = 0;
    hip_check(hipMemcpyAsync(&bits, g, sizeof(bits), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    double vmax;
    std::memcpy(&vmax, &bits, sizeof(vmax));
    if (!(vmax > 0.0) || !std::isfinite(vmax)) throw Error(FN_E_INVALID, "the amplitudes vanish on the sample");
    W = kGenEnvelopeFactor * vmax;
  }
  if (envelope_used) *envelope_used = W;
  if (n == 0) return;
  td4_launch_gen(*m->td4_jit, tc, m->table_td4(), pr, seed, fit, n, W, kGenMaxAttemptsTd4, ev_dev, ld, g + 1, s);
  hip_check(hipGetLastError(), "kernel launch");
  unsigned long long bad[2] = {0, 0};
  hip_check(hipMemcpyAsync(bad, g + 1, sizeof(bad), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (bad[0])
    throw Error(FN_E_DOMAIN, std::to_string(bad[0]) + " accepted events lie above the envelope " + std::to_string(W) +
                                 ": raise it");
  if (bad[1]) throw Error(FN_E_DOMAIN, std::to_string(bad[1]) + " events not resolved within the attempt limit");
}

}  // namespace fn

using namespace fn;

extern "C" {

const char* fn_last_error(void) { return g_last_error.c_str(); }
int32_t fn_version(void) { return 10000; }

fn_status fn_ctx_create(int32_t device, fn_ctx** out) {
  return guard([&] {
    if (!out) throw Error(FN_E_INVALID, "out is NULL");
    int n = 0;
    hip_check(hipGetDeviceCount(&n), "hipGetDeviceCount");
    if (device < 0 || device >= n) throw Error(FN_E_INVALID, "no such device");
    hip_check(hipSetDevice(device), "hipSetDevice");
    double* sp = scratch_address(device);
    fn_ctx* c = new fn_ctx;
    c->device = device;
    c->scratch = sp;
    *out = c;
  });
}

fn_status fn_ctx_destroy(fn_ctx* ctx) {
  return guard([&] { delete ctx; });
}

// Events per thread and loop iteration of a dalitz3 model's events passes
// (1 or 2); the two-event module is compiled when first chosen.
static void set_dalitz_ept(fn_model* m, long ept) {
  if (m->kind != kKindDalitz3) throw Error(FN_E_INVALID, "events_per_thread applies to dalitz3 models");
  if (ept != 1 && ept != 2) throw Error(FN_E_INVALID, "events_per_thread must be 1 or 2");
  if (ept == 2 && !m->dal_jit2) m->dal_jit2 = dalitz_jit(m->dal, 2);
  m->ept = (int)ept;
}

fn_status fn_model_create(fn_ctx* ctx, const char* desc_json, fn_model** out) {
  fn_model* m = nullptr;
  fn_status st = guard([&] {
    if (!ctx || !desc_json || !out) throw Error(FN_E_INVALID, "NULL argument");
    json::Value d;
    try {
      d = json::parse(desc_json);
    } catch (const std::exception& e) {
      throw Error(FN_E_INVALID, e.what());
    }
    hip_check(hipSetDevice(ctx->device), "hipSetDevice");
    m = new fn_model;
    m->ctx = ctx;
    m->device = ctx->device;
    try {
      const std::string& kind = d.at("kind").string();
      if (kind == "mix1d") {
        m->kind = kKindMix1d;
        compile_mix1d(d, m);
      } else if (kind == "dalitz3") {
        m->kind = kKindDalitz3;
        compile_dalitz3(d, m);
      } else if (kind == "td4") {
        m->kind = kKindTd4;
        compile_td4(d, m);
      } else if (kind == "tddp3") {
        m->kind = kKindTddp3;
        compile_tddp3(d, m);
      } else {
        throw Error(FN_E_INVALID, "unknown model kind \"" + kind + "\"");
      }
      if (d.has("chunk")) {
        const long c = d.at("chunk").integer();
        if (c % 256 != 0 || c < 256 || c > kMaxChunk)
          throw Error(FN_E_INVALID, "chunk must be a multiple of 256 in [256, " + std::to_string(kMaxChunk) + "]");
        m->chunk = (int)c;
      }
      if (d.has("events_per_thread")) set_dalitz_ept(m, d.at("events_per_thread").integer());
    } catch (const Error&) {
      throw;
    } catch (const std::exception& e) {
      throw Error(FN_E_INVALID, std::string("model description: ") + e.what());
    }
    m->d_out.reserve(sizeof(double) * (2 + 2 * m->P));
    m->d_count.reserve(sizeof(unsigned long long));
    if (hipHostMalloc((void**)&m->h_out, sizeof(double) * (2 + 2 * m->P) + 64, hipHostMallocDefault) !=
        hipSuccess) {
      m->h_out = nullptr;
      throw Error(FN_E_NOMEM, "hipHostMalloc failed");
    }
    *out = m;
  });
  if (st != FN_OK && m) {
    delete m;
  }
  return st;
}

fn_status fn_model_check_compile(const char* desc_json, const char* arch) {
  return guard([&] {
    if (!desc_json) throw Error(FN_E_INVALID, "NULL argument");
    json::Value d;
    try {
      d = json::parse(desc_json);
    } catch (const std::exception& e) {
      throw Error(FN_E_INVALID, e.what());
    }
    const std::string target = arch && *arch ? arch : "gfx950";
    fn_model tmp;
    try {
      const std::string& kind = d.at("kind").string();
      if (d.has("events_per_thread") && kind != "dalitz3")
        throw Error(FN_E_INVALID, "events_per_thread applies to dalitz3 models");
      if (kind == "dalitz3") {
        compile_dalitz3(d, &tmp, false);
        (void)jit_compile(dalitz_jit_source(tmp.dal, 1), target);
        if (d.has("events_per_thread")) {
          const long e = d.at("events_per_thread").integer();
          if (e != 1 && e != 2) throw Error(FN_E_INVALID, "events_per_thread must be 1 or 2");
          if (e == 2) (void)jit_compile(dalitz_jit_source(tmp.dal, 2), target);
        }
      } else if (kind == "td4") {
        compile_td4(d, &tmp, false);
        (void)jit_compile(td4_jit_source(tmp.td4), target);
      } else if (kind == "tddp3") {
        compile_tddp3(d, &tmp, false);
        (void)jit_compile(tddp_jit_source(tmp.dal), target);
      } else if (kind != "mix1d") {
        throw Error(FN_E_INVALID, "unknown model kind \"" + kind + "\"");
      }
    } catch (const Error&) {
      throw;
    } catch (const std::exception& e) {
      throw Error(FN_E_INVALID, std::string("model description: ") + e.what());
    }
  });
}

fn_status fn_model_info(const fn_model* m, int32_t* n_params, int32_t* n_obs, int32_t* chunk) {
  return guard([&] {
    if (!m) throw Error(FN_E_INVALID, "model is NULL");
    if (n_params) *n_params = m->P;
    if (n_obs) *n_obs = m->n_obs;
    if (chunk) *chunk = m->chunk;
  });
}

fn_status fn_model_destroy(fn_model* m) {
  return guard([&] { delete m; });
}

fn_status fn_model_autotune(fn_model* m, const double* theta_host, const double* ev, int64_t n, int64_t ld,
                            int32_t reps, int32_t* chunk_out, int32_t* ept_out, int32_t* chunks_out, double* us_out,
                            void* stream) {
  return guard([&] {
    if (!m || !theta_host) throw Error(FN_E_INVALID, "NULL argument");
    if (n < 1) throw Error(FN_E_INVALID, "autotuning needs events");
    check_events_args(m, ev, n, ld);
    if (reps < 1) reps = 20;
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const ParamBlock pb = make_block(m, theta_host);
    const int saved = m->chunk, saved_ept = m->ept;
    int cus = 0;
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device),
              "hipDeviceGetAttribute");
    int32_t cand[FN_TUNE_MAX];
    const int count = tune_candidates(n, cus > 0 ? cus : 1, cand);
    // dalitz3 events passes also come with two events per thread and iteration
    const int n_ept = m->kind == kKindDalitz3 ? 2 : 1;
    if (chunks_out)
      for (int c = 0; c < FN_TUNE_MAX; ++c) chunks_out[c] = c < count ? cand[c] : 0;
    if (us_out)
      for (int c = 0; c < FN_TUNE_EPT * FN_TUNE_MAX; ++c) us_out[c] = NAN;
    std::vector<hipEvent_t> evs(2 * (size_t)reps);
    for (auto& e : evs) hip_check(hipEventCreate(&e), "hipEventCreate");
    std::vector<double> med((size_t)n_ept * count, INFINITY);
    try {
      if (n_ept == 2 && !m->dal_jit2) m->dal_jit2 = dalitz_jit(m->dal, 2);
      for (int e = 0; e < n_ept; ++e) {
        m->ept = e + 1;
        for (int c = 0; c < count; ++c) {
          m->chunk = cand[c];
          for (int w = 0; w < 3; ++w) run_nll(m, &pb, nullptr, ev, n, ld, true, nullptr, s);  // warm-up, buffers
          for (int r = 0; r < reps; ++r) {
            hip_check(hipEventRecord(evs[2 * r], s), "hipEventRecord");
            run_nll(m, &pb, nullptr, ev, n, ld, true, nullptr, s);
            hip_check(hipEventRecord(evs[2 * r + 1], s), "hipEventRecord");
          }
          hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
          std::vector<double> t(reps);
          for (int r = 0; r < reps; ++r) {
            float ms = 0.0f;
            hip_check(hipEventElapsedTime(&ms, evs[2 * r], evs[2 * r + 1]), "hipEventElapsedTime");
            t[r] = 1e3 * ms;
          }
          std::nth_element(t.begin(), t.begin() + reps / 2, t.end());
          med[(size_t)e * count + c] = t[reps / 2];
          if (us_out) us_out[e * FN_TUNE_MAX + c] = t[reps / 2];
        }
      }
    } catch (...) {
      m->chunk = saved;
      m->ept = saved_ept;
      for (auto& e : evs) (void)hipEventDestroy(e);
      throw;
    }
    for (auto& e : evs) (void)hipEventDestroy(e);
    // among the candidates within kTuneTie of the fastest: one event per
    // thread when it has one (fewer registers), then the largest chunk (fewer
    // partial rows for the level-2 step, and a stable choice when candidates
    // time alike)
    const double fastest = *std::min_element(med.begin(), med.end());
    int best_e = -1, best_c = 0;
    for (int e = 0; e < n_ept && best_e < 0; ++e)
      for (int c = 0; c < count; ++c)
        if (med[(size_t)e * count + c] <= (1.0 + kTuneTie) * fastest && cand[c] > best_c) {
          best_e = e;
          best_c = cand[c];
        }
    m->chunk = best_c;
    m->ept = best_e + 1;
    if (chunk_out) *chunk_out = best_c;
    if (ept_out) *ept_out = best_e + 1;
  });
}

fn_status fn_events_check(fn_model* m, const double* ev, int64_t n, int64_t ld, int64_t* n_bad, void* stream) {
  return guard([&] {
    if (!m) throw Error(FN_E_INVALID, "model is NULL");
    check_events_args(m, ev, n, ld);
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    hip_check(hipMemsetAsync(m->d_count.ptr, 0, sizeof(unsigned long long), s), "hipMemsetAsync");
    if (m->kind == kKindMix1d) mix1d_launch_check(m->mix, ev, n, (unsigned long long*)m->d_count.ptr, s);
    else if (m->kind == kKindTd4) td4_launch_check(m->td4, ev, ld, n, (unsigned long long*)m->d_count.ptr, s);
    else dalitz_launch_check(m->dal, ev, ld, n, (unsigned long long*)m->d_count.ptr, s);
    hip_check(hipGetLastError(), "kernel launch");
    unsigned long long cnt = 0;
    hip_check(hipMemcpyAsync(m->h_out, m->d_count.ptr, sizeof(cnt), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    std::memcpy(&cnt, m->h_out, sizeof(cnt));
    if (n_bad) *n_bad = (int64_t)cnt;
    if (cnt) throw Error(FN_E_DOMAIN, std::to_string(cnt) + " events outside the observable domain");
  });
}

fn_status fn_nll(fn_model* m, const double* theta_host, const double* ev, int64_t n, int64_t ld,
                 double* nll_out, double* grad_host, void* stream) {
  return guard([&] {
    if (!m) throw Error(FN_E_INVALID, "model is NULL");
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    nll_host(m, theta_host, ev, n, ld, nll_out, grad_host, (hipStream_t)stream);
  });
}

fn_status fn_nll_async(fn_model* m, const double* theta_dev, const double* ev, int64_t n, int64_t ld,
                       double* out_dev, int32_t with_grad, void* stream) {
  return guard([&] {
    if (!m || !theta_dev || !out_dev) throw Error(FN_E_INVALID, "NULL argument");
    check_events_args(m, ev, n, ld);
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    run_nll(m, nullptr, theta_dev, ev, n, ld, with_grad != 0, out_dev, s);
  });
}

fn_status fn_nll_async_noalloc(fn_model* m, const double* theta_dev, const double* ev, int64_t n, int64_t ld,
                               double* out_dev, int32_t with_grad, void* stream) {
  return guard([&] {
    if (!m || !theta_dev || !out_dev) throw Error(FN_E_INVALID, "NULL argument");
    check_events_args(m, ev, n, ld);
    if (!m->ctx || !m->ctx->scratch) throw Error(FN_E_INVALID, "the model's context has no scratch address");
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    Workspace ws;
    ws.base = m->ctx->scratch;
    ws.cap = kScratchDoubles;
    run_nll(m, nullptr, theta_dev, ev, n, ld, with_grad != 0, out_dev, (hipStream_t)stream, &ws);
  });
}

fn_status fn_norm(fn_model* m, const double* theta_host, double* norm_host, double* dnorm_host, void* stream) {
  return guard([&] {
    if (!m) throw Error(FN_E_INVALID, "model is NULL");
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const ParamBlock pb = make_block(m, theta_host);
    run_nll(m, &pb, nullptr, nullptr, 0, 0, true, nullptr, s);
    hip_check(hipMemcpyAsync(m->h_out, m->out(), sizeof(double) * (2 + 2 * m->P), hipMemcpyDeviceToHost, s),
              "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (norm_host) *norm_host = m->h_out[1 + m->P];
    if (dnorm_host)
      for (int p = 0; p < m->P; ++p) dnorm_host[p] = m->h_out[2 + m->P + p];
  });
}

fn_status fn_eval(fn_model* m, const double* theta_host, const double* ev, int64_t n, int64_t ld, double* p_dev,
                  void* stream) {
  return guard([&] {
    if (!m) throw Error(FN_E_INVALID, "model is NULL");
    if (m->kind == kKindTddp3) throw Error(FN_E_INVALID, "fn_eval is not available for tddp3 models");
    if (n > 0 && !p_dev) throw Error(FN_E_INVALID, "output is NULL");
    check_events_args(m, ev, n, ld);
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const ParamBlock pb = make_block(m, theta_host);
    run_nll(m, &pb, nullptr, nullptr, 0, 0, false, nullptr, s);
    if (m->kind == kKindMix1d) mix1d_launch_eval(m->mix, m->table_mix(), ev, n, p_dev, s);
    else if (m->kind == kKindTd4) td4_launch_eval(m->td4, m->table_td4(), ev, ld, n, m->out() + 1 + m->P, p_dev, s);
    else dalitz_launch_eval(m->dal, m->table_dal(), ev, ld, n, m->out() + 1 + m->P, p_dev, s);
    hip_check(hipGetLastError(), "kernel launch");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  });
}

fn_status fn_nll_binned(fn_model* m, const double* theta_host, const double* counts_dev, int64_t n_bins,
                        int32_t stat, double* value_host, double* grad_host, void* stream) {
  return guard([&] {
    if (!m || !theta_host) throw Error(FN_E_INVALID, "NULL argument");
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    nll_binned_host(m, theta_host, BinnedData{counts_dev, n_bins, stat}, value_host, grad_host,
                    (hipStream_t)stream);
  });
}

fn_status fn_generate(fn_model* m, const double* theta_host, uint32_t seed, uint32_t fit, int64_t n,
                      double envelope, double* ev_dev, int64_t ld, double* envelope_used, void* stream) {
  return guard([&] {
    if (!m || !theta_host) throw Error(FN_E_INVALID, "NULL argument");
    if (m->kind == kKindTd4) {
      generate_td4(m, theta_host, seed, fit, n, envelope, ev_dev, ld, envelope_used, (hipStream_t)stream);
      return;
    }
    if (m->kind != kKindDalitz3 && m->kind != kKindTddp3)
      throw Error(FN_E_INVALID, "device generation by model is available for dalitz3, tddp3 and td4 models "
                                "(mix1d: fn_generate_mix1d)");
    const bool td = m->kind == kKindTddp3;
    if (n < 0 || (n > 0 && !ev_dev)) throw Error(FN_E_INVALID, "bad output");
    if (ld < n) throw Error(FN_E_INVALID, "ld must be >= n");
    if (!(envelope >= 0.0) || !std::isfinite(envelope)) throw Error(FN_E_INVALID, "envelope must be finite and >= 0");
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    const DalitzConst& dc = m->dal;
    const ParamBlock pb = make_block(m, theta_host);
    dalitz_launch_prologue(dc, pb, nullptr, m->fixed(), 1, 0, m->table_dal(), s);
    if (td) tddp_launch_copy_theta(pb, m->P, (double*)m->d_theta.ptr, s);
    const double* coef = (const double*)m->d_theta.ptr;
    if (td && !(std::fabs(theta_host[m->P - 1]) < 1.0))
      throw Error(FN_E_INVALID, "tddp3 generation needs |y| < 1");
    m->d_gen.reserve(3 * sizeof(unsigned long long));
    unsigned long long* g = (unsigned long long*)m->d_gen.ptr;
    hip_check(hipMemsetAsync(g, 0, 3 * sizeof(unsigned long long), s), "hipMemsetAsync");
    double valid = 0.0;
    hip_check(hipMemcpyAsync(&valid, &m->table_dal()->valid, sizeof(double), hipMemcpyDeviceToHost, s),
              "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (valid == 0.0) throw Error(FN_E_INVALID, "invalid lineshape parameters");
    double W = envelope;
    if (W == 0.0) {
      if (td) tddp_launch_gridmax(*m->tddp_jit, dc, m->table_dal(), coef, g, s);
      else dalitz_launch_gridmax(*m->dal_jit, dc, m->table_dal(), g, s);
      hip_check(hipGetLastError(), "kernel launch");
      unsigned long long bits = 0;
      hip_check(hipMemcpyAsync(&bits, g, sizeof(bits), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
      hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
      double vmax;
      std::memcpy(&vmax, &bits, sizeof(vmax));
      if (!(vmax > 0.0) || !std::isfinite(vmax)) throw Error(FN_E_INVALID, "the density vanishes on the grid");
      W = kGenEnvelopeFactor * vmax;
    }
    if (envelope_used) *envelope_used = W;
    if (n == 0) return;
    if (td)
      tddp_launch_gen(*m->tddp_jit, dc, m->table_dal(), coef, m->tdt, seed, fit, n, W, m->box, kGenMaxAttemptsModel,
                      ev_dev, ld, g + 1, s);
    else
      dalitz_launch_gen(*m->dal_jit, dc, m->table_dal(), seed, fit, n, W, m->box, kGenMaxAttemptsModel, ev_dev, ld,
                        g + 1, s);
    hip_check(hipGetLastError(), "kernel launch");
    unsigned long long bad[2] = {0, 0};
    hip_check(hipMemcpyAsync(bad, g + 1, sizeof(bad), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (bad[0])
      throw Error(FN_E_DOMAIN, std::to_string(bad[0]) + " accepted events lie above the envelope " +
                                   std::to_string(W) + ": raise it");
    if (bad[1]) throw Error(FN_E_DOMAIN, std::to_string(bad[1]) + " events not resolved within the attempt limit");
  });
}

fn_status fn_model_generate_norm_sample(fn_model* m, uint32_t seed, uint32_t fit, int64_t n_mc, void* stream) {
  return guard([&] {
    if (!m) throw Error(FN_E_INVALID, "model is NULL");
    if (m->kind != kKindTd4) throw Error(FN_E_INVALID, "only td4 models take a normalization sample");
    if (n_mc <= 0) throw Error(FN_E_INVALID, "need n_mc > 0");
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    m->d_mc.reserve(sizeof(double) * 5 * (size_t)n_mc);
    m->d_gen.reserve(3 * sizeof(unsigned long long));
    unsigned long long* g = (unsigned long long*)m->d_gen.ptr;
    hip_check(hipMemsetAsync(g, 0, sizeof(unsigned long long), s), "hipMemsetAsync");
    td4_launch_phase_space(m->td4, seed, fit, kPhaseSpaceStream0, kGenMaxAttemptsModel, n_mc, (double*)m->d_mc.ptr,
                           n_mc, g, s);
    hip_check(hipGetLastError(), "kernel launch");
    unsigned long long bad = 0;
    hip_check(hipMemcpyAsync(&bad, g, sizeof(bad), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    m->n_mc = n_mc;
    m->mc_gen += 1;
    m->M_valid = false;
    if (bad) {
      m->n_mc = 0;
      throw Error(FN_E_DOMAIN, std::to_string(bad) + " phase-space points not resolved within the attempt limit");
    }
  });
}

fn_status fn_model_set_norm_sample(fn_model* m, const double* mc_dev, int64_t n_mc, int64_t ld, void* stream) {
  return guard([&] {
    if (!m) throw Error(FN_E_INVALID, "model is NULL");
    if (m->kind != kKindTd4) throw Error(FN_E_INVALID, "only td4 models take a normalization sample");
    if (n_mc <= 0 || !mc_dev) throw Error(FN_E_INVALID, "need n_mc > 0 and a sample pointer");
    if (ld < n_mc) throw Error(FN_E_INVALID, "ld must be >= n_mc");
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    m->d_mc.reserve(sizeof(double) * 5 * (size_t)n_mc);
    hip_check(hipMemcpy2DAsync(m->d_mc.ptr, sizeof(double) * n_mc, mc_dev, sizeof(double) * ld,
                               sizeof(double) * n_mc, 5, hipMemcpyDeviceToDevice, s),
              "hipMemcpy2DAsync");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    m->n_mc = n_mc;
    m->mc_gen += 1;
    m->M_valid = false;
  });
}

fn_status fn_model_fixed(const fn_model* m, int32_t* n_fixed, double* fixed_host) {
  return guard([&] {
    if (!m) throw Error(FN_E_INVALID, "model is NULL");
    if (m->kind != kKindTd4) throw Error(FN_E_INVALID, "only td4 models have a fixed-constant vector");
    if (n_fixed) *n_fixed = (int32_t)m->fixed_ls.size();
    if (fixed_host) std::memcpy(fixed_host, m->fixed_ls.data(), sizeof(double) * m->fixed_ls.size());
  });
}

// The span record of span mode: summed span and launch count back to zero.
static void span_reset(fn_model* m) {
  const unsigned long long init[2] = {0ull, 0ull};
  hip_check(hipMemcpy(m->d_span.ptr, init, sizeof(init), hipMemcpyHostToDevice), "hipMemcpy");
}

fn_status fn_model_timing(fn_model* m, int32_t every) {
  return guard([&] {
    if (!m) throw Error(FN_E_INVALID, "model is NULL");
    if (every < -1) throw Error(FN_E_INVALID, "every must be >= -1");
    if (every == -1) {
      if (m->kind != kKindDalitz3) throw Error(FN_E_INVALID, "in-kernel span timing is available for dalitz3 models");
      hip_check(hipSetDevice(m->device), "hipSetDevice");
      int khz = 0;
      hip_check(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, m->device), "hipDeviceGetAttribute");
      if (khz <= 0) throw Error(FN_E_HIP, "the device reports no wall-clock rate");
      m->span_khz = khz;
      m->d_span.reserve(2 * sizeof(unsigned long long));
      hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
      span_reset(m);
    }
    m->timing = every;
    m->timing_count = 0;
  });
}

fn_status fn_model_kernel_time(fn_model* m, double* total_ms, int64_t* launches) {
  return guard([&] {
    if (!m) throw Error(FN_E_INVALID, "model is NULL");
    hip_check(hipSetDevice(m->device), "hipSetDevice");
    if (m->timing < 0) {
      // span mode: the launches may sit on any stream or inside graphs
      hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
      unsigned long long rec[2];
      hip_check(hipMemcpy(rec, m->d_span.ptr, sizeof(rec), hipMemcpyDeviceToHost), "hipMemcpy");
      if (total_ms) *total_ms = (double)rec[0] / m->span_khz;
      if (launches) *launches = (int64_t)rec[1];
      span_reset(m);
      return;
    }
    double tot = 0.0;
    for (auto& pr : m->ev_pending) {
      hip_check(hipEventSynchronize(pr.second), "hipEventSynchronize");
      float ms = 0.0f;
      hip_check(hipEventElapsedTime(&ms, pr.first, pr.second), "hipEventElapsedTime");
      tot += ms;
      m->ev_pool.push_back(pr.first);
      m->ev_pool.push_back(pr.second);
    }
    if (launches) *launches = (int64_t)m->ev_pending.size();
    if (total_ms) *total_ms = tot;
    m->ev_pending.clear();
  });
}

}  // extern "C"

hipEvent_t fn_model::take_event() {
  if (!ev_pool.empty()) {
    hipEvent_t e = ev_pool.back();
    ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  fn::hip_check(hipEventCreate(&e), "hipEventCreate");
  return e;
}

fn_model::~fn_model() {
  for (auto& pr : ev_pending) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  for (auto e : ev_pool) (void)hipEventDestroy(e);
  if (h_out) (void)hipHostFree(h_out);
}
