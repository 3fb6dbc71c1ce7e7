// Internal data layouts shared by the host side of the library and its
// kernels: model constants (passed by value as kernel arguments), per-fit
// parameter-derived tables (device memory, written by the prologue kernels),
// and launch constants.
#pragma once
#if !defined(__HIPCC_RTC__)
#include <hip/hip_runtime.h>
#include <stdint.h>
#else  // runtime compilation: the HIP device environment is built in, fixed-width integers live here
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
#endif

namespace fn {

constexpr int kBlock = 256;           // threads per workgroup (4 wave64s)
constexpr int kWaves = kBlock / 64;
constexpr int kMaxParams = 96;

// Parameter vector passed by value (kernel argument segment).
struct ParamBlock {
  double v[kMaxParams];
};

// ---------------------------------------------------------------- mix1d
constexpr int kMixMaxComp = 8;
enum MixType : int { kGauss = 0, kExp = 1, kArgus = 2, kBW = 3 };

struct Mix1dConst {
  double lo, hi;
  int K;                          // components
  int n_params;
  int type[kMixMaxComp];
  int pidx[kMixMaxComp][2];       // parameter indices of each component
  int npar[kMixMaxComp];          // 1 or 2
  int fidx[kMixMaxComp];          // fraction index for k < K-1
  int yidx;                       // expected-yield parameter (extended likelihood), -1 for none
};

// Gradient slots of a mix1d partial: [0] NLL, then 2 per component (its shape
// parameters), then one per fraction.  Slot -> parameter is done at the end.
__host__ __device__ constexpr int mix_nv(int kmax) { return 1 + 2 * kmax + kmax; }

// Per-fit derived constants (prologue output), one record per fit.
struct Mix1dTable {
  double frac[kMixMaxComp];       // weight of each component (last: 1 - sum)
  double invN[kMixMaxComp];       // 1 / integral of the shape on [lo, hi]
  double a[kMixMaxComp];          // gauss: mu     exp: tau  argus: 1/m0^2  bw: m0
  double b[kMixMaxComp];          // gauss: 1/sigma        argus: c       bw: gamma^2/4
  double c[kMixMaxComp];          // argus: 1/m0            bw: gamma
  double dlnN[kMixMaxComp][2];    // d ln N_k / d (its parameters)
  double yield;                   // expected yield (extended likelihood), 0 when none
  double valid;                   // 1 when the parameters define a density
};

// -------------------------------------------------------------- dalitz3
constexpr int kDalMaxRes = 16;

struct DalitzChan {               // a pair AB with bachelor C
  double mA2, mB2, mC2;
  double sum2, dif2;              // (mA+mB)^2, (mA-mB)^2
  double Psum2, Pdif2;            // (M+mC)^2, (M-mC)^2
  double zc;                      // (M^2 - mC^2)(mB^2 - mA^2)
  int useL[3];                    // which L occur in this pair
};

struct DalitzConst {
  double M2, msum;                // M^2, M^2 + m1^2 + m2^2 + m3^2
  double m1s, m2s, m3s;           // squared daughter masses
  double r2, rD2;                 // squared barrier radii
  double a12, d12, a13, d13;      // grid origin and cell sizes
  double dA;                      // cell area
  int nx, ny;
  int K;
  int free_ls;                    // lineshape parameters are in theta
  int chan[kDalMaxRes];           // 0 = "12", 1 = "13", 2 = "23"
  int L[kDalMaxRes];
  DalitzChan ch[3];
};

// A grid cell inside the physical region: column ix (s12) and row iy (s13).
// The grid passes of models with free lineshapes walk the list of these cells
// (built once per model, in column-major order) instead of the whole grid.
struct alignas(8) GridCell {
  int32_t ix, iy;
};

// Per-fit per-resonance record (prologue output).
enum DalField : int {
  dM0SQ = 0, dKW, dKA, dCRE, dCIM,  // m0^2, width scale, 1/F_L(q0), coefficient
  dDLNKA, dDKW_DM0, dKW_W0, dTWOM0, // derivatives for lineshape gradients
  kDalFields
};
struct DalitzTable {
  double r[kDalMaxRes][kDalFields];
  double coef[2 * kDalMaxRes];  // (Re c_k, Im c_k), the layout of theta's first 2K entries
  double valid;
};

}  // namespace fn
