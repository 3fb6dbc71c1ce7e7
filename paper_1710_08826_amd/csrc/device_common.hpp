// Device helpers: the deterministic two-level FP64 reduction.
//
// Level 1 (inside an evaluation kernel): every workgroup owns one fixed chunk
// of events.  Each thread sums its events in index order; every quad of lanes
// combines with two DPP exchanges (lane ^ 1, then lane ^ 2: register moves, no
// LDS traffic); one lane per quad stores its sums to LDS; four threads per
// value then add the workgroup's 64 quad sums, each taking every fourth quad
// in index order, and a last quad exchange combines the four.  The workgroup
// writes one row of NV doubles.
// Level 2 (a single workgroup): rows are summed in a fixed interleaving that
// depends only on the number of rows and NV.
// Nothing depends on scheduling, so results are bitwise reproducible, and a
// fit computes the same bits alone or inside a batch.
#pragma once
#include "model.hpp"

namespace fn {

constexpr int kQuads = kBlock / 4;  // quad sums per workgroup
constexpr int kFinalBlock = 1024;   // level-2 block size

// LDS doubles block_sum_row needs for NV values.
__host__ __device__ constexpr int block_sum_lds(int nv) { return kQuads * nv; }

// Sum over the four lanes of a quad, the same value in all four (fixed order:
// (a + b) + (c + d) pairs by lane ^ 1 first, then lane ^ 2).
__device__ __forceinline__ double quad_sum(double x) {
  x += __builtin_amdgcn_update_dpp(0.0, x, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
  x += __builtin_amdgcn_update_dpp(0.0, x, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
  return x;
}

template <int NV>
__device__ inline void block_sum_row(double (&v)[NV], double* lds /* block_sum_lds(NV) */,
                                     double* __restrict__ out_row) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = quad_sum(v[i]);
  if ((t & 3) == 0) {
    const int q = t >> 2;
#pragma unroll
    for (int i = 0; i < NV; ++i) lds[q * NV + i] = v[i];
  }
  __syncthreads();
  // thread (i, p) = (u >> 2, u & 3) adds quads p, p + 4, ..., p + 60 of value i;
  // the four threads of a value form one quad, so a quad sum combines them
  for (int u = t; u < 4 * NV; u += kBlock) {
    const int i = u >> 2, p = u & 3;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kQuads / 4; ++j) s += lds[(p + 4 * j) * NV + i];
    s = quad_sum(s);
    if (p == 0) out_row[i] = s;
  }
}

// Level 2: res[v] = sum over rows r of part[r*nv + v], for v < nv <= TB (the
// block size).  The rows were just written by other compute units and the
// whole block runs on one compute unit, so the step is bound by load latency,
// by the compute unit's load bandwidth and by its barriers (measured on
// gfx950 with the device wall clock, 1M events of the three-body model, 489
// rows of 17 values: the first thread's rows back after 0.9 us, every
// thread's after 1.6 us).  Thread t takes column v = t % nv and rows g, g+G,
// g+2G, ... (g = t / nv, G = TB / nv): ten rows per round, all loads issued
// before the first is used (rows past the end are not loaded and count zero;
// up to 10 G rows -- 600 of 17 values with a 1024-thread block -- take one
// round trip), added in row order.  Addresses are 32-bit byte offsets from
// the uniform base whenever the rows span less than 4 GB.  The G group sums
// of each column are then added in two levels, one barrier each: J = min(8,
// G) threads per column each add the groups j, j+J, j+2J, ... in order, then
// one thread per column adds the J results in order.  scratch holds TB
// doubles.
template <int TB>
__device__ inline void sum_rows_t(const double* __restrict__ part, int64_t nrows, int nv, double* scratch,
                                  double* res) {
  constexpr int U = 10;
  const int t = threadIdx.x;
  const int G = TB / nv;
  const int g = t / nv;
  const int v = t - g * nv;
  double s = 0.0;
  if (g < G) {
    if ((nrows + (int64_t)U * G) * nv * 8 < (int64_t(1) << 32)) {
      const char* __restrict__ base = reinterpret_cast<const char*>(part);
      const unsigned step = (unsigned)(G * nv) * 8u;
      unsigned o = (unsigned)(g * nv + v) * 8u;
      for (int64_t r = g; r < nrows; r += (int64_t)U * G, o += U * step) {
        double x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          x[u] = 0.0;
          if (r + (int64_t)u * G < nrows) x[u] = *reinterpret_cast<const double*>(base + o + u * step);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) s += x[u];
      }
    } else {
      for (int64_t r = g; r < nrows; r += (int64_t)U * G) {
        double x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          x[u] = 0.0;
          if (r + (int64_t)u * G < nrows) x[u] = part[(r + (int64_t)u * G) * nv + v];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) s += x[u];
      }
    }
    scratch[t] = s;
  }
  __syncthreads();
  // (each level's LDS reads are issued eight at a time, at clamped indices,
  // so that their latencies overlap)
  const int J = G < 8 ? G : 8;
  if (g < J) {
    double a = 0.0;
    for (int h0 = g; h0 < G; h0 += 8 * J) {
      double y[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int h = h0 + i * J;
        y[i] = scratch[(h < G ? h : g) * nv + v];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) a += h0 + i * J < G ? y[i] : 0.0;
    }
    scratch[t] = a;  // read by no other thread of this level
  }
  __syncthreads();
  if (t < nv) {
    double y[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) y[j] = scratch[(j < J ? j : 0) * nv + t];
    double a = y[0];
#pragma unroll
    for (int j = 1; j < 8; ++j) a += j < J ? y[j] : 0.0;
    res[t] = a;
  }
  __syncthreads();
}

__device__ inline void sum_rows(const double* __restrict__ part, int64_t nrows, int nv, double* scratch,
                                double* res) {
  sum_rows_t<kBlock>(part, nrows, nv, scratch, res);
}

// Kernel span (measurement support, used only when a launch is given a span
// record): span[0] the sum over launches of (last workgroup end - earliest
// workgroup start) on the device wall clock, span[1] the number of launches,
// then two stamps per workgroup of the running launch (start, end), written
// with plain stores to distinct addresses -- no atomics or fences in the
// measured kernel -- and reduced by the level-2 kernel that follows it.
__device__ __forceinline__ void span_begin(unsigned long long* span) {
  if (threadIdx.x == 0) span[2 + 2 * (int64_t)blockIdx.x] = wall_clock64();
}
__device__ inline void span_end(unsigned long long* span) {
  __syncthreads();
  if (threadIdx.x == 0) span[3 + 2 * (int64_t)blockIdx.x] = wall_clock64();
}
// In the level-2 kernel (one workgroup of TB threads, after the measured
// launch on the same stream): span_load takes each thread's share of the
// stamps of the launch's `blocks` workgroups (issued before the row sums, so
// that their latency overlaps them), span_add reduces them (wave shuffles,
// then one value per wave) and adds the launch's span to the record.
template <int TB>
__device__ __forceinline__ void span_load(const unsigned long long* span, int64_t blocks, unsigned long long& lo,
                                          unsigned long long& hi) {
  lo = ~0ull;
  hi = 0ull;
  for (int64_t b = threadIdx.x; b < blocks; b += TB) {
    const unsigned long long s0 = span[2 + 2 * b], s1 = span[3 + 2 * b];
    lo = s0 < lo ? s0 : lo;
    hi = s1 > hi ? s1 : hi;
  }
}
template <int TB>
__device__ inline void span_add(unsigned long long* span, int64_t blocks, unsigned long long lo,
                                unsigned long long hi, double* scratch) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    const unsigned long long ol = __shfl_xor(lo, d), oh = __shfl_xor(hi, d);
    lo = ol < lo ? ol : lo;
    hi = oh > hi ? oh : hi;
  }
  unsigned long long* u = reinterpret_cast<unsigned long long*>(scratch);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    u[2 * (threadIdx.x >> 6)] = lo;
    u[2 * (threadIdx.x >> 6) + 1] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0 && blocks > 0) {
    unsigned long long first = u[0], last = u[1];
    for (int w = 1; w < TB / 64; ++w) {
      first = u[2 * w] < first ? u[2 * w] : first;
      last = u[2 * w + 1] > last ? u[2 * w + 1] : last;
    }
    span[0] += last - first;
    span[1] += 1ull;
  }
  __syncthreads();
}

}  // namespace fn
