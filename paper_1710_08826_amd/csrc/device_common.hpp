// Device helpers: the deterministic two-level FP64 reduction.
//
// Level 1 (inside an evaluation kernel): every workgroup owns one fixed chunk
// of events.  Each thread sums its events in index order, the 64 lanes of a
// wave combine with a fixed xor butterfly, and the 4 waves combine through
// LDS in wave order.  The workgroup writes one row of NV doubles.
// Level 2 (a single workgroup): rows are summed in a fixed interleaving that
// depends only on the number of rows and NV.
// Nothing depends on scheduling, so results are bitwise reproducible, and a
// fit computes the same bits alone or inside a batch.
#pragma once
#include "model.hpp"

namespace fn {

template <int NV>
__device__ inline void block_sum_row(double (&v)[NV], double* lds /* kWaves*NV */,
                                     double* __restrict__ out_row) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double x = v[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    v[i] = x;
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) lds[wave * NV + i] = v[i];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NV; i += kBlock) {
    double s = lds[i];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += lds[w * NV + i];
    out_row[i] = s;
  }
}

// Level 2: res[v] = sum over rows r of part[r*nv + v], for v < nv <= kBlock.
// Thread t takes column t % nv and rows g, g+G, g+2G, ... with g = t / nv,
// G = kBlock / nv, in sixteen interleaved partial sums (sixteen independent
// loads in flight per thread: the rows were just written by other compute
// units, so this step is load-latency bound); the partial sums are added
// pairwise and the groups in order of g.  scratch holds kBlock doubles.
__device__ inline void sum_rows(const double* __restrict__ part, int64_t nrows, int nv,
                                double* scratch, double* res) {
  constexpr int U = 16;
  const int t = threadIdx.x;
  const int G = kBlock / nv;
  const int g = t / nv;
  const int v = t - g * nv;
  double s = 0.0;
  if (g < G) {
    double a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] = 0.0;
    int64_t r = g;
    const int64_t step = G;
    for (; r + (U - 1) * step < nrows; r += U * step) {
      double x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = part[(r + u * step) * nv + v];
#pragma unroll
      for (int u = 0; u < U; ++u) a[u] += x[u];
    }
    for (; r < nrows; r += step) a[0] += part[r * nv + v];
#pragma unroll
    for (int w = U / 2; w > 0; w >>= 1)
#pragma unroll
      for (int u = 0; u < w; ++u) a[u] += a[u + w];
    s = a[0];
  }
  scratch[t] = s;
  __syncthreads();
  if (t < nv) {
    double acc = scratch[t];
    for (int gg = 1; gg < G; ++gg) acc += scratch[gg * nv + t];
    res[t] = acc;
  }
  __syncthreads();
}

}  // namespace fn
