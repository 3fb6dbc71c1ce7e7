// Counter-based uniforms for the device event generators: Philox4x32-10
// (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2,
// 3", SC'11).  Counter (i mod 2^32, i >> 32, stream, word), key (k0, k1).
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>

#include <cstdint>
#else
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
#endif

namespace fn {

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64 multiplications with the published multipliers and Weyl key
// increments.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Two uniforms in [0, 1) from counter (i, stream, word): 53-bit mantissas of
// the 64-bit words (w0:w1) and (w2:w3).
__device__ __forceinline__ void philox_uniforms(uint64_t i, uint32_t stream, uint32_t word, uint32_t k0,
                                                uint32_t k1, double& ua, double& ub) {
  uint32_t c[4] = {(uint32_t)i, (uint32_t)(i >> 32), stream, word};
  philox4x32_10(c, k0, k1);
  const uint64_t a = (((uint64_t)c[0] << 32) | c[1]) >> 11;
  const uint64_t b = (((uint64_t)c[2] << 32) | c[3]) >> 11;
  ua = (double)a * 0x1.0p-53;
  ub = (double)b * 0x1.0p-53;
}

}  // namespace fn
