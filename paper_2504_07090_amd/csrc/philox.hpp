// Philox-4x32-10 (Salmon, Moraes, Dror & Shaw 2011, "Parallel random numbers:
// as easy as 1, 2, 3") and Box-Muller normals on the device.  A 4-word
// counter and a 2-word key; each of 10 rounds multiplies counter words 0 and 2
// by 0xD2511F53 and 0xCD9E8D57 and recombines the 64-bit products' halves with
// the other words and the key; the key is bumped by 0x9E3779B9 and 0xBB67AE85
// between rounds.  Counter word 3 names the purpose of a stream: 0 HMC momenta,
// 1 the Metropolis uniform, 2-4 NUTS decisions, 5 Hutchinson probes of the
// mass-matrix estimate.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bv {

__device__ __forceinline__ uint4 philox_round(uint4 c, uint2 k) {
  const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
  const uint32_t hi0 = __umulhi(m0, c.x), lo0 = m0 * c.x;
  const uint32_t hi1 = __umulhi(m1, c.z), lo1 = m1 * c.z;
  return make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
}

__device__ inline uint4 philox10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    c = philox_round(c, k);
  }
  return c;
}

// (x + 1/2) 2^-32, strictly inside (0, 1)
__device__ __forceinline__ double unit_open(uint32_t x) {
  return (static_cast<double>(x) + 0.5) * 2.3283064365386963e-10;  // 2^-32
}

// Four normals from counter (j, c1, c2, purpose) by Box-Muller:
// r = sqrt(-2 ln u1), (r cos 2 pi u2, r sin 2 pi u2) from words (0, 1) and (2, 3).
__device__ __forceinline__ void philox_normals4(uint64_t seed, uint32_t j, uint32_t c1, uint32_t c2,
                                                uint32_t purpose, float z[4]) {
  const uint4 x = philox10(make_uint4(j, c1, c2, purpose),
                           make_uint2(static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32)));
  const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float r = sqrtf(-2.0f * logf(static_cast<float>(unit_open(w[2 * h]))));
    float s, c;
    sincospif(2.0f * static_cast<float>(unit_open(w[2 * h + 1])), &s, &c);
    z[2 * h] = r * c;
    z[2 * h + 1] = r * s;
  }
}

// Normals 4j .. 4j+3 of the (trajectory, stream) momentum sequence.
__device__ __forceinline__ void normals4(uint64_t seed, uint32_t stream, uint32_t traj, uint32_t j,
                                         float z[4]) {
  philox_normals4(seed, j, traj, stream, 0u, z);
}

}  // namespace bv
