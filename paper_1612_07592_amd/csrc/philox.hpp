// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11),
// host and device.  One call maps a 128-bit counter and a 64-bit key to four
// 32-bit words; the step kernels key it with (seed, job) and count with
// (electron id, step, purpose, 0), so a stream never depends on thread order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

struct U4 {
  uint32_t v[4];
};

__host__ __device__ inline U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    // two 32x32->64 products per round; their halves are permuted and keyed
    const uint64_t a = (uint64_t)0xD2511F53u * c0;
    const uint64_t b = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t t0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
    const uint32_t t2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)b;
    c3 = (uint32_t)a;
    c0 = t0;
    c2 = t2;
    k0 += 0x9E3779B9u;  // Weyl key schedule
    k1 += 0xBB67AE85u;
  }
  U4 r;
  r.v[0] = c0; r.v[1] = c1; r.v[2] = c2; r.v[3] = c3;
  return r;
}

// (r + 1/2) 2^-32: a double in (0, 1), exact.
__host__ __device__ inline double unif32(uint32_t r) { return ((double)r + 0.5) * 0x1p-32; }
// float in (0, 1) from the top 23 bits: (k + 1/2) 2^-23 with k < 2^23 needs
// 24 significant bits, so it is exact and never reaches 1.  (With 24 bits,
// k + 1/2 would round to 2^24 for the largest k and the draw would be 1.0.)
__host__ __device__ inline float unif23f(uint32_t r) { return ((float)(r >> 9) + 0.5f) * 0x1p-23f; }
// 52-bit uniform from two words: (k + 1/2) 2^-52, k < 2^52, exact in double.
__host__ __device__ inline double unif52(uint32_t r0, uint32_t r1) {
  const uint64_t k = ((uint64_t)r0 << 20) | (uint64_t)(r1 >> 12);
  return ((double)k + 0.5) * 0x1p-52;
}

}  // namespace pic
