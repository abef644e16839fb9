// philox.h -- Philox4x32-10 counter-based generator for the device (Salmon, Moraes, Dror, Shaw, SC11 2011).
// Each round multiplies counter words 0 and 2 by 0xD2511F53 / 0xCD9E8D57 (32x32 -> 64 bits), xors the high
// halves with the other two counter words and the key, and moves the low halves into the odd slots; the
// key advances by the Weyl increments 0x9E3779B9 / 0xBB67AE85 between rounds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmc {

struct Philox4 {
  uint32_t v[4];
};

// a ^ b ^ c in one gfx950 three-input bitwise instruction (truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                 uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t m0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t m1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t n0 = xor3((uint32_t)(m1 >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(m0 >> 32), c3, k1);
    c1 = (uint32_t)m1;
    c3 = (uint32_t)m0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Philox4 out;
  out.v[0] = c0;
  out.v[1] = c1;
  out.v[2] = c2;
  out.v[3] = c3;
  return out;
}

}  // namespace bmc
