// Counter-based random numbers of the environments and the policy: Philox
// with Box-Muller normals. Counter (env, step lo, step hi, block), key
// (seed lo, seed hi). Blocks 0..3 give the action noise of joints 0..15;
// the tracking task's goal draws use blocks 8 (velocity increment) and 9
// (new episode centre); per-episode re-randomisation uses block 10.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sgk {

enum { RNG_BLOCK_GOAL_ACCEL = 8, RNG_BLOCK_GOAL_RESET = 9, RNG_BLOCK_RERAND = 10 };

// ---- Philox4x32-10 (Salmon et al., SC'11) --------------------------------
// Ten rounds of: two 32x32->64 multiplies by the round constants, with the
// high halves xored into the other two words together with the key; the key
// advances by the Weyl constants between rounds.
struct U4 {
  uint32_t x, y, z, w;
};
__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t p0_hi = __umulhi(0xD2511F53u, c.x), p0_lo = 0xD2511F53u * c.x;
    const uint32_t p1_hi = __umulhi(0xCD9E8D57u, c.z), p1_lo = 0xCD9E8D57u * c.z;
    c = U4{p1_hi ^ c.y ^ k0, p1_lo, p0_hi ^ c.w ^ k1, p0_lo};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Standard normals for joints 0..J-1 of (env, step) by Box-Muller on 24-bit
// uniforms ((x >> 8) + 0.5) / 2^24, pairs (x, y) and (z, w) of each block.
template <int J>
__device__ __forceinline__ void normals(uint64_t seed, uint32_t env, uint64_t step, int n, float (&eps)[J]) {
#pragma unroll
  for (int b = 0; 4 * b < J; ++b) {
    const U4 r = philox10(U4{env, (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)b}, (uint32_t)seed,
                          (uint32_t)(seed >> 32));
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const float u1 = ((float)(w[2 * p] >> 8) + 0.5f) * (1.0f / 16777216.0f);
      const float u2 = ((float)(w[2 * p + 1] >> 8) + 0.5f) * (1.0f / 16777216.0f);
      const float rad = sqrtf(-2.f * logf(u1));
      float s, c;
      sincospif(2.f * u2, &s, &c);
      const int j0 = 4 * b + 2 * p;
      if (j0 < J) eps[j0] = j0 < n ? rad * c : 0.f;
      if (j0 + 1 < J) eps[j0 + 1] = j0 + 1 < n ? rad * s : 0.f;
    }
  }
}

// Four standard normals of one block: Box-Muller pairs (x, y) and (z, w).
__device__ __forceinline__ void normals4(uint64_t seed, uint32_t env, uint64_t step, uint32_t block, float* out) {
  const U4 r = philox10(U4{env, (uint32_t)step, (uint32_t)(step >> 32), block}, (uint32_t)seed,
                        (uint32_t)(seed >> 32));
  const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const float u1 = ((float)(w[2 * p] >> 8) + 0.5f) * (1.0f / 16777216.0f);
    const float u2 = ((float)(w[2 * p + 1] >> 8) + 0.5f) * (1.0f / 16777216.0f);
    const float rad = sqrtf(-2.f * logf(u1));
    float sn, cs;
    sincospif(2.f * u2, &sn, &cs);
    out[2 * p] = rad * cs;
    out[2 * p + 1] = rad * sn;
  }
}

}  // namespace sgk
