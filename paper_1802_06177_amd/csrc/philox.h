// Philox4x32-10 counter-based generator, written from its published definition (J. K.
// Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as
// 1, 2, 3", SC'11): 10 rounds, each multiplying counter words 0 and 2 by the two round
// multipliers and mixing the 64-bit products' halves with words 1 and 3 and the key, the
// key bumped by the two Weyl constants between rounds.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slmc {

struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox(U4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    U4 n;
    n.x = hi1 ^ c.y ^ k0;
    n.y = lo1;
    n.z = hi0 ^ c.w ^ k1;
    n.w = lo0;
    c = n;
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// u = (r + 1/2) 2^-32 in (0, 1), exact in FP64
__device__ __forceinline__ double u01(uint32_t r) {
  return ((double)r + 0.5) * 2.3283064365386962890625e-10;   // 2^-32
}

// The per-proposal coin of the cumulative proposal: forward phase order (and local sweeps
// before cluster moves) iff word 0 at counter (0xFFFFFFFF, 0xFFFFFFFE, proposal, chain)
// is below 2^31.
__device__ __forceinline__ bool proposal_forward(uint32_t prop, uint32_t chain, uint32_t k0,
                                                 uint32_t k1) {
  return philox(U4{0xFFFFFFFFu, 0xFFFFFFFEu, prop, chain}, k0, k1).x < 0x80000000u;
}

}  // namespace slmc
