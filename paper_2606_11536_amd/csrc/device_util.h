// Small device helpers shared by the kernels: exact modular arithmetic for
// primes q < 2^28 in 32-bit registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pir {

// x * w mod q, lazily in [0, 2q), for any x < 2^32 and w < q with
// wsh = floor(w * 2^32 / q) (Shoup's precomputed quotient).
__device__ __forceinline__ uint32_t mul_shoup(uint32_t x, uint32_t w, uint32_t wsh, uint32_t q) {
  return x * w - __umulhi(x, wsh) * q;
}

// x - m if x >= m, else x.
__device__ __forceinline__ uint32_t csub(uint32_t x, uint32_t m) { return x >= m ? x - m : x; }

// Map a block index to a logical work index so that the blocks dispatched to
// one XCD (blocks are dealt round-robin over the 8 XCDs) take a contiguous run
// of logical indices.  `grid` must be a multiple of 8; logical indices at or
// beyond `total` are idle.
__device__ __forceinline__ uint32_t xcd_logical(uint32_t bid, uint32_t grid) {
  const uint32_t per = grid >> 3;
  return (bid & 7u) * per + (bid >> 3);
}

}  // namespace pir
