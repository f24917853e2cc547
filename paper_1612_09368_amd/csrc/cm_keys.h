// Iteration-stamped selection keys of the superior-edge-set partition.
//
// An iteration with stamp ep runs `rounds` claim rounds; round r of it has
// the round number sr = ep * rounds + r.  A claim key is (high word
// 0xFFFFFFFF - sr, low word a bijective hash of the item), so keys of later
// rounds are smaller and win an atomicMin over any claim left from an
// earlier round without clearing the claim array; a vertex matched in round
// r stores sr + 1.  These stay exact while sr fits in 32 bits: before an
// iteration would get a stamp above the handle's stamp limit (at most
// EPOCH_REWIND), the kernel restarts the stamps at an iteration boundary --
// it clears every array that holds a stamp (claim, matched, stamp, chg, cd,
// the selection stamps of the batch) and continues from ep = 0 or 1 (the
// parity of ep selects the remaining-edge list of the next iteration).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cm {

constexpr int MAX_ROUNDS = 8;                // claim rounds per iteration, at most
constexpr int32_t EPOCH_REWIND = 1 << 28;    // largest stamp limit
static_assert((unsigned long long)(EPOCH_REWIND + 1) * MAX_ROUNDS + MAX_ROUNDS < (1ull << 32),
              "round numbers must stay below 2^32");

__host__ __device__ __forceinline__ uint32_t round_no(int32_t ep, int rounds, int r) {
    return (uint32_t)ep * (uint32_t)rounds + (uint32_t)r;
}
// high word of the claim keys of round r of iteration ep (smaller wins)
__host__ __device__ __forceinline__ unsigned long long claim_hi(int32_t ep, int rounds, int r) {
    return (unsigned long long)(0xFFFFFFFFu - round_no(ep, rounds, r)) << 32;
}
// stamp left by a vertex matched in round r of iteration ep
__host__ __device__ __forceinline__ uint32_t matched_stamp(int32_t ep, int rounds, int r) {
    return round_no(ep, rounds, r) + 1u;
}
// m was matched in an earlier round (0 .. r-1) of iteration ep
__host__ __device__ __forceinline__ bool matched_before(uint32_t m, int32_t ep, int rounds, int r) {
    const uint32_t lo = round_no(ep, rounds, 0) + 1u;
    const uint32_t hi = round_no(ep, rounds, r);
    return m >= lo && m <= hi;
}

}  // namespace cm
