// quad_gfx950.h -- four lanes evaluating one PRF block together.
//
// Walking one key's path from the root is a chain of dependent PRF calls, so
// its speed is the latency of one call.  In the quad form the four lanes
// 4j..4j+3 of a quad share a node, lane q owning column q (word q) of the
// state, and exchange words through DPP quad permutes, which are plain VALU
// operands; each lane's chain of dependent operations is then about a quarter
// as long.  All four lanes of a quad must be active when a quad form runs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pir_dev {

struct Quad {
    bool q1, q2, q3;  // this lane's column: 1, 2 or 3 (none: column 0)
    uint32_t lo, hi;  // all-ones where bit 0 / bit 1 of the column is set
    __device__ __forceinline__ explicit Quad(uint32_t lane)
        : q1((lane & 3) == 1), q2((lane & 3) == 2), q3((lane & 3) == 3), lo(0u - (lane & 1)), hi(0u - ((lane >> 1) & 1))
    {
    }
    // k[q] for this lane's column q, as two levels of bit selects (a select
    // chain on q is compiled into an indexed scratch access)
    __device__ __forceinline__ uint32_t own(const uint32_t k[4]) const
    {
        const uint32_t k01 = (k[1] & lo) | (k[0] & ~lo), k23 = (k[3] & lo) | (k[2] & ~lo);
        return (k23 & hi) | (k01 & ~hi);
    }
};

// word of the quad lane (q + K) mod 4
template <int K>
__device__ __forceinline__ uint32_t quad_next(uint32_t x)
{
    constexpr int ctrl = K == 1 ? 0x39 : K == 2 ? 0x4E : 0x93; // quad_perm [1,2,3,0], [2,3,0,1], [3,0,1,2]
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, ctrl, 0xf, 0xf, false);
}
// word of quad lane 0 (column 0)
__device__ __forceinline__ uint32_t quad_first(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x00, 0xf, 0xf, false);
}

} // namespace pir_dev
