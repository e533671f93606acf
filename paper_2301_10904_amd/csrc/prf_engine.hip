// prf_engine.hip -- a measurement kernel, not part of the PIR path: the PRF
// work of the tree walk with nothing else around it, to give the PRF-engine
// ceiling that the fused kernels are compared against.
//
// Every lane evaluates a chain of nodes with the same mix as a depth-first
// walk step: both children of a full node (two blocks and one key expansion),
// then word 0 of both outputs of a bottom node (what a leaf pair needs), with
// each node keyed by the previous one's output so that nothing can be hoisted
// or dropped.  It uses the walk kernels' PRF code, LDS tables and workgroup
// shape (512 lanes; the AES tables take 64 KiB, two workgroups per CU) but no
// codewords, table reads, contraction or atomics.  One checksum word per lane
// keeps the work observable.
//
// Two more chains compare the PRF codes node for node: full nodes only
// (both children of every node) with the T-table rounds, and the same with the
// bitsliced rounds of aes_bitsliced_gfx950.h, where a quad of lanes evaluates
// 32 nodes per step.  pir_prf_bitsliced_pairs evaluates the bitsliced PRF on
// given seeds, so that its outputs can be checked.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aes_bitsliced_gfx950.h"
#include "pir_kernels.h"

namespace {

template <class PRF, bool FULL_ONLY = false>
__global__ __launch_bounds__(NT) void k_prf_engine(uint32_t steps, uint32_t *out)
{
    __shared__ uint32_t tab[PRF::TAB_WORDS ? PRF::TAB_WORDS : 1];
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    const PRF P(tab, lane);
    if (PRF::TAB_WORDS) {
        PRF::fill(tab, tid, NT);
        __syncthreads();
    }
    const uint32_t gid = blockIdx.x * NT + tid;
    uint32_t s[4] = {gid, 0x9e3779b9u * (gid + 1), steps, 0x7f4a7c15u};
    uint32_t acc = 0;
    for (uint32_t m = 0; m < steps; m++) {
        uint32_t a[4], b[4], y0, y1;
        P.pair(s, a, b);            // a full node: both children
        if (FULL_ONLY) {            // the next node is keyed by both outputs
            acc ^= a[0];
            s[0] = b[0] ^ a[1];
            s[1] = b[1] ^ a[2];
            s[2] = b[2] ^ a[3];
            s[3] = b[3] ^ a[0];
            continue;
        }
        P.pair_word0(a, y0, y1);    // a bottom node: word 0 of both leaves
        acc += y0 ^ y1;
        s[0] = b[0];
        s[1] = b[1];
        s[2] = b[2] ^ acc;
        s[3] = b[3];
    }
    out[gid] = acc;
}

constexpr int BS_NT = 256; // lanes per workgroup of the bitsliced kernels (64 quads)

// Full nodes only, bitsliced: every quad evaluates 32 nodes per step, each
// keyed by the XOR of its predecessor's two outputs (as the T-table chain).
__global__ __launch_bounds__(BS_NT) void k_prf_engine_bitsliced(uint32_t steps, uint32_t *out)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    const pir_bs::QuadMasks Q(lane);
    const uint32_t gid = blockIdx.x * BS_NT + tid;
    uint32_t s[32];
#pragma unroll
    for (int i = 0; i < 32; i++)
        s[i] = (gid + 1) * 0x9e3779b9u ^ (uint32_t)i * 0x85ebca6bu ^ steps;
    uint32_t acc = 0;
    for (uint32_t m = 0; m < steps; m++) {
        uint32_t a[32], b[32];
        pir_bs::prf_pair(s, a, b, Q);
        acc ^= a[0];
#pragma unroll
        for (int i = 0; i < 32; i++)
            s[i] = b[i] ^ a[(i + 1) & 31];
    }
    out[gid] = acc;
}

// PRF_s(0) and PRF_s(1) of n seeds (16 bytes each, as four little-endian
// words) into out[8 i .. 8 i + 7]: quad j takes seeds 32 j .. 32 j + 31, lane
// q of it column q, transposed into bit planes and back.
__global__ __launch_bounds__(BS_NT) void k_prf_bitsliced_pairs(const uint32_t *seeds, uint32_t n, uint32_t *out)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63, q = lane & 3;
    const pir_bs::QuadMasks Q(lane);
    const uint32_t node0 = ((blockIdx.x * BS_NT + tid) >> 2) * 32;
    uint32_t s[32], a[32], b[32];
#pragma unroll
    for (int i = 0; i < 32; i++)
        s[i] = node0 + i < n ? seeds[(size_t)(node0 + i) * 4 + q] : 0u;
    pir_bs::transpose32(s);
    pir_bs::prf_pair(s, a, b, Q);
    pir_bs::transpose32(a);
    pir_bs::transpose32(b);
#pragma unroll
    for (int i = 0; i < 32; i++)
        if (node0 + i < n) {
            out[(size_t)(node0 + i) * 8 + q] = a[i];
            out[(size_t)(node0 + i) * 8 + 4 + q] = b[i];
        }
}

} // namespace

extern "C" {

// Runs an engine kernel on `stream` with `blocks` workgroups and `steps`
// steps per lane; out receives one word per lane.  kind:
//   0 = AES-128 T-table, 1 = ChaCha20: 512 lanes per workgroup, a step is one
//       full and one bottom node per lane;
//   2 = AES-128 T-table, full nodes only: 512 lanes, one full node per lane
//       and step;
//   3 = AES-128 bitsliced, full nodes only: 256 lanes, 32 full nodes per quad
//       of lanes and step (8 per lane).
// Returns 0, -1 for bad arguments, -3 for a launch error.
int pir_prf_engine(uint32_t kind, uint32_t blocks, uint32_t steps, uint32_t *d_out, void *stream)
{
    if (!d_out || blocks == 0 || kind > 3)
        return -1;
    hipStream_t st = (hipStream_t)stream;
    if (kind == 0)
        hipLaunchKernelGGL(k_prf_engine<AesPrf>, dim3(blocks), dim3(NT), 0, st, steps, d_out);
    else if (kind == 1)
        hipLaunchKernelGGL(k_prf_engine<ChaChaPrf>, dim3(blocks), dim3(NT), 0, st, steps, d_out);
    else if (kind == 2)
        hipLaunchKernelGGL((k_prf_engine<AesPrf, true>), dim3(blocks), dim3(NT), 0, st, steps, d_out);
    else
        hipLaunchKernelGGL(k_prf_engine_bitsliced, dim3(blocks), dim3(BS_NT), 0, st, steps, d_out);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// Lanes per workgroup of engine kind `kind` (512, or 256 for the bitsliced
// engine), 0 for an unknown kind.
uint32_t pir_prf_engine_lanes(uint32_t kind)
{
    return kind <= 2 ? (uint32_t)NT : kind == 3 ? (uint32_t)BS_NT : 0u;
}

// The bitsliced AES-128 PRF on n seeds: d_seeds holds n 16-byte seeds (four
// little-endian words each), d_out receives 8 n words, PRF_s(0) then PRF_s(1)
// per seed.  Device pointers, 4-byte aligned; runs on `stream`.  Returns 0,
// -1 for bad arguments, -3 for a launch error.
int pir_prf_bitsliced_pairs(const uint32_t *d_seeds, uint32_t n, uint32_t *d_out, void *stream)
{
    if (n == 0)
        return 0;
    if (!d_seeds || !d_out || n > (1u << 26))
        return -1;
    const uint32_t lanes = (n + 31) / 32 * 4, blocks = (lanes + BS_NT - 1) / BS_NT;
    hipLaunchKernelGGL(k_prf_bitsliced_pairs, dim3(blocks), dim3(BS_NT), 0, (hipStream_t)stream, d_seeds, n,
                       d_out);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

} // extern "C"
