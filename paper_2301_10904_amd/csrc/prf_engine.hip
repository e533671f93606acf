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
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pir_kernels.h"

namespace {

template <class PRF>
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
        P.pair_word0(a, y0, y1);    // a bottom node: word 0 of both leaves
        acc += y0 ^ y1;
        s[0] = b[0];
        s[1] = b[1];
        s[2] = b[2] ^ acc;
        s[3] = b[3];
    }
    out[gid] = acc;
}

} // namespace

extern "C" {

// Runs the engine kernel with `blocks` workgroups of 512 lanes, `steps` steps
// (two nodes each) per lane, on `stream`; out receives blocks * 512 words.
// prf_id: 0 = AES-128, 1 = ChaCha20.  Returns 0, or -1 for bad arguments.
int pir_prf_engine(uint32_t prf_id, uint32_t blocks, uint32_t steps, uint32_t *d_out, void *stream)
{
    if (!d_out || blocks == 0 || prf_id > 1)
        return -1;
    hipStream_t st = (hipStream_t)stream;
    if (prf_id == 0)
        hipLaunchKernelGGL(k_prf_engine<AesPrf>, dim3(blocks), dim3(NT), 0, st, steps, d_out);
    else
        hipLaunchKernelGGL(k_prf_engine<ChaChaPrf>, dim3(blocks), dim3(NT), 0, st, steps, d_out);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

} // extern "C"
