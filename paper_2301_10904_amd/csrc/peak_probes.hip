// peak_probes.hip -- measurement kernels, not part of the PIR path: the rates
// this GPU delivers for the four resources the PIR kernels are bounded by,
// each measured with a plain loop rather than taken from the data sheet.
//
//   kind 0  HBM reads: each workgroup streams its own contiguous share of a
//           buffer far larger than the caches with 16-byte non-temporal
//           loads, 16 in flight per lane, summing the words mod 2^32 (one
//           256-lane workgroup per CU reads fastest; a grid-stride loop over
//           the whole buffer, or more workgroups, read up to 15% slower)
//   kind 1  VALU: 16 independent chains of v_xor_b32 per lane
//   kind 2  LDS lookups: 8 independent chains of ds_read_b32 per lane, each
//           address made from the previous load by one v_and_or_b32, in the
//           T-table layout of the AES kernels (256-byte rows, the lane's own
//           copy of the entry; 64 KiB per workgroup).  Two 1024-lane
//           workgroups per CU (8 waves per SIMD): the LDS then serves more
//           lookups than with fewer waves (two 512-lane workgroups, as in the
//           AES kernels: about 7% fewer)
//   kind 3  int8 matrix cores: 8 independent v_mfma_i32_16x16x64_i8
//           accumulators per wave (the double-K form, which gfx950 runs at
//           its full int8 rate)
//   kind 4  the same with v_mfma_i32_16x16x32_i8, the form the PIR
//           contraction uses
//
// Every probe leaves one checksum word per lane, which the host can recompute
// from the probe's inputs: it shows that the loop did the work it is counted
// for.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint32_t PROBE_NT = 256; // lanes per workgroup (the LDS probe: 1024)
constexpr uint32_t LDS_NT = 1024;
constexpr uint32_t LDS_WORDS = 16384; // 256 rows of 64 words

// workgroup b reads vectors [b n4 / blocks, (b + 1) n4 / blocks)
__global__ __launch_bounds__(PROBE_NT) void k_peak_read(const uint32_t *__restrict__ in, uint64_t n4,
                                                        uint32_t *__restrict__ out)
{
    typedef unsigned v4u __attribute__((ext_vector_type(4)));
    constexpr uint32_t U = 16;
    const v4u *p = reinterpret_cast<const v4u *>(in);
    const uint64_t lo = (uint64_t)blockIdx.x * n4 / gridDim.x, hi = (uint64_t)(blockIdx.x + 1) * n4 / gridDim.x;
    uint64_t i = lo + threadIdx.x;
    uint32_t acc = 0;
    // U loads in flight per lane, then the tail one by one
    for (; i + (U - 1) * PROBE_NT < hi; i += U * PROBE_NT) {
        v4u v[U];
#pragma unroll
        for (uint32_t u = 0; u < U; u++)
            v[u] = __builtin_nontemporal_load(p + i + u * PROBE_NT);
#pragma unroll
        for (uint32_t u = 0; u < U; u++)
            acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
    }
    for (; i < hi; i += PROBE_NT) {
        const v4u a = __builtin_nontemporal_load(p + i);
        acc += a.x + a.y + a.z + a.w;
    }
    out[(uint64_t)blockIdx.x * PROBE_NT + threadIdx.x] = acc;
}

// lane g: chain c starts at g * 0x9e3779b9 + c and is XORed with k each
// iteration, so it ends at its start value XOR (k if iters is odd)
__global__ __launch_bounds__(PROBE_NT) void k_peak_valu(uint32_t iters, uint32_t k, uint32_t *__restrict__ out)
{
    const uint32_t g = blockIdx.x * PROBE_NT + threadIdx.x;
    uint32_t x[16];
#pragma unroll
    for (int c = 0; c < 16; c++)
        x[c] = g * 0x9e3779b9u + (uint32_t)c;
    for (uint32_t it = 0; it < iters; it++) {
#pragma unroll
        for (int c = 0; c < 16; c++)
            asm volatile("v_xor_b32 %0, %1, %0" : "+v"(x[c]) : "v"(k));
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < 16; c++)
        acc += x[c];
    out[g] = acc;
}

// word i of the table is i * 0x9e3779b9 ^ (i >> 5); chain c of lane t (t the
// lane's index in the workgroup, l = t mod 64) starts at t * 0x85ebca6b + c
// and steps v <- word ((v & 0xff80) | 4 (l mod 32)) / 4
__global__ __launch_bounds__(LDS_NT) void k_peak_lds(uint32_t iters, uint32_t *__restrict__ out)
{
    __shared__ uint32_t tab[LDS_WORDS];
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    for (uint32_t i = tid; i < LDS_WORDS; i += LDS_NT)
        tab[i] = (i * 0x9e3779b9u) ^ (i >> 5);
    __syncthreads();
    const uint32_t l4 = (lane & 31) << 2;
    const char *base = reinterpret_cast<const char *>(tab);
    uint32_t v[8];
#pragma unroll
    for (int c = 0; c < 8; c++)
        v[c] = tid * 0x85ebca6bu + (uint32_t)c;
    for (uint32_t it = 0; it < iters; it++) {
#pragma unroll
        for (int c = 0; c < 8; c++)
            v[c] = *reinterpret_cast<const uint32_t *>(base + ((v[c] & 0xff80u) | l4));
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < 8; c++)
        acc ^= v[c];
    out[blockIdx.x * LDS_NT + tid] = acc;
}

// lane g: A operand words w0 = g * 0x9e3779b9, w1 = g ^ 0x5bd1e995 (K64:
// also w2 = w0 ^ 0x3c6ef372, w3 = w1 ^ 0xa54ff53a), B operand the same words
// XOR 0x01234567, 0x89abcdef (K64: 0x0f1e2d3c, 0x4b5a6978); every
// accumulator adds the same product each iteration
template <bool K64>
__global__ __launch_bounds__(PROBE_NT) void k_peak_mfma(uint32_t iters, uint32_t *__restrict__ out)
{
    typedef int v4i __attribute__((ext_vector_type(4)));
    const uint32_t g = blockIdx.x * PROBE_NT + threadIdx.x;
    const uint32_t w0 = g * 0x9e3779b9u, w1 = g ^ 0x5bd1e995u;
    const v4i a4 = {(int)w0, (int)w1, (int)(w0 ^ 0x3c6ef372u), (int)(w1 ^ 0xa54ff53au)};
    const v4i b4 = {(int)(w0 ^ 0x01234567u), (int)(w1 ^ 0x89abcdefu), (int)(w0 ^ 0x3c6ef372u ^ 0x0f1e2d3cu),
                    (int)(w1 ^ 0xa54ff53au ^ 0x4b5a6978u)};
    const long a = (long)(((uint64_t)w1 << 32) | w0);
    const long b = (long)(((uint64_t)(w1 ^ 0x89abcdefu) << 32) | (w0 ^ 0x01234567u));
    v4i acc[8];
#pragma unroll
    for (int c = 0; c < 8; c++)
        acc[c] = v4i{0, 0, 0, 0};
    // an empty asm on the accumulators gives each its own registers before the
    // loop (otherwise the allocator rotates them through copies every iteration)
    asm volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5]),
                 "+v"(acc[6]), "+v"(acc[7]));
    for (uint32_t it = 0; it < iters; it++) {
#pragma unroll
        for (int c = 0; c < 8; c++) {
            if constexpr (K64)
                acc[c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a4, b4, acc[c], 0, 0, 0);
            else
                acc[c] = __builtin_amdgcn_mfma_i32_16x16x32_i8(a, b, acc[c], 0, 0, 0);
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int c = 0; c < 8; c++)
        s += (uint32_t)acc[c][0] + (uint32_t)acc[c][1] + (uint32_t)acc[c][2] + (uint32_t)acc[c][3];
    out[g] = s;
}

} // namespace

extern "C" {

// Runs probe `kind` (0 HBM read, 1 VALU, 2 LDS, 3 int8 MFMA 16x16x64, 4 int8
// MFMA 16x16x32) with `blocks` workgroups of 256 lanes (1024 for kind 2) on
// `stream`; `iters` loop iterations per lane for kinds 1..4.  Kind 0 reads in_words words at d_in
// (16-byte aligned, in_words a multiple of 4), workgroup b the b-th of
// `blocks` contiguous shares.  d_out receives one checksum
// word per lane: blocks * 256 words (blocks * 1024 for kind 2).  Returns 0, -1
// for bad arguments, -3 if the launch failed.
int pir_peak_probe(uint32_t kind, uint32_t blocks, uint32_t iters, const uint32_t *d_in, uint64_t in_words,
                   uint32_t *d_out, void *stream)
{
    if (!d_out || blocks == 0 || kind > 4)
        return -1;
    if (kind == 0 && (!d_in || in_words == 0 || in_words % 4 || ((uintptr_t)d_in % 16) ||
                      in_words / 4 > (UINT64_MAX >> 1) / blocks))
        return -1;
    hipStream_t st = (hipStream_t)stream;
    switch (kind) {
    case 0:
        hipLaunchKernelGGL(k_peak_read, dim3(blocks), dim3(PROBE_NT), 0, st, d_in, in_words / 4, d_out);
        break;
    case 1:
        hipLaunchKernelGGL(k_peak_valu, dim3(blocks), dim3(PROBE_NT), 0, st, iters, 0x6a09e667u, d_out);
        break;
    case 2:
        hipLaunchKernelGGL(k_peak_lds, dim3(blocks), dim3(LDS_NT), 0, st, iters, d_out);
        break;
    case 3:
        hipLaunchKernelGGL(k_peak_mfma<true>, dim3(blocks), dim3(PROBE_NT), 0, st, iters, d_out);
        break;
    default:
        hipLaunchKernelGGL(k_peak_mfma<false>, dim3(blocks), dim3(PROBE_NT), 0, st, iters, d_out);
        break;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

} // extern "C"
