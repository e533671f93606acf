// chacha_gfx950.h -- ChaCha20 as the PRF of the DPF tree, for CDNA4 lanes.
//
// The paper's alternative to AES is the ChaCha20 stream cipher (section 3.2.6,
// Table 5).  Here PRF_s(x) is bytes [16x, 16x+16) of the RFC 8439 keystream
// under the 256-bit key s || s with nonce 0 and block counter 0, so one block
// function call yields both children of a node: PRF_s(0) is state words 0..3
// and PRF_s(1) words 4..7 of the first keystream block.
//
// The block function is pure 32-bit VALU work: per quarter round four adds,
// four XORs and four rotations (each rotation is one v_alignbit_b32), eighty
// quarter rounds per block, no memory traffic and no LDS.  The input state is
// four constants, the seed twice and four zero words; the compiler folds the
// zero words into the first round and drops the parts of the last round whose
// outputs are not used (words 8..15 always; all but words 0 and 4 at the
// leaves).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "quad_gfx950.h"

namespace pir_dev {

// "expand 32-byte k" as four little-endian words
constexpr uint32_t CHACHA_C0 = 0x61707865u, CHACHA_C1 = 0x3320646eu, CHACHA_C2 = 0x79622d32u,
                   CHACHA_C3 = 0x6b206574u;

__device__ __forceinline__ uint32_t rotl32(uint32_t x, uint32_t n) { return __builtin_amdgcn_alignbit(x, x, 32 - n); }

__device__ __forceinline__ void quarter(uint32_t &a, uint32_t &b, uint32_t &c, uint32_t &d)
{
    a += b;
    d = rotl32(d ^ a, 16);
    c += d;
    b = rotl32(b ^ c, 12);
    a += b;
    d = rotl32(d ^ a, 8);
    c += d;
    b = rotl32(b ^ c, 7);
}

// The twenty rounds for key s || s, counter 0, nonce 0 (state before the
// input is added back).
__device__ __forceinline__ void chacha_rounds(const uint32_t s[4], uint32_t x[16])
{
    x[0] = CHACHA_C0;
    x[1] = CHACHA_C1;
    x[2] = CHACHA_C2;
    x[3] = CHACHA_C3;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        x[4 + i] = s[i];
        x[8 + i] = s[i];
        x[12 + i] = 0u;
    }
#pragma unroll
    for (int r = 0; r < 10; r++) {
        quarter(x[0], x[4], x[8], x[12]);
        quarter(x[1], x[5], x[9], x[13]);
        quarter(x[2], x[6], x[10], x[14]);
        quarter(x[3], x[7], x[11], x[15]);
        quarter(x[0], x[5], x[10], x[15]);
        quarter(x[1], x[6], x[11], x[12]);
        quarter(x[2], x[7], x[8], x[13]);
        quarter(x[3], x[4], x[9], x[14]);
    }
}

// a = PRF_s(0), b = PRF_s(1)
__device__ __forceinline__ void chacha_pair(const uint32_t s[4], uint32_t a[4], uint32_t b[4])
{
    uint32_t x[16];
    chacha_rounds(s, x);
    a[0] = x[0] + CHACHA_C0;
    a[1] = x[1] + CHACHA_C1;
    a[2] = x[2] + CHACHA_C2;
    a[3] = x[3] + CHACHA_C3;
#pragma unroll
    for (int i = 0; i < 4; i++)
        b[i] = x[4 + i] + s[i];
}

// a = PRF_s(c), c in {0, 1}
__device__ __forceinline__ void chacha_one(const uint32_t s[4], uint32_t c, uint32_t a[4])
{
    uint32_t lo[4], hi[4];
    chacha_pair(s, lo, hi);
#pragma unroll
    for (int i = 0; i < 4; i++)
        a[i] = c ? hi[i] : lo[i];
}

// word 0 of PRF_s(0) and of PRF_s(1): all a leaf share needs
__device__ __forceinline__ void chacha_pair_word0(const uint32_t s[4], uint32_t &y0, uint32_t &y1)
{
    uint32_t x[16];
    chacha_rounds(s, x);
    y0 = x[0] + CHACHA_C0;
    y1 = x[4] + s[0];
}

// Quad form (quad_gfx950.h): lane q of the quad holds column q of the state,
// words q, 4 + q, 8 + q, 12 + q, which start as the constant word q, the seed
// word q (twice) and zero -- the lane's own seed word is all it needs.  The
// column round is one quarter round per lane with no exchange; for the
// diagonal round lane q takes word 4 + (q+1) mod 4, 8 + (q+2) mod 4 and
// 12 + (q+3) mod 4 from its neighbours and gives them back afterwards.  At the
// end lane q holds word q of PRF_s(0) and word q of PRF_s(1) (state word 4 + q).
__device__ __forceinline__ void quad_chacha_pair(uint32_t s, uint32_t &a, uint32_t &b, const Quad &Q)
{
    const uint32_t cw[4] = {CHACHA_C0, CHACHA_C1, CHACHA_C2, CHACHA_C3};
    const uint32_t c = Q.own(cw);
    uint32_t xa = c, xb = s, xc = s, xd = 0u;
#pragma unroll
    for (int r = 0; r < 10; r++) {
        quarter(xa, xb, xc, xd);
        xb = quad_next<1>(xb);
        xc = quad_next<2>(xc);
        xd = quad_next<3>(xd);
        quarter(xa, xb, xc, xd);
        xb = quad_next<3>(xb);
        xc = quad_next<2>(xc);
        xd = quad_next<1>(xd);
    }
    a = xa + c;
    b = xb + s;
}

__device__ __forceinline__ uint32_t quad_chacha_one(uint32_t s, uint32_t c, const Quad &Q)
{
    uint32_t a, b;
    quad_chacha_pair(s, a, b, Q);
    return c ? b : a;
}

} // namespace pir_dev
