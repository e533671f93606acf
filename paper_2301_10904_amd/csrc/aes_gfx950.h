// aes_gfx950.h -- AES-128 for the PRF of the DPF tree, written for CDNA4 lanes.
//
// Every internal node of the tree needs AES-128 under its own seed as key of
// the two counter blocks 0 and 1 (one key expansion, two encryptions).  The
// round function uses the combined SubBytes/MixColumns table TE (see
// aes_tables.h) and its byte rotation TE8 = rotl(TE, 8), both resident in LDS:
//
//   table byte offset  x * 256 + j * 4        (j = lane mod 32):  TE[x]
//   table byte offset  x * 256 + 128 + j * 4  (j = lane mod 32):  TE8[x]
//
// so each lane reads its own copy and a lookup never meets a bank conflict.
// The address of a lookup is one v_perm_b32: byte r of a state word goes to
// address byte 1 and the lane's offset (< 256) to address byte 0.  With TE and
// TE8 a MixColumns column needs one rotation instead of three:
//   out = TE[a0] ^ TE8[b1] ^ rotl16(TE[c2] ^ TE8[d3] ^ rotr16(k)),
// and the three-input XORs are single v_bitop3_b32 instructions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aes_tables.h"
#include "quad_gfx950.h"

namespace pir_dev {

typedef const __attribute__((address_space(3))) uint32_t lds_u32;
typedef const __attribute__((address_space(3))) uint8_t lds_u8;

constexpr uint32_t AES_TAB_WORDS = 256 * 64; // 64 KiB

// The table base and this lane's offsets into the two table halves.  Every
// lookup address is formed from `base`, so the compiler sees the reads of the
// table (an address made from a bare integer would let it drop the fill).
struct Lanes {
    lds_u8 *base;
    uint32_t te, te8;
    __device__ __forceinline__ Lanes(const uint32_t *tab, uint32_t lane)
        : base((lds_u8 *)tab), te((lane & 31) * 4), te8((lane & 31) * 4 + 128)
    {
    }
    __device__ __forceinline__ uint32_t word(uint32_t byte_off) const { return *(lds_u32 *)(base + byte_off); }
};

template <int R>
__device__ __forceinline__ uint32_t addr(uint32_t w, uint32_t off)
{
    return __builtin_amdgcn_perm(w, off, 0x0c0c0000u | ((4u + R) << 8));
}

template <int R>
__device__ __forceinline__ uint32_t te(uint32_t w, const Lanes &L) { return L.word(addr<R>(w, L.te)); }
template <int R>
__device__ __forceinline__ uint32_t te8(uint32_t w, const Lanes &L) { return L.word(addr<R>(w, L.te8)); }

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t rot16(uint32_t x) { return __builtin_amdgcn_alignbit(x, x, 16); }

// S(x) is byte 1 of TE[x].  pick01(hi, lo) = S-bytes of lo, hi into bytes 0, 1;
// pick23(hi, lo) = S-bytes of lo, hi into bytes 2, 3.
__device__ __forceinline__ uint32_t pick01(uint32_t hi, uint32_t lo) { return __builtin_amdgcn_perm(hi, lo, 0x0c0c0501u); }
__device__ __forceinline__ uint32_t pick23(uint32_t hi, uint32_t lo) { return __builtin_amdgcn_perm(hi, lo, 0x05010c0cu); }

// One MixColumns output column; kr = rotl16 (= rotr16) of the round-key word.
__device__ __forceinline__ uint32_t mcol(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t kr, const Lanes &L)
{
    uint32_t u = xor3(te<2>(c, L), te8<3>(d, L), kr);
    return xor3(te<0>(a, L), te8<1>(b, L), rot16(u));
}

// One output column of the last round (SubBytes, ShiftRows, AddRoundKey).
__device__ __forceinline__ uint32_t fcol(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t k, const Lanes &L)
{
    return xor3(pick01(te<1>(b, L), te<0>(a, L)), pick23(te<3>(d, L), te<2>(c, L)), k);
}

// Next round key in place (FIPS-197 5.2, little-endian words).
__device__ __forceinline__ void next_key(uint32_t k[4], uint32_t rcon, const Lanes &L)
{
    const uint32_t w = k[3];
    k[0] = xor3(pick01(te<2>(w, L), te<1>(w, L)), pick23(te<0>(w, L), te<3>(w, L)), k[0] ^ rcon);
    k[1] ^= k[0];
    k[2] ^= k[1];
    k[3] ^= k[2];
}

__device__ __forceinline__ void full_round(uint32_t s[4], const uint32_t kr[4], const Lanes &L)
{
    uint32_t t0 = mcol(s[0], s[1], s[2], s[3], kr[0], L);
    uint32_t t1 = mcol(s[1], s[2], s[3], s[0], kr[1], L);
    uint32_t t2 = mcol(s[2], s[3], s[0], s[1], kr[2], L);
    uint32_t t3 = mcol(s[3], s[0], s[1], s[2], kr[3], L);
    s[0] = t0;
    s[1] = t1;
    s[2] = t2;
    s[3] = t3;
}

// Rounds 1..9 of AES-128 on the counter blocks 0 (state a) and 1 (state b)
// under key s.  The key schedule runs on rotated words kr = rotl16(k): the
// schedule commutes with a 16-bit rotation (SubWord and RotWord act on bytes,
// the rest is XOR), so with Rcon moved to byte 2 the same next_key() yields
// rotl16 of every round key, which is what mcol() consumes.  On return kr
// holds rotl16 of round key 9.  Block 1 differs from block 0 only in byte 15
// (row 3 of column 3), which after round 1 affects column 0 alone, so round 1
// of block 1 reuses columns 1..3 of block 0.
__device__ __forceinline__ void rounds_1_to_9(const uint32_t s[4], uint32_t kr[4], uint32_t a[4], uint32_t b[4],
                                              const Lanes &L)
{
#pragma unroll
    for (int c = 0; c < 4; c++) {
        a[c] = s[c];
        kr[c] = rot16(s[c]);
    }
    const uint32_t b3 = s[3] ^ 0x01000000u;
    next_key(kr, pir_aes::RCON.v[1] << 16, L);
    {
        uint32_t t0 = mcol(a[0], a[1], a[2], a[3], kr[0], L);
        uint32_t u0 = mcol(a[0], a[1], a[2], b3, kr[0], L);
        uint32_t t1 = mcol(a[1], a[2], a[3], a[0], kr[1], L);
        uint32_t t2 = mcol(a[2], a[3], a[0], a[1], kr[2], L);
        uint32_t t3 = mcol(a[3], a[0], a[1], a[2], kr[3], L);
        a[0] = t0;
        a[1] = t1;
        a[2] = t2;
        a[3] = t3;
        b[0] = u0;
        b[1] = t1;
        b[2] = t2;
        b[3] = t3;
    }
#pragma unroll
    for (int r = 2; r <= 9; r++) {
        next_key(kr, pir_aes::RCON.v[r] << 16, L);
        full_round(a, kr, L);
        full_round(b, kr, L);
    }
}

// PRF_s(0), PRF_s(1) in full.
__device__ __forceinline__ void prf_pair(const uint32_t s[4], uint32_t a[4], uint32_t b[4], const Lanes &L)
{
    uint32_t kr[4];
    rounds_1_to_9(s, kr, a, b, L);
    next_key(kr, pir_aes::RCON.v[10] << 16, L);
    const uint32_t k0 = rot16(kr[0]), k1 = rot16(kr[1]), k2 = rot16(kr[2]), k3 = rot16(kr[3]);
    uint32_t a0 = fcol(a[0], a[1], a[2], a[3], k0, L), a1 = fcol(a[1], a[2], a[3], a[0], k1, L);
    uint32_t a2 = fcol(a[2], a[3], a[0], a[1], k2, L), a3 = fcol(a[3], a[0], a[1], a[2], k3, L);
    uint32_t b0 = fcol(b[0], b[1], b[2], b[3], k0, L), b1 = fcol(b[1], b[2], b[3], b[0], k1, L);
    uint32_t b2 = fcol(b[2], b[3], b[0], b[1], k2, L), b3 = fcol(b[3], b[0], b[1], b[2], k3, L);
    a[0] = a0;
    a[1] = a1;
    a[2] = a2;
    a[3] = a3;
    b[0] = b0;
    b[1] = b1;
    b[2] = b2;
    b[3] = b3;
}

// PRF_s(c) alone, for a walk down one path (one block instead of two).
__device__ __forceinline__ void prf_one(const uint32_t s[4], uint32_t c, uint32_t a[4], const Lanes &L)
{
    uint32_t kr[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        a[j] = s[j];
        kr[j] = rot16(s[j]);
    }
    a[3] ^= c << 24; // counter block c: byte 15 = c
#pragma unroll
    for (int r = 1; r <= 9; r++) {
        next_key(kr, pir_aes::RCON.v[r] << 16, L);
        full_round(a, kr, L);
    }
    next_key(kr, pir_aes::RCON.v[10] << 16, L);
    const uint32_t k0 = rot16(kr[0]), k1 = rot16(kr[1]), k2 = rot16(kr[2]), k3 = rot16(kr[3]);
    uint32_t a0 = fcol(a[0], a[1], a[2], a[3], k0, L), a1 = fcol(a[1], a[2], a[3], a[0], k1, L);
    uint32_t a2 = fcol(a[2], a[3], a[0], a[1], k2, L), a3 = fcol(a[3], a[0], a[1], a[2], k3, L);
    a[0] = a0;
    a[1] = a1;
    a[2] = a2;
    a[3] = a3;
}

// Only word 0 (bytes 0..3) of PRF_s(0) and PRF_s(1): what a leaf share uses.
__device__ __forceinline__ void prf_pair_word0(const uint32_t s[4], uint32_t &y0, uint32_t &y1, const Lanes &L)
{
    uint32_t kr[4], a[4], b[4];
    rounds_1_to_9(s, kr, a, b, L);
    const uint32_t w = kr[3];
    const uint32_t k0 = rot16(xor3(pick01(te<2>(w, L), te<1>(w, L)), pick23(te<0>(w, L), te<3>(w, L)),
                                   kr[0] ^ (pir_aes::RCON.v[10] << 16)));
    y0 = fcol(a[0], a[1], a[2], a[3], k0, L);
    y1 = fcol(b[0], b[1], b[2], b[3], k0, L);
}

// ---------------------------------------------------------------------------
// Quad form, for the latency-bound parts of a walk (a single key's path from
// the root): the four lanes 4j..4j+3 of a quad evaluate one node together,
// lane q owning column q of the state.  A round needs the other three columns'
// words, which come from the quad's lanes by DPP quad permutes, and this
// lane's round-key word; every lane runs the (short) key schedule itself.  A
// lane then issues 4 state lookups per block and round instead of 16, which
// shortens a node's dependent chain (measured 3.2 k against 5.7 k cycles for
// the pair of blocks).  All four lanes of a quad must be active.
// ---------------------------------------------------------------------------

// The four words of the seed in column order, in rotated (rotl16) form, from
// this lane's word s of column q.
__device__ __forceinline__ void quad_key(uint32_t s, const Quad &Q, uint32_t k[4])
{
    const uint32_t w0 = rot16(s), w1 = rot16(quad_next<1>(s)), w2 = rot16(quad_next<2>(s)), w3 = rot16(quad_next<3>(s));
    // w_j is column q + j
    k[0] = Q.q3 ? w1 : Q.q2 ? w2 : Q.q1 ? w3 : w0;
    k[1] = Q.q3 ? w2 : Q.q2 ? w3 : Q.q1 ? w0 : w1;
    k[2] = Q.q3 ? w3 : Q.q2 ? w0 : Q.q1 ? w1 : w2;
    k[3] = Q.q3 ? w0 : Q.q2 ? w1 : Q.q1 ? w2 : w3;
}

__device__ __forceinline__ uint32_t quad_mcol(uint32_t w, uint32_t kr, const Lanes &L)
{
    return mcol(w, quad_next<1>(w), quad_next<2>(w), quad_next<3>(w), kr, L);
}
__device__ __forceinline__ uint32_t quad_fcol(uint32_t w, uint32_t k, const Lanes &L)
{
    return fcol(w, quad_next<1>(w), quad_next<2>(w), quad_next<3>(w), k, L);
}

// This lane's words of PRF_s(0) and PRF_s(1); s is this lane's seed word.
__device__ __forceinline__ void quad_prf_pair(uint32_t s, uint32_t &a, uint32_t &b, const Quad &Q, const Lanes &L)
{
    uint32_t k[4];
    quad_key(s, Q, k);
    uint32_t wa = s, wb = s ^ (Q.q3 ? 0x01000000u : 0u); // counter blocks 0 and 1 (byte 15: column 3)
#pragma unroll
    for (int r = 1; r <= 9; r++) {
        next_key(k, pir_aes::RCON.v[r] << 16, L);
        const uint32_t kq = Q.own(k);
        const uint32_t na = quad_mcol(wa, kq, L), nb = quad_mcol(wb, kq, L);
        wa = na;
        wb = nb;
    }
    next_key(k, pir_aes::RCON.v[10] << 16, L);
    const uint32_t kq = rot16(Q.own(k));
    a = quad_fcol(wa, kq, L);
    b = quad_fcol(wb, kq, L);
}

// This lane's word of PRF_s(c), c in {0, 1}.
__device__ __forceinline__ uint32_t quad_prf_one(uint32_t s, uint32_t c, const Quad &Q, const Lanes &L)
{
    uint32_t k[4];
    quad_key(s, Q, k);
    uint32_t w = s ^ (Q.q3 ? c << 24 : 0u);
#pragma unroll
    for (int r = 1; r <= 9; r++) {
        next_key(k, pir_aes::RCON.v[r] << 16, L);
        w = quad_mcol(w, Q.own(k), L);
    }
    next_key(k, pir_aes::RCON.v[10] << 16, L);
    return quad_fcol(w, rot16(Q.own(k)), L);
}

// Fill the LDS table region (called by every lane of the workgroup): one
// global load per half row, then eight 16-byte LDS writes of its 32 copies.
__device__ __forceinline__ void fill_tables(uint32_t *tab, const uint32_t *te_global, uint32_t tid, uint32_t nthreads)
{
    for (uint32_t i = tid; i < 512; i += nthreads) {
        const uint32_t x = i >> 1, upper = i & 1;
        uint32_t v = te_global[x];
        v = upper ? __builtin_amdgcn_alignbit(v, v, 24) : v; // rotl8 in the upper half
        uint4 *dst = reinterpret_cast<uint4 *>(tab + x * 64 + upper * 32);
        const uint4 q = make_uint4(v, v, v, v);
#pragma unroll
        for (int j = 0; j < 8; j++)
            dst[j] = q;
    }
}

} // namespace pir_dev
