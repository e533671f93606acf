// aes_bitsliced_gfx950.h -- AES-128 for the PRF of the DPF tree in bitsliced
// form: the measured alternative to the LDS T-table rounds of aes_gfx950.h.
// The PIR kernels do not use it; the PRF-engine measurement library runs it
// beside the T-table engine so that the choice of PRF code rests on a
// measurement (paper §3.2.6 weighs PRF choices by their cost on the GPU).
//
// Layout ("column slicing").  A quad of lanes (4j..4j+3) evaluates 32 nodes
// at once.  Lane q of the quad owns column q of the AES state as 32 bit
// planes: plane 8r + k holds bit k of the byte in row r, and bit i of every
// plane belongs to node i.  Then
//   * SubBytes is a boolean circuit on the 8 planes of a byte (below, derived
//     through the tower field GF(((2^2)^2)^2));
//   * ShiftRows moves row r from column q + r: a DPP quad permute per plane;
//   * MixColumns and AddRoundKey are XORs within the lane (a column is local);
//   * the key schedule's word chain w'_q = w'_{q-1} ^ w_q is a prefix XOR over
//     the quad (two DPP steps), and SubWord(RotWord(w_3)) costs one S-box per
//     lane: lane q evaluates byte q + 1 of column 3.
// No table and no LDS: the work is VALU operations only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aes_tables.h"
#include "quad_gfx950.h"

namespace pir_bs {

// ---------------------------------------------------------------------------
// The tower field, on integers (compile time).  FIPS-197 4.2 defines the
// S-box through the inverse in GF(2^8) = GF(2)[t]/(t^8 + t^4 + t^3 + t + 1);
// that field is isomorphic to
//   GF(4)   = GF(2)[x]/(x^2 + x + 1),           a1*x + a0  held as (a1 << 1) | a0
//   GF(16)  = GF(4)[y]/(y^2 + y + NU),           A1*y + A0  held as (A1 << 2) | A0
//   GF(256) = GF(16)[z]/(z^2 + z + LAMBDA),      B1*z + B0  held as (B1 << 4) | B0
// where an inverse reduces to operations one level down:
//   (A1 y + A0)^-1 = (A1 d^-1) y + (A1 + A0) d^-1,  d = NU A1^2 + A1 A0 + A0^2
// (the same with LAMBDA one level up), and in GF(4) the inverse is the square.
// ---------------------------------------------------------------------------

constexpr uint32_t g4_mul(uint32_t a, uint32_t b)
{
    const uint32_t a1 = a >> 1, a0 = a & 1, b1 = b >> 1, b0 = b & 1;
    const uint32_t p00 = a0 & b0, m = (a1 ^ a0) & (b1 ^ b0);
    return ((m ^ p00) << 1) | ((a1 & b1) ^ p00); // x^2 = x + 1
}

// y^2 + y takes only the values 0 and 1 on GF(4), so y^2 + y + x has no root
constexpr uint32_t NU = 2;

constexpr uint32_t g16_mul(uint32_t a, uint32_t b)
{
    const uint32_t a1 = a >> 2, a0 = a & 3, b1 = b >> 2, b0 = b & 3;
    const uint32_t p00 = g4_mul(a0, b0), m = g4_mul(a1 ^ a0, b1 ^ b0);
    return ((m ^ p00) << 2) | (g4_mul(g4_mul(a1, b1), NU) ^ p00); // y^2 = y + NU
}

// the first LAMBDA in GF(16) with no root of z^2 + z + LAMBDA
constexpr uint32_t find_lambda()
{
    for (uint32_t l = 1; l < 16; l++) {
        bool root = false;
        for (uint32_t z = 0; z < 16; z++)
            root = root || ((g16_mul(z, z) ^ z) == l);
        if (!root)
            return l;
    }
    return 0;
}
constexpr uint32_t LAMBDA = find_lambda();
static_assert(LAMBDA != 0, "an irreducible z^2 + z + LAMBDA exists over GF(16)");

constexpr uint32_t g256_mul(uint32_t a, uint32_t b)
{
    const uint32_t a1 = a >> 4, a0 = a & 15, b1 = b >> 4, b0 = b & 15;
    const uint32_t p00 = g16_mul(a0, b0), m = g16_mul(a1 ^ a0, b1 ^ b0);
    return ((m ^ p00) << 4) | (g16_mul(g16_mul(a1, b1), LAMBDA) ^ p00);
}

constexpr uint32_t g16_inv(uint32_t a)
{
    const uint32_t a1 = a >> 2, a0 = a & 3;
    const uint32_t d = g4_mul(g4_mul(a1, a1), NU) ^ g4_mul(a1, a0) ^ g4_mul(a0, a0);
    const uint32_t di = g4_mul(d, d);
    return (g4_mul(a1, di) << 2) | g4_mul(a1 ^ a0, di);
}

constexpr uint32_t g256_inv(uint32_t a)
{
    const uint32_t a1 = a >> 4, a0 = a & 15;
    const uint32_t d = g16_mul(g16_mul(a1, a1), LAMBDA) ^ g16_mul(a1, a0) ^ g16_mul(a0, a0);
    const uint32_t di = g16_inv(d);
    return (g16_mul(a1, di) << 4) | g16_mul(a1 ^ a0, di);
}

constexpr bool tower_is_a_field()
{
    for (uint32_t a = 1; a < 256; a++)
        if (g256_mul(a, g256_inv(a)) != 1)
            return false;
    return true;
}
static_assert(tower_is_a_field(), "every nonzero tower element has its inverse");

// The change of basis.  beta is a root in the tower field of the AES
// polynomial, so t -> beta extends to a field isomorphism phi: an AES byte v
// maps to the XOR of beta^i over its set bits i (column i of the input map is
// in[i] = beta^i).  out[j] is the S-box's linear part (FIPS-197 5.1.1, the
// affine map without its constant {63}) applied to phi^-1 of tower bit j.  Of
// the eight roots (beta and its conjugates) the one with the fewest ones in
// the two matrices is kept: fewer XORs in the circuit.
struct Basis {
    uint32_t beta;
    uint8_t in[8], out[8];
};

constexpr uint8_t affine_linear(uint32_t b)
{
    return (uint8_t)(b ^ pir_aes::rotl8((uint8_t)b, 1) ^ pir_aes::rotl8((uint8_t)b, 2) ^
                     pir_aes::rotl8((uint8_t)b, 3) ^ pir_aes::rotl8((uint8_t)b, 4));
}

constexpr int popcount8(uint32_t v)
{
    int n = 0;
    for (int i = 0; i < 8; i++)
        n += (v >> i) & 1;
    return n;
}

constexpr Basis make_basis()
{
    Basis best{};
    int best_ones = 1 << 30;
    for (uint32_t beta = 2; beta < 256; beta++) {
        uint32_t pw[9] = {};
        pw[0] = 1;
        for (int i = 1; i <= 8; i++)
            pw[i] = g256_mul(pw[i - 1], beta);
        if ((pw[8] ^ pw[4] ^ pw[3] ^ pw[1] ^ pw[0]) != 0)
            continue;
        Basis b{};
        b.beta = beta;
        uint32_t inv_col[8] = {};
        for (uint32_t v = 0; v < 256; v++) {
            uint32_t t = 0;
            for (int i = 0; i < 8; i++)
                t ^= ((v >> i) & 1) ? pw[i] : 0u;
            for (int j = 0; j < 8; j++)
                if (t == (1u << j))
                    inv_col[j] = v;
        }
        int ones = 0;
        for (int i = 0; i < 8; i++) {
            b.in[i] = (uint8_t)pw[i];
            b.out[i] = affine_linear(inv_col[i]);
            ones += popcount8(b.in[i]) + popcount8(b.out[i]);
        }
        if (ones < best_ones) {
            best = b;
            best_ones = ones;
        }
    }
    return best;
}

constexpr Basis BASIS = make_basis();

constexpr uint32_t apply_in(uint32_t v)
{
    uint32_t t = 0;
    for (int i = 0; i < 8; i++)
        t ^= ((v >> i) & 1) ? BASIS.in[i] : 0u;
    return t;
}
constexpr uint32_t apply_out(uint32_t t)
{
    uint32_t v = 0;
    for (int j = 0; j < 8; j++)
        v ^= ((t >> j) & 1) ? BASIS.out[j] : 0u;
    return v ^ 0x63u;
}

constexpr bool tower_sbox_ok()
{
    for (uint32_t v = 0; v < 256; v++)
        if (apply_out(g256_inv(apply_in(v))) != pir_aes::SBOX.v[v])
            return false;
    return true;
}
static_assert(BASIS.beta != 0, "the AES polynomial has a root in the tower field");
static_assert(tower_sbox_ok(), "S(v) = out(inverse(in(v))) for every byte");

// ---------------------------------------------------------------------------
// The same arithmetic on bit planes: each uint32_t holds one bit of 32
// independent elements.  The circuit runs unchanged at compile time (checked
// below against the S-box table) and on the device, where three-input XORs
// are v_bitop3_b32 and the compiler fuses other three-input logic likewise.
// ---------------------------------------------------------------------------

// a ^ b ^ c: one v_bitop3_b32 on the device, plain XORs at compile time
constexpr uint32_t x3(uint32_t a, uint32_t b, uint32_t c)
{
    if (__builtin_is_constant_evaluated())
        return a ^ b ^ c;
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

struct P4 {
    uint32_t h, l; // a1, a0
};
struct P16 {
    P4 h, l; // A1, A0
};
struct P256 {
    P16 h, l; // B1, B0
};

constexpr P4 add(P4 a, P4 b) { return {a.h ^ b.h, a.l ^ b.l}; }
constexpr P16 add(P16 a, P16 b) { return {add(a.h, b.h), add(a.l, b.l)}; }
constexpr P4 add3(P4 a, P4 b, P4 c) { return {x3(a.h, b.h, c.h), x3(a.l, b.l, c.l)}; }
constexpr P16 add3(P16 a, P16 b, P16 c) { return {add3(a.h, b.h, c.h), add3(a.l, b.l, c.l)}; }

constexpr P4 mul(P4 a, P4 b)
{
    const uint32_t p00 = a.l & b.l, m = (a.h ^ a.l) & (b.h ^ b.l);
    return {m ^ p00, (a.h & b.h) ^ p00};
}
constexpr P4 sq(P4 a) { return {a.h, a.h ^ a.l}; }        // (a1 x + a0)^2 = a1 x + (a1 + a0)
constexpr P4 mul_nu(P4 a) { return {a.h ^ a.l, a.h}; }    // times x

constexpr P16 mul(P16 a, P16 b)
{
    const P4 p00 = mul(a.l, b.l), m = mul(add(a.h, a.l), add(b.h, b.l));
    return {add(m, p00), add(mul_nu(mul(a.h, b.h)), p00)};
}
constexpr P16 sq(P16 a) { return {sq(a.h), add(mul_nu(sq(a.h)), sq(a.l))}; } // y^2 = y + NU

// a GF(16) constant as planes (all-ones or zero), for multiplying by LAMBDA
constexpr P16 constant16(uint32_t c)
{
    return {{0u - ((c >> 3) & 1), 0u - ((c >> 2) & 1)}, {0u - ((c >> 1) & 1), 0u - (c & 1)}};
}

constexpr P16 inv(P16 a)
{
    const P4 d = add3(mul_nu(sq(a.h)), mul(a.h, a.l), sq(a.l));
    const P4 di = sq(d);
    return {mul(a.h, di), mul(add(a.h, a.l), di)};
}

constexpr P256 inv(P256 a)
{
    const P16 d = add3(mul(sq(a.h), constant16(LAMBDA)), mul(a.h, a.l), sq(a.l));
    const P16 di = inv(d);
    return {mul(a.h, di), mul(add(a.h, a.l), di)};
}

// XOR of v[j] over the set bits j of `mask` (at most 8), onto `init`, three
// inputs per operation
constexpr uint32_t xor_select(uint32_t init, uint32_t mask, const uint32_t *v)
{
    uint32_t acc = init;
    int pend = -1;
#pragma unroll
    for (int j = 0; j < 8; j++)
        if ((mask >> j) & 1) {
            if (pend < 0) {
                pend = j;
            } else {
                acc = x3(acc, v[pend], v[j]);
                pend = -1;
            }
        }
    return pend < 0 ? acc : acc ^ v[pend];
}

// the rows of a column-defined 8 x 8 matrix: bit i of row j = bit j of col[i]
constexpr uint32_t matrix_row(const uint8_t *col, int j)
{
    uint32_t r = 0;
    for (int i = 0; i < 8; i++)
        r |= ((col[i] >> j) & 1u) << i;
    return r;
}

// S-box in place on the planes x[0..7] (x[k] = bit k of the byte): the input
// change of basis, the tower-field inverse, then the output change of basis
// merged with the affine map and its constant {63}.
constexpr void sbox_planes(uint32_t *x)
{
    uint32_t t[8] = {};
#pragma unroll
    for (int j = 0; j < 8; j++)
        t[j] = xor_select(0u, matrix_row(BASIS.in, j), x);
    const P256 a = {{{t[7], t[6]}, {t[5], t[4]}}, {{t[3], t[2]}, {t[1], t[0]}}};
    const P256 r = inv(a);
    const uint32_t u[8] = {r.l.l.l, r.l.l.h, r.l.h.l, r.l.h.h, r.h.l.l, r.h.l.h, r.h.h.l, r.h.h.h};
#pragma unroll
    for (int k = 0; k < 8; k++)
        x[k] = xor_select((0x63u >> k) & 1 ? ~0u : 0u, matrix_row(BASIS.out, k), u);
}

constexpr bool sbox_circuit_ok()
{
    for (uint32_t base = 0; base < 256; base += 32) {
        uint32_t x[8] = {};
        for (uint32_t i = 0; i < 32; i++)
            for (int k = 0; k < 8; k++)
                x[k] |= (((base + i) >> k) & 1u) << i;
        sbox_planes(x);
        for (uint32_t i = 0; i < 32; i++) {
            uint32_t y = 0;
            for (int k = 0; k < 8; k++)
                y |= ((x[k] >> i) & 1u) << k;
            if (y != pir_aes::SBOX.v[base + i])
                return false;
        }
    }
    return true;
}
static_assert(sbox_circuit_ok(), "the plane circuit computes the S-box on all 256 bytes");

// 32 x 32 bit transpose in place: afterwards bit i of w[p] is what bit p of
// w[i] was (five stages of block swaps, halving the block each time).
constexpr void transpose32(uint32_t *w)
{
#pragma unroll
    for (int j = 16, s = 0; j >= 1; j >>= 1, s++) {
        const uint32_t m = s == 0 ? 0x0000ffffu : s == 1 ? 0x00ff00ffu : s == 2 ? 0x0f0f0f0fu
                         : s == 3 ? 0x33333333u : 0x55555555u;
#pragma unroll
        for (int i = 0; i < 32; i++)
            if ((i & j) == 0) {
                const uint32_t t = ((w[i] >> j) ^ w[i + j]) & m;
                w[i + j] ^= t;
                w[i] ^= t << j;
            }
    }
}

constexpr bool transpose_ok()
{
    uint32_t w[32] = {}, v[32] = {};
    for (uint32_t i = 0; i < 32; i++)
        v[i] = w[i] = (i + 1) * 0x9e3779b9u ^ (i << 7);
    transpose32(w);
    for (uint32_t i = 0; i < 32; i++)
        for (uint32_t p = 0; p < 32; p++)
            if (((w[p] >> i) & 1) != ((v[i] >> p) & 1))
                return false;
    return true;
}
static_assert(transpose_ok(), "transpose32");

// ---------------------------------------------------------------------------
// The rounds on a quad (device).  Every lane of a quad must be active.
// ---------------------------------------------------------------------------

// DPP quad permute with a constant control word
template <int CTRL>
__device__ __forceinline__ uint32_t qperm(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xf, 0xf, false);
}

struct QuadMasks {
    uint32_t ge1, ge2; // all ones in columns >= 1 / >= 2
    uint32_t lo, hi;   // all ones where bit 0 / bit 1 of the column is set
    uint32_t is3;      // all ones in column 3
    __device__ __forceinline__ explicit QuadMasks(uint32_t lane)
        : ge1((lane & 3) >= 1 ? ~0u : 0u), ge2((lane & 3) >= 2 ? ~0u : 0u), lo(0u - (lane & 1)),
          hi(0u - ((lane >> 1) & 1)), is3((lane & 3) == 3 ? ~0u : 0u)
    {
    }
};

// The next round key (FIPS-197 5.2) in place: k holds this lane's column.
__device__ __forceinline__ void next_key(uint32_t *k, uint32_t rcon, const QuadMasks &Q)
{
    // S-box input of lane q: byte (q + 1) mod 4 of column 3 (RotWord)
    uint32_t x[8];
#pragma unroll
    for (int b = 0; b < 8; b++) {
        const uint32_t r0 = qperm<0xff>(k[b]), r1 = qperm<0xff>(k[8 + b]);
        const uint32_t r2 = qperm<0xff>(k[16 + b]), r3 = qperm<0xff>(k[24 + b]);
        const uint32_t even = (r2 & Q.lo) | (r1 & ~Q.lo), odd = (r0 & Q.lo) | (r3 & ~Q.lo);
        x[b] = (odd & Q.hi) | (even & ~Q.hi);
    }
    sbox_planes(x);
    // w'_q = w_0 ^ ... ^ w_q ^ SubWord(RotWord(w_3)) ^ Rcon
#pragma unroll
    for (int i = 0; i < 32; i++) {
        uint32_t p = k[i];
        p ^= qperm<0x90>(p) & Q.ge1; // quad_perm [0,0,1,2]: column q - 1
        p ^= qperm<0x40>(p) & Q.ge2; // quad_perm [0,0,0,1]: column q - 2
        k[i] = p;
    }
#pragma unroll
    for (int b = 0; b < 8; b++) {
        k[b] ^= qperm<0x00>(x[b]) ^ (0u - ((rcon >> b) & 1));
        k[8 + b] ^= qperm<0x55>(x[b]);
        k[16 + b] ^= qperm<0xaa>(x[b]);
        k[24 + b] ^= qperm<0xff>(x[b]);
    }
}

// ShiftRows: row r of column q comes from column q + r
__device__ __forceinline__ void shift_rows(uint32_t *s)
{
#pragma unroll
    for (int b = 0; b < 8; b++) {
        s[8 + b] = pir_dev::quad_next<1>(s[8 + b]);
        s[16 + b] = pir_dev::quad_next<2>(s[16 + b]);
        s[24 + b] = pir_dev::quad_next<3>(s[24 + b]);
    }
}

// MixColumns then AddRoundKey on this lane's column:
// out_r = 2 a_r + 3 a_{r+1} + a_{r+2} + a_{r+3} = a_r + t + {02}(a_r + a_{r+1}),
// t = a_0 + a_1 + a_2 + a_3, and {02}u shifts the bits up and folds bit 7
// back into bits 0, 1, 3, 4 (the polynomial {1b}).
__device__ __forceinline__ void mix_add(uint32_t *s, const uint32_t *k)
{
    uint32_t t[8], o[32];
#pragma unroll
    for (int b = 0; b < 8; b++)
        t[b] = x3(s[b], s[8 + b], s[16 + b]) ^ s[24 + b];
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const uint32_t *a = s + 8 * r, *a1 = s + 8 * ((r + 1) & 3);
        uint32_t u[8];
#pragma unroll
        for (int b = 0; b < 8; b++)
            u[b] = a[b] ^ a1[b];
        // bit b of {02}u is u[b - 1] (u[7] for bit 0), with u[7] added into bits 1, 3, 4
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const uint32_t up = u[(b + 7) & 7];
            if (b == 1 || b == 3 || b == 4)
                o[8 * r + b] = x3(x3(a[b], t[b], up), u[7], k[8 * r + b]);
            else
                o[8 * r + b] = x3(a[b], t[b], up) ^ k[8 * r + b];
        }
    }
#pragma unroll
    for (int i = 0; i < 32; i++)
        s[i] = o[i];
}

__device__ __forceinline__ void sub_bytes(uint32_t *s)
{
#pragma unroll
    for (int r = 0; r < 4; r++)
        sbox_planes(s + 8 * r);
}

// PRF_s(0) and PRF_s(1) for the quad's 32 nodes: s holds this lane's column
// of the 32 seeds (the AES keys), a and b receive this lane's column of the
// two output blocks (counter blocks 0 and 1: byte 15 = the counter).
__device__ __forceinline__ void prf_pair(const uint32_t *s, uint32_t *a, uint32_t *b, const QuadMasks &Q)
{
    uint32_t k[32];
#pragma unroll
    for (int i = 0; i < 32; i++) {
        k[i] = s[i];
        a[i] = s[i];
        b[i] = s[i];
    }
    b[24] ^= Q.is3; // byte 15 (row 3 of column 3) of counter block 1 is 1
    uint32_t rcon = 1;
#pragma unroll 1
    for (int r = 1; r <= 9; r++) {
        next_key(k, rcon, Q);
        sub_bytes(a);
        sub_bytes(b);
        shift_rows(a);
        shift_rows(b);
        mix_add(a, k);
        mix_add(b, k);
        rcon = (rcon << 1) ^ ((rcon >> 7) * 0x11bu);
    }
    next_key(k, rcon, Q);
    sub_bytes(a);
    sub_bytes(b);
    shift_rows(a);
    shift_rows(b);
#pragma unroll
    for (int i = 0; i < 32; i++) {
        a[i] ^= k[i];
        b[i] ^= k[i];
    }
}

} // namespace pir_bs
