/*
 * aes_ref.c -- textbook AES-128 for the oracle (test infrastructure only).
 *
 * Written from FIPS-197 byte by byte: the S-box is derived from the
 * multiplicative inverse in GF(2^8) followed by the affine map (FIPS-197
 * 5.1.1), the state is the 4x4 byte array s[r][c] = in[r + 4c] (3.4), and
 * Cipher / KeyExpansion follow 5.1 and 5.2 for Nk = 4, Nr = 10.  Nothing is
 * table-driven beyond the S-box, so every step can be checked against the
 * standard by eye.
 */
#include "oracle.h"

#include <string.h>

/* multiplication in GF(2^8) modulo x^8 + x^4 + x^3 + x + 1 (FIPS-197 4.2) */
static uint8_t gf_mul(uint8_t a, uint8_t b)
{
    uint8_t p = 0;
    for (int i = 0; i < 8; i++) {
        if (b & 1)
            p ^= a;
        uint8_t hi = a & 0x80;
        a = (uint8_t)(a << 1);
        if (hi)
            a ^= 0x1b;
        b >>= 1;
    }
    return p;
}

/* inverse in GF(2^8) as a^254 (a^255 = 1 for a != 0); 0 maps to 0 */
static uint8_t gf_inv(uint8_t a)
{
    uint8_t r = 1;
    for (int i = 0; i < 254; i++)
        r = gf_mul(r, a);
    return a ? r : 0;
}

static uint8_t SBOX[256];
static int sbox_ready;

static void build_sbox(void)
{
    for (int x = 0; x < 256; x++) {
        uint8_t b = gf_inv((uint8_t)x);
        uint8_t s = 0;
        /* b'_i = b_i ^ b_{i+4} ^ b_{i+5} ^ b_{i+6} ^ b_{i+7} ^ c_i, c = 0x63 */
        for (int i = 0; i < 8; i++) {
            int bit = ((b >> i) & 1) ^ ((b >> ((i + 4) % 8)) & 1) ^
                      ((b >> ((i + 5) % 8)) & 1) ^ ((b >> ((i + 6) % 8)) & 1) ^
                      ((b >> ((i + 7) % 8)) & 1) ^ ((0x63 >> i) & 1);
            s |= (uint8_t)(bit << i);
        }
        SBOX[x] = s;
    }
    __atomic_store_n(&sbox_ready, 1, __ATOMIC_RELEASE);
}

static void ensure_sbox(void)
{
    if (!__atomic_load_n(&sbox_ready, __ATOMIC_ACQUIRE))
        build_sbox(); /* idempotent: concurrent builders write equal bytes */
}

void or_aes128_sbox(uint8_t out[256])
{
    ensure_sbox();
    memcpy(out, SBOX, 256);
}

/* FIPS-197 5.2: w holds 44 words of 4 bytes, word i at bytes 4i..4i+3 */
void or_aes128_expand(const uint8_t key[16], uint8_t w[176])
{
    ensure_sbox();
    uint8_t rcon = 0x01;
    memcpy(w, key, 16);
    for (int i = 4; i < 44; i++) {
        uint8_t temp[4];
        memcpy(temp, &w[4 * (i - 1)], 4);
        if (i % 4 == 0) {
            /* RotWord, SubWord, then XOR with Rcon[i/4] = (x^(i/4-1), 0, 0, 0) */
            uint8_t t0 = temp[0];
            temp[0] = SBOX[temp[1]];
            temp[1] = SBOX[temp[2]];
            temp[2] = SBOX[temp[3]];
            temp[3] = SBOX[t0];
            temp[0] ^= rcon;
            rcon = gf_mul(rcon, 0x02);
        }
        for (int k = 0; k < 4; k++)
            w[4 * i + k] = w[4 * (i - 4) + k] ^ temp[k];
    }
}

static void add_round_key(uint8_t s[4][4], const uint8_t *w, int round)
{
    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++)
            s[r][c] ^= w[16 * round + 4 * c + r];
}

static void sub_bytes(uint8_t s[4][4])
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            s[r][c] = SBOX[s[r][c]];
}

/* row r is rotated left by r positions: s'[r][c] = s[r][(c + r) mod 4] */
static void shift_rows(uint8_t s[4][4])
{
    uint8_t t[4];
    for (int r = 1; r < 4; r++) {
        for (int c = 0; c < 4; c++)
            t[c] = s[r][(c + r) % 4];
        for (int c = 0; c < 4; c++)
            s[r][c] = t[c];
    }
}

/* each column times the fixed polynomial {03}x^3 + {01}x^2 + {01}x + {02} */
static void mix_columns(uint8_t s[4][4])
{
    for (int c = 0; c < 4; c++) {
        uint8_t a0 = s[0][c], a1 = s[1][c], a2 = s[2][c], a3 = s[3][c];
        s[0][c] = gf_mul(a0, 2) ^ gf_mul(a1, 3) ^ a2 ^ a3;
        s[1][c] = a0 ^ gf_mul(a1, 2) ^ gf_mul(a2, 3) ^ a3;
        s[2][c] = a0 ^ a1 ^ gf_mul(a2, 2) ^ gf_mul(a3, 3);
        s[3][c] = gf_mul(a0, 3) ^ a1 ^ a2 ^ gf_mul(a3, 2);
    }
}

/* FIPS-197 5.1 */
void or_aes128_encrypt(const uint8_t w[176], const uint8_t in[16], uint8_t out[16])
{
    ensure_sbox();
    uint8_t s[4][4];
    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++)
            s[r][c] = in[r + 4 * c];
    add_round_key(s, w, 0);
    for (int round = 1; round < 10; round++) {
        sub_bytes(s);
        shift_rows(s);
        mix_columns(s);
        add_round_key(s, w, round);
    }
    sub_bytes(s);
    shift_rows(s);
    add_round_key(s, w, 10);
    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++)
            out[r + 4 * c] = s[r][c];
}

void or_aes128(const uint8_t key[16], const uint8_t in[16], uint8_t out[16])
{
    uint8_t w[176];
    or_aes128_expand(key, w);
    or_aes128_encrypt(w, in, out);
}
