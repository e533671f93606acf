/*
 * chacha_ref.c -- textbook ChaCha20 block function for the oracle (test
 * infrastructure only).
 *
 * Written from RFC 8439: the quarter round of section 2.1, the 4x4 word state
 * of section 2.3 (four constants "expand 32-byte k", eight key words, one
 * block-counter word, three nonce words, all little-endian), twenty rounds as
 * ten column-then-diagonal double rounds, the input added back to the state,
 * and the state serialized little-endian (section 2.3).  The paper lists
 * ChaCha20 among its PRFs (section 3.2.6, Table 5).
 */
#include "oracle.h"

#include <string.h>

static uint32_t rotl(uint32_t v, int c) { return (v << c) | (v >> (32 - c)); }

static uint32_t le32(const uint8_t *p)
{
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

void or_chacha20_quarter(uint32_t *a, uint32_t *b, uint32_t *c, uint32_t *d)
{
    *a += *b;
    *d ^= *a;
    *d = rotl(*d, 16);
    *c += *d;
    *b ^= *c;
    *b = rotl(*b, 12);
    *a += *b;
    *d ^= *a;
    *d = rotl(*d, 8);
    *c += *d;
    *b ^= *c;
    *b = rotl(*b, 7);
}

static void qr(uint32_t x[16], int a, int b, int c, int d)
{
    or_chacha20_quarter(&x[a], &x[b], &x[c], &x[d]);
}

void or_chacha20_block(const uint8_t key[32], uint32_t counter, const uint8_t nonce[12], uint8_t out[64])
{
    uint32_t init[16], x[16];
    init[0] = 0x61707865; /* "expa" */
    init[1] = 0x3320646e; /* "nd 3" */
    init[2] = 0x79622d32; /* "2-by" */
    init[3] = 0x6b206574; /* "te k" */
    for (int i = 0; i < 8; i++)
        init[4 + i] = le32(key + 4 * i);
    init[12] = counter;
    for (int i = 0; i < 3; i++)
        init[13 + i] = le32(nonce + 4 * i);
    memcpy(x, init, sizeof x);
    for (int i = 0; i < 10; i++) {
        qr(x, 0, 4, 8, 12); /* columns */
        qr(x, 1, 5, 9, 13);
        qr(x, 2, 6, 10, 14);
        qr(x, 3, 7, 11, 15);
        qr(x, 0, 5, 10, 15); /* diagonals */
        qr(x, 1, 6, 11, 12);
        qr(x, 2, 7, 8, 13);
        qr(x, 3, 4, 9, 14);
    }
    for (int i = 0; i < 16; i++) {
        uint32_t v = x[i] + init[i];
        out[4 * i] = (uint8_t)v;
        out[4 * i + 1] = (uint8_t)(v >> 8);
        out[4 * i + 2] = (uint8_t)(v >> 16);
        out[4 * i + 3] = (uint8_t)(v >> 24);
    }
}
