// aes_tables.h -- compile-time AES-128 tables for the library (host and device).
//
// The S-box is built from its definition in FIPS-197 5.1.1: the inverse in
// GF(2^8) (taken here from log/antilog tables over the generator {03}) followed
// by the affine map b ^ rotl(b,1) ^ rotl(b,2) ^ rotl(b,3) ^ rotl(b,4) ^ {63}.
//
// Words are little-endian: byte r of a state column sits in bits 8r..8r+7, so a
// 16-byte block is four uint32 loaded straight from memory.  With that order
// the combined SubBytes+MixColumns table for an input byte of row 0 is
//   TE[x] = {02}S(x) | S(x) << 8 | S(x) << 16 | {03}S(x) << 24,
// and rows 1..3 use TE rotated left by 8, 16, 24 bits.
#pragma once
#include <stdint.h>

namespace pir_aes {

constexpr uint8_t xtime(uint8_t a) { return (uint8_t)((a << 1) ^ ((a & 0x80) ? 0x1b : 0)); }

constexpr uint8_t rotl8(uint8_t b, int k) { return (uint8_t)((b << k) | (b >> (8 - k))); }

struct Bytes256 {
    uint8_t v[256];
};
struct Words256 {
    uint32_t v[256];
};
struct Words11 {
    uint32_t v[11];
};

constexpr Bytes256 make_sbox()
{
    Bytes256 ex{}, lg{}, s{};
    uint8_t x = 1;
    for (int i = 0; i < 255; i++) { // x = {03}^i
        ex.v[i] = x;
        lg.v[x] = (uint8_t)i;
        x = (uint8_t)(x ^ xtime(x));
    }
    for (int a = 0; a < 256; a++) {
        uint8_t inv = a ? ex.v[(255 - lg.v[a]) % 255] : 0;
        s.v[a] = (uint8_t)(inv ^ rotl8(inv, 1) ^ rotl8(inv, 2) ^ rotl8(inv, 3) ^
                           rotl8(inv, 4) ^ 0x63);
    }
    return s;
}

constexpr Bytes256 SBOX = make_sbox();

constexpr Words256 make_te()
{
    Words256 t{};
    for (int a = 0; a < 256; a++) {
        uint32_t s = SBOX.v[a];
        uint32_t s2 = xtime((uint8_t)s);
        uint32_t s3 = s2 ^ s;
        t.v[a] = s2 | (s << 8) | (s << 16) | (s3 << 24);
    }
    return t;
}

constexpr Words256 TE = make_te();

// round constants as little-endian words (the constant sits in byte 0)
constexpr Words11 make_rcon()
{
    Words11 r{};
    uint8_t c = 1;
    r.v[0] = 0;
    for (int i = 1; i <= 10; i++) {
        r.v[i] = c;
        c = xtime(c);
    }
    return r;
}

constexpr Words11 RCON = make_rcon();

static_assert(SBOX.v[0x00] == 0x63 && SBOX.v[0x53] == 0xed, "S-box");
static_assert(RCON.v[9] == 0x1b && RCON.v[10] == 0x36, "Rcon");

} // namespace pir_aes
