// pir_internal.h -- declarations shared by the library's translation units.
#pragma once
#include <stdint.h>

namespace pir_impl {

// Records the hipError_t of a failed runtime call for pir_last_hip_error().
void set_hip_error(int err);

// Seed / AES block as four little-endian words (byte r of word c is byte
// 4c + r of the 16-byte string).
struct Block {
    uint32_t w[4];
};

// AES-128 of one block under `key` (host).
Block aes128_host(const Block &key, const Block &in);

// The 128-bit big-endian counter block holding x (AES-CTR counter value x).
inline Block counter_block(uint64_t x)
{
    Block b{};
    uint32_t hi = (uint32_t)(x >> 32), lo = (uint32_t)x;
    b.w[2] = __builtin_bswap32(hi);
    b.w[3] = __builtin_bswap32(lo);
    return b;
}

} // namespace pir_impl
