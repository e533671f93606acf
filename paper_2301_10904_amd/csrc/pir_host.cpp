// pir_host.cpp -- host side of the C ABI: Gen, reconstruction, status strings.
//
// Gen follows the construction the library documents for the paper's section
// 3.1 (the paper defers key generation to its DPF reference).  Per level d the
// two parties' on-path seeds s_0, s_1 have different control bits; with
// c = bit (n-d) of alpha and tau = t(s_0), the four codewords are chosen so
// that the off-path children of both parties coincide and the on-path
// children again have different control bits; the last level fixes the
// low 32 bits of the two on-path leaves to differ by beta.
#include <string.h>
#include <sys/random.h>

#include "pir.h"
#include "aes_tables.h"
#include "pir_internal.h"

namespace pir_impl {

static thread_local int g_last_hip_error = 0;

void set_hip_error(int err) { g_last_hip_error = err; }

static inline uint32_t rotl32(uint32_t x, int k) { return (x << k) | (x >> (32 - k)); }
static inline uint32_t byte_of(uint32_t w, int r) { return (w >> (8 * r)) & 0xff; }

Block aes128_host(const Block &key, const Block &in)
{
    using pir_aes::RCON;
    using pir_aes::SBOX;
    using pir_aes::TE;
    uint32_t k[4], s[4], t[4];
    for (int c = 0; c < 4; c++) {
        k[c] = key.w[c];
        s[c] = in.w[c] ^ k[c];
    }
    for (int r = 1; r <= 10; r++) {
        // next round key: SubWord(RotWord(w3)) ^ Rcon, then the running XOR
        uint32_t w3 = k[3];
        uint32_t sub = (uint32_t)SBOX.v[byte_of(w3, 1)] | (uint32_t)SBOX.v[byte_of(w3, 2)] << 8 |
                       (uint32_t)SBOX.v[byte_of(w3, 3)] << 16 | (uint32_t)SBOX.v[byte_of(w3, 0)] << 24;
        k[0] ^= sub ^ RCON.v[r];
        k[1] ^= k[0];
        k[2] ^= k[1];
        k[3] ^= k[2];
        for (int c = 0; c < 4; c++) {
            uint32_t a0 = byte_of(s[c], 0), a1 = byte_of(s[(c + 1) & 3], 1),
                     a2 = byte_of(s[(c + 2) & 3], 2), a3 = byte_of(s[(c + 3) & 3], 3);
            if (r < 10)
                t[c] = TE.v[a0] ^ rotl32(TE.v[a1], 8) ^ rotl32(TE.v[a2], 16) ^
                       rotl32(TE.v[a3], 24) ^ k[c];
            else
                t[c] = ((uint32_t)SBOX.v[a0] | (uint32_t)SBOX.v[a1] << 8 |
                        (uint32_t)SBOX.v[a2] << 16 | (uint32_t)SBOX.v[a3] << 24) ^
                       k[c];
        }
        memcpy(s, t, sizeof s);
    }
    Block out;
    memcpy(out.w, s, sizeof s);
    return out;
}

// ChaCha20 keystream block 0 under key s || s, nonce 0 (RFC 8439 state
// layout): the two children's PRF outputs are its words 0..3 and 4..7.
static void chacha_children_host(const Block &s, Block &p0, Block &p1)
{
    static const uint32_t sigma[4] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u};
    uint32_t in[16], x[16];
    for (int i = 0; i < 4; i++) {
        in[i] = sigma[i];
        in[4 + i] = s.w[i];
        in[8 + i] = s.w[i];
        in[12 + i] = 0;
    }
    memcpy(x, in, sizeof x);
    auto qr = [&](int a, int b, int c, int d) {
        x[a] += x[b];
        x[d] = rotl32(x[d] ^ x[a], 16);
        x[c] += x[d];
        x[b] = rotl32(x[b] ^ x[c], 12);
        x[a] += x[b];
        x[d] = rotl32(x[d] ^ x[a], 8);
        x[c] += x[d];
        x[b] = rotl32(x[b] ^ x[c], 7);
    };
    for (int r = 0; r < 10; r++) {
        for (int i = 0; i < 4; i++)
            qr(i, 4 + i, 8 + i, 12 + i);
        for (int i = 0; i < 4; i++)
            qr(i, 4 + (i + 1) % 4, 8 + (i + 2) % 4, 12 + (i + 3) % 4);
    }
    for (int i = 0; i < 4; i++) {
        p0.w[i] = x[i] + in[i];
        p1.w[i] = x[4 + i] + in[4 + i];
    }
}

// Both PRF outputs of a node with seed s under the PRF prf_id.
static void prf_children_host(uint32_t prf_id, const Block &s, Block out[2])
{
    if (prf_id == PIR_PRF_CHACHA20) {
        chacha_children_host(s, out[0], out[1]);
    } else {
        out[0] = aes128_host(s, counter_block(0));
        out[1] = aes128_host(s, counter_block(1));
    }
}

static Block load_block(const uint8_t *p)
{
    Block b;
    memcpy(b.w, p, 16); // little-endian host
    return b;
}

static void store_block(uint8_t *p, const Block &b) { memcpy(p, b.w, 16); }

static Block xorb(const Block &a, const Block &b)
{
    Block r;
    for (int i = 0; i < 4; i++)
        r.w[i] = a.w[i] ^ b.w[i];
    return r;
}

} // namespace pir_impl

using namespace pir_impl;

extern "C" {

size_t dpf_key_size(uint32_t n)
{
    if (n < 1 || n > PIR_MAX_LOG_DOMAIN)
        return 0;
    return 32 + 64 * (size_t)n;
}

int dpf_gen(uint32_t n, uint64_t alpha, uint32_t beta, const uint8_t *seed16, uint8_t *key0,
            uint8_t *key1)
{
    return dpf_gen_prf(n, alpha, beta, seed16, PIR_PRF_AES128, key0, key1);
}

int dpf_gen_prf(uint32_t n, uint64_t alpha, uint32_t beta, const uint8_t *seed16, uint32_t prf_id,
                uint8_t *key0, uint8_t *key1)
{
    if (!key0 || !key1 || n < 1 || n > PIR_MAX_LOG_DOMAIN)
        return PIR_EINVAL;
    if (prf_id != PIR_PRF_AES128 && prf_id != PIR_PRF_CHACHA20)
        return PIR_EINVAL;
    if (alpha >> n)
        return PIR_EINVAL;
    uint8_t sys_seed[16];
    if (!seed16) {
        size_t got = 0;
        while (got < 16) {
            ssize_t r = getrandom(sys_seed + got, 16 - got, 0);
            if (r <= 0)
                return PIR_EHIP;
            got += (size_t)r;
        }
        seed16 = sys_seed;
    }
    const Block drbg_key = load_block(seed16);
    uint64_t ctr = 0;
    auto draw = [&]() { return aes128_host(drbg_key, counter_block(ctr++)); };

    Block s0 = draw(), s1 = draw();
    s1.w[0] = (s1.w[0] & ~1u) | (1u - (s0.w[0] & 1u));

    const size_t ks = dpf_key_size(n);
    uint8_t *keys[2] = {key0, key1};
    for (int b = 0; b < 2; b++) {
        memset(keys[b], 0, ks);
        keys[b][0] = PIR_KEY_VERSION;
        keys[b][1] = (uint8_t)b;
        keys[b][2] = (uint8_t)n;
        keys[b][3] = (uint8_t)prf_id;
    }
    store_block(key0 + 16, s0);
    store_block(key1 + 16, s1);

    for (uint32_t d = 1; d <= n; d++) {
        const unsigned c = (unsigned)((alpha >> (n - d)) & 1);
        const unsigned tau = s0.w[0] & 1u;
        Block P0[2], P1[2];
        prf_children_host(prf_id, s0, P0);
        prf_children_host(prf_id, s1, P1);
        Block C[2][2]; // C[t][child]

        Block R = draw();
        C[tau][c ^ 1] = R;
        C[tau ^ 1][c ^ 1] = xorb(R, xorb(P0[c ^ 1], P1[c ^ 1]));

        Block R2 = draw();
        C[tau][c] = R2;
        Block ns0 = xorb(P0[c], R2), ns1;
        if (d < n) {
            Block Qb = draw();
            Qb.w[0] = (Qb.w[0] & ~1u) | ((P1[c].w[0] ^ 1u ^ ns0.w[0]) & 1u);
            C[tau ^ 1][c] = Qb;
            ns1 = xorb(P1[c], Qb);
        } else {
            // ns1 = ns0 - beta over 128-bit little-endian integers
            uint64_t borrow = 0;
            for (int i = 0; i < 4; i++) {
                uint64_t sub = (i == 0 ? (uint64_t)beta : 0) + borrow;
                uint64_t v = (uint64_t)ns0.w[i] - sub;
                ns1.w[i] = (uint32_t)v;
                borrow = ((uint64_t)ns0.w[i] < sub) ? 1 : 0;
            }
            C[tau ^ 1][c] = xorb(P1[c], ns1);
        }
        for (int b = 0; b < 2; b++)
            for (int t = 0; t < 2; t++)
                for (int x = 0; x < 2; x++)
                    store_block(keys[b] + 32 + 64 * (size_t)(d - 1) + 32 * t + 16 * x, C[t][x]);
        s0 = ns0;
        s1 = ns1;
    }
    return PIR_OK;
}

int pir_reconstruct(const uint32_t *a0, const uint32_t *a1, uint32_t dim, uint32_t *out)
{
    if (!a0 || !a1 || !out)
        return PIR_EINVAL;
    for (uint32_t k = 0; k < dim; k++)
        out[k] = a0[k] + a1[k];
    return PIR_OK;
}

const char *pir_strerror(int status)
{
    switch (status) {
    case PIR_OK:
        return "ok";
    case PIR_EINVAL:
        return "invalid argument";
    case PIR_ENOMEM:
        return "size beyond the library's limits";
    case PIR_EHIP:
        return "HIP runtime error";
    case PIR_EKEY:
        return "a key had a bad header";
    case PIR_ESTALL:
        return "a kernel gave up a bounded wait (the output is not valid)";
    default:
        return "unknown status";
    }
}

int pir_last_hip_error(void) { return g_last_hip_error; }

} // extern "C"
