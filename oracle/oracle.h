/*
 * oracle.h -- plain, slow, CPU reference for the two-server DPF-PIR server path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path
 * (include/pir.h and the package) shares no code with it and never calls it.
 *
 * What it computes (paper section 3.1, the fundamentals of PIR and DPF):
 *   - PRF_s(x): AES-128 under key s (FIPS-197), used in counter mode: the
 *     plaintext is the 128-bit big-endian integer x (the paper's PRF table,
 *     Table 5, runs AES-128 as a block cipher in counter mode).
 *   - Eval(k, j): the node recurrence of Eq. (p1)-(p3),
 *       P(0,0)  = root of the key,
 *       P(d,j)  = PRF_{P(d-1,j/2)}(j mod 2) XOR C_{t(P(d-1,j/2))}[j mod 2, d],
 *     with t(s) = bit 0 of byte 0 of s, and the share of leaf j is
 *       Eval(k_b, j) = (-1)^b * low32(P(n, j))  (mod 2^32).
 *   - Answer: T x Eval(k, {0..L-1}) for a table T of L rows by D uint32
 *     columns, mod 2^32; reconstruct = a0 + a1 (mod 2^32) = beta * T[alpha].
 *   - Gen(1^lambda, alpha): the paper defers key generation to its DPF
 *     reference; this oracle uses the construction written out in dpf_ref.c.
 *
 *   - ChaCha20 (RFC 8439) as the alternative PRF of section 3.2.6: PRF_s(x)
 *     is keystream bytes [16x, 16x+16) under key s || s, nonce 0.
 *
 * Key byte layout (size 32 + 64 n):
 *   [0] version = 1, [1] party b, [2] n, [3] prf id (0 = AES-128,
 *   1 = ChaCha20),
 *   [4..15] zero, [16..31] root seed P(0,0) of party b,
 *   then for d = 1..n: C_0[0,d], C_0[1,d], C_1[0,d], C_1[1,d] (16 bytes each).
 *   The 64 n codeword bytes equal the key sizes the paper prints (Table 4).
 */
#ifndef PIR_ORACLE_H
#define PIR_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* AES-128, FIPS-197 sections 5.1 (Cipher) and 5.2 (KeyExpansion). */
void or_aes128_sbox(uint8_t out[256]);
void or_aes128_expand(const uint8_t key[16], uint8_t w[176]);
void or_aes128_encrypt(const uint8_t w[176], const uint8_t in[16], uint8_t out[16]);
void or_aes128(const uint8_t key[16], const uint8_t in[16], uint8_t out[16]);

/* ChaCha20, RFC 8439 sections 2.1 (quarter round) and 2.3 (block function):
 * 64 keystream bytes for a 256-bit key, 32-bit block counter, 96-bit nonce. */
void or_chacha20_quarter(uint32_t *a, uint32_t *b, uint32_t *c, uint32_t *d);
void or_chacha20_block(const uint8_t key[32], uint32_t counter, const uint8_t nonce[12],
                       uint8_t out[64]);

#define OR_PRF_AES128 0u
#define OR_PRF_CHACHA20 1u

/* PRF_s(x) = AES-128_s(BE128(x)); one call = one key expansion + one block. */
void or_prf(const uint8_t s[16], uint64_t x, uint8_t out[16]);
/* PRF_s(x) = ChaCha20 keystream bytes [16x, 16x+16) under key s || s, nonce 0. */
void or_prf_chacha(const uint8_t s[16], uint64_t x, uint8_t out[16]);
/* PRF selected by prf id; returns -1 for an unknown id. */
int or_prf_by(uint32_t prf_id, const uint8_t s[16], uint64_t x, uint8_t out[16]);
/* DRBG draw i under a 16-byte seed: AES-128-CTR keystream block i. */
void or_drbg_block(const uint8_t seed[16], uint64_t i, uint8_t out[16]);

size_t or_key_size(uint32_t n);
/* Returns 0, or -1 on bad arguments (n outside [1,32], alpha >= 2^n, null). */
int or_gen(uint32_t n, uint64_t alpha, uint32_t beta, const uint8_t seed[16],
           uint8_t *key0, uint8_t *key1);
/* Same construction with the tree's PRF chosen by prf_id (the random draws
 * stay AES-128-CTR); or_gen is prf_id 0.  -1 also for an unknown prf_id. */
int or_gen_prf(uint32_t n, uint64_t alpha, uint32_t beta, const uint8_t seed[16],
               uint32_t prf_id, uint8_t *key0, uint8_t *key1);
/* Share of one index j (walks root to leaf). */
uint32_t or_eval_point(const uint8_t *key, uint64_t j);
/* All 2^d seeds at depth d (16 bytes each), by the recurrence. */
int or_eval_level(const uint8_t *key, uint32_t d, uint8_t *seeds);
/* All 2^n shares (uint32). */
int or_eval_full(const uint8_t *key, uint32_t *shares);
/* ans[k] = sum_{j<rows} Eval(key, j) * T[j][k] mod 2^32; rows <= 2^n. */
int or_answer(const uint8_t *key, const uint32_t *table, uint64_t rows,
              uint32_t dim, uint32_t *ans);
/* A row slice (one GPU's share of a row-sharded table, section 3.2.7):
 * ans[k] = sum_{i<rows} Eval(key, row0 + i) * T[i][k] mod 2^32, shares by
 * point evaluation; row0 + rows <= 2^n. */
int or_answer_slice(const uint8_t *key, uint64_t row0, const uint32_t *table, uint64_t rows,
                    uint32_t dim, uint32_t *ans);
/* Same, for nkeys keys at byte stride `stride`, spread over nthreads threads
 * (one key per task; the arithmetic per key is or_answer's). */
int or_answer_batch(const uint8_t *keys, uint32_t nkeys, size_t stride,
                    const uint32_t *table, uint64_t rows, uint32_t dim,
                    uint32_t *ans, int nthreads);
/* Partial batch retrieval (section 4.1), server side: bins of 2^bin_log rows,
 * key (c, b) at keys + (c * n_bins + b) * stride with n_bins = ceil(rows /
 * 2^bin_log), every key over the bin domain (n = bin_log);
 * ans[(c * n_bins + b) * dim + k] = sum_{j < rows_b} Eval(key, j) T[b 2^bin_log + j][k]. */
int or_answer_bins(const uint8_t *keys, uint32_t n_clients, size_t stride, const uint32_t *table,
                   uint64_t rows, uint32_t dim, uint32_t bin_log, uint32_t *ans, int nthreads);
void or_reconstruct(const uint32_t *a0, const uint32_t *a1, uint32_t dim,
                    uint32_t *out);

/* Per-thread call counters (for the O(L) work claims of section 3.1). */
uint64_t or_count_prf(void);
uint64_t or_count_drbg(void);
void or_reset_counts(void);

#ifdef __cplusplus
}
#endif
#endif
