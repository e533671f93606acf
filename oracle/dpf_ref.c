/*
 * dpf_ref.c -- the oracle's DPF and PIR answer (test infrastructure only).
 *
 * Paper section 3.1: keys k_a, k_b are produced by Gen; a server expands its
 * key over every index with the node recurrence of Eq. (p1)-(p3) and takes
 * the product of the resulting share vector with the table; the client adds
 * the two answers.  Every function below does exactly one of those steps, in
 * the paper's order and notation, with no blocking or reordering.
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes of the repository):
 *   - "+" inside the tree is XOR (the codewords live in F_{2^lambda}); the
 *     share of a leaf is its low 32 bits read little-endian, times (-1)^b,
 *     in Z_{2^32}.
 *   - "P mod 2" is bit 0 of byte 0 of the seed.
 *   - PRF_s(x) is AES-128 in counter mode: block x of the keystream under key
 *     s, i.e. AES_s(BE128(x)).  With prf id 1 (ChaCha20, the stream cipher of
 *     section 3.2.6) it is bytes [16x, 16x+16) of the RFC 8439 keystream under
 *     the 256-bit key s || s, nonce zero, block counter from zero.
 *   - Index bits are consumed most significant first (the parent of (d, j)
 *     is (d-1, floor(j/2)), as in the L = 4 walk-through).
 *   - The root sits in the key beside the codewords; the two keys share
 *     their codewords and differ only in party and root.
 *   - Gen, which the paper defers to its DPF reference, is the construction
 *     in or_gen; its randomness is AES-128-CTR under a 16-byte seed.
 */
#include "oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

static _Thread_local uint64_t n_prf_calls;
static _Thread_local uint64_t n_drbg_draws;

uint64_t or_count_prf(void) { return n_prf_calls; }
uint64_t or_count_drbg(void) { return n_drbg_draws; }
void or_reset_counts(void)
{
    n_prf_calls = 0;
    n_drbg_draws = 0;
}

/* counter block for counter value x: 128-bit big-endian integer */
static void counter_block(uint64_t x, uint8_t blk[16])
{
    memset(blk, 0, 16);
    for (int i = 0; i < 8; i++)
        blk[15 - i] = (uint8_t)(x >> (8 * i));
}

void or_prf(const uint8_t s[16], uint64_t x, uint8_t out[16])
{
    uint8_t blk[16];
    counter_block(x, blk);
    or_aes128(s, blk, out);
    n_prf_calls++;
}

/* ChaCha20 keystream bytes [16x, 16x+16) under the key s || s */
void or_prf_chacha(const uint8_t s[16], uint64_t x, uint8_t out[16])
{
    uint8_t key[32], nonce[12] = {0}, blk[64];
    memcpy(key, s, 16);
    memcpy(key + 16, s, 16);
    or_chacha20_block(key, (uint32_t)(x / 4), nonce, blk);
    memcpy(out, blk + 16 * (x % 4), 16);
    n_prf_calls++;
}

int or_prf_by(uint32_t prf_id, const uint8_t s[16], uint64_t x, uint8_t out[16])
{
    if (prf_id == OR_PRF_AES128)
        or_prf(s, x, out);
    else if (prf_id == OR_PRF_CHACHA20)
        or_prf_chacha(s, x, out);
    else
        return -1;
    return 0;
}

void or_drbg_block(const uint8_t seed[16], uint64_t i, uint8_t out[16])
{
    uint8_t blk[16];
    counter_block(i, blk);
    or_aes128(seed, blk, out);
    n_drbg_draws++;
}

size_t or_key_size(uint32_t n) { return 32 + 64 * (size_t)n; }

/* control bit t(s) = "s mod 2" */
static int tbit(const uint8_t s[16]) { return s[0] & 1; }

static uint32_t low32(const uint8_t s[16])
{
    return (uint32_t)s[0] | ((uint32_t)s[1] << 8) | ((uint32_t)s[2] << 16) |
           ((uint32_t)s[3] << 24);
}

static void xor16(uint8_t *dst, const uint8_t *a, const uint8_t *b)
{
    for (int i = 0; i < 16; i++)
        dst[i] = a[i] ^ b[i];
}

/* the codeword C_t[c, d] inside a key, d = 1..n */
static const uint8_t *cw(const uint8_t *key, int t, int c, uint32_t d)
{
    return key + 32 + 64 * (size_t)(d - 1) + 32 * t + 16 * c;
}

static int key_ok(const uint8_t *key)
{
    return key && key[0] == 1 && key[1] <= 1 && key[2] >= 1 && key[2] <= 32 &&
           key[3] <= OR_PRF_CHACHA20;
}

static uint32_t share_of(const uint8_t *key, const uint8_t leaf[16])
{
    uint32_t v = low32(leaf);
    return key[1] ? (uint32_t)(0u - v) : v; /* (-1)^b mod 2^32 */
}

/* one step of Eq. (p3): child j mod 2 = c of the node with seed `parent` */
static void child(const uint8_t *key, const uint8_t parent[16], int c, uint32_t d,
                  uint8_t out[16])
{
    uint8_t p[16];
    or_prf_by(key[3], parent, (uint64_t)c, p);
    xor16(out, p, cw(key, tbit(parent), c, d));
}

int or_gen(uint32_t n, uint64_t alpha, uint32_t beta, const uint8_t seed[16],
           uint8_t *key0, uint8_t *key1)
{
    return or_gen_prf(n, alpha, beta, seed, OR_PRF_AES128, key0, key1);
}

int or_gen_prf(uint32_t n, uint64_t alpha, uint32_t beta, const uint8_t seed[16],
               uint32_t prf_id, uint8_t *key0, uint8_t *key1)
{
    if (!seed || !key0 || !key1 || n < 1 || n > 32 || prf_id > OR_PRF_CHACHA20)
        return -1;
    if (n < 64 && alpha >= ((uint64_t)1 << n))
        return -1;
    uint64_t draw = 0;
    uint8_t s[2][16];

    /* roots with opposite control bits */
    or_drbg_block(seed, draw++, s[0]);
    or_drbg_block(seed, draw++, s[1]);
    s[1][0] = (uint8_t)((s[1][0] & 0xfe) | (1 - tbit(s[0])));

    uint8_t *keys[2] = {key0, key1};
    for (int b = 0; b < 2; b++) {
        memset(keys[b], 0, or_key_size(n));
        keys[b][0] = 1;
        keys[b][1] = (uint8_t)b;
        keys[b][2] = (uint8_t)n;
        keys[b][3] = (uint8_t)prf_id;
        memcpy(keys[b] + 16, s[b], 16);
    }

    for (uint32_t d = 1; d <= n; d++) {
        int c = (int)((alpha >> (n - d)) & 1); /* on-path child */
        int cb = 1 - c;                        /* off-path child */
        int tau = tbit(s[0]);                  /* party 1 holds 1 - tau */
        uint8_t P[2][2][16];                   /* P[b][x] = PRF_{s_b}(x) */
        for (int b = 0; b < 2; b++)
            for (int x = 0; x < 2; x++)
                or_prf_by(prf_id, s[b], (uint64_t)x, P[b][x]);

        uint8_t C[2][2][16]; /* C[t][c] at this depth */

        /* off-path: both parties land on the same seed P_0 ^ R */
        uint8_t R[16];
        or_drbg_block(seed, draw++, R);
        memcpy(C[tau][cb], R, 16);
        for (int i = 0; i < 16; i++)
            C[1 - tau][cb][i] = R[i] ^ P[0][cb][i] ^ P[1][cb][i];

        /* on-path: party 0 gets P_0 ^ R', party 1 is steered below */
        uint8_t R2[16], ns0[16], ns1[16];
        or_drbg_block(seed, draw++, R2);
        memcpy(C[tau][c], R2, 16);
        xor16(ns0, P[0][c], R2);

        if (d < n) {
            /* keep the two on-path control bits different */
            uint8_t Q[16];
            or_drbg_block(seed, draw++, Q);
            Q[0] = (uint8_t)((Q[0] & 0xfe) | ((P[1][c][0] & 1) ^ 1 ^ tbit(ns0)));
            memcpy(C[1 - tau][c], Q, 16);
            xor16(ns1, P[1][c], Q);
        } else {
            /* last level: s1 = s0 - beta as little-endian 128-bit integers,
             * so low32(s0) - low32(s1) = beta (mod 2^32) */
            uint32_t borrow = 0;
            for (int i = 0; i < 16; i++) {
                uint32_t sub = (i < 4) ? ((beta >> (8 * i)) & 0xff) : 0;
                int32_t v = (int32_t)ns0[i] - (int32_t)sub - (int32_t)borrow;
                borrow = v < 0;
                ns1[i] = (uint8_t)(v & 0xff);
            }
            xor16(C[1 - tau][c], P[1][c], ns1);
        }

        for (int b = 0; b < 2; b++)
            for (int t = 0; t < 2; t++)
                for (int x = 0; x < 2; x++)
                    memcpy(keys[b] + 32 + 64 * (size_t)(d - 1) + 32 * t + 16 * x,
                           C[t][x], 16);
        memcpy(s[0], ns0, 16);
        memcpy(s[1], ns1, 16);
    }
    return 0;
}

uint32_t or_eval_point(const uint8_t *key, uint64_t j)
{
    uint32_t n = key[2];
    uint8_t s[16], nx[16];
    memcpy(s, key + 16, 16); /* P(0,0) */
    for (uint32_t d = 1; d <= n; d++) {
        int c = (int)((j >> (n - d)) & 1);
        child(key, s, c, d, nx);
        memcpy(s, nx, 16);
    }
    return share_of(key, s);
}

int or_eval_level(const uint8_t *key, uint32_t d, uint8_t *seeds)
{
    if (!key_ok(key) || !seeds || d > key[2] || d > 24)
        return -1;
    uint8_t *cur = malloc(16 << d), *nxt = malloc(16 << d);
    if (!cur || !nxt) {
        free(cur);
        free(nxt);
        return -1;
    }
    memcpy(cur, key + 16, 16);
    for (uint32_t e = 1; e <= d; e++) {
        for (uint64_t j = 0; j < ((uint64_t)1 << e); j++)
            child(key, cur + 16 * (j >> 1), (int)(j & 1), e, nxt + 16 * j);
        uint8_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
    memcpy(seeds, cur, 16 << d);
    free(cur);
    free(nxt);
    return 0;
}

/* depth-first walk of the tree; every node is evaluated once by Eq. (p3) */
static void expand(const uint8_t *key, const uint8_t P[16], uint32_t d, uint64_t j,
                   uint32_t *shares)
{
    uint32_t n = key[2];
    if (d == n) {
        shares[j] = share_of(key, P);
        return;
    }
    for (int c = 0; c < 2; c++) {
        uint8_t ch[16];
        child(key, P, c, d + 1, ch);
        expand(key, ch, d + 1, 2 * j + (uint64_t)c, shares);
    }
}

int or_eval_full(const uint8_t *key, uint32_t *shares)
{
    if (!key_ok(key) || !shares)
        return -1;
    expand(key, key + 16, 0, 0, shares);
    return 0;
}

int or_answer(const uint8_t *key, const uint32_t *table, uint64_t rows,
              uint32_t dim, uint32_t *ans)
{
    if (!key_ok(key) || !table || !ans || dim == 0 || rows == 0)
        return -1;
    uint32_t n = key[2];
    if (n > 30 || rows > ((uint64_t)1 << n))
        return -1;
    uint32_t *y = malloc(sizeof(uint32_t) << n);
    if (!y)
        return -1;
    or_eval_full(key, y);
    for (uint32_t k = 0; k < dim; k++)
        ans[k] = 0;
    for (uint64_t j = 0; j < rows; j++)
        for (uint32_t k = 0; k < dim; k++)
            ans[k] += y[j] * table[j * dim + k]; /* uint32 wraps mod 2^32 */
    free(y);
    return 0;
}

/* One GPU's share of a table whose rows are split over several GPUs (section
 * 3.2.7): each GPU evaluates the DPF on its own subset of the indices and the
 * partial results are summed.  Here the subset is the slice row0 .. row0 +
 * rows - 1, table row i holding index row0 + i, every share by point
 * evaluation:  ans[k] = sum_{i<rows} Eval(key, row0 + i) * T[i][k] mod 2^32. */
int or_answer_slice(const uint8_t *key, uint64_t row0, const uint32_t *table, uint64_t rows,
                    uint32_t dim, uint32_t *ans)
{
    if (!key_ok(key) || !table || !ans || dim == 0 || rows == 0)
        return -1;
    uint32_t n = key[2];
    if (n > 62 || row0 + rows > ((uint64_t)1 << n) || row0 + rows < row0)
        return -1;
    for (uint32_t k = 0; k < dim; k++)
        ans[k] = 0;
    for (uint64_t i = 0; i < rows; i++) {
        const uint32_t y = or_eval_point(key, row0 + i);
        for (uint32_t k = 0; k < dim; k++)
            ans[k] += y * table[i * dim + k]; /* uint32 wraps mod 2^32 */
    }
    return 0;
}

struct batch_job {
    const uint8_t *keys;
    uint32_t nkeys;
    size_t stride;
    const uint32_t *table;
    uint64_t rows;
    uint32_t dim;
    uint32_t *ans;
    int nthreads, tid, status;
};

static void *batch_worker(void *arg)
{
    struct batch_job *jb = arg;
    for (uint32_t q = (uint32_t)jb->tid; q < jb->nkeys; q += (uint32_t)jb->nthreads)
        if (or_answer(jb->keys + (size_t)q * jb->stride, jb->table, jb->rows, jb->dim,
                      jb->ans + (size_t)q * jb->dim))
            jb->status = -1;
    return NULL;
}

int or_answer_batch(const uint8_t *keys, uint32_t nkeys, size_t stride,
                    const uint32_t *table, uint64_t rows, uint32_t dim,
                    uint32_t *ans, int nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    struct batch_job jobs[256];
    pthread_t th[256];
    int started[256];
    for (int i = 0; i < nthreads; i++) {
        jobs[i] = (struct batch_job){keys, nkeys, stride, table, rows, dim, ans,
                                     nthreads, i, 0};
        started[i] = pthread_create(&th[i], NULL, batch_worker, &jobs[i]) == 0;
        if (!started[i])
            batch_worker(&jobs[i]); /* run this share on the calling thread */
    }
    int st = 0;
    for (int i = 0; i < nthreads; i++) {
        if (started[i])
            pthread_join(th[i], NULL);
        st |= jobs[i].status;
    }
    return st;
}

/* Partial batch retrieval, server side (paper section 4.1): the table is cut
 * into bins of 2^bin_log consecutive rows (the last bin may be shorter) and
 * key (c, b) -- client c, bin b, at keys + (c * n_bins + b) * stride -- is a
 * DPF over the domain of one bin.  Its answer is that key's answer over the
 * bin's rows: ans[c][b][k] = sum_{j < rows_b} Eval(key, j) * T[b 2^bin_log + j][k]. */
struct bins_job {
    const uint8_t *keys;
    uint32_t n_clients, n_bins, bin_log, dim;
    size_t stride;
    const uint32_t *table;
    uint64_t rows;
    uint32_t *ans;
    int nthreads, tid, status;
};

static void *bins_worker(void *arg)
{
    struct bins_job *jb = arg;
    uint64_t total = (uint64_t)jb->n_clients * jb->n_bins;
    for (uint64_t i = (uint64_t)jb->tid; i < total; i += (uint64_t)jb->nthreads) {
        uint64_t b = i % jb->n_bins;
        uint64_t first = b << jb->bin_log;
        uint64_t rows_b = jb->rows - first;
        if (rows_b > ((uint64_t)1 << jb->bin_log))
            rows_b = (uint64_t)1 << jb->bin_log;
        const uint8_t *key = jb->keys + i * jb->stride;
        if (key[2] != jb->bin_log ||
            or_answer(key, jb->table + first * jb->dim, rows_b, jb->dim, jb->ans + i * jb->dim))
            jb->status = -1;
    }
    return NULL;
}

int or_answer_bins(const uint8_t *keys, uint32_t n_clients, size_t stride, const uint32_t *table,
                   uint64_t rows, uint32_t dim, uint32_t bin_log, uint32_t *ans, int nthreads)
{
    if (!keys || !table || !ans || rows == 0 || dim == 0 || bin_log < 1 || bin_log > 30)
        return -1;
    uint64_t n_bins = (rows + ((uint64_t)1 << bin_log) - 1) >> bin_log;
    if (n_bins > 0xffffffffu)
        return -1;
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    struct bins_job jobs[256];
    pthread_t th[256];
    int started[256];
    for (int i = 0; i < nthreads; i++) {
        jobs[i] = (struct bins_job){keys, n_clients, (uint32_t)n_bins, bin_log, dim, stride,
                                    table, rows, ans, nthreads, i, 0};
        started[i] = pthread_create(&th[i], NULL, bins_worker, &jobs[i]) == 0;
        if (!started[i])
            bins_worker(&jobs[i]);
    }
    int st = 0;
    for (int i = 0; i < nthreads; i++) {
        if (started[i])
            pthread_join(th[i], NULL);
        st |= jobs[i].status;
    }
    return st;
}

void or_reconstruct(const uint32_t *a0, const uint32_t *a1, uint32_t dim, uint32_t *out)
{
    for (uint32_t k = 0; k < dim; k++)
        out[k] = a0[k] + a1[k];
}
