/*
 * pir.h -- C ABI of the MI355X two-server DPF-PIR library (libpir.so).
 *
 * The calls follow the problem statement of the paper's section 3.1 (the
 * fundamentals of PIR and DPF):
 *   - the client runs Gen(1^lambda, alpha) -> (k_a, k_b)          : dpf_gen
 *   - each server computes T x Eval(k, {0 .. L-1}) over its table   : pir_answer,
 *     which fuses the full-domain evaluation of the node recurrence, Eq.
 *     (p1)-(p3), with the share-vector x table product (section 3.2.3,
 *     the memory-bounded tree traversal, and 3.2.4, the fused product)
 *   - the client adds the two answers                                : pir_reconstruct
 *
 * Conventions
 *   - Every call returns an int status (PIR_OK or a negative PIR_E* code) and
 *     never throws or aborts across the ABI.
 *   - Pointers named d_* are device (HBM) pointers on the current HIP device;
 *     all others are host pointers.  The caller owns every buffer; the library
 *     keeps no pointer after a call returns.
 *   - Device calls are asynchronous and ordered on the caller's HIP stream
 *     (`stream` is a hipStream_t passed as void*; NULL is the default stream).
 *     Launch errors are returned as PIR_EHIP (pir_last_hip_error() gives the
 *     hipError_t); faults inside a kernel surface at the caller's next
 *     synchronisation of that stream.
 *   - Arithmetic on shares and answers is in Z_{2^32} (uint32 wrap-around).
 *
 * DPF key layout (bytes; dpf_key_size(n) = 32 + 64 n):
 *   [0] version = 1   [1] party b in {0,1}   [2] n = log2 of the domain
 *   [3] PRF id: PIR_PRF_AES128 (0) or PIR_PRF_CHACHA20 (1)   [4..15] zero
 *   [16..31] root seed P(0,0) of party b (16 bytes)
 *   [32 + 64 (d-1) + 32 t + 16 c .. +15] codeword C_t[c, d], d = 1..n,
 *                                        t, c in {0,1}
 *   The codeword part, 64 n bytes, is the key size the paper prints in its
 *   Table 4 (896 / 1280 / 1408 bytes for 2^14 / 2^20 / 2^22 entries).
 *
 * Evaluation (what pir_answer computes for each key; Eq. (p1)-(p3)):
 *   P(0,0) = root;  P(d,j) = AES128_{P(d-1, j/2)}(BE128(j mod 2))
 *                            XOR C_{t(P(d-1, j/2))}[j mod 2, d]
 *   with t(s) = bit 0 of byte 0 of s; the share of row j is
 *   (-1)^b * (bytes 0..3 of P(n,j) read little-endian) mod 2^32.
 *   With PRF id 1 the AES block is replaced by the ChaCha20 stream cipher
 *   the paper also evaluates (section 3.2.6, Table 5): PRF_s(x) is bytes
 *   [16x, 16x+16) of the RFC 8439 keystream under the 256-bit key s || s,
 *   nonce 0, block counter 0.
 */
#ifndef PIR_H
#define PIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PIR_OK 0
#define PIR_EINVAL (-1) /* a bad argument: null pointer, size or shape     */
#define PIR_ENOMEM (-2) /* a size beyond what the library supports          */
#define PIR_EHIP (-3)   /* a HIP runtime call or kernel launch failed       */
#define PIR_EKEY (-4)   /* a device-resident key had a bad header           */
#define PIR_ESTALL (-5) /* a kernel gave up a bounded wait: output invalid  */

#define PIR_KEY_VERSION 1
#define PIR_MAX_LOG_DOMAIN 32 /* n <= 32: tables of at most 2^32 rows */
#define PIR_MAX_DIM 256       /* uint32 columns per row (1 KiB rows)  */

/* PRF ids (key byte 3) */
#define PIR_PRF_AES128 0u   /* AES-128 of the counter block BE128(x)          */
#define PIR_PRF_CHACHA20 1u /* ChaCha20 keystream bytes [16x, 16x+16), s || s */

/* Size in bytes of one DPF key over a domain of 2^n indices: 32 + 64 n.
 * Returns 0 for n outside [1, 32]. */
size_t dpf_key_size(uint32_t n);

/* Client side Gen (paper section 3.1; the construction the paper defers to
 * its DPF reference is written out in the library's design notes).
 *   n      log2 of the domain, 1..32
 *   alpha  the secret index, alpha < 2^n
 *   beta   the value at alpha: Eval(k0, j) + Eval(k1, j) = beta * [j == alpha]
 *   seed16 16 bytes of randomness; the 3n+1 random 16-byte draws of Gen are
 *          the AES-128-CTR keystream under this key from counter 0.  NULL
 *          draws the seed from the operating system (getrandom).
 *   key0, key1  caller-owned host buffers of dpf_key_size(n) bytes each.
 * Returns PIR_EINVAL for null key buffers, n outside [1,32] or alpha >= 2^n,
 * and PIR_EHIP if the operating system refuses randomness. */
int dpf_gen(uint32_t n, uint64_t alpha, uint32_t beta, const uint8_t *seed16,
            uint8_t *key0, uint8_t *key1);

/* Gen with the tree's PRF chosen by prf_id (section 3.2.6: the PRF is a free
 * choice of the construction; PIR_PRF_AES128 or PIR_PRF_CHACHA20).  The
 * random draws stay the AES-128-CTR keystream under seed16, so two calls with
 * the same seed and different prf_id share their roots and random codewords.
 * dpf_gen is prf_id = PIR_PRF_AES128.  PIR_EINVAL also for an unknown prf_id. */
int dpf_gen_prf(uint32_t n, uint64_t alpha, uint32_t beta, const uint8_t *seed16,
                uint32_t prf_id, uint8_t *key0, uint8_t *key1);

/* Server side answer for one table (paper section 3.1: T x Eval(k, {0..L-1});
 * fused evaluation as in sections 3.2.3-3.2.4).
 *   d_keys     n_keys keys, key q at d_keys + q * key_stride (16-byte aligned,
 *              key_stride a multiple of 16 and >= dpf_key_size(n))
 *   d_table    row-major uint32 [rows][dim], 4-byte aligned, resident in HBM
 *              (16-byte aligned tables are read with vector loads)
 *   rows       L, 1 <= rows <= 2^32; the keys' domain is n = ceil(log2 rows)
 *              (n = 1 when rows = 1) and every key header must carry that n
 *   dim        D, 1 <= dim <= PIR_MAX_DIM
 *   d_out      uint32 [n_keys][dim]; fully overwritten:
 *              d_out[q][k] = sum_{j<rows} Eval(key_q, j) * T[j][k] mod 2^32
 *   stream     hipStream_t (void*), NULL for the default stream
 * Keys may be of either party and mixed in one call.  A key whose header is
 * bad (version, party, n or PRF id) gets an all-zero output row and sets
 * PIR_STATUS_BAD_KEY in the call's status word (pir_workspace_status,
 * pir_check_status).  n_keys = 0 is a no-op returning PIR_OK (the status
 * word is left as it was).
 * Returns PIR_EINVAL on null pointers, bad sizes or misalignment (nothing is
 * launched), PIR_ENOMEM if the call's work items reach 2^31 (tens of
 * thousands of keys on a table of 2^32 rows), PIR_EHIP if a launch fails. */
int pir_answer(const uint8_t *d_keys, uint32_t n_keys, uint32_t key_stride,
               const uint32_t *d_table, uint64_t rows, uint32_t dim, uint32_t *d_out,
               void *stream);

/* pir_answer for keys of the PRF prf_id (section 3.2.6): every key of the
 * call must carry prf_id in byte 3, else it is treated as a bad header (zero
 * output row, PIR_STATUS_BAD_KEY in the status word).  pir_answer is prf_id =
 * PIR_PRF_AES128.  PIR_EINVAL also for an unknown prf_id. */
int pir_answer_prf(uint32_t prf_id, const uint8_t *d_keys, uint32_t n_keys,
                   uint32_t key_stride, const uint32_t *d_table, uint64_t rows,
                   uint32_t dim, uint32_t *d_out, void *stream);

/* One GPU's share of a table whose rows are split over several GPUs (paper
 * section 3.2.7: each GPU evaluates the DPF on its own subset of the indices,
 * and the partial answers are summed, which is exact because the reduction
 * is a sum).  Keys of domain 2^n are evaluated on the indices row0 .. row0 +
 * rows - 1 only, table row i holding index row0 + i:
 *     d_out[q][k] = sum_{i<rows} Eval(key_q, row0 + i) * T[i][k]   mod 2^32,
 * so the outputs of slices that cover 0 .. L - 1, added mod 2^32, equal
 * pir_answer_prf over the whole table.  Each lane descends from the key's
 * root to the slice, which costs the n - m extra path nodes per key that
 * splitting over 2^(n-m) GPUs implies.
 *   n          the keys' domain, 1..32; every key header must carry it
 *   row0       first index of the slice; with m = max(1, ceil(log2 rows)) it
 *              must be a multiple of 2^m (the slice lies in one aligned
 *              subtree; equal slices of 2^(n-g) rows for 2^g GPUs do), and
 *              row0 + rows <= 2^n
 *   d_table    the slice: row-major uint32 [rows][dim], rows >= 1
 * Other arguments, bad keys and errors as for pir_answer_prf; PIR_EINVAL also
 * for an unaligned or out-of-domain slice. */
int pir_answer_slice(uint32_t prf_id, uint32_t n, uint64_t row0, const uint8_t *d_keys, uint32_t n_keys,
                     uint32_t key_stride, const uint32_t *d_table, uint64_t rows, uint32_t dim,
                     uint32_t *d_out, void *stream);

/* One table of a multi-table call (a batch grouped by table; the paper's
 * batching of section 3.2.1 over tables of different sizes, section 3.2.5). */
typedef struct {
    const uint32_t *d_table; /* row-major uint32 [rows][dim] in HBM */
    uint64_t rows;           /* L_t >= 1 */
    uint32_t dim;            /* D_t, 1..PIR_MAX_DIM */
    uint32_t n_keys;         /* keys for this table (may be 0) */
} pir_table_t;

/* Server side answer for keys over several tables of different sizes in one
 * stream-ordered call (paper section 3.1: each key is answered as
 * T_t x Eval(k, {0..L_t-1}) over its own table t; sections 3.2.1 and 3.2.5:
 * one launch serves a batch of queries of uneven domain sizes).
 *   tables     host array of n_tables descriptors
 *   d_keys     all keys, grouped by table in the order of `tables`: the first
 *              tables[0].n_keys keys query table 0, and so on; key stride and
 *              alignment as for pir_answer; each table's keys carry that
 *              table's n = ceil(log2 rows)
 *   d_out      answers packed in key order: key i of table t occupies dim_t
 *              words starting at sum over earlier keys of their dim
 * Errors as for pir_answer; any bad descriptor rejects the whole call. */
int pir_answer_multi(const pir_table_t *tables, uint32_t n_tables, const uint8_t *d_keys,
                     uint32_t key_stride, uint32_t *d_out, void *stream);

/* pir_answer_multi for keys of the PRF prf_id (section 3.2.6), as
 * pir_answer_prf. */
int pir_answer_multi_prf(uint32_t prf_id, const pir_table_t *tables, uint32_t n_tables,
                         const uint8_t *d_keys, uint32_t key_stride, uint32_t *d_out,
                         void *stream);

/* Partial batch retrieval, server side (paper section 4.1): a table is cut
 * into n_bins = ceil(rows / 2^bin_log) bins of 2^bin_log consecutive rows (the
 * last may be shorter) and every client sends one DPF key per bin, over the
 * bin's domain (n = bin_log); key (c, b) answers
 *     sum_{j < rows_b} Eval(key, j) * T[b 2^bin_log + j][k]   (mod 2^32).
 * A client wanting up to n_bins entries in distinct bins retrieves them all at
 * the cost of one full-table query.  Which entry each bin serves, and dummy
 * keys for bins it does not need, are the client's business. */
#define PIR_BINS_MIN_LOG 3  /* bins of at least 8 rows   */
#define PIR_BINS_MAX_DIM 128 /* rows of at most 128 words */
typedef struct {
    const uint32_t *d_table; /* row-major uint32 [rows][dim] in HBM, 4-byte aligned */
    uint64_t rows;           /* 1 <= rows <= 2^32 */
    uint32_t dim;            /* 1..PIR_BINS_MAX_DIM */
    uint32_t n_clients;      /* clients querying this table (may be 0) */
    uint32_t bin_log;        /* PIR_BINS_MIN_LOG..32; >= ceil(log2 rows) is one bin */
} pir_bins_t;

/* Server side answer of partial batch retrieval over one or more tables in
 * one stream-ordered call.
 *   tables     host array of n_tables descriptors
 *   d_keys     keys grouped by table in the order of `tables`; within table
 *              t, client-major: key (c, b) is the (c * n_bins_t + b)-th key
 *              of the table; every key carries n = bin_log_t and prf_id;
 *              stride and alignment as for pir_answer
 *   d_out      answers in key order, dim_t words each; fully overwritten
 * Bad key headers as for pir_answer.  PIR_EINVAL for an unknown prf_id, bad
 * sizes (including dim > PIR_BINS_MAX_DIM or bin_log < PIR_BINS_MIN_LOG),
 * null pointers or misalignment; nothing is launched then. */
int pir_answer_bins(uint32_t prf_id, const pir_bins_t *tables, uint32_t n_tables,
                    const uint8_t *d_keys, uint32_t key_stride, uint32_t *d_out,
                    void *stream);

/* The work plan pir_answer / pir_answer_prf would use for one table (the
 * batch scheduling of sections 3.2.1 and 3.2.5), for inspection and tests; it
 * launches nothing and needs no GPU.  PIR_EINVAL for an unknown prf_id, no
 * keys, or sizes pir_answer rejects; PIR_ENOMEM where pir_answer would. */
#define PIR_KERNEL_WAVES 1       /* batched: up to 16 keys per wave, int8 matrix cores; rows of
                                    65-128 words run as wave pairs (two waves on the same keys
                                    and adjacent chunks trade leaf shares, each multiplies one
                                    64-column half), items counted per wave, in pairs */
#define PIR_KERNEL_SMALL_BATCH 2 /* small batches (or rows > 128 words): 512-lane workgroups */
#define PIR_KERNEL_STREAM 3      /* one AES-128 key on a table above 256 MiB with rows of at
                                    most 64 words (a multiple of 4, 16-byte aligned): tree
                                    and table-stream waves in 512-lane workgroups */
typedef struct {
    uint32_t kernel;              /* PIR_KERNEL_* */
    uint32_t n;                   /* key domain: ceil(log2 rows), at least 1 */
    uint64_t items;               /* work items (waves or workgroups) */
    uint64_t workgroups;          /* workgroups launched */
    uint32_t lanes_per_workgroup;
    uint32_t lds_bytes;           /* static LDS per workgroup */
    uint32_t keys_per_item;       /* keys sharing one item's table rows */
    uint32_t subtree_log;         /* each lane walks a subtree of 2^subtree_log leaves */
    uint64_t rows_per_item;
    uint32_t descent_levels;      /* tree levels walked from the root to an item's subtree */
    uint32_t bfs_levels;          /* breadth-first levels in LDS (small-batch kernel) */
    uint32_t tail_keys;           /* the last tail_keys keys (1..8 past whole groups of 16) go to a
                                     second launch, planned as a batch of their own; the fields
                                     above describe the first launch, over the other keys */
    uint32_t source;              /* PIR_PLAN_MODEL or PIR_PLAN_TUNED: where the first launch's
                                     plan came from */
} pir_plan_t;
#define PIR_PLAN_MODEL 0 /* the library's cost model and measured thresholds */
#define PIR_PLAN_TUNED 1 /* an entry of the tuned plan table (pir_set_tuning) */
int pir_plan(uint32_t prf_id, uint32_t n_keys, uint64_t rows, uint32_t dim, pir_plan_t *out);

/* Tuned plans (sections 3.2.1 and 3.2.5 tune the batch scheduling, and
 * section 3.2.3 its node budget K, by measurement; here the project's
 * autotuner, paper_2301_10904_amd/autotune.py, times the candidate plans of
 * each shape on the GPU and hands the winners to the library).  An entry
 * covers single-table calls (pir_answer, pir_answer_prf, pir_answer_slice)
 * of one PRF whose rows lie in an aligned subtree of height n, with row
 * widths dim_lo..dim_hi and batches of keys_lo..keys_hi keys; the first
 * matching entry fixes the fields it sets, the model the rest.  Multi-table
 * and bins calls always use the model.  A field value the call cannot use
 * (the wave kernel on rows wider than 128 words, 16 keys per workgroup on
 * rows of 65..128 words, a height above what the rows allow) falls back to
 * the model or is clamped, so any entry gives correct answers. */
#define PIR_TUNE_MODEL 0xffffffffu /* tail_keys: keep the model's rule */
typedef struct {
    uint32_t prf_id;             /* PIR_PRF_* */
    uint32_t n;                  /* 1..32 */
    uint32_t dim_lo, dim_hi;     /* 1 <= dim_lo <= dim_hi <= PIR_MAX_DIM */
    uint32_t keys_lo, keys_hi;   /* 1 <= keys_lo <= keys_hi */
    uint32_t kernel;             /* 0 (the model's), PIR_KERNEL_WAVES or PIR_KERNEL_SMALL_BATCH */
    uint32_t subtree_log;        /* wave kernel: 0 (the model's) or 1..9 */
    uint32_t keys_per_item;      /* small-batch kernel: 0 (the model's), 1, 2, 4, 8 or 16 */
    uint32_t tail_keys;          /* PIR_TUNE_MODEL, 0 (never split off a remainder) or 1..8: a
                                    remainder of 1..tail_keys keys past whole groups of 16 gets
                                    a launch of its own */
} pir_tune_t;
#define PIR_TUNE_MAX_ENTRIES 65536

/* Replaces the tuned plan table with a copy of entries[0..count); count = 0
 * clears it (every plan from the model).  Process-wide; calls already
 * enqueued are unaffected, and calls planned concurrently see either table.
 * PIR_EINVAL (the table unchanged) for a null pointer with count > 0, more
 * than PIR_TUNE_MAX_ENTRIES entries, or an entry outside the ranges above. */
int pir_set_tuning(const pir_tune_t *entries, uint32_t count);

/* Entries of the tuned plan table. */
uint32_t pir_tuning_count(void);

/* Static, NUL-terminated fingerprint of the kernel sources this library was
 * built from (comments and layout ignored): a tuned plan table is only valid
 * for the kernels it was measured on. */
const char *pir_kernel_digest(void);

/* The work plan pir_answer_bins would use for a call over this one table
 * (section 4.1: n_clients clients, one key per bin of 2^bin_log rows), for
 * inspection and tests; it launches nothing and needs no GPU.  PIR_EINVAL for
 * an unknown prf_id, no clients, or sizes pir_answer_bins rejects; PIR_ENOMEM
 * where it would.  subtree_log is always in 1 .. bin_log. */
int pir_plan_bins(uint32_t prf_id, uint64_t rows, uint32_t dim, uint32_t n_clients, uint32_t bin_log,
                  pir_plan_t *out);

/* Client side reconstruction (paper section 3.1): out[k] = a0[k] + a1[k]
 * mod 2^32 for k < dim; host buffers.  PIR_EINVAL on null pointers. */
int pir_reconstruct(const uint32_t *a0, const uint32_t *a1, uint32_t dim, uint32_t *out);

/* Call status (section 3.1: each server answers its own keys, so the report
 * that a key was malformed belongs to the call that saw it).
 *
 * Every answer call (pir_answer*, pir_answer_slice, pir_answer_multi*,
 * pir_answer_bins) reports into one 32-bit status word: its first kernel
 * clears the word, in stream order, and a key with a bad header sets
 * PIR_STATUS_BAD_KEY in it.  Once the call has completed, the word holds that
 * call's status.  The word is the first word of the status workspace:
 *   - the workspace the calling host thread bound with pir_set_workspace, or
 *   - if it bound none, the library's own workspace on the current device (a
 *     static device array; nothing is ever allocated), read by
 *     pir_check_status().  That one is shared by every thread and stream of
 *     the process: calls that overlap in time on one device overwrite each
 *     other's status in it, so concurrent streams should each bind their own.
 * The calls clear the word with a kernel, never a memset, so they may be
 * captured in a HIP graph; a replay reports its own status.
 *
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the answer calls never
 * allocate, and with no workspace bound they use the library's own array of
 * PIR_WORKSPACE_BYTES per device (held until the process ends), so they need
 * no buffer beyond their inputs and outputs. */
#define PIR_WORKSPACE_BYTES 256u  /* size of a status workspace */
#define PIR_STATUS_BAD_KEY 1u     /* status bit: a key had a bad header */
#define PIR_STATUS_STALLED 2u     /* status bit: a kernel gave up a bounded wait (never expected;
                                     the call's output is then not valid) */
#define PIR_WAIT_LIMIT_DEFAULT (1u << 22) /* tries of a bounded wait (see pir_set_wait_limit) */

/* Bytes of a status workspace: PIR_WORKSPACE_BYTES. */
size_t pir_workspace_size(void);

/* Binds d_ws, a device buffer of at least pir_workspace_size() bytes,
 * 16-byte aligned, on the device the calls will run on, as the status
 * workspace of the answer calls this host thread makes from now on; NULL
 * unbinds (back to the library's own).  The caller owns the buffer and keeps
 * it alive while calls that use it may run; it needs no initialisation.
 * PIR_EINVAL for a short or misaligned buffer (the binding is unchanged). */
int pir_set_workspace(void *d_ws, size_t bytes);

/* The status of the last call that used workspace d_ws, in the order of
 * `stream`: enqueues a read of the word on `stream` and waits for it, so the
 * calls enqueued on `stream` before have completed.  PIR_ESTALL if one of
 * that call's kernels gave up a bounded wait (its output is not valid), else
 * PIR_EKEY if it saw a key with a bad header (version, party, n or PRF id),
 * else PIR_OK; PIR_EINVAL for a null or misaligned d_ws; PIR_EHIP if the read
 * fails. */
int pir_workspace_status(const void *d_ws, void *stream);

/* After the caller has synchronised the stream of the last call that used the
 * library's own workspace on the current device: PIR_ESTALL, PIR_EKEY or
 * PIR_OK as for pir_workspace_status; PIR_EHIP if the word cannot be read. */
int pir_check_status(void);

/* The number of tries a kernel's bounded wait makes before it gives up
 * (waves of one workgroup handing work to each other; a wait that gives up
 * sets PIR_STATUS_STALLED and the kernel ends).  Correct code never reaches
 * the default, PIR_WAIT_LIMIT_DEFAULT; tests of the stalled-wait path set a
 * small limit to force it, and 0 restores the default.  Applies to calls
 * launched afterwards from any thread.  Returns PIR_OK. */
int pir_set_wait_limit(uint32_t tries);

/* Static, NUL-terminated description of a status code. */
const char *pir_strerror(int status);

/* The hipError_t of the last failed HIP call in this thread (0 if none). */
int pir_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif
