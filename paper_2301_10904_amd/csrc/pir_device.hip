// pir_device.hip -- fused full-domain DPF evaluation x table product on gfx950.
//
// For every key q of a batch, one server computes (paper section 3.1)
//     out[q][k] = sum_j Eval(k_q, j) * T[j][k]   (mod 2^32),
// where Eval expands the key's GGM tree with the node recurrence of Eq.
// (p1)-(p3): each internal node with seed s yields its two children
// AES128_s(BE128(c)) ^ C_{t(s)}[c, d], c in {0,1}.
//
// Work decomposition (sections 3.2.1, 3.2.3 and 3.2.4 of the paper give the
// V100 design: a batch over blocks, a depth-first traversal holding K nodes
// per level, and the product fused at the leaves; here it is re-planned for
// 64-wide wavefronts and a large LDS):
//   * A work item is (group of Q keys, chunk of 2^H rows).  One workgroup of
//     256 lanes owns an item: S = 256/Q lanes per key.
//   * Descent: Q lanes walk from each root to the chunk's subtree root.
//   * Breadth-first expansion in LDS until every lane holds one node.
//   * Each lane then walks its own subtree of height h depth-first with the
//     path (both children of every node on it) in registers: every node is
//     evaluated once and no seed below the lane's root ever leaves the VGPRs.
//   * Each step of that walk yields two leaf shares per lane; they go to LDS
//     and the workgroup immediately multiplies them into the streamed table
//     rows (coalesced: one wave reads one 256-byte row per instruction).
//   * Partial sums are reduced across waves in LDS and added with 32-bit
//     atomics into out; integer addition mod 2^32 makes the result exact and
//     independent of the order.
//
// AES-128 runs on little-endian column words with the combined
// SubBytes/MixColumns table TE replicated 32 times across the LDS banks, so
// lane l always reads bank (l mod 32) and table lookups never conflict.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "aes_tables.h"
#include "pir.h"
#include "pir_internal.h"

namespace {

constexpr int NT = 256;            // lanes per workgroup
constexpr int NW = NT / 64;        // waves per workgroup
constexpr int HMAX = 10;           // largest per-lane subtree height
constexpr int TAB_REPL = 32;       // TE copies, one per LDS bank
constexpr int TAB_WORDS = 256 * TAB_REPL;

__constant__ pir_aes::Words256 c_TE = pir_aes::TE;
__device__ uint32_t g_key_error;

struct Seed {
    uint32_t w[4];
};

struct Tab {
    const uint32_t *lds;
    uint32_t lane;
    __device__ __forceinline__ uint32_t te(uint32_t x) const { return lds[(x << 5) | lane]; }
};

__device__ __forceinline__ uint32_t b0(uint32_t w) { return w & 0xff; }
__device__ __forceinline__ uint32_t b1(uint32_t w) { return (w >> 8) & 0xff; }
__device__ __forceinline__ uint32_t b2(uint32_t w) { return (w >> 16) & 0xff; }
__device__ __forceinline__ uint32_t b3(uint32_t w) { return w >> 24; }
__device__ __forceinline__ uint32_t rotl(uint32_t x, int k) { return (x << k) | (x >> (32 - k)); }

// SubWord(RotWord(w)) ^ rcon, little-endian words; S(x) is byte 1 of TE(x)
__device__ __forceinline__ uint32_t ks_word(const Tab &T, uint32_t w, uint32_t rcon)
{
    uint32_t t0 = T.te(b1(w)), t1 = T.te(b2(w)), t2 = T.te(b3(w)), t3 = T.te(b0(w));
    return (((t0 >> 8) & 0xffu) | (t1 & 0xff00u) | ((t2 << 8) & 0xff0000u) |
            ((t3 << 16) & 0xff000000u)) ^
           rcon;
}

__device__ __forceinline__ void next_round_key(const Tab &T, uint32_t k[4], uint32_t rcon)
{
    k[0] ^= ks_word(T, k[3], rcon);
    k[1] ^= k[0];
    k[2] ^= k[1];
    k[3] ^= k[2];
}

__device__ __forceinline__ uint32_t mix_col(const Tab &T, uint32_t a, uint32_t b, uint32_t c,
                                            uint32_t d, uint32_t k)
{
    return T.te(b0(a)) ^ rotl(T.te(b1(b)), 8) ^ rotl(T.te(b2(c)), 16) ^ rotl(T.te(b3(d)), 24) ^ k;
}

__device__ __forceinline__ uint32_t last_col(const Tab &T, uint32_t a, uint32_t b, uint32_t c,
                                             uint32_t d, uint32_t k)
{
    uint32_t ta = T.te(b0(a)), tb = T.te(b1(b)), tc = T.te(b2(c)), td = T.te(b3(d));
    return (((ta >> 8) & 0xffu) | (tb & 0xff00u) | (tc & 0xff0000u) | ((td << 16) & 0xff000000u)) ^ k;
}

__device__ __forceinline__ void full_round(const Tab &T, uint32_t s[4], const uint32_t k[4])
{
    uint32_t t0 = mix_col(T, s[0], s[1], s[2], s[3], k[0]);
    uint32_t t1 = mix_col(T, s[1], s[2], s[3], s[0], k[1]);
    uint32_t t2 = mix_col(T, s[2], s[3], s[0], s[1], k[2]);
    uint32_t t3 = mix_col(T, s[3], s[0], s[1], s[2], k[3]);
    s[0] = t0;
    s[1] = t1;
    s[2] = t2;
    s[3] = t3;
}

__device__ __forceinline__ void final_round(const Tab &T, uint32_t s[4], const uint32_t k[4])
{
    uint32_t t0 = last_col(T, s[0], s[1], s[2], s[3], k[0]);
    uint32_t t1 = last_col(T, s[1], s[2], s[3], s[0], k[1]);
    uint32_t t2 = last_col(T, s[2], s[3], s[0], s[1], k[2]);
    uint32_t t3 = last_col(T, s[3], s[0], s[1], s[2], k[3]);
    s[0] = t0;
    s[1] = t1;
    s[2] = t2;
    s[3] = t3;
}

// PRF_s(0) and PRF_s(1): AES-128 under key s of the counter blocks 0 and 1.
// The key schedule runs once, interleaved with the two encryptions.
__device__ __forceinline__ void prf_pair(const Tab &T, const Seed &s, uint32_t a[4], uint32_t b[4])
{
    uint32_t k[4] = {s.w[0], s.w[1], s.w[2], s.w[3]};
    a[0] = k[0];
    a[1] = k[1];
    a[2] = k[2];
    a[3] = k[3];
    b[0] = k[0];
    b[1] = k[1];
    b[2] = k[2];
    b[3] = k[3] ^ 0x01000000u; // counter 1 = byte 15
#pragma unroll
    for (int r = 1; r <= 9; r++) {
        next_round_key(T, k, pir_aes::RCON.v[r]);
        full_round(T, a, k);
        full_round(T, b, k);
    }
    next_round_key(T, k, pir_aes::RCON.v[10]);
    final_round(T, a, k);
    final_round(T, b, k);
}

// Only the first output word (bytes 0..3) of both blocks: all a leaf needs.
__device__ __forceinline__ void prf_pair_low32(const Tab &T, const Seed &s, uint32_t &y0, uint32_t &y1)
{
    uint32_t k[4] = {s.w[0], s.w[1], s.w[2], s.w[3]};
    uint32_t a[4] = {k[0], k[1], k[2], k[3]};
    uint32_t b[4] = {k[0], k[1], k[2], k[3] ^ 0x01000000u};
#pragma unroll
    for (int r = 1; r <= 9; r++) {
        next_round_key(T, k, pir_aes::RCON.v[r]);
        full_round(T, a, k);
        full_round(T, b, k);
    }
    next_round_key(T, k, pir_aes::RCON.v[10]);
    y0 = last_col(T, a[0], a[1], a[2], a[3], k[0]);
    y1 = last_col(T, b[0], b[1], b[2], b[3], k[0]);
}

struct KeyView {
    const uint8_t *p; // key base (16-byte aligned)
    __device__ __forceinline__ Seed root() const
    {
        uint4 v = *reinterpret_cast<const uint4 *>(p + 16);
        return Seed{{v.x, v.y, v.z, v.w}};
    }
    // C_t[0, d] and C_t[1, d]
    __device__ __forceinline__ void cw(uint32_t d, uint32_t t, uint4 &c0, uint4 &c1) const
    {
        const uint4 *q = reinterpret_cast<const uint4 *>(p + 32 + 64 * (size_t)(d - 1) + 32 * t);
        c0 = q[0];
        c1 = q[1];
    }
    __device__ __forceinline__ uint32_t cw_low32(uint32_t d, uint32_t t, uint32_t c) const
    {
        return *reinterpret_cast<const uint32_t *>(p + 32 + 64 * (size_t)(d - 1) + 32 * t + 16 * c);
    }
};

// Both children of the node with seed s at depth d - 1 (codeword level d).
__device__ __forceinline__ void children(const Tab &T, const KeyView &K, const Seed &s, uint32_t d,
                                         Seed &c0, Seed &c1)
{
    uint4 w0, w1;
    K.cw(d, s.w[0] & 1u, w0, w1);
    uint32_t a[4], b[4];
    prf_pair(T, s, a, b);
    c0 = Seed{{a[0] ^ w0.x, a[1] ^ w0.y, a[2] ^ w0.z, a[3] ^ w0.w}};
    c1 = Seed{{b[0] ^ w1.x, b[1] ^ w1.y, b[2] ^ w1.z, b[3] ^ w1.w}};
}

__global__ void k_fill_zero(uint32_t *out, size_t count)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride)
        out[i] = 0;
}

struct Geometry {
    uint32_t n;        // log2 of the key domain
    uint32_t H;        // rows per item = 2^H
    uint32_t lgS;      // lanes used per key = 2^lgS (lgS < H)
    uint32_t n_groups; // key groups of Q
    uint32_t n_chunks; // row chunks
};

// Q keys per group; KCH column chunks of 64 (dim <= 64 KCH).
template <int Q, int KCH>
__global__ __launch_bounds__(NT) void k_pir_fused(const uint8_t *__restrict__ keys, uint32_t n_keys,
                                                  uint32_t stride, const uint32_t *__restrict__ table,
                                                  uint64_t rows, uint32_t dim, uint32_t *__restrict__ out,
                                                  Geometry g)
{
    constexpr int S = NT / Q;
    __shared__ uint32_t s_tab[TAB_WORDS];
    __shared__ Seed s_bfs[2][NT];
    __shared__ uint32_t s_sh[2 * S][Q];
    __shared__ uint32_t s_keyok[Q];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63, wave = tid >> 6;
    const uint32_t grp = blockIdx.x % g.n_groups;
    const uint32_t chunk = blockIdx.x / g.n_groups;
    const uint64_t row_base = (uint64_t)chunk << g.H;

    for (uint32_t i = tid; i < TAB_WORDS; i += NT)
        s_tab[i] = c_TE.v[i / TAB_REPL];
    const Tab T{s_tab, lane & 31};

    // key header check and the descent to the chunk's subtree root
    const uint32_t dtop = g.n - g.H;
    if (tid < Q) {
        uint32_t kq = grp * Q + tid;
        Seed s{{0, 0, 0, 0}};
        uint32_t ok = 0;
        if (kq < n_keys) {
            KeyView K{keys + (size_t)kq * stride};
            uint32_t hdr = *reinterpret_cast<const uint32_t *>(K.p);
            uint32_t ver = hdr & 0xff, party = (hdr >> 8) & 0xff, kn = (hdr >> 16) & 0xff, prf = hdr >> 24;
            ok = (ver == PIR_KEY_VERSION && party <= 1 && kn == g.n && prf == 0) ? 1u + party : 0u;
            if (!ok)
                atomicOr(&g_key_error, 1u);
        }
        s_keyok[tid] = ok; // 0 = skip, 1 = party 0, 2 = party 1
        if (ok) {
            KeyView K{keys + (size_t)kq * stride};
            s = K.root();
            // the descent needs T, which every lane of this wave is still filling
        }
        s_bfs[0][tid] = s;
    }
    __syncthreads();
    if (tid < Q && s_keyok[tid]) {
        KeyView K{keys + (size_t)(grp * Q + tid) * stride};
        Seed s = s_bfs[0][tid];
        for (uint32_t d = 1; d <= dtop; d++) {
            Seed c0, c1;
            children(T, K, s, d, c0, c1);
            s = ((row_base >> (g.n - d)) & 1) ? c1 : c0;
        }
        s_bfs[0][tid] = s;
    }
    __syncthreads();

    // breadth-first expansion in LDS: Q * 2^lgS nodes at depth dtop + lgS
    int cur = 0;
    for (uint32_t l = 1; l <= g.lgS; l++) {
        uint32_t half = 1u << (l - 1);
        if (tid < Q * half) {
            uint32_t q = tid >> (l - 1), j = tid & (half - 1);
            if (s_keyok[q]) {
                KeyView K{keys + (size_t)(grp * Q + q) * stride};
                Seed c0, c1;
                children(T, K, s_bfs[cur][tid], dtop + l, c0, c1);
                s_bfs[cur ^ 1][q * 2 * half + 2 * j] = c0;
                s_bfs[cur ^ 1][q * 2 * half + 2 * j + 1] = c1;
            }
        }
        __syncthreads();
        cur ^= 1;
    }

    // per-lane depth-first walk of a subtree of height h
    const uint32_t q = tid / S, ln = tid % S;
    const uint32_t S_used = 1u << g.lgS;
    const bool active = ln < S_used && s_keyok[q];
    const uint32_t h = g.H - g.lgS;            // >= 1
    const uint32_t d0 = g.n - h;               // depth of the lane's root
    const uint32_t steps = 1u << (h - 1);      // bottom nodes per lane
    const KeyView K{keys + (size_t)(grp * Q + (q < Q ? q : 0)) * stride};
    Seed node = active ? s_bfs[cur][q * S_used + ln] : Seed{{0, 0, 0, 0}};
    const Seed root = node;
    Seed right[HMAX];
#pragma unroll
    for (int i = 0; i < HMAX; i++)
        right[i] = Seed{{0, 0, 0, 0}};

    uint32_t acc[Q][KCH];
#pragma unroll
    for (int i = 0; i < Q; i++)
#pragma unroll
        for (int c = 0; c < KCH; c++)
            acc[i][c] = 0;

    for (uint32_t m = 0; m < steps; m++) {
        uint32_t kst;
        if (m == 0) {
            node = root;
            kst = 1;
        } else {
            uint32_t kf = h - 1 - __builtin_ctz(m);
#pragma unroll
            for (int i = 1; i < HMAX; i++)
                if ((uint32_t)i == kf)
                    node = right[i];
            kst = kf + 1;
        }
        if (active) {
            for (uint32_t k = kst; k < h; k++) {
                Seed c0, c1;
                children(T, K, node, d0 + k, c0, c1);
#pragma unroll
                for (int i = 1; i < HMAX; i++)
                    if ((uint32_t)i == k)
                        right[i] = c1;
                node = c0;
            }
        }
        uint32_t y0 = 0, y1 = 0;
        if (active) {
            uint32_t t = node.w[0] & 1u;
            prf_pair_low32(T, node, y0, y1);
            y0 ^= K.cw_low32(g.n, t, 0);
            y1 ^= K.cw_low32(g.n, t, 1);
        }
        __syncthreads(); // the previous step's readers are done with s_sh
        if (ln < S_used) {
            s_sh[2 * ln][q] = y0;
            s_sh[2 * ln + 1][q] = y1;
        }
        __syncthreads();
        for (uint32_t i = wave; i < 2 * S_used; i += NW) {
            uint64_t row = row_base + ((uint64_t)(i >> 1) << h) + 2 * m + (i & 1);
            if (row >= rows)
                continue;
            const uint32_t *trow = table + row * dim;
            uint32_t tv[KCH];
#pragma unroll
            for (int c = 0; c < KCH; c++) {
                uint32_t col = lane + 64 * c;
                tv[c] = col < dim ? trow[col] : 0u;
            }
#pragma unroll
            for (int qq = 0; qq < Q; qq++) {
                uint32_t y = s_sh[i][qq];
#pragma unroll
                for (int c = 0; c < KCH; c++)
                    acc[qq][c] += y * tv[c];
            }
        }
    }

    // reduce the waves' partial sums in LDS (the table copy is no longer needed)
    __syncthreads();
    uint32_t *s_acc = s_tab;
    for (uint32_t i = tid; i < Q * dim; i += NT)
        s_acc[i] = 0;
    __syncthreads();
#pragma unroll
    for (int qq = 0; qq < Q; qq++)
#pragma unroll
        for (int c = 0; c < KCH; c++) {
            uint32_t col = lane + 64 * c;
            if (col < dim)
                atomicAdd(&s_acc[qq * dim + col], acc[qq][c]);
        }
    __syncthreads();
    for (uint32_t i = tid; i < Q * dim; i += NT) {
        uint32_t qq = i / dim, col = i % dim;
        uint32_t ok = s_keyok[qq];
        if (!ok)
            continue;
        uint32_t v = s_acc[i];
        if (ok == 2)
            v = 0u - v; // party 1 holds the negated share
        atomicAdd(&out[(size_t)(grp * Q + qq) * dim + col], v);
    }
}

static uint32_t ceil_log2(uint64_t x)
{
    uint32_t r = 0;
    while (((uint64_t)1 << r) < x)
        r++;
    return r;
}

template <int Q>
static void launch_q(uint32_t kch, dim3 grid, hipStream_t st, const uint8_t *keys, uint32_t n_keys,
                     uint32_t stride, const uint32_t *table, uint64_t rows, uint32_t dim, uint32_t *out,
                     const Geometry &g)
{
    if (kch == 1)
        hipLaunchKernelGGL((k_pir_fused<Q, 1>), grid, dim3(NT), 0, st, keys, n_keys, stride, table, rows,
                           dim, out, g);
    else if (kch == 2)
        hipLaunchKernelGGL((k_pir_fused<Q, 2>), grid, dim3(NT), 0, st, keys, n_keys, stride, table, rows,
                           dim, out, g);
    else
        hipLaunchKernelGGL((k_pir_fused<Q, 4>), grid, dim3(NT), 0, st, keys, n_keys, stride, table, rows,
                           dim, out, g);
}

static int fail_hip(hipError_t e)
{
    pir_impl::set_hip_error((int)e);
    return PIR_EHIP;
}

// Validates one table's call and enqueues its kernels.
static int answer_one(const uint8_t *d_keys, uint32_t n_keys, uint32_t key_stride, const uint32_t *d_table,
                      uint64_t rows, uint32_t dim, uint32_t *d_out, hipStream_t st)
{
    if (n_keys == 0)
        return PIR_OK;
    if (!d_keys || !d_table || !d_out || rows == 0 || dim == 0)
        return PIR_EINVAL;
    if (rows > ((uint64_t)1 << PIR_MAX_LOG_DOMAIN) || dim > PIR_MAX_DIM)
        return PIR_EINVAL;
    const uint32_t n = rows <= 2 ? 1 : ceil_log2(rows);
    if (key_stride % 16 || key_stride < dpf_key_size(n) || ((uintptr_t)d_keys % 16) ||
        ((uintptr_t)d_table % 4) || ((uintptr_t)d_out % 4))
        return PIR_EINVAL;

    const uint32_t Q = n_keys >= 16 ? 16 : (uint32_t)1 << ceil_log2(n_keys);
    const uint32_t lgS_max = ceil_log2(NT / Q);
    const uint32_t groups = (n_keys + Q - 1) / Q;
    const uint32_t want = ceil_log2((2048 + groups - 1) / groups);
    uint32_t H = n > want ? n - want : 1;
    H = std::min(H, lgS_max + (uint32_t)HMAX);
    H = std::max(H, std::min(n, lgS_max + 1));
    H = std::min(H, n);
    Geometry g;
    g.n = n;
    g.H = H;
    g.lgS = std::min(lgS_max, H - 1);
    g.n_groups = groups;
    const uint64_t chunks = (rows + ((uint64_t)1 << H) - 1) >> H;
    if (chunks * groups >= ((uint64_t)1 << 31))
        return PIR_ENOMEM;
    g.n_chunks = (uint32_t)chunks;
    const uint32_t kch = dim <= 64 ? 1 : dim <= 128 ? 2 : 4;

    const size_t count = (size_t)n_keys * dim;
    const uint32_t fill_blocks = (uint32_t)std::min<size_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_zero, dim3(fill_blocks), dim3(256), 0, st, d_out, count);
    const dim3 grid((uint32_t)(chunks * groups));
    switch (Q) {
    case 1: launch_q<1>(kch, grid, st, d_keys, n_keys, key_stride, d_table, rows, dim, d_out, g); break;
    case 2: launch_q<2>(kch, grid, st, d_keys, n_keys, key_stride, d_table, rows, dim, d_out, g); break;
    case 4: launch_q<4>(kch, grid, st, d_keys, n_keys, key_stride, d_table, rows, dim, d_out, g); break;
    case 8: launch_q<8>(kch, grid, st, d_keys, n_keys, key_stride, d_table, rows, dim, d_out, g); break;
    default: launch_q<16>(kch, grid, st, d_keys, n_keys, key_stride, d_table, rows, dim, d_out, g); break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PIR_OK : fail_hip(e);
}

} // namespace

extern "C" {

int pir_answer(const uint8_t *d_keys, uint32_t n_keys, uint32_t key_stride, const uint32_t *d_table,
               uint64_t rows, uint32_t dim, uint32_t *d_out, void *stream)
{
    return answer_one(d_keys, n_keys, key_stride, d_table, rows, dim, d_out, (hipStream_t)stream);
}

int pir_answer_multi(const pir_table_t *tables, uint32_t n_tables, const uint8_t *d_keys, uint32_t key_stride,
                     uint32_t *d_out, void *stream)
{
    if (!tables && n_tables)
        return PIR_EINVAL;
    // validate every descriptor before anything is enqueued
    for (uint32_t t = 0; t < n_tables; t++) {
        const pir_table_t &T = tables[t];
        if (T.n_keys == 0)
            continue;
        if (!T.d_table || T.rows == 0 || T.dim == 0 || T.dim > PIR_MAX_DIM ||
            T.rows > ((uint64_t)1 << PIR_MAX_LOG_DOMAIN) || !d_keys || !d_out)
            return PIR_EINVAL;
        uint32_t n = T.rows <= 2 ? 1 : ceil_log2(T.rows);
        if (key_stride % 16 || key_stride < dpf_key_size(n))
            return PIR_EINVAL;
    }
    size_t key_off = 0, out_off = 0;
    for (uint32_t t = 0; t < n_tables; t++) {
        const pir_table_t &T = tables[t];
        int st = answer_one(d_keys + key_off * key_stride, T.n_keys, key_stride, T.d_table, T.rows, T.dim,
                            d_out + out_off, (hipStream_t)stream);
        if (st != PIR_OK)
            return st;
        key_off += T.n_keys;
        out_off += (size_t)T.n_keys * T.dim;
    }
    return PIR_OK;
}

int pir_check_status(void)
{
    uint32_t v = 0;
    hipError_t e = hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_key_error), sizeof v, 0, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return fail_hip(e);
    if (v) {
        v = 0;
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_key_error), &v, sizeof v, 0, hipMemcpyHostToDevice);
        if (e != hipSuccess)
            return fail_hip(e);
        return PIR_EKEY;
    }
    return PIR_OK;
}

} // extern "C"
