// pir_kernels.h -- device side of the fused full-domain DPF evaluation x table
// product on gfx950: the PRF policies, the small-batch kernel k_pir_fused and
// the batched kernel k_pir_waves, with the work-item structures their launchers
// (pir_device.hip) fill in.  Included by pir_device.hip (and by the
// measurement kernel in prf_engine.hip); everything here has internal linkage.
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
//     512 lanes owns an item: S = 512/Q lanes per key.
//   * Descent: Q lanes walk from each root to the chunk's subtree root.
//   * Breadth-first expansion in LDS until every lane holds one node.
//   * Each lane then walks its own subtree of height h depth-first with the
//     path (both children of every node on it) in registers: every node is
//     evaluated once and no seed below the lane's root ever leaves the VGPRs.
//   * Each step of that walk yields two leaf shares per lane.  A wave holds
//     all Q keys over its own subtrees, so it passes the shares through a
//     private LDS slot and immediately multiplies them into the table rows
//     of those subtrees (coalesced 256-byte rows); no workgroup barrier is
//     needed in the walk.  With 16 keys and rows of at most 64 words the
//     shares are the matrix cores' operand directly (mfma_step), as in the
//     batched kernel.
//   * Partial sums are reduced across waves in LDS and added with 32-bit
//     atomics into out; integer addition mod 2^32 makes the result exact and
//     independent of the order.
//
// AES-128 (aes_gfx950.h) runs on little-endian column words with the combined
// SubBytes/MixColumns tables replicated per lane in LDS, so table lookups never
// conflict; the tables fill the first 64 KiB, and two workgroups share a CU.
// Keys with the ChaCha20 PRF (chacha_gfx950.h, section 3.2.6) run the same
// kernels instantiated with a register-only PRF and no table in LDS.
#pragma once
#include <hip/hip_runtime.h>

#include "aes_gfx950.h"
#include "aes_tables.h"
#include "chacha_gfx950.h"
#include "pir.h"

namespace {

using namespace pir_dev;

constexpr int NT = 512;      // lanes per workgroup
constexpr int NW = NT / 64;  // waves per workgroup
constexpr int HMAX = 10;     // largest per-lane subtree height
constexpr int QMAX = 16;     // keys per workgroup

__constant__ pir_aes::Words256 c_TE = pir_aes::TE;

struct Seed {
    uint32_t w[4];
};

// The PRF of a launch.  Each provides both children's PRF outputs of a node,
// one child's, and word 0 of both (all a leaf share needs); TAB_WORDS is the
// LDS table it reads (filled by fill()), 0 for none.
// QUAD: the PRF also has the quad form (four lanes per node, lane q holding
// word q), used where a walk is latency-bound.
struct AesPrf {
    static constexpr uint32_t id = PIR_PRF_AES128;
    static constexpr uint32_t TAB_WORDS = AES_TAB_WORDS;
    static constexpr bool QUAD = true;
    Lanes L;
    __device__ __forceinline__ AesPrf(const uint32_t *tab, uint32_t lane) : L(tab, lane) {}
    static __device__ __forceinline__ void fill(uint32_t *tab, uint32_t tid, uint32_t nt)
    {
        fill_tables(tab, c_TE.v, tid, nt);
    }
    __device__ __forceinline__ void pair(const uint32_t s[4], uint32_t a[4], uint32_t b[4]) const
    {
        prf_pair(s, a, b, L);
    }
    __device__ __forceinline__ void one(const uint32_t s[4], uint32_t c, uint32_t a[4]) const { prf_one(s, c, a, L); }
    __device__ __forceinline__ void pair_word0(const uint32_t s[4], uint32_t &y0, uint32_t &y1) const
    {
        prf_pair_word0(s, y0, y1, L);
    }
    __device__ __forceinline__ void quad_pair(uint32_t s, uint32_t &a, uint32_t &b, const Quad &Qd) const
    {
        quad_prf_pair(s, a, b, Qd, L);
    }
    __device__ __forceinline__ uint32_t quad_one(uint32_t s, uint32_t c, const Quad &Qd) const
    {
        return quad_prf_one(s, c, Qd, L);
    }
};

struct ChaChaPrf {
    static constexpr uint32_t id = PIR_PRF_CHACHA20;
    static constexpr uint32_t TAB_WORDS = 0;
    static constexpr bool QUAD = true;
    __device__ __forceinline__ void quad_pair(uint32_t s, uint32_t &a, uint32_t &b, const Quad &Qd) const
    {
        quad_chacha_pair(s, a, b, Qd);
    }
    __device__ __forceinline__ uint32_t quad_one(uint32_t s, uint32_t c, const Quad &Qd) const
    {
        return quad_chacha_one(s, c, Qd);
    }
    __device__ __forceinline__ ChaChaPrf(const uint32_t *, uint32_t) {}
    static __device__ __forceinline__ void fill(uint32_t *, uint32_t, uint32_t) {}
    __device__ __forceinline__ void pair(const uint32_t s[4], uint32_t a[4], uint32_t b[4]) const
    {
        chacha_pair(s, a, b);
    }
    __device__ __forceinline__ void one(const uint32_t s[4], uint32_t c, uint32_t a[4]) const { chacha_one(s, c, a); }
    __device__ __forceinline__ void pair_word0(const uint32_t s[4], uint32_t &y0, uint32_t &y1) const
    {
        chacha_pair_word0(s, y0, y1);
    }
};

// The whole LDS of a workgroup: the PRF's table (if any), which is reused for
// the cross-wave sums of up to QMAX x PIR_MAX_DIM words.
template <uint32_t TABW>
struct Smem {
    static constexpr uint32_t W = TABW > QMAX * PIR_MAX_DIM ? TABW : QMAX * PIR_MAX_DIM;
    uint32_t tab[W];
    union {
        Seed bfs[NT];              // breadth-first nodes, then the waves' share slots
    } u;
    uint32_t keyok[QMAX];          // 0 = skip, 1 = party 0, 2 = party 1
};

struct KeyView {
    const uint8_t *p; // key base (16-byte aligned)
    __device__ __forceinline__ Seed root() const
    {
        uint4 v = *reinterpret_cast<const uint4 *>(p + 16);
        return Seed{{v.x, v.y, v.z, v.w}};
    }
};

// The codewords of a key, C_t[c, d] for d = 1..n, read from the key in HBM
// (CwGlobal) or from a copy in LDS (CwLds); both point at C_0[0, 1].  The
// casts keep the pointer's address space, so LDS copies are read with ds_read.
typedef unsigned v4u __attribute__((ext_vector_type(4)));
template <class Byte, class V4, class U32>
struct CwViewT {
    Byte *p;
    __device__ __forceinline__ uint4 vec(size_t off) const
    {
        const v4u x = *(V4 *)(p + off);
        return make_uint4(x.x, x.y, x.z, x.w);
    }
    // C_t[0, d] and C_t[1, d]
    __device__ __forceinline__ void cw(uint32_t d, uint32_t t, uint4 &c0, uint4 &c1) const
    {
        c0 = vec(64 * (size_t)(d - 1) + 32 * t);
        c1 = vec(64 * (size_t)(d - 1) + 32 * t + 16);
    }
    __device__ __forceinline__ uint4 one(uint32_t d, uint32_t t, uint32_t c) const
    {
        return vec(64 * (size_t)(d - 1) + 32 * t + 16 * c);
    }
    // word w of C_t[c, d]
    __device__ __forceinline__ uint32_t word(uint32_t d, uint32_t t, uint32_t c, uint32_t w) const
    {
        return *(U32 *)(p + 64 * (size_t)(d - 1) + 32 * t + 16 * c + 4 * w);
    }
    __device__ __forceinline__ uint2 cw_word0(uint32_t d, uint32_t t) const
    {
        return make_uint2(word(d, t, 0, 0), word(d, t, 1, 0));
    }
};
typedef const __attribute__((address_space(3))) v4u lds_v4u;
typedef CwViewT<const uint8_t, const v4u, const uint32_t> CwGlobal;
typedef CwViewT<lds_u8, lds_v4u, lds_u32> CwLds;
__device__ __forceinline__ CwGlobal cw_global(const KeyView &K) { return CwGlobal{K.p + 32}; }

// Both children of the node with seed s, codeword level d (Eq. (p3)).
template <class PRF, class CW>
__device__ __forceinline__ void children(const PRF &P, const CW &C, const Seed &s, uint32_t d, Seed &c0, Seed &c1)
{
    uint4 w0, w1;
    C.cw(d, s.w[0] & 1u, w0, w1);
    uint32_t a[4], b[4];
    P.pair(s.w, a, b);
    c0 = Seed{{a[0] ^ w0.x, a[1] ^ w0.y, a[2] ^ w0.z, a[3] ^ w0.w}};
    c1 = Seed{{b[0] ^ w1.x, b[1] ^ w1.y, b[2] ^ w1.z, b[3] ^ w1.w}};
}

// Child c of the node with seed s, codeword level d (Eq. (p3)), for descents.
template <class PRF, class CW>
__device__ __forceinline__ Seed child_on_path(const PRF &P, const CW &C, const Seed &s, uint32_t d, uint32_t c)
{
    const uint4 w = C.one(d, s.w[0] & 1u, c);
    uint32_t a[4];
    P.one(s.w, c, a);
    return Seed{{a[0] ^ w.x, a[1] ^ w.y, a[2] ^ w.z, a[3] ^ w.w}};
}

// Logical block index of this workgroup.  The hardware deals workgroups to the
// 8 XCDs in turn (block b to XCD b mod 8), and each XCD has its own L2; work
// items that read the same table rows sit at consecutive logical indices, so
// the map gives every XCD one contiguous range of logical blocks (a bijection
// on [0, gridDim.x)) and rows shared by neighbouring blocks stay in one L2.
__device__ __forceinline__ uint32_t xcd_block()
{
    constexpr uint32_t XCDS = 8;
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    const uint32_t x = b % XCDS, k = b / XCDS, per = nb / XCDS, extra = nb % XCDS;
    return x * per + (x < extra ? x : extra) + k;
}

// Clears out[0 .. count) and, if status is not null, the call's status word
// (the first launch of every call clears it, in stream order before the
// kernels that may set it).
__global__ __attribute__((unused)) void k_fill_zero(uint32_t *out, size_t count, uint32_t *status)
{
    if (status && blockIdx.x == 0 && threadIdx.x == 0)
        *status = 0;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride)
        out[i] = 0;
}

struct Geometry {
    uint64_t row0;     // index of table row 0 in the key domain (a slice; 0 for a whole table)
    uint32_t n;        // log2 of the key domain
    uint32_t H;        // rows per item = 2^H
    uint32_t lgS;      // lanes used per key = 2^lgS (lgS < H)
    uint32_t n_groups; // key groups of Q
    uint32_t n_chunks; // row chunks
};

// ---------------------------------------------------------------------------
// The share x table product on the int8 matrix cores (v_mfma_i32_16x16x32_i8:
// A lane l holds row l mod 16, K slice (l / 16) * 8 .. +7).
//
// Exactness mod 2^32 on int8 units: a uint32 x has balanced base-256 digits
// d_0..d_3 in [-128, 127] with x = sum d_a 256^a (mod 2^32); they are the bytes
// of (x + 0x80808080) ^ 0x80808080.  Then
//     y * T = sum_{s=0..3} 256^s * sum_{a+b=s} d_a(y) e_b(T)      (mod 2^32),
// so for each s one MFMA with A = digits of y arranged d_s, d_{s-1}, .., d_0
// and B = digits of T gives the s-th term; the int32 accumulators wrap mod 2^32.
// Each step folds its four terms into one running sum per tile.
// ---------------------------------------------------------------------------
typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t balanced(uint32_t x) { return (x + 0x80808080u) ^ 0x80808080u; }

// digits of x arranged for shift s: byte j holds d_{s-j} (0 where j > s)
template <int S>
__device__ __forceinline__ uint32_t arrange(uint32_t x)
{
    if (S == 0)
        return x & 0xffu;
    constexpr uint32_t sel = S == 1 ? 0x0c0c0001u : S == 2 ? 0x0c000102u : 0x00010203u;
    return __builtin_amdgcn_perm(x, x, sel);
}

__device__ __forceinline__ long pack2(uint32_t lo, uint32_t hi) { return (long)(((uint64_t)hi << 32) | lo); }

// The table column a lane feeds to the product as column n (= lane mod 16)
// of 16-column tile t.  PACKED: the lane's KT tiles are KT consecutive words
// (one vector load where the row allows it); otherwise tile t is columns
// 16 t .. 16 t + 15, so that the 16 lanes of a row read 64 contiguous bytes
// per word load.
template <int KT, bool PACKED>
__device__ __forceinline__ uint32_t col_of(uint32_t n, int t)
{
    return PACKED ? n * KT + (uint32_t)t : n + 16u * (uint32_t)t;
}

// The words v[t] = p[col_of<KT, PACKED>(n, t)] of the row at p, t < KT;
// columns past dim read zero.  VEC (PACKED): dim == 16 KT, so the words are in
// bounds and 4 KT-byte aligned, and one vector load reads them.
template <int KT, bool VEC, bool PACKED = VEC>
__device__ __forceinline__ void load_cols(const uint32_t *__restrict__ p, uint32_t dim, uint32_t n,
                                          uint32_t (&v)[KT])
{
    static_assert(PACKED || !VEC, "vector loads read packed columns");
    if (VEC) {
        const uint32_t c0 = n * KT;
        if (KT == 4) {
            const uint4 x = *reinterpret_cast<const uint4 *>(p + c0);
            v[0] = x.x;
            v[KT > 1 ? 1 : 0] = x.y;
            v[KT > 2 ? 2 : 0] = x.z;
            v[KT > 3 ? 3 : 0] = x.w;
        } else if (KT == 2) {
            const uint2 x = *reinterpret_cast<const uint2 *>(p + c0);
            v[0] = x.x;
            v[KT > 1 ? 1 : 0] = x.y;
        } else {
            v[0] = p[c0];
        }
    } else {
#pragma unroll
        for (int t = 0; t < KT; t++) {
            const uint32_t c = col_of<KT, PACKED>(n, t);
            const uint32_t x = p[c < dim ? c : dim - 1];
            v[t] = c < dim ? x : 0u;
        }
    }
}

// One walk step's product on the matrix cores: the 64 lanes hold the shares
// y0, y1 of rows 2m, 2m+1 of their subtrees (lane l: key l mod 16, subtree
// l / 16) and the table words t0, t1 of those rows at columns
// (l mod 16) KT + t; tot[t] accumulates the [16 keys x 16 columns] tile t.
template <int KT>
__device__ __forceinline__ void mfma_step(uint32_t y0, uint32_t y1, const uint32_t (&t0)[KT],
                                          const uint32_t (&t1)[KT], v4i (&tot)[KT])
{
    const uint32_t e0 = balanced(y0), e1 = balanced(y1);
    const long a0 = pack2(arrange<0>(e0), arrange<0>(e1));
    const long a1 = pack2(arrange<1>(e0), arrange<1>(e1));
    const long a2 = pack2(arrange<2>(e0), arrange<2>(e1));
    const long a3 = pack2(arrange<3>(e0), arrange<3>(e1));
    const v4i zero = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < KT; t++) {
        // tot += D_0 + 2^8 (D_1 + 2^8 (D_2 + 2^8 D_3)): D_0 accumulates in
        // the matrix core, the rest is three shift-and-add steps per word
        const long b = pack2(balanced(t0[t]), balanced(t1[t]));
        const v4i c1 = __builtin_amdgcn_mfma_i32_16x16x32_i8(a1, b, zero, 0, 0, 0);
        const v4i c2 = __builtin_amdgcn_mfma_i32_16x16x32_i8(a2, b, zero, 0, 0, 0);
        const v4i c3 = __builtin_amdgcn_mfma_i32_16x16x32_i8(a3, b, zero, 0, 0, 0);
        v4i acc = tot[t];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            // the empty asm keeps each (x << 8) + y a single v_lshl_add_u32
            // (the compiler would otherwise expand the chain into separate shifts)
            uint32_t hi = ((uint32_t)c3[i] << 8) + (uint32_t)c2[i];
            asm volatile("" : "+v"(hi));
            hi = (hi << 8) + (uint32_t)c1[i];
            asm volatile("" : "+v"(hi));
            acc[i] = (int)((uint32_t)acc[i] + (hi << 8));
        }
        tot[t] = __builtin_amdgcn_mfma_i32_16x16x32_i8(a0, b, acc, 0, 0, 0);
    }
}

// 16 bytes of a table row; STREAM: without allocating in the caches (a
// table read once per call and larger than the memory-side cache)
template <bool STREAM>
__device__ __forceinline__ uint4 row_load4(const uint32_t *p)
{
    if constexpr (STREAM) {
        typedef unsigned v4u __attribute__((ext_vector_type(4)));
        const v4u v = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(p));
        return make_uint4(v.x, v.y, v.z, v.w);
    } else {
        return *reinterpret_cast<const uint4 *>(p);
    }
}

// Q keys per group (Q <= QMAX); KCH column chunks of 64 (dim <= 64 KCH);
// VEC4: dim is a multiple of 4 and the table 16-byte aligned (16-byte row
// segments are aligned); STREAM:
// table rows are read with row_load4<true> (single keys on large tables).
// The top of a small-batch item's trees, shared by k_pir_fused and
// k_pir_stream (all lanes of the workgroup call it): the PRF's tables in LDS,
// the Q keys' headers (sm.keyok, a bad one flagged in *status), the descent
// from each root to the chunk's subtree root at depth n - H, and lgS
// breadth-first levels below it, after which sm.u.bfs holds each key's 2^lgS
// nodes at depth n - H + lgS, key-major.  cw_of(q) gives key q's codewords.
template <class PRF, int Q, class CWOF>
__device__ __forceinline__ void expand_top(Smem<PRF::TAB_WORDS> &sm, const PRF &P, const CWOF &cw_of,
                                           const uint8_t *__restrict__ keys, uint32_t n_keys, uint32_t stride,
                                           uint32_t grp, uint64_t row_base, const Geometry &g, uint32_t lgS,
                                           uint32_t *status)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    PRF::fill(sm.tab, tid, NT);

    // key headers; roots of the keys
    const uint32_t dtop = g.n - g.H;
    if (tid < Q) {
        const uint32_t kq = grp * Q + tid;
        uint32_t ok = 0;
        Seed s{{0, 0, 0, 0}};
        if (kq < n_keys) {
            const KeyView K{keys + (size_t)kq * stride};
            const uint32_t hdr = *reinterpret_cast<const uint32_t *>(K.p);
            const uint32_t ver = hdr & 0xff, party = (hdr >> 8) & 0xff, kn = (hdr >> 16) & 0xff, prf = hdr >> 24;
            ok = (ver == PIR_KEY_VERSION && party <= 1 && kn == g.n && prf == PRF::id) ? 1u + party : 0u;
            if (!ok)
                atomicOr(status, PIR_STATUS_BAD_KEY);
            else
                s = K.root();
        }
        sm.keyok[tid] = ok;
        sm.u.bfs[tid] = s;
    }
    __syncthreads(); // tables and roots are in place

    // descent from each root to the chunk's subtree root at depth n - H: a
    // dependent chain, walked by a quad of lanes per key where the PRF has the
    // quad form (lane w holds word w of the seed)
    const Quad Qd(lane);
    if constexpr (PRF::QUAD) {
        const uint32_t qk = tid >> 2, w = tid & 3;
        if (tid < 4 * Q && sm.keyok[qk]) { // whole quads: qk is the same for the four lanes
            const auto C = cw_of(qk);
            uint32_t s = sm.u.bfs[qk].w[w];
            for (uint32_t d = 1; d <= dtop; d++) {
                const uint32_t c = (uint32_t)((g.row0 + row_base) >> (g.n - d)) & 1u;
                const uint32_t t = quad_first(s) & 1u;
                s = P.quad_one(s, c, Qd) ^ C.word(d, t, c, w);
            }
            sm.u.bfs[qk].w[w] = s;
        }
    } else if (tid < Q && sm.keyok[tid]) {
        const auto C = cw_of(tid);
        Seed s = sm.u.bfs[tid];
        for (uint32_t d = 1; d <= dtop; d++)
            s = child_on_path(P, C, s, d, (uint32_t)((g.row0 + row_base) >> (g.n - d)) & 1u);
        sm.u.bfs[tid] = s;
    }
    __syncthreads();

    // breadth-first expansion in LDS, in place: Q * 2^lgS nodes at depth dtop + lgS
    for (uint32_t l = 1; l <= lgS; l++) {
        const uint32_t half = 1u << (l - 1);
        if (PRF::QUAD && 4 * Q * half <= NT) {
            // a quad of lanes per node while the level is narrow
            const uint32_t nd = tid >> 2, w = tid & 3;
            const bool mine = nd < Q * half; // whole quads
            const uint32_t q = nd >> (l - 1), j = nd & (half - 1);
            uint32_t c0 = 0, c1 = 0;
            if (mine && sm.keyok[q]) {
                const auto C = cw_of(q);
                const uint32_t s = sm.u.bfs[nd].w[w];
                const uint32_t t = quad_first(s) & 1u;
                uint32_t a, b;
                P.quad_pair(s, a, b, Qd);
                c0 = a ^ C.word(dtop + l, t, 0, w);
                c1 = b ^ C.word(dtop + l, t, 1, w);
            }
            __syncthreads(); // every parent has been read
            if (mine) {
                sm.u.bfs[q * 2 * half + 2 * j].w[w] = c0;
                sm.u.bfs[q * 2 * half + 2 * j + 1].w[w] = c1;
            }
            __syncthreads();
            continue;
        }
        const bool mine = tid < Q * half;
        const uint32_t q = tid >> (l - 1), j = tid & (half - 1);
        Seed c0{{0, 0, 0, 0}}, c1{{0, 0, 0, 0}};
        if (mine && sm.keyok[q])
            children(P, cw_of(q), sm.u.bfs[tid], dtop + l, c0, c1);
        __syncthreads(); // every parent has been read
        if (mine) {
            sm.u.bfs[q * 2 * half + 2 * j] = c0;
            sm.u.bfs[q * 2 * half + 2 * j + 1] = c1;
        }
        __syncthreads();
    }

}

template <class PRF, int Q, int KCH, bool VEC4, bool STREAM>
__global__ __launch_bounds__(NT) void k_pir_fused(const uint8_t *__restrict__ keys, uint32_t n_keys,
                                                  uint32_t stride, const uint32_t *__restrict__ table,
                                                  uint64_t rows, uint32_t dim, uint32_t *__restrict__ out,
                                                  Geometry g, uint32_t *status)
{
    __shared__ Smem<PRF::TAB_WORDS> sm;
    // CWL: one or two keys per workgroup keep their codewords in LDS (2 KiB
    // each at most), so that the dependent chain of node evaluations from the
    // root down never waits on a load from memory
    constexpr bool CWL = Q <= 2;
    constexpr uint32_t CW_WORDS = 64 * PIR_MAX_LOG_DOMAIN / 4; // one key's codewords
    __shared__ uint4 s_cw[CWL ? Q * CW_WORDS / 4 : 1];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63, wave = tid >> 6;
    const uint32_t blk = xcd_block();
    const uint32_t grp = blk % g.n_groups;
    const uint32_t chunk = blk / g.n_groups;
    const uint64_t row_base = (uint64_t)chunk << g.H;
    const PRF P(sm.tab, lane);

    if constexpr (CWL) {
        // key q's 4n codeword vectors to s_cw[q CW_WORDS / 4 ..]; a key past
        // the batch leaves its slots unused
        const uint32_t per = 4 * g.n;
        for (uint32_t i = tid; i < Q * per; i += NT) {
            const uint32_t q = i / per, j = i % per, kq = grp * Q + q;
            if (kq < n_keys)
                s_cw[q * (CW_WORDS / 4) + j] = reinterpret_cast<const uint4 *>(keys + (size_t)kq * stride + 32)[j];
        }
    }
    // the codewords of key q of the group
    auto cw_of = [&](uint32_t q) {
        if constexpr (CWL)
            return CwLds{(lds_u8 *)(s_cw + q * (CW_WORDS / 4))};
        else
            return cw_global(KeyView{keys + (size_t)(grp * Q + q) * stride});
    };

    expand_top<PRF, Q>(sm, P, cw_of, keys, n_keys, stride, grp, row_base, g, g.lgS, status);

    // per-lane depth-first walk of a subtree of height h.  Lane l of wave w
    // evaluates key q = l mod Q over subtree position w P + l / Q (P = 64 / Q
    // positions per wave), so each wave holds every key of the item over its
    // own P subtrees.
    constexpr uint32_t P_W = 64 / Q;
    const uint32_t q = lane % Q, lnw = lane / Q, ln = wave * P_W + lnw;
    const uint32_t S_used = 1u << g.lgS;
    const bool active = ln < S_used && sm.keyok[q];
    const uint32_t h = g.H - g.lgS;       // >= 1
    const uint32_t d0 = g.n - h;          // depth of the lane's root
    const uint32_t steps = 1u << (h - 1); // bottom nodes per lane
    const auto C = cw_of(q);
    Seed node = active ? sm.u.bfs[q * S_used + ln] : Seed{{0, 0, 0, 0}};
    const Seed root = node;
    Seed right[HMAX];
#pragma unroll
    for (int i = 0; i < HMAX; i++)
        right[i] = Seed{{0, 0, 0, 0}};

    // WIDE: few accumulators per column; a lane then owns 4 columns of one of
    // 4 row slots, otherwise one column of every row.  MF: sixteen keys and
    // rows of at most 64 words; the lanes are then laid out as the matrix
    // cores' operands (key lane mod 16, subtree position lane / 16) and the
    // product runs on them (mfma_step), four tiles of 16 columns.
    constexpr bool WIDE = Q * KCH <= 4;
    constexpr bool MF = Q == 16 && KCH == 1;
    uint32_t acc[WIDE || MF ? 1 : Q][WIDE || MF ? 1 : KCH];
    uint32_t accw[WIDE ? Q : 1][WIDE ? KCH : 1][4];
    v4i tot[MF ? 4 : 1];
#pragma unroll
    for (int t = 0; t < (MF ? 4 : 1); t++)
        tot[t] = v4i{0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < (WIDE || MF ? 1 : Q); i++)
#pragma unroll
        for (int c = 0; c < (WIDE || MF ? 1 : KCH); c++)
            acc[i][c] = 0;
#pragma unroll
    for (int i = 0; i < (WIDE ? Q : 1); i++)
#pragma unroll
        for (int c = 0; c < (WIDE ? KCH : 1); c++)
#pragma unroll
            for (int e = 0; e < 4; e++)
                accw[i][c][e] = 0;

    // Every row of the chunk lies in exactly one subtree position, and the
    // wave owning that position holds the shares of all Q keys for it: each
    // wave multiplies the R = 2 P rows of its step into its accumulators
    // (every row is read once per item) and needs no other wave.  With no
    // workgroup barrier in the walk the waves drift apart, and the tree work
    // of some overlaps the table loads of others.  Wave-row r is leaf r mod 2
    // of the step at position r / 2; its share for key q goes through a
    // wave-private LDS slot at (r mod 4) SHP + (r / 4) Q + q, rows padded to
    // SHP = 36 words so that the four row slots fall in different banks.
    constexpr uint32_t R_W = 2 * P_W, SHP = 36;
    uint32_t *shw = reinterpret_cast<uint32_t *>(sm.u.bfs) + wave * 4 * SHP;
    __syncthreads(); // every lane has read its node: the breadth-first area is free
    const uint32_t n_steps = wave * P_W >= S_used ? 0u : steps; // a wave with no position in use
    for (uint32_t m = 0; m < n_steps; m++) {
        // MF: this lane's two rows (leaves 2m, 2m+1 of its subtree), loaded
        // before the step's tree work so that their latency hides behind it; a
        // row past the table reads the last row and gets a zero share
        uint32_t t0[MF ? 4 : 1], t1[MF ? 4 : 1];
        const uint64_t mrow = MF ? row_base + ((uint64_t)ln << h) + 2 * m : 0;
        if constexpr (MF) {
            const uint32_t *p0 = table + (mrow < rows ? mrow : rows - 1) * dim;
            const uint32_t *p1 = table + (mrow + 1 < rows ? mrow + 1 : rows - 1) * dim;
            if (VEC4 && dim == 64) {
                load_cols<4, true>(p0, dim, lane & 15, t0);
                load_cols<4, true>(p1, dim, lane & 15, t1);
            } else {
                load_cols<4, false, true>(p0, dim, lane & 15, t0);
                load_cols<4, false, true>(p1, dim, lane & 15, t1);
            }
        }
        uint32_t kst;
        if (m == 0) {
            node = root;
            kst = 1;
        } else {
            const uint32_t kf = h - 1 - __builtin_ctz(m);
#pragma unroll
            for (int i = 1; i < HMAX; i++)
                if ((uint32_t)i == kf)
                    node = right[i];
            kst = kf + 1;
        }
        uint32_t y0 = 0, y1 = 0;
        if (active) {
            for (uint32_t k = kst; k < h; k++) {
                Seed c0, c1;
                children(P, C, node, d0 + k, c0, c1);
#pragma unroll
                for (int i = 1; i < HMAX; i++)
                    if ((uint32_t)i == k)
                        right[i] = c1;
                node = c0;
            }
            const uint2 cw = C.cw_word0(g.n, node.w[0] & 1u);
            P.pair_word0(node.w, y0, y1);
            y0 ^= cw.x;
            y1 ^= cw.y;
        }
        if constexpr (MF) {
            mfma_step<4>(mrow < rows ? y0 : 0u, mrow + 1 < rows ? y1 : 0u, t0, t1, tot);
        } else {
            // the previous step's reads of the slot come first in this wave's LDS order
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            shw[(2 * (lnw & 1)) * SHP + (lnw >> 1) * Q + q] = y0;
            shw[(2 * (lnw & 1) + 1) * SHP + (lnw >> 1) * Q + q] = y1;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if constexpr (WIDE) {
                // lane = (row slot rs = lane / 16, column group cg = lane mod 16):
                // one 16-byte load covers 4 columns of row 4 k + rs, and U rows of
                // a slot are in flight before any is used
                constexpr uint32_t U = 8 / (Q * KCH);
                const uint32_t rs = lane >> 4, cg = lane & 15;
    #pragma unroll 1 // one group of U rows in flight per wave; more costs occupancy
                for (uint32_t k0 = 0; k0 < R_W / 4; k0 += U) {
                    uint32_t tv[U][KCH][4], yv[U][Q];
    #pragma unroll
                    for (int u = 0; u < (int)U; u++) {
                        const uint32_t k = k0 + u, j = wave * P_W + 2 * k + (rs >> 1);
                        const uint64_t row = row_base + ((uint64_t)j << h) + 2 * m + (rs & 1);
                        const bool ok = j < S_used && row < rows;
                        const uint32_t *trow = table + (ok ? row : 0) * dim;
    #pragma unroll
                        for (int c = 0; c < KCH; c++) {
                            const uint32_t col = 64 * c + 4 * cg;
                            if (VEC4) {
                                const uint4 x =
                                    col < dim ? row_load4<STREAM>(trow + col) : make_uint4(0, 0, 0, 0);
                                tv[u][c][0] = ok ? x.x : 0u;
                                tv[u][c][1] = ok ? x.y : 0u;
                                tv[u][c][2] = ok ? x.z : 0u;
                                tv[u][c][3] = ok ? x.w : 0u;
                            } else {
    #pragma unroll
                                for (int e = 0; e < 4; e++) {
                                    const uint32_t cc = col + e;
                                    const uint32_t x = trow[cc < dim ? cc : dim - 1];
                                    tv[u][c][e] = (ok && cc < dim) ? x : 0u;
                                }
                            }
                        }
    #pragma unroll
                        for (int qq = 0; qq < Q; qq++)
                            yv[u][qq] = shw[rs * SHP + k * Q + qq];
                    }
    #pragma unroll
                    for (int u = 0; u < (int)U; u++)
    #pragma unroll
                        for (int qq = 0; qq < Q; qq++)
    #pragma unroll
                            for (int c = 0; c < KCH; c++)
    #pragma unroll
                                for (int e = 0; e < 4; e++)
                                    accw[qq][c][e] += yv[u][qq] * tv[u][c][e];
                }
            } else {
                // lane = column: U rows per round, their words loaded together
                // (clamped addresses, masked values) so the loads overlap
                constexpr uint32_t U = (Q * KCH >= 32) ? 2 : (Q * KCH >= 8 ? 4 : 8);
    #pragma unroll 1
                for (uint32_t r0 = 0; r0 < R_W; r0 += U) {
                    uint32_t tv[U][KCH];
    #pragma unroll
                    for (int u = 0; u < (int)U; u++) {
                        const uint32_t r = r0 + u, j = wave * P_W + (r >> 1);
                        const uint64_t row = row_base + ((uint64_t)j << h) + 2 * m + (r & 1);
                        const bool ok = j < S_used && row < rows;
                        const uint32_t *trow = table + (ok ? row : 0) * dim;
    #pragma unroll
                        for (int c = 0; c < KCH; c++) {
                            const uint32_t col = lane + 64 * c;
                            const uint32_t x = trow[col < dim ? col : dim - 1];
                            tv[u][c] = (ok && col < dim) ? x : 0u;
                        }
                    }
    #pragma unroll
                    for (int u = 0; u < (int)U; u++) {
                        const uint32_t r = r0 + u;
    #pragma unroll
                        for (int qq = 0; qq < Q; qq++) {
                            const uint32_t y = shw[(r & 3) * SHP + (r >> 2) * Q + qq];
    #pragma unroll
                            for (int c = 0; c < KCH; c++)
                                acc[qq][c] += y * tv[u][c];
                        }
                    }
                }
            }
        }
    }

    // reduce the waves' partial sums in LDS (the tables are no longer needed)
    __syncthreads();
    uint32_t *s_acc = sm.tab;
    for (uint32_t i = tid; i < Q * dim; i += NT)
        s_acc[i] = 0;
    __syncthreads();
    if constexpr (MF) {
        // lane l holds D[(l / 16) 4 + i][l mod 16] of tile t, table column
        // (l mod 16) 4 + t (packed columns)
#pragma unroll
        for (int t = 0; t < (MF ? 4 : 1); t++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const uint32_t col = col_of<4, true>(lane & 15, t);
                if (col < dim)
                    atomicAdd(&s_acc[((lane >> 4) * 4 + i) * dim + col], (uint32_t)tot[t][i]);
            }
    } else if constexpr (WIDE) {
#pragma unroll
        for (int qq = 0; qq < (WIDE ? Q : 1); qq++)
#pragma unroll
            for (int c = 0; c < (WIDE ? KCH : 1); c++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const uint32_t col = 64 * c + 4 * (lane & 15) + e;
                    if (col < dim)
                        atomicAdd(&s_acc[qq * dim + col], accw[qq][c][e]);
                }
    } else {
#pragma unroll
        for (int qq = 0; qq < (WIDE ? 1 : Q); qq++)
#pragma unroll
            for (int c = 0; c < (WIDE ? 1 : KCH); c++) {
                const uint32_t col = lane + 64 * c;
                if (col < dim)
                    atomicAdd(&s_acc[qq * dim + col], acc[qq][c]);
            }
    }
    __syncthreads();
    for (uint32_t i = tid; i < Q * dim; i += NT) {
        const uint32_t qq = i / dim, col = i % dim;
        const uint32_t ok = sm.keyok[qq];
        if (!ok)
            continue;
        uint32_t v = s_acc[i];
        if (ok == 2)
            v = 0u - v; // party 1 holds the negated share
        atomicAdd(&out[(size_t)(grp * Q + qq) * dim + col], v);
    }
}

// ---------------------------------------------------------------------------
// One key: the table stream, not the tree, bounds the call on large tables,
// and on small ones the rows wait on the tree's dependent chain; so the waves
// of a workgroup split the work.  STREAM: rows read without allocating in the
// caches (a table above the memory-side cache, read once).
// Waves 0 .. SP_WAVES-1 (producers) walk the key's subtrees, one lane per
// subtree as in k_pir_fused, and write each step's leaf shares into an LDS ring
// of SP_RING steps; the other waves (consumers) stream the table rows of each
// step from HBM as soon as its shares are in the ring and multiply them in.
// The consumers carry no tree state, so they keep 16 row loads of 16 bytes
// in flight per lane whatever the tree work is doing.  The ring's slots are
// handed over with workgroup-scope counters in LDS: a producer wave adds one
// to ready[slot] after writing its part of a step, a consumer wave adds one to
// freed[slot] after its last read of it.  Every wait is bounded (wait_limit
// tries): a wait that runs out (which correct code never reaches) sets
// PIR_STATUS_STALLED and the waves leave their loops, so the kernel always ends.
// ---------------------------------------------------------------------------
constexpr uint32_t SP_WAVES = 4;                 // producer waves
constexpr uint32_t SP_LANES = 64 * SP_WAVES;      // subtrees per workgroup
constexpr uint32_t SP_LGS = 8;                    // log2 SP_LANES: breadth-first levels
constexpr uint32_t SP_RING = 4;                   // steps of shares in the ring
constexpr uint32_t SP_STEP_WORDS = 2 * SP_LANES;  // shares of one step
constexpr uint32_t SP_CONS = NW - SP_WAVES;       // consumer waves
constexpr uint32_t SP_ROWS_PER_WAVE = SP_STEP_WORDS / SP_CONS; // rows of a step per consumer wave
constexpr uint32_t SP_U = 16;                     // row loads in flight per consumer lane
static_assert(SP_RING * SP_STEP_WORDS * 4 <= sizeof(Seed) * NT, "the ring lives in the breadth-first area");
static_assert(SP_ROWS_PER_WAVE % (4 * SP_U) == 0, "whole rounds of loads per step");

// Waits until the LDS counter reaches target, for at most `limit` tries;
// false if the wait ran out.
__device__ __forceinline__ bool wait_count(uint32_t *ctr, uint32_t target, uint32_t limit)
{
    for (uint32_t it = 0; it < limit; it++) {
        if (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) >= target)
            return true;
        __builtin_amdgcn_s_sleep(1);
    }
    return false;
}

template <class PRF, bool STREAM>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_pir_stream(const uint8_t *__restrict__ keys,
                                                   const uint32_t *__restrict__ table, uint64_t rows, uint32_t dim,
                                                   uint32_t *__restrict__ out, Geometry g, uint32_t *status,
                                                   uint32_t wait_limit)
{
    __shared__ Smem<PRF::TAB_WORDS> sm;
    constexpr uint32_t CW_WORDS = 64 * PIR_MAX_LOG_DOMAIN / 4;
    __shared__ uint4 s_cw[CW_WORDS / 4];
    __shared__ uint32_t ready[SP_RING], freed[SP_RING], stalled;

    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t chunk = xcd_block();
    const uint64_t row_base = (uint64_t)chunk << g.H;
    const PRF P(sm.tab, lane);
    if (tid < SP_RING) {
        ready[tid] = 0;
        freed[tid] = 0;
    }
    if (tid == 0)
        stalled = 0;
    for (uint32_t i = tid; i < 4 * g.n; i += NT)
        s_cw[i] = reinterpret_cast<const uint4 *>(keys + 32)[i];
    auto cw_of = [&](uint32_t) { return CwLds{(lds_u8 *)s_cw}; };
    expand_top<PRF, 1>(sm, P, cw_of, keys, 1, 0, 0, row_base, g, SP_LGS, status);
    const uint32_t ok = sm.keyok[0];
    if (!ok)
        return; // uniform: the output row stays zero

    const uint32_t h = g.H - SP_LGS; // >= 1
    const uint32_t steps = 1u << (h - 1);
    const Seed root = wave < SP_WAVES ? sm.u.bfs[tid] : Seed{{0, 0, 0, 0}};
    __syncthreads(); // every producer has its subtree root: the breadth-first area becomes the ring
    uint32_t *const ring = reinterpret_cast<uint32_t *>(sm.u.bfs);
    uint32_t accw[4] = {0, 0, 0, 0};

    if (wave < SP_WAVES) {
        // producer lane p walks subtree p (rows p 2^h .. of the chunk) depth-first
        const uint32_t p = tid;
        const CwLds C = cw_of(0);
        const uint32_t d0 = g.n - h;
        const uint64_t lane_row0 = row_base + ((uint64_t)p << h);
        Seed node = root;
        Seed right[HMAX];
#pragma unroll
        for (int i = 0; i < HMAX; i++)
            right[i] = Seed{{0, 0, 0, 0}};
        for (uint32_t m = 0; m < steps; m++) {
            const uint32_t slot = m % SP_RING;
            uint32_t kst = 1;
            if (m != 0) {
                const uint32_t kf = h - 1 - __builtin_ctz(m);
#pragma unroll
                for (int i = 1; i < HMAX; i++)
                    if ((uint32_t)i == kf)
                        node = right[i];
                kst = kf + 1;
            }
            for (uint32_t k = kst; k < h; k++) {
                Seed c0, c1;
                children(P, C, node, d0 + k, c0, c1);
#pragma unroll
                for (int i = 1; i < HMAX; i++)
                    if ((uint32_t)i == k)
                        right[i] = c1;
                node = c0;
            }
            const uint2 cw = C.cw_word0(g.n, node.w[0] & 1u);
            uint32_t y0, y1;
            P.pair_word0(node.w, y0, y1);
            const uint64_t r0 = lane_row0 + 2 * m;
            y0 = r0 < rows ? y0 ^ cw.x : 0u; // rows past the table add nothing
            y1 = r0 + 1 < rows ? y1 ^ cw.y : 0u;
            // the slot is free once every consumer wave is done with step m - SP_RING
            if (m >= SP_RING && !wait_count(&freed[slot], SP_CONS * (m / SP_RING), wait_limit)) {
                stalled = 1;
                break;
            }
            ring[slot * SP_STEP_WORDS + 2 * p] = y0;
            ring[slot * SP_STEP_WORDS + 2 * p + 1] = y1;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0)
                __hip_atomic_fetch_add(&ready[slot], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    } else {
        // consumer wave c takes rows c R .. (c + 1) R - 1 of each step (R =
        // SP_ROWS_PER_WAVE; step row k is leaf k mod 2 of subtree k / 2);
        // lane (rs = lane / 16, cg = lane mod 16) loads 16 bytes, columns
        // 4 cg .. 4 cg + 3, of every fourth of them
        const uint32_t c = wave - SP_WAVES, rs = lane >> 4, cg = lane & 15, col = 4 * cg;
        const bool col_ok = col < dim;
#pragma unroll 1
        for (uint32_t m = 0; m < steps; m++) {
            const uint32_t slot = m % SP_RING;
            // issue the step's first round of loads before waiting for its shares
            uint4 tv[SP_U];
            auto load_round = [&](uint32_t r0) {
#pragma unroll
                for (uint32_t u = 0; u < SP_U; u++) {
                    const uint32_t k = c * SP_ROWS_PER_WAVE + r0 + 4 * u + rs;
                    const uint64_t row = row_base + ((uint64_t)(k >> 1) << h) + 2 * m + (k & 1);
                    const uint32_t *trow = table + (row < rows ? row : rows - 1) * dim;
                    tv[u] = col_ok ? row_load4<STREAM>(trow + col) : make_uint4(0, 0, 0, 0);
                }
            };
            load_round(0);
            if (!wait_count(&ready[slot], SP_WAVES * (m / SP_RING + 1), wait_limit)) {
                stalled = 1;
                break;
            }
            const uint32_t *sh = ring + slot * SP_STEP_WORDS + c * SP_ROWS_PER_WAVE + rs;
#pragma unroll 1 // one round of loads in flight: unrolled, the rounds' loads all hoist and spill
            for (uint32_t r0 = 0; r0 < SP_ROWS_PER_WAVE; r0 += 4 * SP_U) {
                if (r0)
                    load_round(r0);
#pragma unroll
                for (uint32_t u = 0; u < SP_U; u++) {
                    const uint32_t y = sh[r0 + 4 * u]; // zero for rows past the table
                    accw[0] += y * tv[u].x;
                    accw[1] += y * tv[u].y;
                    accw[2] += y * tv[u].z;
                    accw[3] += y * tv[u].w;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0)
                __hip_atomic_fetch_add(&freed[slot], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }

    // the consumers' sums per column, reduced in LDS (the tables are no longer needed)
    __syncthreads();
    uint32_t *s_acc = sm.tab;
    for (uint32_t i = tid; i < dim; i += NT)
        s_acc[i] = 0;
    __syncthreads();
    if (wave >= SP_WAVES) {
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const uint32_t cc = 4 * (lane & 15) + e;
            if (cc < dim)
                atomicAdd(&s_acc[cc], accw[e]);
        }
    }
    __syncthreads();
    if (tid == 0 && stalled)
        atomicOr(status, PIR_STATUS_STALLED);
    for (uint32_t i = tid; i < dim; i += NT) {
        uint32_t v = s_acc[i];
        if (ok == 2)
            v = 0u - v; // party 1 holds the negated share
        atomicAdd(&out[i], v);
    }
}

// ---------------------------------------------------------------------------
// Batched kernel: every wave is an independent work item, and the share x
// table product runs on the int8 matrix cores.
//
// A wave item is (16 keys, chunk of 4 * 2^h rows).  Lane l evaluates key
// (l mod 16) over subtree (l / 16) of the chunk: it walks from the key's root
// to the subtree root itself (n - h nodes, so no lane waits for another), then
// depth-first over the subtree with the path in registers.  Each walk step
// gives a lane the shares of two consecutive rows, so the 64 lanes together
// hold an [16 keys x 8 rows] share tile, exactly the A operand layout of
// v_mfma_i32_16x16x32_i8 (lane l: row l mod 16, K slice (l / 16) * 8 .. +7),
// and mfma_step() multiplies it into the table rows: KT output tiles of 16
// columns, for rows of up to 16 KT words (KT <= 4, two workgroups per CU at
// 4 waves per SIMD).  Rows of 65-128 words run as wave pairs
// (k_pir_waves_pairs below), each wave with four tiles.
// ---------------------------------------------------------------------------
// Adds a wave's answer tiles into out: tile t of lane l holds
// D[(l / 16) 4 + i][l mod 16], the total of key key0 + (l / 16) 4 + i at column
// col0 + col_of<KT, PACKED>(l mod 16, t); ok is the lane's key status (0 =
// skip, 1 or 2 = party 0 or 1, which negates).  Packed columns (lane n holds
// columns n KT .. n KT + KT - 1) are first regrouped across the 16 lanes of a
// key row, so that each atomic instruction adds 16 consecutive columns of four
// keys: 64 bytes a key instead of words 4 KT bytes apart, a quarter of the
// memory footprint at KT = 4.
template <int KT, bool PACKED>
__device__ __forceinline__ void add_tiles(const v4i (&tot)[KT], uint32_t ok, uint32_t lane, uint32_t ncols,
                                          uint32_t *__restrict__ out, size_t out_step, uint32_t key0, uint32_t col0)
{
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const uint32_t key = (lane >> 4) * 4 + i;
        const uint32_t kok = __shfl(ok, (int)key);
#pragma unroll
        for (int t = 0; t < KT; t++) {
            uint32_t col, v;
            if constexpr (PACKED && KT > 1) {
                // column 16 t + n of the row is tile (16 t + n) mod KT of lane (16 t + n) / KT
                col = 16 * (uint32_t)t + (lane & 15);
                const uint32_t src = (lane & 48) | (col / KT), ts = col % KT;
                v = 0;
#pragma unroll
                for (int u = 0; u < KT; u++) {
                    const uint32_t x = (uint32_t)__shfl(tot[u][i], (int)src); // every lane takes part
                    v = (uint32_t)u == ts ? x : v;
                }
            } else {
                col = col_of<KT, PACKED>(lane & 15, t);
                v = (uint32_t)tot[t][i];
            }
            if (kok && col < ncols)
                atomicAdd(&out[(size_t)(key0 + key) * out_step + col0 + col], kok == 2 ? 0u - v : v);
        }
    }
}

constexpr int NW3 = 8;             // waves per workgroup
constexpr int HMAX3 = 9;           // largest per-lane subtree height of the wave kernel
constexpr int NT3 = 64 * NW3;

// One table's share of a wave-kernel launch.  The table is cut into n_bins
// bins of 2^n rows (the last may be shorter; one bin for a whole-table query)
// and every client sends one key per bin: key (c, b) at keys + (c n_bins + b)
// * stride, answer at out + (c n_bins + b) * dim.
struct WaveTask {
    const uint32_t *table; // row-major uint32 [rows][dim]
    const uint8_t *keys;   // this table's first key
    uint32_t *out;         // this table's first answer word
    uint64_t rows;
    uint64_t row0;                   // index of table row 0 in the key domain (a slice; else 0)
    uint32_t dim, n_keys, n, h, n_groups, item_begin;
    uint32_t n_bins, chunks_per_bin; // n_keys counts clients
};
constexpr int MAX_TASKS = 16;
struct WaveTasks {
    WaveTask t[MAX_TASKS];
    uint32_t count, n_items;
    uint32_t *status; // the call's status word
};

template <class PRF, int KT, bool VEC>
__global__ __launch_bounds__(NT3) __attribute__((amdgpu_waves_per_eu(4))) void k_pir_waves(const WaveTasks tasks,
                                                                                           uint32_t stride)
{
    static_assert(KT <= 4, "rows of 65-128 words run as wave pairs");
    __shared__ uint32_t tab[PRF::TAB_WORDS ? PRF::TAB_WORDS : 1];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const PRF P(tab, lane);
    if (PRF::TAB_WORDS) {
        PRF::fill(tab, tid, NT3);
        __syncthreads();
    }

    const uint32_t item0 = __builtin_amdgcn_readfirstlane(xcd_block() * NW3 + wave); // uniform over the wave
    if (item0 >= tasks.n_items)
        return; // whole wave; no barrier follows
    uint32_t ti = 0; // the table this item belongs to (tasks are in item order)
    while (ti + 1 < tasks.count && item0 >= tasks.t[ti + 1].item_begin)
        ti++;
    const WaveTask &g = tasks.t[ti];
    const uint32_t item = item0 - g.item_begin;
    const uint32_t dim = g.dim, n_keys = g.n_keys;
    const uint32_t grp = item % g.n_groups, bin_chunk = item / g.n_groups;
    const uint32_t bin = bin_chunk / g.chunks_per_bin, chunk = bin_chunk % g.chunks_per_bin;
    // this bin's rows, keys (one per client, n_bins apart) and answers
    const uint64_t first_row = (uint64_t)bin << g.n;
    const uint64_t rows_left = g.rows - first_row;
    const uint64_t rows = rows_left < ((uint64_t)1 << g.n) ? rows_left : ((uint64_t)1 << g.n);
    const uint32_t *__restrict__ table = g.table + first_row * dim;
    const uint8_t *__restrict__ keys = g.keys + (size_t)bin * stride;
    uint32_t *__restrict__ out = g.out + (size_t)bin * dim;
    const size_t key_step = (size_t)g.n_bins * stride, out_step = (size_t)g.n_bins * dim;
    const uint32_t q = lane & 15, sub = lane >> 4;
    const uint32_t kq = grp * 16 + q;
    const uint32_t h = g.h;
    if (h == 0 || h > g.n || h > HMAX3)
        return; // the planner keeps 1 <= h <= min(n, HMAX3); no barrier follows

    uint32_t ok = 0;
    const KeyView K{keys + (size_t)(kq < n_keys ? kq : 0) * key_step};
    const CwGlobal C = cw_global(K);
    if (kq < n_keys) {
        const uint32_t hdr = *reinterpret_cast<const uint32_t *>(K.p);
        const uint32_t ver = hdr & 0xff, party = (hdr >> 8) & 0xff, kn = (hdr >> 16) & 0xff, prf = hdr >> 24;
        ok = (ver == PIR_KEY_VERSION && party <= 1 && kn == g.n && prf == PRF::id) ? 1u + party : 0u;
        if (!ok && sub == 0)
            atomicOr(tasks.status, PIR_STATUS_BAD_KEY);
    }
    const uint64_t lane_row0 = ((uint64_t)chunk * 4 + sub) << h;
    const bool active = ok && lane_row0 < rows;

    // walk from the root to this lane's subtree root (depth n - h)
    Seed node{{0, 0, 0, 0}};
    if (active) {
        node = K.root();
        for (uint32_t d = 1; d + h <= g.n; d++)
            node = child_on_path(P, C, node, d, (uint32_t)((g.row0 + lane_row0) >> (g.n - d)) & 1u);
    }
    const uint32_t d0 = g.n - h;
    Seed right[HMAX3];
#pragma unroll
    for (int i = 0; i < HMAX3; i++)
        right[i] = Seed{{0, 0, 0, 0}};

    // running sum over steps of sum_s 256^s D_s, per tile (wraps mod 2^32)
    v4i tot[KT];
#pragma unroll
    for (int t = 0; t < KT; t++)
        tot[t] = v4i{0, 0, 0, 0};

    // this lane's table columns: tile t, column n = lane mod 16 -> col_of(n, t)
    const uint32_t ncol = lane & 15;
    const uint32_t steps = 1u << (h - 1);
    // The item's rows: a chunk of at most 4 2^h <= 2048 rows from chunk_row0,
    // read through 32-bit word offsets from the chunk's first row; a row past
    // the table reads the chunk's last row instead (its share is zero).
    const uint64_t chunk_row0 = ((uint64_t)chunk * 4) << h;
    const uint32_t *__restrict__ ctab = table + chunk_row0 * dim;
    const uint64_t chunk_rows = rows - chunk_row0 < ((uint64_t)4 << h) ? rows - chunk_row0 : ((uint64_t)4 << h);
    const uint32_t last_off = (uint32_t)(chunk_rows - 1) * dim;
    uint32_t row_off = (sub << h) * dim; // this lane's row 2m
    for (uint32_t m = 0; m < steps; m++, row_off += 2 * dim) {
        // table words of the two rows this lane feeds to the product; issued
        // first and unconditionally (clamped rows), so their latency hides
        // behind this step's AES work
        const uint64_t r0 = lane_row0 + 2 * m;
        uint32_t t0[KT], t1[KT];
        load_cols<KT, VEC>(ctab + (row_off < last_off ? row_off : last_off), dim, ncol, t0);
        load_cols<KT, VEC>(ctab + (row_off + dim < last_off ? row_off + dim : last_off), dim, ncol, t1);

        uint32_t kst = 1; // step 0 starts at the lane's root, already in `node`
        if (m != 0) {
            // uniform over the wave: scalar compares select the path entry
            const uint32_t kf = __builtin_amdgcn_readfirstlane(h - 1 - __builtin_ctz(m));
#pragma unroll
            for (int i = 1; i < HMAX3; i++)
                if ((uint32_t)i == kf)
                    node = right[i];
            kst = kf + 1;
        }
        uint32_t y0 = 0, y1 = 0;
        if (active) {
            for (uint32_t k = __builtin_amdgcn_readfirstlane(kst); k < h; k++) {
                Seed c0, c1;
                children(P, C, node, d0 + k, c0, c1);
#pragma unroll
                for (int i = 1; i < HMAX3; i++)
                    if ((uint32_t)i == k)
                        right[i] = c1;
                node = c0;
            }
            const uint2 cw = C.cw_word0(g.n, node.w[0] & 1u);
            P.pair_word0(node.w, y0, y1);
            y0 = r0 < rows ? y0 ^ cw.x : 0u; // rows past the table add nothing
            y1 = r0 + 1 < rows ? y1 ^ cw.y : 0u;
        }

        mfma_step<KT>(y0, y1, t0, t1, tot);
    }

    add_tiles<KT, VEC>(tot, ok, lane, dim, out, out_step, grp * 16, 0);
}


// ---------------------------------------------------------------------------
// Rows of 65-128 words: wave pairs.  Eight column tiles in one wave need more
// than 128 VGPRs, so the two waves of a pair share the work instead: both take
// the same 16 keys, wave j of the pair walks chunk 2 c + j of the bin (its own
// subtrees, as in k_pir_waves), and each step the two trade their leaf shares
// through LDS; wave j then multiplies both chunks' shares into column half j
// (columns 64 j .. 64 j + 63), four tiles of 16 columns: its own shares of
// the step, and its partner's of the step before, so that a wave can run a
// step ahead of its partner before it waits.  Per wave that is the register
// and table-row footprint of a 64-word row (4 waves per SIMD), at the cost of
// two LDS accesses and two bounded waits per step.  Items come in pairs
// (2 p, 2 p + 1): pair p is (key group, pair of chunks); a pair whose second
// chunk is past the bin gives that wave no rows (zero shares).
// ---------------------------------------------------------------------------
constexpr uint32_t PAIR_RING = 3; // steps of shares in a wave's LDS slots (two workgroups per CU)

template <uint32_t TABW>
struct PairSmem {
    uint32_t tab[TABW];                  // first: at LDS address 0
    uint2 ring[NW3][PAIR_RING][64];       // (y0, y1) of each lane, per wave and slot
    uint32_t wdone[NW3], rdone[NW3];      // steps written by a wave / of its partner's read by it
};

template <class PRF, bool VEC>
__global__ __launch_bounds__(NT3) __attribute__((amdgpu_waves_per_eu(4))) void k_pir_waves_pairs(const WaveTasks tasks,
                                                                                          uint32_t stride,
                                                                                          uint32_t wait_limit)
{
    __shared__ PairSmem<PRF::TAB_WORDS ? PRF::TAB_WORDS : 1> sm;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const PRF P(sm.tab, lane);
    if (PRF::TAB_WORDS)
        PRF::fill(sm.tab, tid, NT3);
    if (lane == 0) {
        sm.wdone[wave] = 0;
        sm.rdone[wave] = 0;
    }
    __syncthreads();

    // pairs are whole: every task's item count is even and starts even
    const uint32_t item0 = __builtin_amdgcn_readfirstlane(xcd_block() * NW3 + wave);
    if (item0 >= tasks.n_items)
        return; // the partner (item0 ^ 1) returns too; no barrier follows
    uint32_t ti = 0;
    while (ti + 1 < tasks.count && item0 >= tasks.t[ti + 1].item_begin)
        ti++;
    const WaveTask &g = tasks.t[ti];
    const uint32_t item = item0 - g.item_begin;
    const uint32_t j = item & 1, pw = wave ^ 1; // this wave's half; its partner
    const uint32_t pair = item >> 1;
    const uint32_t dim = g.dim, n_keys = g.n_keys;
    const uint32_t pchunks = (g.chunks_per_bin + 1) / 2;
    const uint32_t grp = pair % g.n_groups, bin_pchunk = pair / g.n_groups;
    const uint32_t bin = bin_pchunk / pchunks, pchunk = bin_pchunk % pchunks;
    const uint64_t first_row = (uint64_t)bin << g.n;
    const uint64_t rows_left = g.rows - first_row;
    const uint64_t rows = rows_left < ((uint64_t)1 << g.n) ? rows_left : ((uint64_t)1 << g.n);
    const uint32_t *__restrict__ table = g.table + first_row * dim;
    const uint8_t *__restrict__ keys = g.keys + (size_t)bin * stride;
    uint32_t *__restrict__ out = g.out + (size_t)bin * dim;
    const size_t key_step = (size_t)g.n_bins * stride, out_step = (size_t)g.n_bins * dim;
    const uint32_t q = lane & 15, sub = lane >> 4, ncol = lane & 15;
    const uint32_t kq = grp * 16 + q;
    const uint32_t h = g.h;
    if (h == 0 || h > g.n || h > HMAX3)
        return; // the same for both waves of the pair; no barrier follows

    uint32_t ok = 0;
    const KeyView K{keys + (size_t)(kq < n_keys ? kq : 0) * key_step};
    const CwGlobal C = cw_global(K);
    if (kq < n_keys) {
        const uint32_t hdr = *reinterpret_cast<const uint32_t *>(K.p);
        const uint32_t ver = hdr & 0xff, party = (hdr >> 8) & 0xff, kn = (hdr >> 16) & 0xff, prf = hdr >> 24;
        ok = (ver == PIR_KEY_VERSION && party <= 1 && kn == g.n && prf == PRF::id) ? 1u + party : 0u;
        if (!ok && sub == 0 && j == 0)
            atomicOr(tasks.status, PIR_STATUS_BAD_KEY);
    }
    // the two chunks of the pair; a chunk past the bin reads chunk 2 pchunk's rows
    // (with zero shares)
    const uint32_t c_own = 2 * pchunk + j, c_par = 2 * pchunk + (1 - j);
    const bool own_ok = c_own < g.chunks_per_bin, par_ok = c_par < g.chunks_per_bin;
    auto chunk_base = [&](uint32_t c, bool valid, uint32_t &last_off) {
        const uint64_t r0 = ((uint64_t)(valid ? c : 2 * pchunk) * 4) << h;
        const uint64_t n_r = rows - r0 < ((uint64_t)4 << h) ? rows - r0 : ((uint64_t)4 << h);
        last_off = (uint32_t)(n_r - 1) * dim;
        return table + r0 * dim + 64 * j; // column half j
    };
    uint32_t last_own, last_par;
    const uint32_t *__restrict__ ctab_own = chunk_base(c_own, own_ok, last_own);
    const uint32_t *__restrict__ ctab_par = chunk_base(c_par, par_ok, last_par);
    const uint32_t hdim = dim - 64 * j < 64 ? dim - 64 * j : 64; // columns in this half (>= 1)
    // VEC (dim a multiple of 4): lane n reads columns 4 n .. 4 n + 3 of the
    // half with one 16-byte load; a lane past the half's end reads the last
    // four columns instead, which only feed output columns that are never
    // written (column n of a tile takes only table column n)
    const uint32_t nld = VEC ? (ncol < hdim / 4 ? ncol : hdim / 4 - 1) : ncol;

    const uint64_t lane_row0 = ((uint64_t)c_own * 4 + sub) << h;
    const bool active = ok && own_ok && lane_row0 < rows;

    Seed node{{0, 0, 0, 0}};
    if (active) {
        node = K.root();
        for (uint32_t d = 1; d + h <= g.n; d++)
            node = child_on_path(P, C, node, d, (uint32_t)((g.row0 + lane_row0) >> (g.n - d)) & 1u);
    }
    const uint32_t d0 = g.n - h;
    Seed right[HMAX3];
#pragma unroll
    for (int i = 0; i < HMAX3; i++)
        right[i] = Seed{{0, 0, 0, 0}};

    v4i tot[4];
#pragma unroll
    for (int t = 0; t < 4; t++)
        tot[t] = v4i{0, 0, 0, 0};
    const uint32_t steps = 1u << (h - 1);
    bool stalled = false;
    // The partner's shares of step m - 1 are multiplied in at step m (and its
    // last step's after the loop), so that a wave waits only when its partner
    // is more than a step behind.
    auto partner_step = [&](uint32_t m, uint32_t off) { // the partner's step m, rows at off
        uint32_t u0[4], u1[4];
        load_cols<4, VEC>(ctab_par + (off < last_par ? off : last_par), hdim, nld, u0);
        load_cols<4, VEC>(ctab_par + (off + dim < last_par ? off + dim : last_par), hdim, nld, u1);
        if (!wait_count(&sm.wdone[pw], m + 1, wait_limit))
            return false;
        const uint2 z = sm.ring[pw][m % PAIR_RING][lane];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup"); // the read is done before it is reported
        if (lane == 0)
            __hip_atomic_store(&sm.rdone[wave], m + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        mfma_step<4>(z.x, z.y, u0, u1, tot);
        return true;
    };
    uint32_t row_off = (sub << h) * dim; // this lane's row 2m in either chunk
    for (uint32_t m = 0; m < steps; m++, row_off += 2 * dim) {
        const uint64_t r0 = lane_row0 + 2 * m;
        uint32_t t0[4], t1[4];
        load_cols<4, VEC>(ctab_own + (row_off < last_own ? row_off : last_own), hdim, nld, t0);
        load_cols<4, VEC>(ctab_own + (row_off + dim < last_own ? row_off + dim : last_own), hdim, nld, t1);

        uint32_t kst = 1;
        if (m != 0) {
            const uint32_t kf = __builtin_amdgcn_readfirstlane(h - 1 - __builtin_ctz(m));
#pragma unroll
            for (int i = 1; i < HMAX3; i++)
                if ((uint32_t)i == kf)
                    node = right[i];
            kst = kf + 1;
        }
        uint32_t y0 = 0, y1 = 0;
        if (active) {
            for (uint32_t k = __builtin_amdgcn_readfirstlane(kst); k < h; k++) {
                Seed c0, c1;
                children(P, C, node, d0 + k, c0, c1);
#pragma unroll
                for (int i = 1; i < HMAX3; i++)
                    if ((uint32_t)i == k)
                        right[i] = c1;
                node = c0;
            }
            const uint2 cw = C.cw_word0(g.n, node.w[0] & 1u);
            P.pair_word0(node.w, y0, y1);
            y0 = r0 < rows ? y0 ^ cw.x : 0u;
            y1 = r0 + 1 < rows ? y1 ^ cw.y : 0u;
        }

        // hand this step's shares to the partner: slot m mod PAIR_RING is free
        // once the partner has read step m - PAIR_RING from it
        if (m >= PAIR_RING && !wait_count(&sm.rdone[pw], m - PAIR_RING + 1, wait_limit)) {
            stalled = true;
            break;
        }
        sm.ring[wave][m % PAIR_RING][lane] = make_uint2(y0, y1);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0)
            __hip_atomic_store(&sm.wdone[wave], m + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);

        mfma_step<4>(y0, y1, t0, t1, tot); // own rows, column half j
        if (m != 0 && !partner_step(m - 1, row_off - 2 * dim)) {
            stalled = true;
            break;
        }
    }
    if (!stalled && !partner_step(steps - 1, row_off - 2 * dim))
        stalled = true;
    if (stalled && lane == 0)
        atomicOr(tasks.status, PIR_STATUS_STALLED);

    add_tiles<4, VEC>(tot, ok, lane, hdim, out, out_step, grp * 16, 64 * j); // column half j
}

} // namespace
