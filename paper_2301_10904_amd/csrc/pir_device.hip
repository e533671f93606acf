// pir_device.hip -- host side of the fused DPF evaluation x table product:
// argument validation, the work plan of each call (which kernel, subtree
// height, work items, grid), the launches on the caller's stream and the C ABI
// entry points of include/pir.h.  The kernels are in pir_kernels.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <memory>
#include <mutex>
#include <vector>

#include "pir.h"
#include "pir_internal.h"
#include "pir_kernels.h"

namespace {

static uint32_t ceil_log2(uint64_t x)
{
    uint32_t r = 0;
    while (((uint64_t)1 << r) < x)
        r++;
    return r;
}

// Rows are read with 16-byte (or 8-byte) vector loads only from a table whose
// base is 16-byte aligned; a table at any other 4-byte boundary takes the
// instantiations that read single words.
static bool vec_aligned(const uint32_t *d_table) { return (uintptr_t)d_table % 16 == 0; }

// tries of a kernel's bounded wait (pir_set_wait_limit)
static std::atomic<uint32_t> g_wait_limit{PIR_WAIT_LIMIT_DEFAULT};

template <class PRF, int Q>
static void launch_q(uint32_t kch, dim3 grid, hipStream_t st, const uint8_t *keys, uint32_t n_keys,
                     uint32_t stride, const uint32_t *table, uint64_t rows, uint32_t dim, uint32_t *out,
                     const Geometry &g, uint32_t *status)
{
#define PIR_LAUNCH_FUSED(KCH, V4, S)                                                                              \
    hipLaunchKernelGGL((k_pir_fused<PRF, Q, KCH, V4, S>), grid, dim3(NT), 0, st, keys, n_keys, stride, table, rows,  \
                       dim, out, g, status)
    const bool v4 = dim % 4 == 0 && vec_aligned(table);
    if constexpr (Q == 1) {
        // one key streams the table once per call: past the size of the
        // memory-side cache (256 MiB) its rows are read without allocating in
        // the caches (measured with AES-128: 2^22 x 64 0.235 -> 0.215 ms, 2^25
        // x 64 1.48 -> 1.44 ms; at 2^20 x 64, 256 MiB, cached reads are faster)
        const bool big = rows * dim * 4ull > (256ull << 20);
        if constexpr (PRF::TAB_WORDS != 0) {
            if (v4 && kch == 1 && n_keys == 1 && g.H > SP_LGS && g.H <= SP_LGS + HMAX) {
                // one key, rows of up to 64 words, AES-128: tree waves and
                // table-stream waves (k_pir_stream; measured, 1 key: 2^25 x
                // 64 1.476 -> 1.404 ms, 2^22 x 64 0.224 -> 0.206, 2^24 x 32
                // 0.625 -> 0.587, 2^23 x 16 0.309 -> 0.281; with cached row
                // reads up to 256 MiB: 2^20 x 64 0.080 -> 0.074, 2^19 x 64
                // 0.060 -> 0.055, 2^14 x 16 0.036 -> 0.035).  ChaCha20 keeps
                // k_pir_fused, where the split gained at most 3% and lost at
                // some sizes (2^25 x 64 1.541 against 1.568 ms, 2^20 x 64
                // 0.068 against 0.066)
                if (big)
                    hipLaunchKernelGGL((k_pir_stream<PRF, true>), grid, dim3(NT), 0, st, keys, table, rows, dim, out,
                                       g, status, g_wait_limit.load(std::memory_order_relaxed));
                else
                    hipLaunchKernelGGL((k_pir_stream<PRF, false>), grid, dim3(NT), 0, st, keys, table, rows, dim, out,
                                       g, status, g_wait_limit.load(std::memory_order_relaxed));
                return;
            }
        }
        if (v4 && big) {
            if (kch == 1)
                PIR_LAUNCH_FUSED(1, true, true);
            else if (kch == 2)
                PIR_LAUNCH_FUSED(2, true, true);
            else
                PIR_LAUNCH_FUSED(4, true, true);
            return;
        }
    }
    if (kch == 1) {
        if (v4)
            PIR_LAUNCH_FUSED(1, true, false);
        else
            PIR_LAUNCH_FUSED(1, false, false);
    } else if (kch == 2) {
        if (v4)
            PIR_LAUNCH_FUSED(2, true, false);
        else
            PIR_LAUNCH_FUSED(2, false, false);
    } else {
        if (v4)
            PIR_LAUNCH_FUSED(4, true, false);
        else
            PIR_LAUNCH_FUSED(4, false, false);
    }
#undef PIR_LAUNCH_FUSED
}

static int fail_hip(hipError_t e)
{
    pir_impl::set_hip_error((int)e);
    return PIR_EHIP;
}

// The library's own status workspace, one per device: used by calls from a
// thread that has bound no workspace of its own (pir_set_workspace).  Host
// code never names the array itself: its device address comes from
// hipGetSymbolAddress, once per device with that device current.
static __device__ __align__(256) uint32_t scratch[PIR_WORKSPACE_BYTES / 4];
constexpr int MAX_DEVICES = 64;
static std::atomic<uint32_t *> g_scratch_ptr[MAX_DEVICES];
static std::mutex g_scratch_mu;

static uint32_t *default_workspace()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        pir_impl::set_hip_error((int)(e != hipSuccess ? e : hipErrorInvalidDevice));
        return nullptr;
    }
    if (uint32_t *p = g_scratch_ptr[dev].load(std::memory_order_acquire))
        return p;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (uint32_t *p = g_scratch_ptr[dev].load(std::memory_order_relaxed))
        return p;
    uint32_t *p = nullptr;
    e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        pir_impl::set_hip_error((int)(e != hipSuccess ? e : hipErrorInvalidSymbol));
        return nullptr;
    }
    g_scratch_ptr[dev].store(p, std::memory_order_release);
    return p;
}

// The workspace bound by this thread (pir_set_workspace), or null.
static thread_local uint32_t *t_workspace = nullptr;

// Per-call state: the status word the call's kernels report into, located on
// first use (so that argument errors are found without touching the GPU), and
// cleared by the call's first launch.
struct CallCtx {
    uint32_t *status = nullptr;
    bool cleared = false;
    // The status word, or null if the default workspace cannot be located.
    // Called before the call's first launch: it also drops an error code left
    // in this thread by an earlier runtime call of the caller (an event or
    // stream query that returned "not ready", say), so that the launch checks
    // that follow see only the call's own launches.
    uint32_t *word()
    {
        if (!status) {
            (void)hipGetLastError();
            status = t_workspace ? t_workspace : default_workspace();
        }
        return status;
    }
    // For the first k_fill_zero of the call: the word to clear, then null.
    uint32_t *clear_once()
    {
        if (cleared)
            return nullptr;
        cleared = true;
        return status;
    }
};

constexpr uint64_t WAVE_SLOTS = 256 * 16; // waves resident at once: 256 CUs x two 8-wave workgroups

// Subtree height of a single-table wave launch.  A lane's work per item is its
// descent (n - h single-block nodes, a dependent chain that runs at about half
// the rate of the walk, so weighted 2) plus the 2^h - 1 nodes of its subtree;
// the launch takes about max(items, slots) / slots rounds of that, and a
// launch of at most one round pays about 10% for its unfilled tail.  Small
// batches have few key groups, so a lower h gives more items but a relatively
// longer descent; the model picks the balance (measured: 16 keys on 2^20 rows
// 0.84 -> 0.61 ms against a fixed minimum of 8192 items).
static uint32_t wave_height(uint64_t n_bins, uint64_t bin_rows, uint64_t groups, uint32_t n, uint32_t hmax)
{
    uint32_t best_h = hmax;
    double best = 0.0;
    for (uint32_t h = hmax; h >= 3 && h <= hmax; h--) {
        const uint64_t chunks = (bin_rows + ((uint64_t)4 << h) - 1) / ((uint64_t)4 << h);
        const uint64_t items = n_bins * chunks * groups;
        const double per_lane = 2.0 * (double)(n - h) + (double)((1u << h) - 1);
        const double t = per_lane * (double)std::max<uint64_t>(items, WAVE_SLOTS) / (double)WAVE_SLOTS *
                         (items <= WAVE_SLOTS ? 1.1 : 1.0);
        if (h == hmax || t < best) {
            best = t;
            best_h = h;
        }
    }
    return best_h;
}

// Largest subtree height of a wave item whose rows lie in an aligned subtree
// of height m (1 <= m <= n): at most what the path registers allow (HMAX3),
// and m - 2 where m >= 3, so that the item's four subtrees fill it; below that
// (a bin or slice of at most 4 rows) subtrees of height 1, whose unused lanes
// are inactive.  Always 1 <= h <= m <= n, which the kernel relies on.
static uint32_t wave_hmax(uint32_t m) { return m >= 3 ? std::min<uint32_t>(HMAX3, m - 2) : 1u; }

// Work plan of a wave-kernel launch over `count` tasks: fills h, n_groups,
// chunks_per_bin and item_begin of every task and returns the number of wave
// items (0 if it reaches 2^31).  The subtree height h is at most
// wave_hmax(m) for the aligned subtree of height m holding a bin (or a table
// slice); a single table gets the height of wave_height(), a launch of several
// tables the largest (the tables together fill the GPU).
static uint64_t plan_waves(WaveTask *ts, uint32_t count, uint32_t h_want = 0, bool pairs = false)
{
    uint64_t items = 0;
    for (uint32_t i = 0; i < count; i++) {
        WaveTask &t = ts[i];
        t.n_groups = (t.n_keys + 15) / 16;
        const uint64_t bin_rows = std::min<uint64_t>(t.rows, (uint64_t)1 << t.n);
        auto chunks_per_bin = [&](uint32_t hh) { return (bin_rows + ((uint64_t)4 << hh) - 1) / ((uint64_t)4 << hh); };
        // a slice of a table lies in an aligned subtree of height m < n, and a
        // lane's subtree must lie in it too; whole tables and bins have m = n
        const uint32_t m = std::min<uint32_t>(t.n, bin_rows <= 2 ? 1 : ceil_log2(bin_rows));
        const uint32_t hmax = wave_hmax(m);
        // a single table: the tuned height (clamped to what the rows allow) or the model's
        const uint32_t h = count != 1 ? hmax
                           : h_want   ? std::min(h_want, hmax)
                                      : wave_height(t.n_bins, bin_rows, t.n_groups, t.n, hmax);
        t.h = h;
        t.chunks_per_bin = (uint32_t)chunks_per_bin(h);
        t.item_begin = (uint32_t)items;
        // wave pairs (rows of 65-128 words) take a bin's chunks two at a time
        const uint64_t per_bin = pairs ? 2 * (((uint64_t)t.chunks_per_bin + 1) / 2) : t.chunks_per_bin;
        items += (uint64_t)t.n_bins * per_bin * t.n_groups;
        if (items >= ((uint64_t)1 << 31))
            return 0;
    }
    return items;
}

// Column class of the wave kernel, which picks its instantiation (KT, VEC):
// tables in one launch must share it.  The vector-load classes 0..2 need a
// 16-byte aligned table; others of those widths read single words.  Rows of
// 65-128 words run as wave pairs (k_pir_waves_pairs), with 16-byte loads
// (class 7) when the width is a multiple of 4 and the table is aligned.
static int wave_class(uint32_t dim, bool aligned)
{
    if (dim == 64 && aligned) return 0;
    if (dim == 32 && aligned) return 1;
    if (dim == 16 && aligned) return 2;
    if (dim <= 16) return 3;
    if (dim <= 32) return 4;
    if (dim <= 64) return 5;
    if (dim > 64 && dim <= 128 && dim % 4 == 0 && aligned) return 7;
    if (dim <= 128) return 6;
    return -1;
}
constexpr int WAVE_CLASSES = 8;
static bool wave_pairs(uint32_t dim) { return dim > 64; }
// Static LDS of a wave-kernel workgroup for rows of dim words.
static uint32_t wave_lds_bytes(bool aes, uint32_t dim)
{
    if (wave_pairs(dim))
        return aes ? (uint32_t)sizeof(PairSmem<AesPrf::TAB_WORDS>) : (uint32_t)sizeof(PairSmem<1>);
    return aes ? AES_TAB_WORDS * 4 : 0;
}

// Wave-kernel launch for up to MAX_TASKS tables of column class cls.  Plans
// the tasks and clears their outputs first.
template <class PRF>
static int launch_waves(WaveTask *ts, uint32_t count, uint32_t key_stride, int cls, CallCtx &ctx, hipStream_t st,
                        uint32_t h_want = 0)
{
    WaveTasks W;
    bool any = false;
    for (uint32_t i = 0; i < count; i++)
        any |= ts[i].n_keys > 0;
    const uint64_t items = plan_waves(ts, count, h_want, cls >= 6);
    if (items == 0 && any)
        return PIR_ENOMEM;
    if (!ctx.word())
        return PIR_EHIP;
    for (uint32_t i = 0; i < count; i++)
        W.t[i] = ts[i];
    W.count = count;
    W.n_items = (uint32_t)items;
    W.status = ctx.status;
    for (uint32_t i = 0; i < count; i++) {
        const size_t words = (size_t)ts[i].n_keys * ts[i].n_bins * ts[i].dim;
        const uint32_t blocks = (uint32_t)std::max<size_t>(1, std::min<size_t>((words + 255) / 256, 4096));
        hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, st, ts[i].out, words, ctx.clear_once());
    }
    if (items == 0)
        return PIR_OK;
    const dim3 grid((uint32_t)((items + NW3 - 1) / NW3));
#define PIR_LAUNCH_WAVES(KT, VEC) hipLaunchKernelGGL((k_pir_waves<PRF, KT, VEC>), grid, dim3(NT3), 0, st, W, key_stride)
#define PIR_LAUNCH_PAIRS(VEC)                                                                                      \
    hipLaunchKernelGGL((k_pir_waves_pairs<PRF, VEC>), grid, dim3(NT3), 0, st, W, key_stride,                        \
                       g_wait_limit.load(std::memory_order_relaxed))
    switch (cls) {
    case 0: PIR_LAUNCH_WAVES(4, true); break;
    case 1: PIR_LAUNCH_WAVES(2, true); break;
    case 2: PIR_LAUNCH_WAVES(1, true); break;
    case 3: PIR_LAUNCH_WAVES(1, false); break;
    case 4: PIR_LAUNCH_WAVES(2, false); break;
    case 5: PIR_LAUNCH_WAVES(4, false); break;
    case 6: PIR_LAUNCH_PAIRS(false); break;
    case 7: PIR_LAUNCH_PAIRS(true); break;
    default: return PIR_EINVAL;
    }
#undef PIR_LAUNCH_PAIRS
#undef PIR_LAUNCH_WAVES
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PIR_OK : fail_hip(e);
}

// Which kernel answers one table: the wave kernel (int8 matrix cores, up to 16
// keys per wave) from a batch size on that depends on the PRF, the domain and
// the row width, else the small-batch kernel, which also takes rows wider than
// 128 words.  Every lane of the wave kernel walks its own path from the root,
// while the small-batch kernel shares the path above its chunks; for small
// domains that repeated descent outweighs everything else.  Measured (p50 per
// call, rows of 64 words): 9..16 keys on 2^20 rows take 0.42 ms on the
// small-batch kernel against 0.59 on the wave kernel with AES-128, 0.46
// against 1.02 with ChaCha20.
// On domains up to 2^20 with rows of at most 64 words the small-batch kernel,
// whose workgroups share the path above their chunk, stays ahead until the
// batch is large enough for the wave kernel's matrix-core product to pay:
// from 32 2^(20-n) keys with AES-128 and 256 2^(20-n) with ChaCha20.
// Measured (1 table x 64 words, one build against the other): AES-128 on
// 2^14 rows 25 keys 0.042 against 0.101 ms, 1024 keys 0.411 against 0.432;
// on 2^18 rows 64 keys 0.417 against 0.428, 128 keys 0.809 against 0.776; on
// 2^20 rows 25 keys 0.806 against 0.817, 48 keys 1.196 against 1.127.
// ChaCha20 on 2^20 rows 128 keys 3.58 against 3.65 ms, 256 keys 7.15 against
// 7.09; on 2^14 rows 25 keys 0.033 against 0.112.  (Remainders of 1..8 keys
// past whole groups of 16 run as launches of their own, split_tail.)  Above
// 2^20 rows the wave kernel takes AES-128 batches from 9 keys and ChaCha20
// ones from 17: 9..16 keys on 2^22 rows take 1.56 against 1.60 ms with
// AES-128.  Rows of 65..128 words (two column chunks): the small-batch
// kernel holds at most 8 keys per workgroup (plan_fused), and the wave kernel
// takes batches from 17 keys on 2^17..2^20 rows, above 2^20 rows from 9
// (ChaCha20 on 2^22 rows: 9..16 keys 3.6 ms there against 2.2-2.4 ms on the
// wave kernel), and on smaller domains from 64 2^(16-n) keys with AES-128 and
// 128 2^(16-n) with ChaCha20 (2^14 x 128: 25 keys 0.048 against 0.068 ms
// with AES-128, 0.038 against 0.081 with ChaCha20; 512 keys 0.317 against
// 0.283 and 0.343 against 0.307; 2^18 x 128, 25 keys: 0.357 against 0.295).
static uint32_t wave_min_keys(uint32_t prf_id, uint32_t n, uint32_t dim)
{
    const bool chacha = prf_id == PIR_PRF_CHACHA20;
    if (dim > 64) {
        if (n > 16)
            return n > 20 ? 9u : 17u;
        const uint32_t shift = 16 - n; // at most 15
        return (chacha ? 128u : 64u) << shift;
    }
    if (n > 20)
        return chacha ? 17u : 9u;
    const uint32_t shift = 20 - n;
    const uint32_t base = chacha ? 256u : 32u; // 2^8 and 2^5
    return shift + (chacha ? 8u : 5u) >= 32 ? 0xffffffffu : base << shift;
}
static bool use_wave_kernel(uint32_t prf_id, uint32_t n_keys, uint32_t n, uint32_t dim)
{
    return n_keys >= wave_min_keys(prf_id, n, dim) && n >= 3 && dim <= 128;
}

// Keys of a batch that go to a launch of their own: a remainder of 1..8 keys
// past whole groups of 16 runs on the small-batch kernel, where in the wave
// kernel it would cost a whole group of items (and often a round of wave slots
// of its own).  Measured with AES-128 (ChaCha20 alike): 17 keys on 2^20 rows
// 0.81 -> 0.51 ms, 132 keys 4.42 -> 3.05 ms; 520 keys on 2^18 rows 4.46 ->
// 2.95 ms; 17 keys on 2^22 rows 2.81 -> 1.87 ms.  Not below 2^17 rows (launch
// bound).  On 2^17 and 2^18 rows a batch of at most 64 keys splits off only a
// remainder of up to 4 keys: 33 keys on 2^18 rows 0.324 -> 0.264 ms (AES-128),
// 49 keys 0.585 -> 0.387 ms (ChaCha20), but 56 keys 0.221 -> 0.245 ms and 24
// keys 0.123 -> 0.140 ms on 2^17 rows with a remainder of 8.  m is the log2
// of the rows' aligned subtree.
static uint32_t split_tail(uint32_t n_keys, uint32_t m)
{
    const uint32_t rem = n_keys % 16;
    if (n_keys <= 16 || rem == 0 || rem > 8 || m < 17)
        return 0;
    if (m < 19 && n_keys <= 64 && rem > 4)
        return 0;
    return rem;
}

// The same for one table of a multi-table call, whose tables share one wave
// launch: a remainder of 1..8 keys (of any batch) on a table of at least 2^20
// rows gets a small-batch launch of its own, while its partial group on a
// smaller table costs little in the shared launch.  Measured with AES-128 on
// tables of 2^18, 2^20, 2^22 and 2^24 rows x 32 words: key counts (5, 7, 3, 2)
// 8.21 -> 2.18 ms, (37, 53, 21, 19) 15.2 -> 11.7 ms, (33, 65, 129, 17) 23.9 ->
// 19.5 ms; counts without remainders unchanged.  In the serving loop over
// those tables the 1/L-weighted mix at 20k requests/s went from 30 to 2 ms
// p50 (38 to 5 ms p99).
static uint32_t multi_tail(uint32_t n_keys, uint32_t n)
{
    const uint32_t rem = n_keys % 16;
    return n >= 20 && rem >= 1 && rem <= 8 ? rem : 0;
}

// Work plan of the small-batch kernel: Q keys per workgroup, chunks of 2^H
// rows, breadth-first expansion to 2^lgS lanes per key, per-lane subtrees of
// height H - lgS.  H is chosen so that the grid is about one round of
// workgroup slots (two per CU), which spreads even a single key over every CU.
struct FusedPlan {
    Geometry g;
    uint32_t Q, kch;
    uint64_t grid;
};

// n is the keys' domain; the rows lie in an aligned subtree of height m <= n
// from index row0 (m = n and row0 = 0 for a whole table), and chunks of 2^H
// rows, H <= m, stay inside it.
static FusedPlan plan_fused(uint32_t n_keys, uint64_t rows, uint32_t dim, uint32_t n, uint32_t m, uint64_t row0,
                            uint32_t q_want = 0)
{
    FusedPlan p{};
    p.kch = dim <= 64 ? 1 : dim <= 128 ? 2 : 4;
    // 16 keys with two column chunks need 138-141 VGPRs, one workgroup per
    // CU; two groups of 8 keep two (9..16 keys on 2^20 x 128: 0.92 -> 0.77
    // ms with AES-128, 0.97 -> 0.92 with ChaCha20).  With four chunks 16
    // keys stay faster than groups of 4 (1.45 against 1.85-2.05 ms at 200
    // words) despite their two waves per SIMD.
    const uint32_t qmax = p.kch == 2 ? 8u : (uint32_t)QMAX;
    p.Q = n_keys >= qmax ? qmax : (uint32_t)1 << ceil_log2(n_keys);
    if (q_want && q_want <= qmax && (q_want & (q_want - 1)) == 0)
        p.Q = q_want; // a tuned group size (a power of two the kernels are built for)
    const uint32_t lgS_max = ceil_log2(NT / p.Q);
    const uint32_t groups = (n_keys + p.Q - 1) / p.Q;
    const uint32_t want = ceil_log2((512 + groups - 1) / groups); // about one round of workgroup slots
    uint32_t H = m > want ? m - want : 1;
    H = std::min(H, lgS_max + (uint32_t)HMAX);
    H = std::max(H, std::min(m, lgS_max + 1));
    H = std::min(H, m);
    p.g.row0 = row0;
    p.g.n = n;
    p.g.H = H;
    p.g.lgS = std::min(lgS_max, H - 1);
    p.g.n_groups = groups;
    const uint64_t chunks = (rows + ((uint64_t)1 << H) - 1) >> H;
    p.g.n_chunks = (uint32_t)std::min<uint64_t>(chunks, 0xffffffffu);
    p.grid = chunks * groups;
    return p;
}

// ---------------------------------------------------------------------------
// Tuned plans (pir_set_tuning): a table of entries measured by the project's
// autotuner; a single-table call looks up its (PRF, aligned row height, row
// width, batch size) and takes the fields the entry sets, the model the rest.
struct TuneTable {
    std::vector<pir_tune_t> e;
};
static std::shared_ptr<const TuneTable> g_tune;

static std::shared_ptr<const TuneTable> tune_table() { return std::atomic_load(&g_tune); }

static const pir_tune_t *find_tune(const TuneTable *T, uint32_t prf, uint32_t m, uint32_t dim, uint32_t keys)
{
    if (!T)
        return nullptr;
    for (const pir_tune_t &e : T->e)
        if (e.prf_id == prf && e.n == m && dim >= e.dim_lo && dim <= e.dim_hi && keys >= e.keys_lo &&
            keys <= e.keys_hi)
            return &e;
    return nullptr;
}

static bool tune_entry_ok(const pir_tune_t &e)
{
    return (e.prf_id == PIR_PRF_AES128 || e.prf_id == PIR_PRF_CHACHA20) && e.n >= 1 &&
           e.n <= PIR_MAX_LOG_DOMAIN && e.dim_lo >= 1 && e.dim_lo <= e.dim_hi && e.dim_hi <= PIR_MAX_DIM &&
           e.keys_lo >= 1 && e.keys_lo <= e.keys_hi && e.kernel <= PIR_KERNEL_SMALL_BATCH &&
           e.subtree_log <= (uint32_t)HMAX3 && e.keys_per_item <= (uint32_t)QMAX &&
           (e.keys_per_item & (e.keys_per_item - 1)) == 0 && (e.tail_keys <= 8 || e.tail_keys == PIR_TUNE_MODEL);
}

// How one table's call is planned: the remainder split off to a call of its
// own, then (for a call without one) the kernel and its tuned parameters.
struct Choice {
    uint32_t tail = 0; // keys split off the end (0: none)
    bool waves = false;
    uint32_t h = 0;    // wave kernel: subtree height (0: the model's)
    uint32_t q = 0;    // small-batch kernel: keys per workgroup (0: the model's)
    bool tuned = false;
};

static Choice choose(uint32_t prf, uint32_t n_keys, uint32_t m, uint32_t dim)
{
    const std::shared_ptr<const TuneTable> T = tune_table();
    const pir_tune_t *e = find_tune(T.get(), prf, m, dim, n_keys);
    Choice c;
    c.tuned = e != nullptr;
    if (e && e->tail_keys != PIR_TUNE_MODEL) {
        const uint32_t rem = n_keys % 16;
        c.tail = (n_keys > 16 && rem >= 1 && rem <= e->tail_keys) ? rem : 0;
    } else {
        c.tail = split_tail(n_keys, m);
    }
    if (c.tail)
        return c; // the head and the remainder are planned as calls of their own
    const bool can_wave = m >= 3 && dim <= 128;
    if (e && e->kernel == PIR_KERNEL_WAVES)
        c.waves = can_wave;
    else if (e && e->kernel == PIR_KERNEL_SMALL_BATCH)
        c.waves = false;
    else
        c.waves = use_wave_kernel(prf, n_keys, m, dim);
    if (e) {
        c.h = e->subtree_log;
        c.q = e->keys_per_item;
    }
    return c;
}

// Validates a call over the table rows holding indices row0 .. row0 + rows -
// 1 of keys of domain 2^n (a whole table: row0 = 0, n = ceil(log2 rows)) and
// enqueues its kernels.
template <class PRF>
static int answer_range(const uint8_t *d_keys, uint32_t n_keys, uint32_t key_stride, uint32_t n, uint64_t row0,
                        const uint32_t *d_table, uint64_t rows, uint32_t dim, uint32_t *d_out, CallCtx &ctx,
                        hipStream_t st)
{
    if (n_keys == 0)
        return PIR_OK;
    if (!d_keys || !d_table || !d_out || rows == 0 || dim == 0)
        return PIR_EINVAL;
    if (n == 0 || n > PIR_MAX_LOG_DOMAIN || dim > PIR_MAX_DIM)
        return PIR_EINVAL;
    const uint32_t m = rows <= 2 ? 1 : ceil_log2(rows); // the slice's aligned subtree
    if (m > n || row0 % ((uint64_t)1 << m) || row0 + rows > ((uint64_t)1 << n))
        return PIR_EINVAL;
    if (key_stride % 16 || key_stride < dpf_key_size(n) || ((uintptr_t)d_keys % 16) ||
        ((uintptr_t)d_table % 4) || ((uintptr_t)d_out % 4))
        return PIR_EINVAL;

    const Choice ch = choose(PRF::id, n_keys, m, dim);
    if (const uint32_t tail = ch.tail) {
        const uint32_t head = n_keys - tail;
        const int rc = answer_range<PRF>(d_keys, head, key_stride, n, row0, d_table, rows, dim, d_out, ctx, st);
        if (rc != PIR_OK)
            return rc;
        return answer_range<PRF>(d_keys + (size_t)head * key_stride, tail, key_stride, n, row0, d_table, rows, dim,
                                 d_out + (size_t)head * dim, ctx, st);
    }

    if (ch.waves) {
        WaveTask t{};
        t.table = d_table;
        t.keys = d_keys;
        t.out = d_out;
        t.rows = rows;
        t.row0 = row0;
        t.dim = dim;
        t.n_keys = n_keys;
        t.n = n;
        t.n_bins = 1;
        return launch_waves<PRF>(&t, 1, key_stride, wave_class(dim, vec_aligned(d_table)), ctx, st, ch.h);
    }

    const FusedPlan p = plan_fused(n_keys, rows, dim, n, m, row0, ch.q);
    if (p.grid >= ((uint64_t)1 << 31))
        return PIR_ENOMEM;
    const Geometry &g = p.g;
    const uint32_t Q = p.Q, kch = p.kch;

    if (!ctx.word())
        return PIR_EHIP;
    uint32_t *const status = ctx.status;
    const size_t count = (size_t)n_keys * dim;
    const uint32_t fill_blocks = (uint32_t)std::max<size_t>(1, std::min<size_t>((count + 255) / 256, 4096));
    hipLaunchKernelGGL(k_fill_zero, dim3(fill_blocks), dim3(256), 0, st, d_out, count, ctx.clear_once());
    const dim3 grid((uint32_t)p.grid);
    switch (Q) {
    case 1: launch_q<PRF, 1>(kch, grid, st, d_keys, n_keys, key_stride, d_table, rows, dim, d_out, g, status); break;
    case 2: launch_q<PRF, 2>(kch, grid, st, d_keys, n_keys, key_stride, d_table, rows, dim, d_out, g, status); break;
    case 4: launch_q<PRF, 4>(kch, grid, st, d_keys, n_keys, key_stride, d_table, rows, dim, d_out, g, status); break;
    case 8: launch_q<PRF, 8>(kch, grid, st, d_keys, n_keys, key_stride, d_table, rows, dim, d_out, g, status); break;
    default: launch_q<PRF, 16>(kch, grid, st, d_keys, n_keys, key_stride, d_table, rows, dim, d_out, g, status); break;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? PIR_OK : fail_hip(e);
}

// One whole table.
template <class PRF>
static int answer_one(const uint8_t *d_keys, uint32_t n_keys, uint32_t key_stride, const uint32_t *d_table,
                      uint64_t rows, uint32_t dim, uint32_t *d_out, CallCtx &ctx, hipStream_t st)
{
    if (rows == 0 || rows > ((uint64_t)1 << PIR_MAX_LOG_DOMAIN))
        return n_keys == 0 ? PIR_OK : PIR_EINVAL;
    const uint32_t n = rows <= 2 ? 1 : ceil_log2(rows);
    return answer_range<PRF>(d_keys, n_keys, key_stride, n, 0, d_table, rows, dim, d_out, ctx, st);
}

template <class PRF>
static int answer_multi(const pir_table_t *tables, uint32_t n_tables, const uint8_t *d_keys, uint32_t key_stride,
                        uint32_t *d_out, void *stream)
{
    CallCtx ctx;
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
        if (key_stride % 16 || key_stride < dpf_key_size(n) || ((uintptr_t)d_keys % 16) ||
            ((uintptr_t)T.d_table % 4) || ((uintptr_t)d_out % 4))
            return PIR_EINVAL;
    }
    // tables the wave kernel takes go out grouped by column class, up to
    // MAX_TASKS per launch; the rest one by one, and the remainders split off
    // large tables after the wave launches
    std::vector<WaveTask> cls[WAVE_CLASSES];
    struct Tail {
        uint32_t table, n_keys; // the last n_keys keys of table `table`, at keys, answered into out
        const uint8_t *keys;
        uint32_t *out;
    };
    std::vector<Tail> tails;
    size_t key_off = 0, out_off = 0;
    for (uint32_t t = 0; t < n_tables; t++) {
        const pir_table_t &T = tables[t];
        const uint8_t *kp = d_keys + key_off * key_stride;
        uint32_t *op = d_out + out_off;
        key_off += T.n_keys;
        out_off += (size_t)T.n_keys * T.dim;
        if (T.n_keys == 0)
            continue;
        const uint32_t n = T.rows <= 2 ? 1 : ceil_log2(T.rows);
        const int c = wave_class(T.dim, vec_aligned(T.d_table));
        if (n >= 3 && c >= 0) { // several tables share a launch, so even small batches go to waves
            const uint32_t tail = multi_tail(T.n_keys, n);
            const uint32_t head = T.n_keys - tail;
            if (head) {
                WaveTask w{};
                w.table = T.d_table;
                w.keys = kp;
                w.out = op;
                w.rows = T.rows;
                w.dim = T.dim;
                w.n_keys = head;
                w.n = n;
                w.n_bins = 1;
                cls[c].push_back(w);
            }
            if (tail)
                tails.push_back({t, tail, kp + (size_t)head * key_stride, op + (size_t)head * T.dim});
        } else {
            int st = answer_one<PRF>(kp, T.n_keys, key_stride, T.d_table, T.rows, T.dim, op, ctx,
                                     (hipStream_t)stream);
            if (st != PIR_OK)
                return st;
        }
    }
    for (int c = 0; c < WAVE_CLASSES; c++)
        for (size_t i = 0; i < cls[c].size(); i += MAX_TASKS) {
            const uint32_t cnt = (uint32_t)std::min<size_t>(MAX_TASKS, cls[c].size() - i);
            int st = launch_waves<PRF>(cls[c].data() + i, cnt, key_stride, c, ctx, (hipStream_t)stream);
            if (st != PIR_OK)
                return st;
        }
    for (const Tail &r : tails) {
        const pir_table_t &T = tables[r.table];
        int st = answer_one<PRF>(r.keys, r.n_keys, key_stride, T.d_table, T.rows, T.dim, r.out, ctx,
                                 (hipStream_t)stream);
        if (st != PIR_OK)
            return st;
    }
    return PIR_OK;
}

// Partial batch retrieval: every table cut into bins of 2^bin_log rows, one
// key per (client, bin), all on the wave kernel.
template <class PRF>
static int answer_bins(const pir_bins_t *tables, uint32_t n_tables, const uint8_t *d_keys, uint32_t key_stride,
                       uint32_t *d_out, void *stream)
{
    CallCtx ctx;
    if (!tables && n_tables)
        return PIR_EINVAL;
    for (uint32_t t = 0; t < n_tables; t++) {
        const pir_bins_t &T = tables[t];
        if (T.n_clients == 0)
            continue;
        if (!T.d_table || !d_keys || !d_out || T.rows == 0 || T.dim == 0 || T.dim > PIR_BINS_MAX_DIM ||
            T.rows > ((uint64_t)1 << PIR_MAX_LOG_DOMAIN) || T.bin_log < PIR_BINS_MIN_LOG ||
            T.bin_log > PIR_MAX_LOG_DOMAIN)
            return PIR_EINVAL;
        if (key_stride % 16 || key_stride < dpf_key_size(T.bin_log) || ((uintptr_t)d_keys % 16) ||
            ((uintptr_t)T.d_table % 4) || ((uintptr_t)d_out % 4))
            return PIR_EINVAL;
    }
    std::vector<WaveTask> cls[WAVE_CLASSES];
    size_t key_off = 0, out_off = 0;
    for (uint32_t t = 0; t < n_tables; t++) {
        const pir_bins_t &T = tables[t];
        const uint64_t n_bins = (T.rows + ((uint64_t)1 << T.bin_log) - 1) >> T.bin_log;
        const uint8_t *kp = d_keys + key_off * key_stride;
        uint32_t *op = d_out + out_off;
        key_off += (size_t)T.n_clients * n_bins;
        out_off += (size_t)T.n_clients * n_bins * T.dim;
        if (T.n_clients == 0)
            continue;
        WaveTask w{};
        w.table = T.d_table;
        w.keys = kp;
        w.out = op;
        w.rows = T.rows;
        w.dim = T.dim;
        w.n_keys = T.n_clients;
        w.n = T.bin_log;
        w.n_bins = (uint32_t)n_bins;
        cls[wave_class(T.dim, vec_aligned(T.d_table))].push_back(w);
    }
    for (int c = 0; c < WAVE_CLASSES; c++)
        for (size_t i = 0; i < cls[c].size(); i += MAX_TASKS) {
            const uint32_t cnt = (uint32_t)std::min<size_t>(MAX_TASKS, cls[c].size() - i);
            int st = launch_waves<PRF>(cls[c].data() + i, cnt, key_stride, c, ctx, (hipStream_t)stream);
            if (st != PIR_OK)
                return st;
        }
    return PIR_OK;
}

} // namespace

extern "C" {

int pir_plan(uint32_t prf_id, uint32_t n_keys, uint64_t rows, uint32_t dim, pir_plan_t *out)
{
    if (!out || (prf_id != PIR_PRF_AES128 && prf_id != PIR_PRF_CHACHA20) || n_keys == 0 || rows == 0 ||
        dim == 0 || dim > PIR_MAX_DIM || rows > ((uint64_t)1 << PIR_MAX_LOG_DOMAIN))
        return PIR_EINVAL;
    const uint32_t n = rows <= 2 ? 1 : ceil_log2(rows);
    const bool aes = prf_id == PIR_PRF_AES128;
    *out = pir_plan_t{};
    out->n = n;
    Choice c = choose(prf_id, n_keys, n, dim);
    bool tuned = c.tuned;
    out->tail_keys = c.tail;
    if (c.tail) { // the rest describes the first launch, over the head
        n_keys -= c.tail;
        c = choose(prf_id, n_keys, n, dim);
        tuned |= c.tuned;
    }
    out->source = tuned ? PIR_PLAN_TUNED : PIR_PLAN_MODEL;
    if (c.waves) {
        WaveTask t{};
        t.rows = rows;
        t.dim = dim;
        t.n_keys = n_keys;
        t.n = n;
        t.n_bins = 1;
        const uint64_t items = plan_waves(&t, 1, c.h, wave_pairs(dim));
        if (items == 0)
            return PIR_ENOMEM;
        out->kernel = PIR_KERNEL_WAVES;
        out->items = items;
        out->workgroups = (items + NW3 - 1) / NW3;
        out->lanes_per_workgroup = NT3;
        out->lds_bytes = wave_lds_bytes(aes, dim);
        out->keys_per_item = 16;
        out->rows_per_item = (uint64_t)4 << t.h;
        out->subtree_log = t.h;
        out->descent_levels = n - t.h;
        out->bfs_levels = 0;
        return PIR_OK;
    }
    const FusedPlan p = plan_fused(n_keys, rows, dim, n, n, 0, c.q);
    if (p.grid >= ((uint64_t)1 << 31))
        return PIR_ENOMEM;
    out->kernel = PIR_KERNEL_SMALL_BATCH;
    out->items = p.grid;
    out->workgroups = p.grid;
    out->lanes_per_workgroup = NT;
    if (aes && p.Q == 1 && n_keys == 1 && p.kch == 1 && dim % 4 == 0 && p.g.H > SP_LGS &&
        p.g.H <= SP_LGS + HMAX) { // (for a 16-byte aligned table)
        out->kernel = PIR_KERNEL_STREAM;
        out->lds_bytes = (uint32_t)sizeof(Smem<AesPrf::TAB_WORDS>) + 64 * PIR_MAX_LOG_DOMAIN;
        out->keys_per_item = 1;
        out->rows_per_item = (uint64_t)1 << p.g.H;
        out->subtree_log = p.g.H - SP_LGS;
        out->descent_levels = n - p.g.H;
        out->bfs_levels = SP_LGS;
        return PIR_OK;
    }
    out->lds_bytes = (aes ? (uint32_t)sizeof(Smem<AesPrf::TAB_WORDS>) : (uint32_t)sizeof(Smem<ChaChaPrf::TAB_WORDS>)) +
                     (p.Q <= 2 ? p.Q * 64 * PIR_MAX_LOG_DOMAIN : 0u); // one or two keys' codewords
    out->keys_per_item = p.Q;
    out->rows_per_item = (uint64_t)1 << p.g.H;
    out->subtree_log = p.g.H - p.g.lgS;
    out->descent_levels = n - p.g.H;
    out->bfs_levels = p.g.lgS;
    return PIR_OK;
}

int pir_set_tuning(const pir_tune_t *entries, uint32_t count)
{
    if ((count && !entries) || count > PIR_TUNE_MAX_ENTRIES)
        return PIR_EINVAL;
    for (uint32_t i = 0; i < count; i++)
        if (!tune_entry_ok(entries[i]))
            return PIR_EINVAL;
    std::shared_ptr<const TuneTable> T;
    if (count) {
        auto t = std::make_shared<TuneTable>();
        t->e.assign(entries, entries + count);
        T = t;
    }
    std::atomic_store(&g_tune, T);
    return PIR_OK;
}

uint32_t pir_tuning_count(void)
{
    const std::shared_ptr<const TuneTable> T = tune_table();
    return T ? (uint32_t)T->e.size() : 0u;
}

#ifndef PIR_KERNEL_DIGEST
#define PIR_KERNEL_DIGEST "unknown"
#endif
const char *pir_kernel_digest(void) { return PIR_KERNEL_DIGEST; }

int pir_plan_bins(uint32_t prf_id, uint64_t rows, uint32_t dim, uint32_t n_clients, uint32_t bin_log,
                  pir_plan_t *out)
{
    if (!out || (prf_id != PIR_PRF_AES128 && prf_id != PIR_PRF_CHACHA20) || n_clients == 0 || rows == 0 ||
        dim == 0 || dim > PIR_BINS_MAX_DIM || rows > ((uint64_t)1 << PIR_MAX_LOG_DOMAIN) ||
        bin_log < PIR_BINS_MIN_LOG || bin_log > PIR_MAX_LOG_DOMAIN)
        return PIR_EINVAL;
    WaveTask t{};
    t.rows = rows;
    t.dim = dim;
    t.n_keys = n_clients;
    t.n = bin_log;
    t.n_bins = (uint32_t)((rows + ((uint64_t)1 << bin_log) - 1) >> bin_log);
    const uint64_t items = plan_waves(&t, 1, 0, wave_pairs(dim));
    if (items == 0)
        return PIR_ENOMEM;
    *out = pir_plan_t{};
    out->kernel = PIR_KERNEL_WAVES;
    out->n = bin_log;
    out->items = items;
    out->workgroups = (items + NW3 - 1) / NW3;
    out->lanes_per_workgroup = NT3;
    out->lds_bytes = wave_lds_bytes(prf_id == PIR_PRF_AES128, dim);
    out->keys_per_item = 16;
    out->subtree_log = t.h;
    out->rows_per_item = (uint64_t)4 << t.h;
    out->descent_levels = bin_log - t.h;
    return PIR_OK;
}

int pir_answer_bins(uint32_t prf_id, const pir_bins_t *tables, uint32_t n_tables, const uint8_t *d_keys,
                    uint32_t key_stride, uint32_t *d_out, void *stream)
{
    if (prf_id == PIR_PRF_AES128)
        return answer_bins<AesPrf>(tables, n_tables, d_keys, key_stride, d_out, stream);
    if (prf_id == PIR_PRF_CHACHA20)
        return answer_bins<ChaChaPrf>(tables, n_tables, d_keys, key_stride, d_out, stream);
    return PIR_EINVAL;
}

int pir_answer_prf(uint32_t prf_id, const uint8_t *d_keys, uint32_t n_keys, uint32_t key_stride,
                   const uint32_t *d_table, uint64_t rows, uint32_t dim, uint32_t *d_out, void *stream)
{
    CallCtx ctx;
    const hipStream_t st = (hipStream_t)stream;
    if (prf_id == PIR_PRF_AES128)
        return answer_one<AesPrf>(d_keys, n_keys, key_stride, d_table, rows, dim, d_out, ctx, st);
    if (prf_id == PIR_PRF_CHACHA20)
        return answer_one<ChaChaPrf>(d_keys, n_keys, key_stride, d_table, rows, dim, d_out, ctx, st);
    return PIR_EINVAL;
}

int pir_answer_slice(uint32_t prf_id, uint32_t n, uint64_t row0, const uint8_t *d_keys, uint32_t n_keys,
                     uint32_t key_stride, const uint32_t *d_table, uint64_t rows, uint32_t dim, uint32_t *d_out,
                     void *stream)
{
    CallCtx ctx;
    const hipStream_t st = (hipStream_t)stream;
    if (prf_id == PIR_PRF_AES128)
        return answer_range<AesPrf>(d_keys, n_keys, key_stride, n, row0, d_table, rows, dim, d_out, ctx, st);
    if (prf_id == PIR_PRF_CHACHA20)
        return answer_range<ChaChaPrf>(d_keys, n_keys, key_stride, n, row0, d_table, rows, dim, d_out, ctx, st);
    return PIR_EINVAL;
}

int pir_answer(const uint8_t *d_keys, uint32_t n_keys, uint32_t key_stride, const uint32_t *d_table,
               uint64_t rows, uint32_t dim, uint32_t *d_out, void *stream)
{
    return pir_answer_prf(PIR_PRF_AES128, d_keys, n_keys, key_stride, d_table, rows, dim, d_out, stream);
}

int pir_answer_multi_prf(uint32_t prf_id, const pir_table_t *tables, uint32_t n_tables, const uint8_t *d_keys,
                         uint32_t key_stride, uint32_t *d_out, void *stream)
{
    if (prf_id == PIR_PRF_AES128)
        return answer_multi<AesPrf>(tables, n_tables, d_keys, key_stride, d_out, stream);
    if (prf_id == PIR_PRF_CHACHA20)
        return answer_multi<ChaChaPrf>(tables, n_tables, d_keys, key_stride, d_out, stream);
    return PIR_EINVAL;
}

int pir_answer_multi(const pir_table_t *tables, uint32_t n_tables, const uint8_t *d_keys, uint32_t key_stride,
                     uint32_t *d_out, void *stream)
{
    return pir_answer_multi_prf(PIR_PRF_AES128, tables, n_tables, d_keys, key_stride, d_out, stream);
}

} // extern "C"

// The status code of a status word: a stalled wait first (the output is not
// valid), then a bad key.
static int status_code(uint32_t v)
{
    return (v & PIR_STATUS_STALLED) ? PIR_ESTALL : (v & PIR_STATUS_BAD_KEY) ? PIR_EKEY : PIR_OK;
}

extern "C" {

int pir_check_status(void)
{
    uint32_t *p = default_workspace();
    if (!p)
        return PIR_EHIP;
    uint32_t v = 0;
    const hipError_t e = hipMemcpy(&v, p, sizeof v, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return fail_hip(e);
    return status_code(v);
}

int pir_set_wait_limit(uint32_t tries)
{
    g_wait_limit.store(tries ? tries : PIR_WAIT_LIMIT_DEFAULT, std::memory_order_relaxed);
    return PIR_OK;
}

size_t pir_workspace_size(void) { return PIR_WORKSPACE_BYTES; }

int pir_set_workspace(void *d_ws, size_t bytes)
{
    if (d_ws && (bytes < PIR_WORKSPACE_BYTES || (uintptr_t)d_ws % 16))
        return PIR_EINVAL;
    t_workspace = static_cast<uint32_t *>(d_ws);
    return PIR_OK;
}

int pir_workspace_status(const void *d_ws, void *stream)
{
    if (!d_ws || (uintptr_t)d_ws % 16)
        return PIR_EINVAL;
    const hipStream_t st = (hipStream_t)stream;
    uint32_t v = 0;
    hipError_t e = hipMemcpyAsync(&v, d_ws, sizeof v, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return fail_hip(e);
    return status_code(v);
}

} // extern "C"
