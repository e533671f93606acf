"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Keys always come from the oracle's Gen, tables from the seeded generator, and
expected values from the oracle (or from the closed form beta * T[alpha]); no
input or expected value is taken from the HIP path.  The bar is bit-exact:
every comparison below is on uint32 words.
"""
import numpy as np
import pytest

from conftest import cpu_threads
from paper_2301_10904_amd import workloads as W

pytestmark = pytest.mark.gpu


def oracle_keys(O, n, alphas, seed):
    seeds = W.key_seeds(len(alphas), seed)
    return O.gen_batch(n, alphas, seeds)


def gpu_answer(pir, keys_np, table_dev, prf=0):
    import torch

    keys = torch.from_numpy(np.ascontiguousarray(keys_np)).cuda()
    out = pir.answer(keys, table_dev, prf=prf)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


def log_domain(rows):
    return max(1, (rows - 1).bit_length())


@pytest.fixture(scope="module")
def pirmod(gpu_lib):
    from paper_2301_10904_amd import pir

    return pir


def test_single_pair_2p14_x16(O, pirmod):
    """One table of 2^14 rows x 16 uint32, one key pair over a 14-bit domain,
    beta = 1: both per-server answers bit-exact and the reconstruction."""
    import torch

    rows, dim, seed = 1 << 14, 16, 1
    T = W.make_table(rows, dim, seed)
    alpha = W.uniform_indices(rows, 1, seed)
    K0, K1 = oracle_keys(O, 14, alpha, seed)
    keys = np.concatenate([K0, K1])
    got = gpu_answer(pirmod, keys, T.cuda())
    Tn = T.numpy().view(np.uint32)
    want = O.answer_batch(keys, Tn, nthreads=2)
    assert (got == want).all()
    assert (O.reconstruct(got[0], got[1]) == Tn[alpha[0]]).all()
    torch.cuda.synchronize()


SHAPES = [
    # rows, dim, key pairs: empty-ish, ragged tails, several tiles, wide rows
    (1, 1, 1), (2, 3, 1), (3, 5, 2), (5, 1, 3), (100, 7, 2), (1000, 16, 9),
    (4097, 64, 8), (5000, 65, 3), (3000, 130, 5), (2048, 256, 10), (1 << 16, 32, 20),
    (50000, 64, 1), (1 << 15, 64, 40),
]


@pytest.mark.parametrize("rows,dim,pairs", SHAPES)
def test_parity_shapes(O, pirmod, rows, dim, pairs):
    seed = rows * 7 + dim
    n = log_domain(rows)
    T = W.make_table(rows, dim, seed)
    alphas = W.uniform_indices(rows, pairs, seed)
    alphas[0] = rows - 1  # the last row is always queried
    K0, K1 = oracle_keys(O, n, alphas, seed)
    # both parties mixed in one call, interleaved
    keys = np.empty((2 * pairs, K0.shape[1]), np.uint8)
    keys[0::2], keys[1::2] = K0, K1
    got = gpu_answer(pirmod, keys, T.cuda())
    Tn = T.numpy().view(np.uint32)
    want = O.answer_batch(keys, Tn, nthreads=cpu_threads())
    assert (got == want).all()
    for p in range(pairs):
        assert (O.reconstruct(got[2 * p], got[2 * p + 1]) == Tn[alphas[p]]).all()


def test_beta_values(O, pirmod):
    rows, dim = 3000, 8
    T = W.make_table(rows, dim, 5)
    Tn = T.numpy().view(np.uint32).astype(np.uint64)
    keys, expect = [], []
    for i, beta in enumerate((0, 2, 2**31, 2**32 - 1, 0x12345678)):
        seed = W.key_seeds(1, 100 + i)[0].tobytes()
        k0, k1 = O.gen(12, 17 * i, beta, seed)
        keys += [k0, k1]
        expect.append(((Tn[17 * i] * beta) & 0xFFFFFFFF).astype(np.uint32))
    keys = np.stack(keys)
    got = gpu_answer(pirmod, keys, T.cuda())
    want = O.answer_batch(keys, T.numpy().view(np.uint32), nthreads=cpu_threads())
    assert (got == want).all()
    for i, e in enumerate(expect):
        assert (O.reconstruct(got[2 * i], got[2 * i + 1]) == e).all()


def test_full_size_2p20_x64_batch512(O, pirmod):
    """The benchmark's workload and launch: 2^20 rows x 64 uint32 (256 MiB),
    512 key pairs (1024 keys, both servers in one call).  Every reconstruction
    must equal T[alpha]; per-server answers are compared with the oracle on a
    sample of keys."""
    import torch

    rows, dim, pairs, seed = 1 << 20, 64, 512, 2
    T = W.make_table(rows, dim, seed, device="cuda")
    alphas = W.uniform_indices(rows, pairs, seed)
    K0, K1 = oracle_keys(O, 20, alphas, seed)
    keys = np.concatenate([K0, K1])
    got = gpu_answer(pirmod, keys, T)
    Trows = W.table_rows_np(alphas, dim, seed)
    for p in range(pairs):
        assert (O.reconstruct(got[p], got[pairs + p]) == Trows[p]).all(), p
    # the device table is the generator's table
    Tn = T.cpu().numpy().view(np.uint32)
    assert (Tn[alphas[:16]] == Trows[:16]).all()
    sample = np.array([0, 1, 255, 511, 512, 700, 1022, 1023])
    want = O.answer_batch(keys[sample], Tn, nthreads=cpu_threads())
    assert (got[sample] == want).all()
    del T
    torch.cuda.empty_cache()


def test_bad_key_header_gives_zero_row(O, pirmod):
    rows, dim = 1024, 16
    T = W.make_table(rows, dim, 9)
    K0, K1 = oracle_keys(O, 10, np.array([3, 600]), 9)
    keys = np.concatenate([K0, K1])
    keys[1, 0] = 7          # bad version
    keys[2, 2] = 11         # wrong domain size
    good = gpu_answer(pirmod, keys[[0, 3]], T.cuda())
    assert pirmod.check_status() == pirmod.PIR_OK
    got = gpu_answer(pirmod, keys, T.cuda())
    assert pirmod.check_status() == pirmod.PIR_EKEY
    assert pirmod.check_status() == pirmod.PIR_EKEY  # reading leaves the call's status
    assert (got[1] == 0).all() and (got[2] == 0).all()
    want = O.answer_batch(keys[[0, 3]], T.numpy().view(np.uint32), nthreads=2)
    assert (got[[0, 3]] == want).all() and (good == want).all()
    gpu_answer(pirmod, keys[[0, 3]], T.cuda())
    assert pirmod.check_status() == pirmod.PIR_OK  # the next call reports its own status


def test_repeat_launches_identical(O, pirmod):
    import torch

    rows, dim = 1 << 14, 64
    T = W.make_table(rows, dim, 4).cuda()
    K0, K1 = oracle_keys(O, 14, W.uniform_indices(rows, 24, 4), 4)
    keys = torch.from_numpy(np.concatenate([K0, K1])).cuda()
    first = pirmod.answer(keys, T).clone()
    for _ in range(5):
        out = pirmod.answer(keys, T)
        torch.cuda.synchronize()
        assert torch.equal(out, first)


def test_side_stream(O, pirmod):
    import torch

    rows, dim = 3000, 32
    T = W.make_table(rows, dim, 6)
    K0, K1 = oracle_keys(O, 12, W.uniform_indices(rows, 3, 6), 6)
    keys_np = np.concatenate([K0, K1])
    s = torch.cuda.Stream()
    Td = T.cuda()
    keys = torch.from_numpy(keys_np).cuda()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        out = pirmod.answer(keys, Td, stream=s)
    s.synchronize()
    want = O.answer_batch(keys_np, T.numpy().view(np.uint32), nthreads=cpu_threads())
    assert (out.cpu().numpy().view(np.uint32) == want).all()


def test_answer_multi_ragged(O, pirmod):
    import torch

    specs = [(1 << 12, 32, 5), (3000, 16, 0), (1 << 14, 64, 7), (777, 8, 2)]
    tables, counts, all_keys, expect = [], [], [], []
    for i, (rows, dim, pairs) in enumerate(specs):
        T = W.make_table(rows, dim, 40 + i)
        tables.append(T.cuda())
        counts.append(2 * pairs)
        if pairs == 0:
            expect.append(None)
            continue
        K0, K1 = oracle_keys(O, log_domain(rows), W.zipf_indices(rows, pairs, 40 + i), 40 + i)
        keys = np.concatenate([K0, K1])
        all_keys.append(keys)
        expect.append(O.answer_batch(keys, T.numpy().view(np.uint32), nthreads=cpu_threads()))
    stride = max(k.shape[1] for k in all_keys)
    stride = (stride + 15) // 16 * 16
    padded = [np.pad(k, ((0, 0), (0, stride - k.shape[1]))) for k in all_keys]
    keys_dev = torch.from_numpy(np.concatenate(padded)).cuda()
    _, views = pirmod.answer_multi(tables, counts, keys_dev)
    torch.cuda.synchronize()
    for v, e in zip(views, expect):
        if e is not None:
            assert (v.cpu().numpy().view(np.uint32) == e).all()


def sparse_answers(O, keys, support_rows, support_vals):
    """Per-server answers over a table that is zero except `support_rows`:
    sum_j Eval(key, j) * T[j] over the support only, with point evaluation."""
    out = np.zeros((len(keys), support_vals.shape[1]), np.uint64)
    for q, key in enumerate(keys):
        for j, row in zip(support_rows, support_vals):
            y = np.uint64(O.eval_point(key, int(j)))
            out[q] = (out[q] + y * row.astype(np.uint64)) & 0xFFFFFFFF
    return out.astype(np.uint32)


def make_sparse(rows, dim, seed, n_support, device):
    import torch

    rng = np.random.default_rng([seed, 77])
    support = np.sort(rng.choice(rows, n_support, replace=False))
    support[0] = rows - 1
    vals = W.table_rows_np(support, dim, seed)
    T = torch.zeros((rows, dim), dtype=torch.int32, device=device)
    T[torch.from_numpy(support).to(device)] = torch.from_numpy(vals.view(np.int32)).to(device)
    return T, np.sort(support), vals[np.argsort(support)]


def test_multi_table_ragged_zipf(O, pirmod):
    """Eight tables of 2^16 .. 2^23 rows x 32 uint32 (about 2 GiB), ragged
    batches of 32..1024 queries (both servers' keys), Zipf(1.05) indices, one
    call.  Every reconstruction equals T_t[alpha]; per-server answers are
    bit-exact on sparse copies of the two largest tables (all their keys) and
    against the full oracle on samples of the smallest table."""
    import torch

    seed = 3
    sizes = W.ragged_batch_sizes(8, seed)
    tables, counts, keysets, alphas = [], [], [], []
    for t in range(8):
        rows = 1 << (16 + t)
        tables.append(W.make_table(rows, 32, seed + t, device="cuda"))
        a = W.zipf_indices(rows, int(sizes[t]), seed + t)
        K0, K1 = oracle_keys(O, 16 + t, a, seed + t)
        keysets.append(np.concatenate([K0, K1]))
        counts.append(2 * int(sizes[t]))
        alphas.append(a)
    stride = (max(k.shape[1] for k in keysets) + 15) // 16 * 16
    keys = np.concatenate([np.pad(k, ((0, 0), (0, stride - k.shape[1]))) for k in keysets])
    keys_dev = torch.from_numpy(keys).cuda()
    _, views = pirmod.answer_multi(tables, counts, keys_dev)
    torch.cuda.synchronize()
    for t in range(8):
        got = views[t].cpu().numpy().view(np.uint32)
        want = W.table_rows_np(alphas[t], 32, seed + t)
        B = int(sizes[t])
        recon = (got[:B].astype(np.uint64) + got[B:]) & 0xFFFFFFFF
        assert (recon.astype(np.uint32) == want).all(), t
    # full oracle on a sample of the smallest table
    T0 = tables[0].cpu().numpy().view(np.uint32)
    sample = [0, 1, counts[0] - 1]
    want = O.answer_batch(keysets[0][sample], T0, nthreads=cpu_threads())
    assert (views[0].cpu().numpy().view(np.uint32)[sample] == want).all()
    # sparse copies of the two largest tables: every key, per server
    for t in (6, 7):
        rows = 1 << (16 + t)
        Ts, sup, vals = make_sparse(rows, 32, seed + t, 12, "cuda")
        sub = [tables[i] if i != t else Ts for i in range(8)]
        _, v2 = pirmod.answer_multi(sub, counts, keys_dev)
        torch.cuda.synchronize()
        got = v2[t].cpu().numpy().view(np.uint32)
        assert (got == sparse_answers(O, keysets[t], sup, vals)).all(), t
        del Ts
    del tables
    torch.cuda.empty_cache()


def test_large_table_2p25_x64(O, pirmod):
    """One table of 2^25 rows x 64 uint32 (8 GiB) resident in HBM, 512 key
    pairs with uniform indices: every reconstruction equals T[alpha], and on a
    sparse copy of the same shape every per-server answer is bit-exact."""
    import torch

    rows, dim, pairs, seed = 1 << 25, 64, 512, 4
    T = W.make_table(rows, dim, seed, device="cuda")
    alphas = W.uniform_indices(rows, pairs, seed)
    K0, K1 = oracle_keys(O, 25, alphas, seed)
    keys = np.concatenate([K0, K1])
    keys_dev = torch.from_numpy(keys).cuda()
    out = pirmod.answer(keys_dev, T)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    want = W.table_rows_np(alphas, dim, seed)
    recon = (got[:pairs].astype(np.uint64) + got[pairs:]) & 0xFFFFFFFF
    assert (recon.astype(np.uint32) == want).all()
    del T, out
    torch.cuda.empty_cache()
    Ts, sup, vals = make_sparse(rows, dim, seed, 8, "cuda")
    out = pirmod.answer(keys_dev, Ts)
    torch.cuda.synchronize()
    sample = np.arange(0, 2 * pairs, 37)
    got = out.cpu().numpy().view(np.uint32)
    assert (got[sample] == sparse_answers(O, keys[sample], sup, vals)).all()
    # reconstruction on the sparse table: T[alpha] if alpha is in the support, else 0
    dense_rows = {int(j): v for j, v in zip(sup, vals)}
    for p in range(pairs):
        r = (got[p].astype(np.uint64) + got[pairs + p]) & 0xFFFFFFFF
        w = dense_rows.get(int(alphas[p]), np.zeros(dim, np.uint32))
        assert (r.astype(np.uint32) == w).all()
    del Ts
    torch.cuda.empty_cache()


@pytest.mark.parametrize("pairs", [1024, 2048])
def test_large_table_2p25_x64_large_batches(O, pirmod, pairs):
    """The 2^25 x 64 table (8 GiB) with the large batches of the 1024..4096
    key workload: 2048 and 4096 keys per launch.  Every reconstruction equals
    T[alpha] on the dense table; on a sparse copy of the same shape one key
    of every group of 16 (the wave kernel's key group) is checked per server
    against the oracle's point evaluation, and every reconstruction against
    the support."""
    import torch

    rows, dim, seed = 1 << 25, 64, 40 + pairs
    T = W.make_table(rows, dim, seed, device="cuda")
    alphas = W.uniform_indices(rows, pairs, seed)
    K0, K1 = oracle_keys(O, 25, alphas, seed)
    keys = np.concatenate([K0, K1])
    keys_dev = torch.from_numpy(keys).cuda()
    assert pirmod.plan(2 * pairs, rows, dim)["kernel"] == pirmod.KERNEL_WAVES
    out = pirmod.answer(keys_dev, T)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    recon = (got[:pairs].astype(np.uint64) + got[pairs:]) & 0xFFFFFFFF
    assert (recon.astype(np.uint32) == W.table_rows_np(alphas, dim, seed)).all()
    del T, out
    torch.cuda.empty_cache()
    Ts, sup, vals = make_sparse(rows, dim, seed, 8, "cuda")
    out = pirmod.answer(keys_dev, Ts)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    rng = np.random.default_rng(seed)
    sample = np.arange(0, 2 * pairs, 16) + rng.integers(0, 16, size=2 * pairs // 16)
    assert (got[sample] == sparse_answers(O, keys[sample], sup, vals)).all()
    dense_rows = {int(j): v for j, v in zip(sup, vals)}
    for p in range(pairs):
        r = (got[p].astype(np.uint64) + got[pairs + p]) & 0xFFFFFFFF
        w = dense_rows.get(int(alphas[p]), np.zeros(dim, np.uint32))
        assert (r.astype(np.uint32) == w).all()
    del Ts
    torch.cuda.empty_cache()


@pytest.mark.parametrize("pairs,dim", [(1, 64), (1, 32), (2, 64), (3, 16), (7, 32)])
def test_small_batches_deep_tree(O, pirmod, pairs, dim):
    """Fewer than 16 keys on a 2^18-row table: the small-batch kernel with a
    per-lane walk of height > 1, bit-exact against the full oracle."""
    rows, seed = 1 << 18, 11 + pairs
    T = W.make_table(rows, dim, seed)
    alphas = W.uniform_indices(rows, pairs, seed)
    K0, K1 = oracle_keys(O, 18, alphas, seed)
    keys = np.concatenate([K0, K1])
    got = gpu_answer(pirmod, keys, T.cuda())
    Tn = T.numpy().view(np.uint32)
    want = O.answer_batch(keys, Tn, nthreads=cpu_threads())
    assert (got == want).all()


@pytest.mark.parametrize("log_rows,dim,nkeys", [(20, 64, 1), (24, 32, 1), (22, 32, 2), (20, 32, 5)])
def test_small_batches_sparse_full_size(O, pirmod, log_rows, dim, nkeys):
    """Single keys and small batches at full domain sizes, per server, on a
    sparse table of the full shape (oracle by point evaluation)."""
    import torch

    rows, seed = 1 << log_rows, log_rows + nkeys
    Ts, sup, vals = make_sparse(rows, dim, seed, 16, "cuda")
    alphas = W.uniform_indices(rows, nkeys, seed)
    alphas[0] = sup[3]  # one query hits a non-zero row
    K0, K1 = oracle_keys(O, log_rows, alphas, seed)
    keys = np.concatenate([K0, K1])[:nkeys]
    got = gpu_answer(pirmod, keys, Ts)
    assert (got == sparse_answers(O, keys, sup, vals)).all()
    del Ts
    torch.cuda.empty_cache()


@pytest.mark.parametrize("nkeys", [2, 16])
def test_max_domain_2p32_rows(O, pirmod, nkeys):
    """The largest table the ABI takes: 2^32 rows (n = 32) x 1 uint32, 16 GiB,
    sparse; a key pair on the small-batch kernel and 16 keys on the wave
    kernel, every per-server answer against the oracle's point evaluation and
    the pairs reconstructing T[alpha]."""
    import torch

    rows, dim, seed = 1 << 32, 1, 32
    Ts, sup, vals = make_sparse(rows, dim, seed, 16, "cuda")
    pairs = nkeys // 2
    alphas = W.uniform_indices(rows, pairs, seed + nkeys)
    alphas[0] = sup[-1]  # the last row, 2^32 - 1 (make_sparse puts it in the support)
    if pairs > 1:
        alphas[1] = sup[7]
    K0, K1 = oracle_keys(O, 32, alphas, seed + nkeys)
    keys = np.concatenate([K0, K1])
    got = gpu_answer(pirmod, keys, Ts)
    assert (got == sparse_answers(O, keys, sup, vals)).all()
    dense = {int(j): v for j, v in zip(sup, vals)}
    for p in range(pairs):
        r = ((got[p].astype(np.uint64) + got[pairs + p]) & 0xFFFFFFFF).astype(np.uint32)
        assert (r == dense.get(int(alphas[p]), np.zeros(dim, np.uint32))).all(), p
    del Ts
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prf", [0, 1])
def test_small_groups_every_shape(O, pirmod, prf):
    """1..16 keys (every key-group size of the small-batch kernel, and the
    wave kernel above its threshold) on tiny to mid-size domains, where some
    waves of a workgroup hold no subtree, with row widths of every column
    class (1, 7, 64, 65, 200 words): every per-server answer bit-exact."""
    import torch

    for rows in (1, 2, 7, 64, 300, 5000):
        n = log_domain(rows)
        for dim in (1, 7, 64, 65, 200):
            T = W.make_table(rows, dim, rows + dim)
            Tn = T.numpy().view(np.uint32)
            Td = T.cuda()
            for nk in (1, 2, 3, 5, 8, 16):
                seed = 7 * rows + dim + nk
                alphas = W.uniform_indices(rows, nk, seed)
                K, _ = O.gen_batch(n, alphas, W.key_seeds(nk, seed), prf_id=prf)
                out = pirmod.answer(torch.from_numpy(K).cuda(), Td, prf=prf)
                torch.cuda.synchronize()
                got = out.cpu().numpy().view(np.uint32)
                want = O.answer_batch(K, Tn, nthreads=cpu_threads())
                assert (got == want).all(), (rows, dim, nk)


@pytest.mark.parametrize("prf", [0, 1])
@pytest.mark.parametrize("rows,dim", [(1 << 20, 64), ((1 << 20) - 3, 40)])
def test_sixteen_keys_full_size_dense(O, pirmod, prf, rows, dim):
    """Sixteen keys on a dense 2^20-row table (the small-batch kernel with the
    product on the matrix cores), also with a ragged row count and rows of 40
    words: every per-server answer against the oracle's full evaluation."""
    import torch

    seed = 31 + prf + dim
    T = W.make_table(rows, dim, seed)
    alphas = W.uniform_indices(rows, 16, seed)
    K, _ = O.gen_batch(20, alphas, W.key_seeds(16, seed), prf_id=prf)
    out = pirmod.answer(torch.from_numpy(K).cuda(), T.cuda(), prf=prf)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    want = O.answer_batch(K, T.numpy().view(np.uint32), nthreads=cpu_threads())
    assert (got == want).all()


SLICE_CASES = [
    # n, shards, dim, keys: both kernels, wide and narrow rows, tiny slices
    (12, 4, 16, 3), (14, 8, 64, 40), (16, 2, 7, 20), (13, 16, 33, 1), (10, 64, 4, 17), (15, 4, 130, 5),
    (14, 4, 100, 20),
    (18, 2, 16, 36),  # slices of 2^17 rows: a remainder of 4 keys runs as a launch of its own
    (18, 2, 100, 24),  # slices of 2^17 rows of 100 words on the wave pairs
]


@pytest.mark.parametrize("prf", [0, 1])
@pytest.mark.parametrize("n,shards,dim,nkeys", SLICE_CASES)
def test_slices_sum_to_the_answer(O, pirmod, prf, n, shards, dim, nkeys):
    """Row sharding (section 3.2.7) on one GPU: each slice's per-server answer
    against the oracle's, and the slices' answers summed mod 2^32 against the
    library's own whole-table answer for the same keys."""
    import torch

    rows, seed = 1 << n, n * 100 + shards + prf
    size = rows // shards
    T = W.make_table(rows, dim, seed)
    Tn = T.numpy().view(np.uint32)
    Td = T.cuda()
    alphas = W.uniform_indices(rows, nkeys, seed)
    K, _ = O.gen_batch(n, alphas, W.key_seeds(nkeys, seed), prf_id=prf)
    keys = torch.from_numpy(K).cuda()
    full = pirmod.answer(keys, Td, prf=prf)
    total = torch.zeros_like(full)
    ys = [O.eval_full(k) for k in K]
    for s in range(shards):
        r0 = s * size
        part = pirmod.answer_slice(keys, Td[r0:r0 + size], n, r0, prf=prf)
        torch.cuda.synchronize()
        got = part.cpu().numpy().view(np.uint32)
        for q in range(nkeys):
            want = ((ys[q][r0:r0 + size, None].astype(np.uint64) * Tn[r0:r0 + size]).sum(0) & 0xFFFFFFFF)
            assert (got[q] == want.astype(np.uint32)).all(), (s, q)
        total += part  # int32 addition wraps mod 2^32
    torch.cuda.synchronize()
    assert (total.cpu().numpy() == full.cpu().numpy()).all()
    # one slice also straight from the oracle's definition (point evaluation)
    r0 = (shards // 2) * size
    want = O.answer_slice(K[0], Tn[r0:r0 + size], r0)
    got = pirmod.answer_slice(keys[:1].contiguous(), Td[r0:r0 + size], n, r0, prf=prf)
    assert (got.cpu().numpy().view(np.uint32)[0] == want).all()


@pytest.mark.parametrize("prf", [0, 1])
def test_ragged_slice(O, pirmod, prf):
    """A slice shorter than its aligned subtree (the last GPU's share of a
    table whose rows are not a power of two)."""
    import torch

    n, dim, r0, cnt = 12, 24, 3072, 1000
    T = W.make_table(r0 + cnt, dim, 5 + prf)
    Tn = T.numpy().view(np.uint32)
    for nk in (3, 18):  # the small-batch and the wave kernel
        alphas = W.uniform_indices(r0 + cnt, nk, 5)
        K, _ = O.gen_batch(n, alphas, W.key_seeds(nk, 5), prf_id=prf)
        got = pirmod.answer_slice(torch.from_numpy(K).cuda(), T[r0:].contiguous().cuda(), n, r0, prf=prf)
        torch.cuda.synchronize()
        got = got.cpu().numpy().view(np.uint32)
        for q in sorted({0, nk // 2, nk - 1}):
            assert (got[q] == O.answer_slice(K[q], Tn[r0:], r0)).all(), (nk, q)


@pytest.mark.parametrize("prf", [0, 1])
@pytest.mark.parametrize("dim", [100, 200])
def test_single_key_streamed_wide_rows(O, pirmod, prf, dim):
    """A single key on a dense table above 256 MiB (rows read with
    non-temporal loads) with rows of 100 and 200 words (two and four column
    chunks): the per-server answer against the oracle."""
    import torch

    rows, seed = 1 << 20, 61 + dim + prf
    T = W.make_table(rows, dim, seed)
    alphas = W.uniform_indices(rows, 1, seed)
    K, _ = O.gen_batch(20, alphas, W.key_seeds(1, seed), prf_id=prf)
    out = pirmod.answer(torch.from_numpy(K).cuda(), T.cuda(), prf=prf)
    torch.cuda.synchronize()
    want = O.answer_batch(K, T.numpy().view(np.uint32), nthreads=1)
    assert (out.cpu().numpy().view(np.uint32) == want).all()


WIDE_WAVE_CASES = [
    # rows, dim, keys: rows of 65..128 words on the wave kernel (wave pairs,
    # four column tiles a wave), several key groups, ragged row counts and
    # key groups
    ((1 << 16) + 3, 65, 41), ((1 << 17) - 1, 100, 25), ((1 << 17) + 5, 128, 48), ((1 << 16) + 9, 127, 32),
    ((1 << 14) - 3, 100, 528),
]


@pytest.mark.parametrize("prf", [0, 1])
@pytest.mark.parametrize("rows,dim,nkeys", WIDE_WAVE_CASES)
def test_wide_rows_wave_kernel(O, pirmod, prf, rows, dim, nkeys):
    """Batches on rows of 65 to 128 words, which the wave kernel takes as wave
    pairs (each wave one 64-column half of both chunks' rows): every
    per-server answer against the oracle and every reconstruction against
    T[alpha]."""
    import torch

    assert pirmod.plan(nkeys, rows, dim, prf=prf)["kernel"] == pirmod.KERNEL_WAVES
    seed = rows + dim + nkeys + prf
    n = log_domain(rows)
    T = W.make_table(rows, dim, seed)
    alphas = W.uniform_indices(rows, nkeys, seed)
    alphas[0] = rows - 1
    K0, K1 = O.gen_batch(n, alphas, W.key_seeds(nkeys, seed), prf_id=prf)
    keys = np.concatenate([K0, K1])
    out = pirmod.answer(torch.from_numpy(keys).cuda(), T.cuda(), prf=prf)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    Tn = T.numpy().view(np.uint32)
    want = O.answer_batch(keys, Tn, nthreads=cpu_threads())
    assert (got == want).all()
    for i, a in enumerate(alphas):
        assert (O.reconstruct(got[i], got[nkeys + i]) == Tn[a]).all(), i



@pytest.mark.parametrize("prf", [0, 1])
def test_wave_pairs_several_tables_one_launch(O, pirmod, prf):
    """Rows of 65..128 words run as wave pairs: two waves on the same 16 keys
    and adjacent chunks trade their leaf shares, and each multiplies one
    64-column half.  Six such tables in one call share the launches of their
    column classes (every table's pairs start at an even item); odd chunk
    counts leave the last pair's second wave without rows; the second half
    is full, partial with a width that is a multiple of 4 (16-byte loads
    kept inside the row), or of any width (single words); and one table sits
    at a 4-byte offset.  Every per-server answer against the oracle."""
    import torch

    specs = [  # rows, dim, keys, at a 4-byte offset; chunks of 2048 rows
        (9000, 128, 33, False),  # 5 chunks
        (3000, 100, 21, False),  # 2 chunks, second half of 36 columns
        (7000, 68, 40, False),   # 4 chunks, second half of 4 columns
        (5000, 99, 17, False),   # 3 chunks, single words
        (4100, 128, 18, True),   # 3 chunks, single words (unaligned)
        (4100, 128, 18, False),  # the same rows and keys, aligned
    ]
    tables, counts, keysets, expect = [], [], [], []
    for t, (rows, dim, nk, offset) in enumerate(specs):
        seed = 900 + (t if t < 5 else 4) + prf
        T = W.make_table(rows, dim, seed)
        if offset:
            buf = torch.empty(rows * dim + 4, dtype=torch.int32, device="cuda")
            Td = buf[1:1 + rows * dim].view(rows, dim)
            Td.copy_(T.cuda())
            assert Td.data_ptr() % 16 != 0
        else:
            Td = T.cuda()
        tables.append(Td)
        counts.append(nk)
        K, _ = O.gen_batch(log_domain(rows), W.uniform_indices(rows, nk, seed), W.key_seeds(nk, seed), prf_id=prf)
        keysets.append(K)
        expect.append(O.answer_batch(K, T.numpy().view(np.uint32), nthreads=cpu_threads()))
    stride = (max(k.shape[1] for k in keysets) + 15) // 16 * 16
    keys = np.concatenate([np.pad(k, ((0, 0), (0, stride - k.shape[1]))) for k in keysets])
    _, views = pirmod.answer_multi(tables, counts, torch.from_numpy(keys).cuda(), prf=prf)
    torch.cuda.synchronize()
    for t, (v, e) in enumerate(zip(views, expect)):
        assert (v.cpu().numpy().view(np.uint32) == e).all(), specs[t]
    assert (views[4].cpu() == views[5].cpu()).all()

@pytest.mark.parametrize("prf", [0, 1])
def test_full_size_2p20_x128_batch64(O, pirmod, prf):
    """2^20 rows of 128 words (512 MiB, the 512-byte entries of the paper's
    larger tables) with 32 key pairs on the wave kernel: every reconstruction
    equals T[alpha]; per-server answers against the oracle on a sample."""
    import torch

    rows, dim, pairs, seed = 1 << 20, 128, 32, 71 + prf
    T = W.make_table(rows, dim, seed, device="cuda")
    alphas = W.uniform_indices(rows, pairs, seed)
    K0, K1 = O.gen_batch(20, alphas, W.key_seeds(pairs, seed), prf_id=prf)
    keys = np.concatenate([K0, K1])
    out = pirmod.answer(torch.from_numpy(keys).cuda(), T, prf=prf)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    Trows = W.table_rows_np(alphas, dim, seed)
    for p in range(pairs):
        assert (O.reconstruct(got[p], got[pairs + p]) == Trows[p]).all(), p
    Tn = T.cpu().numpy().view(np.uint32)
    sample = np.array([0, 17, 31, 32, 63])
    want = O.answer_batch(keys[sample], Tn, nthreads=cpu_threads())
    assert (got[sample] == want).all()
    del T
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prf", [0, 1])
@pytest.mark.parametrize("rows,dim,nkeys", [((1 << 14) + 3, 100, 12), (4096, 128, 16), (3000, 65, 9)])
def test_wide_rows_small_batches(O, pirmod, prf, rows, dim, nkeys):
    """9..16 keys on rows of 65..128 words: the small-batch kernel in groups of
    8 keys (two column chunks), the last group partial; per-server answers
    against the oracle."""
    import torch

    p = pirmod.plan(nkeys, rows, dim, prf=prf)
    assert p["kernel"] == pirmod.KERNEL_SMALL_BATCH and p["keys_per_item"] == 8
    seed = 3 * rows + dim + nkeys + prf
    n = log_domain(rows)
    T = W.make_table(rows, dim, seed)
    alphas = W.uniform_indices(rows, nkeys, seed)
    K, _ = O.gen_batch(n, alphas, W.key_seeds(nkeys, seed), prf_id=prf)
    out = pirmod.answer(torch.from_numpy(K).cuda(), T.cuda(), prf=prf)
    torch.cuda.synchronize()
    want = O.answer_batch(K, T.numpy().view(np.uint32), nthreads=cpu_threads())
    assert (out.cpu().numpy().view(np.uint32) == want).all()


def test_chacha20_wide_rows_above_2p20_on_waves(O, pirmod):
    """ChaCha20 keys on 2^21 + 77 rows of 100 words (839 MB): 10 key pairs take
    the wave kernel.  Every reconstruction equals T[alpha]; the per-server
    answers of two keys against the oracle."""
    import torch

    rows, dim, pairs, seed = (1 << 21) + 77, 100, 10, 83
    assert pirmod.plan(2 * pairs, rows, dim, prf=1)["kernel"] == pirmod.KERNEL_WAVES
    T = W.make_table(rows, dim, seed, device="cuda")
    alphas = W.uniform_indices(rows, pairs, seed)
    alphas[0] = rows - 1
    K0, K1 = O.gen_batch(22, alphas, W.key_seeds(pairs, seed), prf_id=1)
    keys = np.concatenate([K0, K1])
    out = pirmod.answer(torch.from_numpy(keys).cuda(), T, prf=1)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    Trows = W.table_rows_np(alphas, dim, seed)
    for p in range(pairs):
        assert (O.reconstruct(got[p], got[pairs + p]) == Trows[p]).all(), p
    Tn = T.cpu().numpy().view(np.uint32)
    sample = np.array([0, pairs + 3])
    want = O.answer_batch(keys[sample], Tn, nthreads=cpu_threads())
    assert (got[sample] == want).all()
    del T
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prf", [0, 1])
@pytest.mark.parametrize("rows,dim,nkeys", [((1 << 17) - 3, 40, 20), ((1 << 18) + 1, 16, 37), (1 << 17, 8, 70),
                                            ((1 << 19) + 3, 8, 264)])
def test_ragged_batches_split_off_the_remainder(O, pirmod, prf, rows, dim, nkeys):
    """A remainder of 1..8 keys past whole groups of 16 is answered by a second
    launch on the small-batch kernel (the first: the small-batch kernel, or
    for 256 keys on 2^20 rows' domain the wave kernel): every per-server
    answer against the oracle, both parties mixed."""
    import torch

    p = pirmod.plan(nkeys, rows, dim, prf=prf)
    assert p["tail_keys"] == nkeys % 16 and p["tail_keys"] > 0
    assert (p["kernel"] == pirmod.KERNEL_WAVES) == (nkeys == 264)
    seed = rows + dim + 5 * nkeys + prf
    n = log_domain(rows)
    T = W.make_table(rows, dim, seed)
    half = (nkeys + 1) // 2
    alphas = W.uniform_indices(rows, half, seed)
    alphas[0] = rows - 1
    K0, K1 = O.gen_batch(n, alphas, W.key_seeds(half, seed), prf_id=prf)
    keys = np.empty((2 * half, K0.shape[1]), np.uint8)
    keys[0::2], keys[1::2] = K0, K1
    keys = keys[:nkeys]
    out = pirmod.answer(torch.from_numpy(keys).cuda(), T.cuda(), prf=prf)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    Tn = T.numpy().view(np.uint32)
    want = O.answer_batch(keys, Tn, nthreads=cpu_threads())
    assert (got == want).all()
    for i in range(nkeys // 2):
        assert (O.reconstruct(got[2 * i], got[2 * i + 1]) == Tn[alphas[i]]).all(), i


@pytest.mark.parametrize("prf", [0, 1])
def test_answer_multi_tails_on_large_tables(O, pirmod, prf):
    """Tables of at least 2^20 rows send a remainder of 1..8 keys to a
    small-batch launch of their own, the rest stays in the shared wave launch
    (here: tails only, a group plus a tail, a group of exactly 16, and a
    small table that keeps its partial group); every per-server answer
    against the oracle."""
    import torch

    specs = [((1 << 20) + 3, 16, 5), (1 << 20, 8, 21), ((1 << 21) - 7, 4, 3), (1 << 20, 8, 16), (5000, 16, 7)]
    tables, counts, keysets, expect = [], [], [], []
    for i, (rows, dim, nk) in enumerate(specs):
        seed = 90 + i + 10 * prf
        T = W.make_table(rows, dim, seed)
        tables.append(T.cuda())
        counts.append(nk)
        K, _ = O.gen_batch(log_domain(rows), W.uniform_indices(rows, nk, seed), W.key_seeds(nk, seed), prf_id=prf)
        keysets.append(K)
        expect.append(O.answer_batch(K, T.numpy().view(np.uint32), nthreads=cpu_threads()))
    stride = (max(k.shape[1] for k in keysets) + 15) // 16 * 16
    keys = np.concatenate([np.pad(k, ((0, 0), (0, stride - k.shape[1]))) for k in keysets])
    _, views = pirmod.answer_multi(tables, counts, torch.from_numpy(keys).cuda(), prf=prf)
    torch.cuda.synchronize()
    for t, (v, e) in enumerate(zip(views, expect)):
        assert (v.cpu().numpy().view(np.uint32) == e).all(), t


def random_cases(rng):
    """(rows, dim, keys, prf): random small cases; narrow rows at and above the
    wave kernel's batch threshold (AES-128 on 2^14..2^18 rows, ChaCha20 just
    above 2^20 rows); rows of 65..128 words on 2^17..2^18 rows."""
    cases = []
    for _ in range(20):
        n = int(rng.integers(1, 20))
        rows = int(rng.integers((1 << (n - 1)) + 1, (1 << n) + 1)) if n > 1 else int(rng.integers(1, 3))
        dim = int(rng.choice([1, 3, 16, 33, 64, 65, 100, 128, 130]))
        cap = max(1, min(600, (1 << 22) // rows, (1 << 26) // (rows * dim)))
        cases.append((rows, dim, int(rng.integers(1, cap + 1)), int(rng.integers(0, 2))))
    for _ in range(4):
        n = int(rng.choice([14, 16, 18]))
        rows = int(rng.integers((1 << (n - 1)) + 1, (1 << n) + 1))
        cases.append((rows, int(rng.choice([8, 16])), (32 << (20 - n)) + int(rng.integers(0, 24)), 0))
    for _ in range(2):
        rows = int(rng.integers((1 << 20) + 1, (1 << 20) + 5000))
        cases.append((rows, 8, int(rng.integers(17, 40)), 1))
    for _ in range(4):
        n = int(rng.choice([17, 18]))
        rows = int(rng.integers((1 << (n - 1)) + 1, (1 << n) + 1))
        cases.append((rows, int(rng.choice([65, 100, 128])), int(rng.integers(17, 41)), int(rng.integers(0, 2))))
    return cases


def test_random_shapes_against_the_oracle(O, pirmod):
    """A seeded sweep over table sizes, row widths, batch sizes and both PRFs,
    bounded so the oracle answers each case in about a second at most; it
    reaches both kernels and the split-off remainder.  Every per-server answer
    against the oracle."""
    import torch

    seen = set()
    for case, (rows, dim, nkeys, prf) in enumerate(random_cases(np.random.default_rng(2301))):
        p = pirmod.plan(nkeys, rows, dim, prf=prf)
        seen.add((p["kernel"], p["tail_keys"] > 0))
        seed = 7000 + case
        T = W.make_table(rows, dim, seed)
        alphas = W.uniform_indices(rows, nkeys, seed)
        K, _ = O.gen_batch(log_domain(rows), alphas, W.key_seeds(nkeys, seed), prf_id=prf)
        out = pirmod.answer(torch.from_numpy(K).cuda(), T.cuda(), prf=prf)
        torch.cuda.synchronize()
        want = O.answer_batch(K, T.numpy().view(np.uint32), nthreads=cpu_threads())
        assert (out.cpu().numpy().view(np.uint32) == want).all(), (case, rows, dim, nkeys, prf, p)
    assert {(pirmod.KERNEL_WAVES, False), (pirmod.KERNEL_SMALL_BATCH, False)} <= seen, seen
    assert any(tail for _, tail in seen), seen


@pytest.mark.parametrize("prf", [0, 1])
@pytest.mark.parametrize("rows,dim,nkeys", [
    (1 << 12, 64, 64),    # wave kernel, vector loads of 16 bytes when aligned
    (1 << 12, 32, 64),    # wave kernel, 8-byte loads when aligned
    (1 << 12, 16, 64),    # wave kernel, 16 columns
    (1 << 14, 64, 3),     # small-batch kernel (16-byte row segments when aligned)
    (1 << 14, 64, 16),    # small-batch kernel, matrix-core product over 16 keys
    (1 << 12, 100, 40),   # wave pairs: single words here, 16-byte loads on the aligned copy
])
def test_table_at_a_4_byte_offset(O, pirmod, prf, rows, dim, nkeys):
    """A table whose base is 4-byte but not 16-byte aligned (a contiguous view
    one word into a buffer) is read with single-word loads and answers exactly
    as an aligned copy does."""
    import torch

    seed = rows + dim + nkeys + prf
    T = W.make_table(rows, dim, seed)
    buf = torch.empty(rows * dim + 4, dtype=torch.int32, device="cuda")
    buf[1:1 + rows * dim].copy_(T.reshape(-1).cuda())
    Tview = buf[1:1 + rows * dim].view(rows, dim)
    assert Tview.data_ptr() % 16 == 4 and Tview.is_contiguous()
    a = W.uniform_indices(rows, nkeys, seed)
    K0, _ = O.gen_batch(log_domain(rows), a, W.key_seeds(nkeys, seed), prf_id=prf)
    keys = torch.from_numpy(K0).cuda()
    got = pirmod.answer(keys, Tview, prf=prf)
    torch.cuda.synchronize()
    want = O.answer_batch(K0, T.numpy().view(np.uint32), nthreads=cpu_threads())
    assert (got.cpu().numpy().view(np.uint32) == want).all()
    # the same table, aligned, in a multi-table call beside the offset one
    Ta = T.cuda()
    out, views = pirmod.answer_multi([Tview, Ta], [nkeys, nkeys], torch.cat([keys, keys]), prf=prf)
    torch.cuda.synchronize()
    for v in views:
        assert (v.cpu().numpy().view(np.uint32) == want).all()


@pytest.mark.parametrize("rows,dim", [(257, 4), (1000, 16), (3000, 64), (5000, 32), (1 << 16, 64), (100000, 16)])
def test_single_key_stream_kernel_small_tables(O, pirmod, rows, dim):
    """One AES-128 key on tables of 257 to 100,000 rows (most of them ragged)
    takes k_pir_stream with cached row reads; both parties' answers against
    the full oracle and the reconstruction of the last row and of a random one."""
    assert pirmod.plan(1, rows, dim)["kernel"] == pirmod.KERNEL_STREAM
    seed = rows + dim
    n = log_domain(rows)
    T = W.make_table(rows, dim, seed)
    Tn, Td = T.numpy().view(np.uint32), T.cuda()
    alphas = [rows - 1, int(W.uniform_indices(rows, 1, seed)[0])]
    K0, K1 = O.gen_batch(n, np.array(alphas, dtype=np.int64), W.key_seeds(2, seed), prf_id=0)
    for i, a in enumerate(alphas):
        g0 = gpu_answer(pirmod, K0[i:i + 1], Td)
        g1 = gpu_answer(pirmod, K1[i:i + 1], Td)
        assert (g0 == O.answer_batch(K0[i:i + 1], Tn, nthreads=cpu_threads())).all(), (rows, dim, a)
        assert (g1 == O.answer_batch(K1[i:i + 1], Tn, nthreads=cpu_threads())).all(), (rows, dim, a)
        assert (O.reconstruct(g0[0], g1[0]) == Tn[a]).all()
    assert pirmod.check_status() == pirmod.PIR_OK


@pytest.mark.parametrize("prf", [0, 1])
@pytest.mark.parametrize("rows,dim", [(1 << 21, 64), ((1 << 22) + 12345, 40), (1 << 23, 16)])
def test_single_key_stream_kernel_dense(O, pirmod, prf, rows, dim):
    """One key on a table above 256 MiB with rows of at most 64 words: with
    AES-128 it runs on k_pir_stream (tree waves and table-stream waves), with
    ChaCha20 on k_pir_fused; both parties' answers against the full oracle,
    and the reconstruction, on dense tables (one of them ragged)."""
    import torch

    want_kernel = pirmod.KERNEL_STREAM if prf == 0 else pirmod.KERNEL_SMALL_BATCH
    assert pirmod.plan(1, rows, dim, prf=prf)["kernel"] == want_kernel
    seed = rows % 1000 + dim + prf
    n = log_domain(rows)
    T = W.make_table(rows, dim, seed)
    Tn = T.numpy().view(np.uint32)
    Td = T.cuda()
    a = W.uniform_indices(rows, 1, seed)
    K0, K1 = O.gen_batch(n, a, W.key_seeds(1, seed), prf_id=prf)
    g0 = gpu_answer(pirmod, K0, Td, prf)
    g1 = gpu_answer(pirmod, K1, Td, prf)
    assert pirmod.check_status() == pirmod.PIR_OK
    assert (g0 == O.answer_batch(K0, Tn, nthreads=cpu_threads())).all()
    assert (g1 == O.answer_batch(K1, Tn, nthreads=cpu_threads())).all()
    assert (O.reconstruct(g0[0], g1[0]) == Tn[a[0]]).all()
    bad = K0.copy()
    bad[0, 2] = n + 1  # wrong domain: zero row, status
    assert (gpu_answer(pirmod, bad, Td, prf) == 0).all()
    assert pirmod.check_status() == pirmod.PIR_EKEY
    del Td
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prf", [0, 1])
def test_single_key_stream_kernel_2p25_and_a_slice(O, pirmod, prf):
    """One key on the 2^25 x 64 table (sparse copy, per server against point
    evaluation) and on a 2^23-row slice of it at row 3 * 2^23
    (pir_answer_slice, per server against point evaluation of the slice's
    indices): the stream kernel with AES-128, k_pir_fused with ChaCha20."""
    import torch

    rows, dim, seed = 1 << 25, 64, 70 + prf
    Ts, sup, vals = make_sparse(rows, dim, seed, 24, "cuda")
    a = [int(sup[5])]  # a queried row in the support
    K0, K1 = O.gen_batch(25, a, W.key_seeds(1, seed), prf_id=prf)
    g0, g1 = gpu_answer(pirmod, K0, Ts, prf), gpu_answer(pirmod, K1, Ts, prf)
    assert (g0 == sparse_answers(O, K0, sup, vals)).all() and (g1 == sparse_answers(O, K1, sup, vals)).all()
    assert (O.reconstruct(g0[0], g1[0]) == vals[5]).all()
    # a slice holding indices 3 * 2^23 .. 4 * 2^23 - 1
    size, row0 = 1 << 23, 3 << 23
    keep = (sup >= row0) & (sup < row0 + size)
    assert keep.any()
    sl = Ts[row0:row0 + size].contiguous()
    out = pirmod.answer_slice(torch.from_numpy(K0).cuda(), sl, 25, row0, prf=prf)
    torch.cuda.synchronize()
    want = sparse_answers(O, K0, sup[keep], vals[keep])
    assert (out.cpu().numpy().view(np.uint32) == want).all()
    del Ts, sl
    torch.cuda.empty_cache()
