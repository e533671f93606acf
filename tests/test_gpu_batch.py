"""GPU parity of batch retrieval (paper section 4) against the oracle.

Partial batch retrieval: many small-domain DPFs, one per (client, bin), over
one or several resident tables in one call (pir_answer_bins).  Keys come from
the oracle's Gen, expected per-server answers from the oracle's binned answer,
and every reconstruction is checked against T[b I + alpha] (or, through the
client plan, against the wanted rows).  The hot/full split runs as a two-table
call.  All comparisons are bit-exact uint32.
"""
import numpy as np
import pytest

from conftest import cpu_threads
from oracle import client as oc
from paper_2301_10904_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pirmod(gpu_lib):
    from paper_2301_10904_amd import pir

    return pir


def oracle_bin_keys(O, alphas, bin_log, seed, prf_id=0):
    """alphas [clients][bins] -> both parties' keys, client-major."""
    C, B = len(alphas), len(alphas[0])
    seeds = W.key_seeds(C * B, seed)
    flat = [int(a) for row in alphas for a in row]
    return O.gen_batch(bin_log, flat, seeds, prf_id=prf_id)


def random_alphas(rows, bin_log, clients, seed):
    size = 1 << bin_log
    nb = -(-rows // size)
    rng = np.random.default_rng([rows, bin_log, clients, seed])
    return [[int(rng.integers(0, min(size, rows - b * size))) for b in range(nb)] for _ in range(clients)]


def run_bins(pir, tables_np, keysets, clients, bin_logs, prf):
    import torch

    stride = (max(k.shape[1] for k in keysets) + 15) // 16 * 16
    keys = np.concatenate([np.pad(k, ((0, 0), (0, stride - k.shape[1]))) for k in keysets])
    tabs = [torch.from_numpy(t.view(np.int32)).cuda() for t in tables_np]
    _, views = pir.answer_bins(tabs, clients, bin_logs, torch.from_numpy(keys).cuda(), prf=prf)
    torch.cuda.synchronize()
    return [v.cpu().numpy().view(np.uint32) for v in views]


CASES = [
    # rows, dim, bin_log, clients: one group, partial groups, several groups, ragged last bin
    (1 << 12, 16, 8, 1), (1 << 12, 64, 10, 5), (3000, 7, 6, 17), (5000, 32, 9, 40),
    (1 << 14, 64, 12, 16), (777, 3, 3, 2), (1 << 13, 33, 13, 20),
    # rows of 65..128 words (wave pairs, four column tiles a wave)
    (1 << 12, 128, 9, 6), (3000, 100, 7, 17), (2000, 65, 11, 3),
    # tables of 1..4 rows: a single bin shorter than any wave item's subtrees
    (1, 16, 3, 3), (2, 64, 3, 2), (3, 5, 4, 17), (4, 128, 3, 1), (4, 32, 12, 16),
]


@pytest.mark.parametrize("prf", [0, 1])
@pytest.mark.parametrize("rows,dim,bin_log,clients", CASES)
def test_bins_parity(O, pirmod, rows, dim, bin_log, clients, prf):
    seed = rows + dim + bin_log + clients + prf
    T = W.make_table(rows, dim, seed).numpy().view(np.uint32)
    alphas = random_alphas(rows, bin_log, clients, seed)
    K0, K1 = oracle_bin_keys(O, alphas, bin_log, seed, prf)
    got0, got1 = run_bins(pirmod, [T, T], [K0, K1], [clients, clients], [bin_log, bin_log], prf)
    want0 = O.answer_bins(K0, T, bin_log, clients, nthreads=cpu_threads())
    want1 = O.answer_bins(K1, T, bin_log, clients, nthreads=cpu_threads())
    assert (got0 == want0).all() and (got1 == want1).all()
    size = 1 << bin_log
    rec = ((got0.astype(np.uint64) + got1) & 0xFFFFFFFF).astype(np.uint32)
    for c in range(clients):
        for b, a in enumerate(alphas[c]):
            assert (rec[c, b] == T[b * size + a]).all(), (c, b)


def test_bins_full_size_2p20_x64(O, pirmod):
    """2^20 x 64 table in 256 bins of 2^12 rows, 64 clients per server (16384
    keys per server, both servers in one call): Zipf-wanted sets planned by the
    oracle's client; every served entry reconstructs exactly, every dropped one
    collided; per-server answers against the oracle on a sample of bins."""
    import torch

    rows, dim, bin_log, clients, seed = 1 << 20, 64, 12, 64, 5
    Tt = W.make_table(rows, dim, seed, device="cuda")
    plans = []
    for c in range(clients):
        wanted = W.zipf_indices(rows, 128, seed * 1000 + c)
        plans.append(oc.pbr_plan(wanted, rows, bin_log))
    alphas = [p[0] for p in plans]
    K0, K1 = oracle_bin_keys(O, alphas, bin_log, seed)
    keys = torch.from_numpy(np.concatenate([K0, K1])).cuda()
    _, views = pirmod.answer_bins([Tt, Tt], [clients, clients], [bin_log, bin_log], keys)
    torch.cuda.synchronize()
    g0, g1 = (v.cpu().numpy().view(np.uint32) for v in views)
    rec = ((g0.astype(np.uint64) + g1) & 0xFFFFFFFF).astype(np.uint32)
    for c, (al, served, dropped) in enumerate(plans):
        idx = [x for x in served if x is not None]
        bins = [b for b, x in enumerate(served) if x is not None]
        assert (rec[c, bins] == W.table_rows_np(idx, dim, seed)).all(), c
        for x in dropped:
            assert served[x >> bin_log] is not None
    Tn = Tt.cpu().numpy().view(np.uint32)
    for c, b in ((0, 0), (3, 17), (63, 255), (31, 128)):
        key = K0[c * 256 + b]
        want = O.answer(key, Tn[b << bin_log:(b + 1) << bin_log])
        assert (g0[c, b] == want).all(), (c, b)
    del Tt
    torch.cuda.empty_cache()


def test_hot_full_two_tables_one_call(O, pirmod):
    """Hot/full split (section 4.2): a hot table gathered from the most
    frequent rows of a Zipf access log and the full table, Q_hot and Q_full
    queries per client (dummies included), answered in one call as two
    one-bin tables; every served entry reconstructs exactly."""
    rows, dim, seed, clients, q_hot, q_full = 1 << 16, 32, 12, 24, 6, 2
    T = W.make_table(rows, dim, seed).numpy().view(np.uint32)
    log = W.zipf_indices(rows, 20000, seed)
    counts = np.bincount(log, minlength=rows)
    order = np.lexsort((np.arange(rows), -counts))
    hot_rows = np.sort(order[:rows // 16])
    hot_map = {int(x): i for i, x in enumerate(hot_rows)}
    H = np.ascontiguousarray(T[hot_rows])
    ha_all, fa_all, plans = [], [], []
    for c in range(clients):
        wanted = W.zipf_indices(rows, 7, seed * 100 + c)
        p = oc.hot_full_plan(wanted, hot_map, q_hot, q_full)
        plans.append(p)
        ha_all.append(p[0])
        fa_all.append(p[1])
    n_hot, n_full = 12, 16  # hot table 2^12 rows, full table 2^16 rows: one bin each
    KH0, KH1 = oracle_bin_keys(O, [[a] for row in ha_all for a in row], n_hot, seed)
    KF0, KF1 = oracle_bin_keys(O, [[a] for row in fa_all for a in row], n_full, seed + 1)
    got = run_bins(pirmod, [H, T, H, T], [KH0, KF0, KH1, KF1],
                   [clients * q_hot, clients * q_full] * 2, [n_hot, n_full] * 2, 0)
    assert (got[0][:, 0] == O.answer_batch(KH0, H, nthreads=cpu_threads())).all()
    assert (got[1][:, 0] == O.answer_batch(KF0, T, nthreads=cpu_threads())).all()
    hot = ((got[0][:, 0].astype(np.uint64) + got[2][:, 0]) & 0xFFFFFFFF).astype(np.uint32)
    full = ((got[1][:, 0].astype(np.uint64) + got[3][:, 0]) & 0xFFFFFFFF).astype(np.uint32)
    for c, (ha, fa, sh, sf, dropped) in enumerate(plans):
        for i, x in enumerate(sh):
            assert (hot[c * q_hot + i] == (T[x] if x is not None else H[0])).all()
        for i, x in enumerate(sf):
            assert (full[c * q_full + i] == (T[x] if x is not None else T[0])).all()


def test_answer_multi_many_tables(O, pirmod):
    """41 tables of every column class in one call (more than a launch takes,
    so several launches per class), some without keys, small and wave-kernel
    batches mixed: every per-server answer bit-exact."""
    import torch

    rng = np.random.default_rng(41)
    dims = [1, 5, 16, 17, 32, 33, 64, 70, 130, 256]
    tables, counts, keysets, expect = [], [], [], []
    for t in range(41):
        rows = int(rng.integers(2, 3000))
        dim = dims[t % len(dims)]
        n = max(1, (rows - 1).bit_length())
        T = W.make_table(rows, dim, 300 + t)
        tables.append(T.cuda())
        nk = int(rng.choice([0, 1, 3, 16, 21]))
        counts.append(nk)
        if nk == 0:
            expect.append(None)
            continue
        K, _ = O.gen_batch(n, W.uniform_indices(rows, nk, 300 + t), W.key_seeds(nk, 300 + t))
        keysets.append(K)
        expect.append(O.answer_batch(K, T.numpy().view(np.uint32), nthreads=cpu_threads()))
    stride = (max(k.shape[1] for k in keysets) + 15) // 16 * 16
    keys = np.concatenate([np.pad(k, ((0, 0), (0, stride - k.shape[1]))) for k in keysets])
    _, views = pirmod.answer_multi(tables, counts, torch.from_numpy(keys).cuda())
    torch.cuda.synchronize()
    for t, (v, e) in enumerate(zip(views, expect)):
        if e is not None:
            assert (v.cpu().numpy().view(np.uint32) == e).all(), t


def test_bins_bad_key_header(O, pirmod):
    """A binned key with a wrong domain or PRF id answers zero and raises the
    key flag; the other keys of the call are unaffected."""
    rows, dim, bin_log, clients, seed = 1000, 8, 7, 2, 44
    T = W.make_table(rows, dim, seed).numpy().view(np.uint32)
    alphas = random_alphas(rows, bin_log, clients, seed)
    K0, _ = oracle_bin_keys(O, alphas, bin_log, seed)
    K0[3, 2] = bin_log + 1   # wrong domain
    K0[10, 3] = 1            # ChaCha20 id in an AES call
    assert pirmod.check_status() == pirmod.PIR_OK
    (got,) = run_bins(pirmod, [T], [K0], [clients], [bin_log], 0)
    assert pirmod.check_status() == pirmod.PIR_EKEY
    flat = got.reshape(-1, dim)
    assert (flat[3] == 0).all() and (flat[10] == 0).all()
    good = [i for i in range(len(K0)) if i not in (3, 10)]
    nb = -(-rows // (1 << bin_log))
    for i in good:
        c, b = divmod(i, nb)
        want = O.answer(K0[i], T[b << bin_log:(b + 1) << bin_log])
        assert (flat[i] == want).all(), i


@pytest.mark.parametrize("prf", [0, 1])
def test_bins_tiny_tables_beside_a_large_one(O, pirmod, prf):
    """Tables of 1..4 rows share one wave launch with larger tables of the same
    row width (the multi-table plan gives every table its own subtree height):
    every per-server answer bit-exact, every reconstruction T[b I + alpha]."""
    specs = [(3, 16, 3, 5), (1 << 12, 16, 9, 20), (1, 16, 4, 2), (4, 16, 3, 17), (2, 16, 5, 1)]
    tabs, keysets, want, alphas_l = [], [], [], []
    for i, (rows, dim, bin_log, clients) in enumerate(specs):
        seed = 500 + 10 * i + prf
        T = W.make_table(rows, dim, seed).numpy().view(np.uint32)
        alphas = random_alphas(rows, bin_log, clients, seed)
        K0, _ = oracle_bin_keys(O, alphas, bin_log, seed, prf)
        tabs.append(T)
        keysets.append(K0)
        alphas_l.append(alphas)
        want.append(O.answer_bins(K0, T, bin_log, clients, nthreads=cpu_threads()))
    got = run_bins(pirmod, tabs, keysets, [s[3] for s in specs], [s[2] for s in specs], prf)
    for i in range(len(specs)):
        assert (got[i] == want[i]).all(), specs[i]
