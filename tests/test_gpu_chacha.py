"""GPU parity of the ChaCha20-PRF path (paper section 3.2.6) against the oracle.

Same bar and rules as the AES-128 parity tests: keys come from the oracle's
Gen with prf id 1, tables from the seeded generator, expected values from the
oracle (or the closed form beta * T[alpha]); every comparison is on uint32
words and bit-exact.  Both kernels are covered: fewer than 16 keys take the
small-batch kernel, 16 or more the wave kernel on the matrix cores.
"""
import numpy as np
import pytest

from conftest import cpu_threads
from paper_2301_10904_amd import workloads as W
from test_gpu_parity import log_domain, make_sparse, sparse_answers

pytestmark = pytest.mark.gpu

CHACHA = 1


def chacha_keys(O, n, alphas, seed, beta=1):
    return O.gen_batch(n, alphas, W.key_seeds(len(alphas), seed), beta=beta, prf_id=CHACHA)


def gpu_answer(pir, keys_np, table_dev):
    import torch

    keys = torch.from_numpy(np.ascontiguousarray(keys_np)).cuda()
    out = pir.answer(keys, table_dev, prf="chacha20")
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


@pytest.fixture(scope="module")
def pirmod(gpu_lib):
    from paper_2301_10904_amd import pir

    return pir


SHAPES = [
    # rows, dim, key pairs: tiny, ragged tails, several tiles, wide rows, both kernels
    (1, 1, 1), (3, 5, 2), (100, 7, 2), (1000, 16, 9), (4097, 64, 8), (5000, 65, 3),
    (2048, 256, 10), (1 << 16, 32, 20), (1 << 15, 64, 40),
]


@pytest.mark.parametrize("rows,dim,pairs", SHAPES)
def test_parity_shapes(O, pirmod, rows, dim, pairs):
    seed = rows * 5 + dim + 1
    T = W.make_table(rows, dim, seed)
    alphas = W.uniform_indices(rows, pairs, seed)
    alphas[0] = rows - 1
    K0, K1 = chacha_keys(O, log_domain(rows), alphas, seed)
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
    T = W.make_table(rows, dim, 15)
    Tn = T.numpy().view(np.uint32)
    keys, expect = [], []
    for i, beta in enumerate((0, 2, 2**31, 2**32 - 1, 0x12345678)):
        seed = W.key_seeds(1, 300 + i)[0].tobytes()
        k0, k1 = O.gen(12, 31 * i, beta, seed, prf_id=CHACHA)
        keys += [k0, k1]
        expect.append(((Tn[31 * i].astype(np.uint64) * beta) & 0xFFFFFFFF).astype(np.uint32))
    keys = np.stack(keys)
    got = gpu_answer(pirmod, keys, T.cuda())
    assert (got == O.answer_batch(keys, Tn, nthreads=cpu_threads())).all()
    for i, e in enumerate(expect):
        assert (O.reconstruct(got[2 * i], got[2 * i + 1]) == e).all()


def test_full_size_2p20_x64_batch512(O, pirmod):
    """2^20 rows x 64 uint32, 512 ChaCha20 key pairs in one call (the shape
    of the paper's PRF comparison): every reconstruction equals T[alpha];
    per-server answers match the oracle on a sample of keys."""
    import torch

    rows, dim, pairs, seed = 1 << 20, 64, 512, 22
    T = W.make_table(rows, dim, seed, device="cuda")
    alphas = W.uniform_indices(rows, pairs, seed)
    K0, K1 = chacha_keys(O, 20, alphas, seed)
    keys = np.concatenate([K0, K1])
    got = gpu_answer(pirmod, keys, T)
    Trows = W.table_rows_np(alphas, dim, seed)
    recon = (got[:pairs].astype(np.uint64) + got[pairs:]) & 0xFFFFFFFF
    assert (recon.astype(np.uint32) == Trows).all()
    Tn = T.cpu().numpy().view(np.uint32)
    sample = np.array([0, 1, 511, 512, 1023])
    want = O.answer_batch(keys[sample], Tn, nthreads=cpu_threads())
    assert (got[sample] == want).all()
    del T
    torch.cuda.empty_cache()


def test_keys_of_the_other_prf_are_rejected(O, pirmod):
    """An AES key in a ChaCha20 call (and the reverse) answers zero and
    raises the key flag; the other keys of the call are unaffected."""
    rows, dim = 1024, 16
    T = W.make_table(rows, dim, 19)
    Tn = T.numpy().view(np.uint32)
    Kc0, Kc1 = chacha_keys(O, 10, np.array([5, 900]), 19)
    Ka0, _ = O.gen_batch(10, np.array([7]), W.key_seeds(1, 19))
    keys = np.concatenate([Kc0, Ka0, Kc1])
    assert pirmod.check_status() == pirmod.PIR_OK
    got = gpu_answer(pirmod, keys, T.cuda())
    assert pirmod.check_status() == pirmod.PIR_EKEY
    assert (got[2] == 0).all()
    ok = [0, 1, 3, 4]
    assert (got[ok] == O.answer_batch(keys[ok], Tn, nthreads=2)).all()
    import torch

    out = pirmod.answer(torch.from_numpy(keys).cuda(), T.cuda(), prf="aes128")
    torch.cuda.synchronize()
    assert pirmod.check_status() == pirmod.PIR_EKEY
    got = out.cpu().numpy().view(np.uint32)
    assert (got[ok] == 0).all()
    assert (got[2] == O.answer(keys[2], Tn)).all()


@pytest.mark.parametrize("pairs,dim", [(1, 64), (3, 16), (7, 32)])
def test_small_batches_deep_tree(O, pirmod, pairs, dim):
    rows, seed = 1 << 17, 50 + pairs
    T = W.make_table(rows, dim, seed)
    alphas = W.uniform_indices(rows, pairs, seed)
    K0, K1 = chacha_keys(O, 17, alphas, seed)
    keys = np.concatenate([K0, K1])
    got = gpu_answer(pirmod, keys, T.cuda())
    want = O.answer_batch(keys, T.numpy().view(np.uint32), nthreads=cpu_threads())
    assert (got == want).all()


@pytest.mark.parametrize("log_rows,dim,nkeys", [(20, 64, 1), (22, 32, 3)])
def test_small_batches_sparse_full_size(O, pirmod, log_rows, dim, nkeys):
    import torch

    rows, seed = 1 << log_rows, 60 + log_rows
    Ts, sup, vals = make_sparse(rows, dim, seed, 16, "cuda")
    alphas = W.uniform_indices(rows, nkeys, seed)
    alphas[0] = sup[5]
    K0, K1 = chacha_keys(O, log_rows, alphas, seed)
    keys = np.concatenate([K0, K1])[:nkeys]
    got = gpu_answer(pirmod, keys, Ts)
    assert (got == sparse_answers(O, keys, sup, vals)).all()
    del Ts
    torch.cuda.empty_cache()


def test_answer_multi_ragged(O, pirmod):
    import torch

    specs = [(1 << 12, 32, 5), (3000, 16, 0), (1 << 14, 64, 9), (777, 8, 2), (1 << 13, 64, 12)]
    tables, counts, all_keys, expect = [], [], [], []
    for i, (rows, dim, pairs) in enumerate(specs):
        T = W.make_table(rows, dim, 70 + i)
        tables.append(T.cuda())
        counts.append(2 * pairs)
        if pairs == 0:
            expect.append(None)
            continue
        K0, K1 = chacha_keys(O, log_domain(rows), W.zipf_indices(rows, pairs, 70 + i), 70 + i)
        keys = np.concatenate([K0, K1])
        all_keys.append(keys)
        expect.append(O.answer_batch(keys, T.numpy().view(np.uint32), nthreads=cpu_threads()))
    stride = (max(k.shape[1] for k in all_keys) + 15) // 16 * 16
    padded = [np.pad(k, ((0, 0), (0, stride - k.shape[1]))) for k in all_keys]
    keys_dev = torch.from_numpy(np.concatenate(padded)).cuda()
    _, views = pirmod.answer_multi(tables, counts, keys_dev, prf="chacha20")
    torch.cuda.synchronize()
    for v, e in zip(views, expect):
        if e is not None:
            assert (v.cpu().numpy().view(np.uint32) == e).all()
