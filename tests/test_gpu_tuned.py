"""Tuned plans on the GPU: whatever plan an entry of the tuned table picks
(kernel, subtree height, keys per workgroup, remainder split), the answers
are the oracle's, bit for bit; and the committed cache, where it applies to
this system, changes plans but not answers."""
import numpy as np
import pytest

from conftest import cpu_threads
from paper_2301_10904_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pirmod(gpu_lib):
    from paper_2301_10904_amd import pir

    yield pir
    pir.set_tuning([])


def entry(pir, prf, n, **kw):
    from paper_2301_10904_amd import autotune as A

    return A.entry(prf, n, 1, 256, 1, A.ALL_KEYS, **kw)


PLANS = [
    dict(kernel=1, subtree_log=3), dict(kernel=1, subtree_log=9), dict(kernel=1, subtree_log=1),
    dict(kernel=2, keys_per_item=1), dict(kernel=2, keys_per_item=2), dict(kernel=2, keys_per_item=4),
    dict(kernel=2, keys_per_item=16), dict(tail_keys=0), dict(tail_keys=8), dict(kernel=1, tail_keys=0),
]


@pytest.mark.parametrize("prf", [0, 1])
@pytest.mark.parametrize("plan", range(len(PLANS)))
def test_any_tuned_plan_answers_exactly(O, pirmod, prf, plan):
    import torch

    rows, dim, nkeys = 5000, 48, 37  # 2^13 aligned rows, a ragged table, a remainder of 5 keys
    seed = 60 + plan + 10 * prf
    T = W.make_table(rows, dim, seed)
    a = W.uniform_indices(rows, nkeys, seed)
    K0, _ = O.gen_batch(13, a, W.key_seeds(nkeys, seed), prf_id=prf)
    pirmod.set_tuning([entry(pirmod, prf, 13, **PLANS[plan])])
    try:
        p = pirmod.plan(nkeys, rows, dim, prf=prf)
        assert p["source"] == pirmod.PLAN_TUNED
        got = pirmod.answer(torch.from_numpy(K0).cuda(), T.cuda(), prf=prf)
        torch.cuda.synchronize()
    finally:
        pirmod.set_tuning([])
    want = O.answer_batch(K0, T.numpy().view(np.uint32), nthreads=cpu_threads())
    assert (got.cpu().numpy().view(np.uint32) == want).all(), p


def test_committed_cache_keeps_answers(O, pirmod):
    import torch

    from paper_2301_10904_amd import autotune as A

    r = A.load()
    if not r["applied"]:
        pytest.skip(f"committed cache does not apply here: {r['reason']}")
    try:
        for rows, dim, nkeys, prf in [(1 << 14, 16, 9, 0), (1 << 14, 64, 100, 1), (1 << 16, 64, 17, 0),
                                      (1 << 14, 16, 520, 1)]:
            n = rows.bit_length() - 1
            a = W.uniform_indices(rows, nkeys, nkeys)
            K0, _ = O.gen_batch(n, a, W.key_seeds(nkeys, nkeys), prf_id=prf)
            T = W.make_table(rows, dim, nkeys)
            got = pirmod.answer(torch.from_numpy(K0).cuda(), T.cuda(), prf=prf)
            torch.cuda.synchronize()
            want = O.answer_batch(K0, T.numpy().view(np.uint32), nthreads=cpu_threads())
            assert (got.cpu().numpy().view(np.uint32) == want).all(), (rows, dim, nkeys, prf)
    finally:
        pirmod.set_tuning([])


@pytest.mark.parametrize("q", [1, 2])
def test_tuned_small_groups_on_a_streamed_table(O, pirmod, q):
    """Tuned plans of 1 or 2 keys per workgroup over 3 keys on a 1 GiB table
    (2^22 x 64, AES-128, where one key alone takes the stream kernel): every
    key is answered (both servers' calls reconstruct T[alpha] for all three),
    and server 0's first and last keys match the oracle's point evaluation on
    a sparse copy of the table."""
    import torch

    rows, dim, nkeys, seed = 1 << 22, 64, 3, 71
    Td = W.make_table(rows, dim, seed, device="cuda")
    a = W.uniform_indices(rows, nkeys, seed)
    K0, K1 = O.gen_batch(22, a, W.key_seeds(nkeys, seed), prf_id=0)
    pirmod.set_tuning([entry(pirmod, 0, 22, kernel=2, keys_per_item=q)])
    try:
        p = pirmod.plan(nkeys, rows, dim)
        assert p["kernel"] == pirmod.KERNEL_SMALL_BATCH and p["keys_per_item"] == q, p
        o0 = pirmod.answer(torch.from_numpy(K0).cuda(), Td)
        o1 = pirmod.answer(torch.from_numpy(K1).cuda(), Td)
        assert pirmod.check_status() == pirmod.PIR_OK
        # the sparse copy: zero except 64 rows, so each key's answer is a sum of 64 point evaluations
        rng = np.random.default_rng(seed)
        keep = np.unique(np.concatenate([a, rng.integers(0, rows, 61)]))
        vals = rng.integers(0, 1 << 32, (len(keep), dim), dtype=np.uint64).astype(np.uint32)
        Sd = torch.zeros((rows, dim), dtype=torch.int32, device="cuda")
        Sd[torch.from_numpy(keep).cuda()] = torch.from_numpy(vals.view(np.int32)).cuda()
        s0 = pirmod.answer(torch.from_numpy(K0).cuda(), Sd)
        torch.cuda.synchronize()
    finally:
        pirmod.set_tuning([])
    rec = pirmod.reconstruct(o0.cpu().numpy().view(np.uint32).ravel(), o1.cpu().numpy().view(np.uint32).ravel())
    assert (rec.reshape(nkeys, dim) == W.table_rows_np(a, dim, seed)).all()
    got = s0.cpu().numpy().view(np.uint32)
    for k in (0, nkeys - 1):
        want = np.zeros(dim, np.uint64)
        for r, v in zip(keep, vals):
            want += np.uint64(O.eval_point(K0[k], int(r))) * v.astype(np.uint64)
        assert (got[k] == (want & 0xFFFFFFFF).astype(np.uint32)).all(), k
