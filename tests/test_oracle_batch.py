"""Pins for the oracle's batch retrieval (paper section 4): the server side of
partial batch retrieval (one DPF per bin of I rows) and the client planning of
partial batch retrieval and of the hot/full table split.

Fixed by the paper or by mathematics, not by the oracle itself:
  - after both servers answer, bin b of a client reconstructs T[b I + alpha_b]
    (the closed form of a DPF-PIR query over the bin);
  - the per-server answer of a bin equals an independent numpy product of the
    key's full evaluation with the bin's rows;
  - with one bin spanning the table, the answer is the plain answer;
  - the plans issue exactly one query per bin (or exactly Q_hot and Q_full
    queries), serve at most one wanted index per bin, and every wanted index is
    either served or dropped.
"""
import numpy as np
import pytest

from oracle.client import hot_full_plan, pbr_plan
from test_oracle_dpf import numpy_answer, seed_for


def table(rows, dim, seed):
    rng = np.random.default_rng([rows, dim, seed])
    return rng.integers(0, 2**32, (rows, dim), dtype=np.uint64).astype(np.uint32)


def bin_keys(O, alphas, bin_log, n_clients, seed, prf_id=0):
    """Both parties' keys, client-major: [n_clients * n_bins, key_size]."""
    k0, k1 = [], []
    for c in range(n_clients):
        for b, a in enumerate(alphas[c]):
            x0, x1 = O.gen(bin_log, int(a), 1, seed_for(seed, c, b), prf_id=prf_id)
            k0.append(x0)
            k1.append(x1)
    return np.stack(k0), np.stack(k1)


@pytest.mark.parametrize("rows,dim,bin_log,n_clients", [
    (256, 4, 5, 2), (200, 3, 6, 3), (1000, 8, 7, 1), (64, 2, 3, 4), (130, 5, 7, 2)])
def test_bins_reconstruct_closed_form(O, rows, dim, bin_log, n_clients):
    """Every bin of every client reconstructs T[b I + alpha_b], ragged last bin
    included (rows not a multiple of I)."""
    T = table(rows, dim, 1)
    size = 1 << bin_log
    n_bins = -(-rows // size)
    rng = np.random.default_rng([rows, bin_log, n_clients])
    alphas = [[int(rng.integers(0, min(size, rows - b * size))) for b in range(n_bins)]
              for _ in range(n_clients)]
    k0, k1 = bin_keys(O, alphas, bin_log, n_clients, rows)
    a0 = O.answer_bins(k0, T, bin_log, n_clients, nthreads=4)
    a1 = O.answer_bins(k1, T, bin_log, n_clients, nthreads=4)
    for c in range(n_clients):
        for b in range(n_bins):
            got = O.reconstruct(a0[c, b], a1[c, b])
            assert (got == T[b * size + alphas[c][b]]).all(), (c, b)


def test_bins_per_server_independent_product(O):
    rows, dim, bin_log = 300, 6, 6
    T = table(rows, dim, 2)
    size, n_bins = 1 << bin_log, -(-rows // (1 << bin_log))
    alphas = [[(7 * b + 3) % min(size, rows - b * size) for b in range(n_bins)] for _ in range(2)]
    k0, _ = bin_keys(O, alphas, bin_log, 2, 9)
    got = O.answer_bins(k0, T, bin_log, 2, nthreads=3)
    for c in range(2):
        for b in range(n_bins):
            key = k0[c * n_bins + b]
            want = numpy_answer(O.eval_full(key), T[b * size:(b + 1) * size])
            assert (got[c, b] == want).all(), (c, b)


def test_one_bin_is_the_plain_answer(O):
    rows, dim, n = 100, 5, 7
    T = table(rows, dim, 3)
    k0, _ = O.gen(n, 42, 1, seed_for(3))
    got = O.answer_bins(k0[None, :], T, n, 1)
    assert (got[0, 0] == O.answer(k0, T)).all()


def test_bins_chacha_keys(O):
    rows, dim, bin_log = 96, 4, 5
    T = table(rows, dim, 4)
    alphas = [[1, 30, 17]]
    k0, k1 = bin_keys(O, alphas, bin_log, 1, 4, prf_id=1)
    a0 = O.answer_bins(k0, T, bin_log, 1)
    a1 = O.answer_bins(k1, T, bin_log, 1)
    for b, a in enumerate(alphas[0]):
        assert (O.reconstruct(a0[0, b], a1[0, b]) == T[32 * b + a]).all()


def test_bins_reject_wrong_domain(O):
    T = table(64, 2, 5)
    k0, _ = O.gen(6, 3, 1, seed_for(5))  # n = 6, but bins of 2^5 rows
    with pytest.raises(ValueError):
        O.answer_bins(np.stack([k0, k0]), T, 5, 1)


def test_pbr_plan_invariants():
    rng = np.random.default_rng(6)
    rows, bin_log = 1000, 6
    size, n_bins = 64, 16
    for trial in range(50):
        wanted = rng.integers(0, rows, int(rng.integers(0, 40)))
        alphas, served, dropped = pbr_plan(wanted, rows, bin_log)
        assert len(alphas) == len(served) == n_bins
        assert sorted([x for x in served if x is not None] + dropped) == sorted(int(x) for x in wanted)
        for b, x in enumerate(served):
            if x is None:
                assert alphas[b] == 0
            else:
                assert x // size == b and alphas[b] == x - b * size
                # the first wanted index of the bin is the one served
                first = next(int(w) for w in wanted if int(w) // size == b)
                assert x == first
        for x in dropped:
            assert served[x // size] is not None
        assert all(0 <= a < size for a in alphas)


def test_pbr_plan_spread_indices_are_all_served():
    """The best case of section 4.1: L/I wanted indices in distinct bins are
    all retrieved by L/I queries."""
    rows, bin_log = 512, 5
    wanted = [b * 32 + (b * 7) % 32 for b in range(16)]
    alphas, served, dropped = pbr_plan(wanted[::-1], rows, bin_log)
    assert dropped == [] and sorted(served) == sorted(wanted)


def test_hot_full_plan_fixed_counts_and_dummies():
    hot_map = {10: 0, 20: 1, 30: 2, 40: 3}
    rng = np.random.default_rng(7)
    for trial in range(50):
        wanted = rng.choice([10, 20, 30, 40, 5, 6, 7, 8, 9, 11], int(rng.integers(0, 9)))
        q_hot, q_full = 2, 3
        ha, fa, sh, sf, dropped = hot_full_plan(wanted, hot_map, q_hot, q_full)
        assert len(ha) == len(sh) == q_hot and len(fa) == len(sf) == q_full
        served = [x for x in sh + sf if x is not None]
        assert sorted(served + dropped) == sorted(int(x) for x in wanted)
        for a, x in zip(ha, sh):
            assert (x is None and a == 0) or (x in hot_map and a == hot_map[x])
        for a, x in zip(fa, sf):
            assert (x is None and a == 0) or (x not in hot_map and a == x)
        n_hot = sum(1 for x in wanted if int(x) in hot_map)
        n_full = len(wanted) - n_hot
        assert len(dropped) == max(0, n_hot - q_hot) + max(0, n_full - q_full)


def test_hot_full_reconstructs_through_both_tables(O):
    """A client plan over a hot table (a gather of the full table's hottest
    rows) and the full table retrieves every served index exactly."""
    rows, dim = 200, 4
    T = table(rows, dim, 8)
    hot_rows = [150, 3, 77, 199, 42, 8, 120, 64]
    hot_map = {x: i for i, x in enumerate(hot_rows)}
    H = T[hot_rows]
    wanted = [3, 5, 150, 199, 11, 64, 13]
    ha, fa, sh, sf, dropped = hot_full_plan(wanted, hot_map, 3, 3)
    assert dropped == [64]  # four hot requests for three hot queries; the three others fit
    for tab, alphas, served, n in ((H, ha, sh, 3), (T, fa, sf, 8)):
        for i, (a, x) in enumerate(zip(alphas, served)):
            k0, k1 = O.gen(n, a, 1, seed_for(8, n, i))
            r = O.reconstruct(O.answer(k0, tab), O.answer(k1, tab))
            assert (r == (T[x] if x is not None else tab[0])).all()
