"""Admission bookkeeping of the serving loop (host only, no GPU).

WorkQueues keeps per-table FIFO rings of request ids and the total queued
work; a batch of arrivals is admitted as its longest prefix that fits under
the work limit, and a table whose ring is full rejects its excess.  Checked
against a plain deque model on random traffic.
"""
from collections import deque

import numpy as np

from paper_2301_10904_amd.serve import WorkQueues


def test_fifo_per_table():
    q = WorkQueues([1.0, 2.0], capacity=8)
    ids = np.arange(6)
    tids = np.array([0, 1, 0, 1, 1, 0])
    assert q.admit(ids, tids, np.inf) == 6
    assert q.work == 3 * 1.0 + 3 * 2.0
    assert q.take(1, 2).tolist() == [1, 3]
    assert q.take(0, 5).tolist() == [0, 2, 5]
    assert q.take(1, 5).tolist() == [4]
    assert not q.any() and q.work == 0.0


def test_work_limit_admits_a_prefix():
    q = WorkQueues([1.0, 10.0], capacity=64)
    ids = np.arange(5)
    tids = np.array([0, 1, 0, 0, 0])  # costs 1, 10, 1, 1, 1
    # limit 12: 1 + 10 + 1 = 12 fits, the fourth (13) does not, nor anything after it
    assert q.admit(ids, tids, 12.0) == 3
    assert q.length == [2, 1] and q.work == 12.0
    # queued work counts against the next arrivals
    assert q.admit(np.array([5]), np.array([0]), 12.0) == 0
    q.take(1, 1)
    assert q.admit(np.array([6, 7]), np.array([0, 0]), 12.0) == 2
    assert q.take(0, 10).tolist() == [0, 2, 6, 7]


def test_full_ring_rejects_its_excess():
    q = WorkQueues([1.0, 1.0], capacity=3)
    ids = np.arange(6)
    tids = np.array([0, 0, 0, 0, 1, 0])
    assert q.admit(ids, tids, np.inf) == 4  # table 0 keeps its first three, table 1 its one
    assert q.take(0, 9).tolist() == [0, 1, 2]
    assert q.take(1, 9).tolist() == [4]


def test_random_traffic_matches_a_deque_model():
    rng = np.random.default_rng(3)
    cost = [1.0, 4.0, 16.0]
    cap = 7
    q = WorkQueues(cost, capacity=cap)
    model = [deque() for _ in cost]
    nxt = 0
    for _ in range(2000):
        n = int(rng.integers(0, 6))
        ids = np.arange(nxt, nxt + n)
        tids = rng.integers(0, 3, n)
        nxt += n
        limit = float(rng.choice([np.inf, 40.0, 80.0]))
        work = sum(len(m) * c for m, c in zip(model, cost))
        want = 0
        cum = 0.0
        for i, t in zip(ids, tids):
            cum += cost[t]
            if work + cum > limit:  # the rest of this batch is rejected
                break
            if len(model[t]) < cap:
                model[t].append(int(i))
                want += 1
        assert q.admit(ids, tids, limit) == want
        for t in range(3):
            k = int(rng.integers(0, 4))
            got = q.take(t, k).tolist()
            exp = [model[t].popleft() for _ in range(min(k, len(model[t])))]
            assert got == exp
        assert q.length == [len(m) for m in model]
        assert abs(q.work - sum(len(m) * c for m, c in zip(model, cost))) < 1e-9
