"""Client side of the paper's batch retrieval (section 4): which DPF queries a
client sends for a set of wanted table indices, and how it reads the answers.

Partial batch retrieval (section 4.1) cuts a table of L rows into bins of
I = 2^m rows and sends exactly one query per bin: a bin holding wanted indices
serves the first of them and drops the rest; a bin holding none gets a dummy
query (index 0 of the bin), so the servers see the same number of queries
whatever is wanted.  The hot/full split (section 4.2) sends exactly Q_hot
queries to a small hot table (a gather of the most frequently used rows, found
through a client-side map) and Q_full to the full table; requests beyond a
table's budget are dropped, missing ones are dummy queries (index 0).

Keys come from the library's Gen (``pir.gen``); the servers' side is
``pir.answer_bins`` / ``pir.answer_multi``.  Plans are computed with numpy.
"""
from __future__ import annotations

import numpy as np

from . import pir


def pbr_plan(indices, rows: int, bin_log: int):
    """(alphas, served, dropped) for partial batch retrieval.

    alphas  uint64 [n_bins]: the in-bin index each bin's query asks for
    served  int64 [n_bins]: the wanted index a bin retrieves, -1 for a dummy
    dropped int64 array of wanted indices that lost their bin to an earlier one
    """
    idx = np.asarray(indices, dtype=np.int64).reshape(-1)
    if idx.size and (idx.min() < 0 or idx.max() >= rows):
        raise ValueError("wanted index outside the table")
    nb = pir.n_bins(rows, bin_log)
    bins = idx >> bin_log
    uniq, first = np.unique(bins, return_index=True)  # first occurrence per bin
    served = np.full(nb, -1, dtype=np.int64)
    served[uniq] = idx[first]
    alphas = np.zeros(nb, dtype=np.uint64)
    alphas[uniq] = (idx[first] - (uniq << bin_log)).astype(np.uint64)
    keep = np.zeros(idx.size, dtype=bool)
    keep[first] = True
    return alphas, served, idx[~keep]


def pbr_keys(indices, rows: int, bin_log: int, seeds=None, prf=pir.PRF_AES128):
    """Keys for both servers: (keys0, keys1) uint8 [n_bins, key_size(bin_log)],
    plus (served, dropped) of the plan.  seeds: optional [n_bins, 16]."""
    alphas, served, dropped = pbr_plan(indices, rows, bin_log)
    K0, K1 = pir.gen_batch(bin_log, alphas, seeds, prf=prf)
    return K0, K1, served, dropped


def pbr_read(a0, a1, served):
    """Entries retrieved by one client: {wanted index: row (uint32 [dim])}
    from both servers' answers [n_bins, dim] of that client."""
    rec = (np.asarray(a0).view(np.uint32).astype(np.uint64) +
           np.asarray(a1).view(np.uint32)) & 0xFFFFFFFF
    rec = rec.astype(np.uint32)
    return {int(x): rec[b] for b, x in enumerate(served) if x >= 0}


def hot_full_plan(indices, hot_of, q_hot: int, q_full: int):
    """(hot_alphas, full_alphas, served_hot, served_full, dropped).

    hot_of      int64 array over the full table: hot row of each index, -1 if cold
    hot_alphas  uint64 [q_hot]; full_alphas uint64 [q_full] (dummies are 0)
    served_*    int64 arrays of the wanted index each query retrieves, -1 for dummies
    """
    idx = np.asarray(indices, dtype=np.int64).reshape(-1)
    hot_row = np.asarray(hot_of)[idx] if idx.size else np.zeros(0, np.int64)
    is_hot = hot_row >= 0
    hot_pos = np.flatnonzero(is_hot)
    cold_pos = np.flatnonzero(~is_hot)
    take_h, take_c = hot_pos[:q_hot], cold_pos[:q_full]
    served_hot = np.full(q_hot, -1, np.int64)
    served_hot[:take_h.size] = idx[take_h]
    served_full = np.full(q_full, -1, np.int64)
    served_full[:take_c.size] = idx[take_c]
    hot_alphas = np.zeros(q_hot, np.uint64)
    hot_alphas[:take_h.size] = hot_row[take_h].astype(np.uint64)
    full_alphas = np.zeros(q_full, np.uint64)
    full_alphas[:take_c.size] = idx[take_c].astype(np.uint64)
    drop = np.sort(np.concatenate([hot_pos[q_hot:], cold_pos[q_full:]]))
    return hot_alphas, full_alphas, served_hot, served_full, idx[drop]


def hot_rows_by_frequency(counts, k: int):
    """The k most frequent rows (ties to the lower index) and the map from a
    full-table index to its hot row (-1 if not hot): the hot table is
    T[hot_rows], built once ahead of serving from access statistics."""
    counts = np.asarray(counts)
    order = np.lexsort((np.arange(counts.size), -counts))
    hot_rows = np.sort(order[:k])
    hot_of = np.full(counts.size, -1, np.int64)
    hot_of[hot_rows] = np.arange(k)
    return hot_rows, hot_of
