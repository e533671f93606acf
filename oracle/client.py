"""Client-side planning of the paper's batch retrieval (section 4), for the
oracle: which DPF queries a client issues for a set of wanted indices.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

Partial batch retrieval (section 4.1): the table of L rows is cut into bins of
I consecutive rows and the client issues exactly one query per bin.  A bin
that holds one or more wanted indices serves one of them; the others that fall
into it are dropped.  A bin that holds none gets a dummy query.

Hot/full split (section 4.2): a hot table holds the top-K rows; the client
issues exactly Q_hot queries to it and Q_full to the full table.  A wanted
index found in the hot map is a hot request, any other a full request;
requests beyond a table's budget are dropped and missing ones are filled with
dummy queries.

Readings (the paper leaves these open): within a bin, and within a budget,
requests are taken in the client's order (first come, first served); a dummy
query is a DPF for index 0 of its table; an over-budget hot request is
dropped, not moved to the full table.
"""
from __future__ import annotations


def pbr_plan(indices, rows: int, bin_log: int):
    """Return (alphas, served, dropped).

    alphas[b]  the in-bin index queried in bin b (0 for a dummy query)
    served[b]  the wanted index bin b retrieves, or None for a dummy
    dropped    wanted indices that shared a bin with an earlier one
    """
    size = 1 << bin_log
    n_bins = (rows + size - 1) // size
    alphas = [0] * n_bins
    served = [None] * n_bins
    dropped = []
    for x in indices:
        x = int(x)
        if not 0 <= x < rows:
            raise ValueError(f"index {x} outside the table")
        b = x // size
        if served[b] is None:
            served[b] = x
            alphas[b] = x - b * size
        else:
            dropped.append(x)
    return alphas, served, dropped


def hot_full_plan(indices, hot_map: dict, q_hot: int, q_full: int):
    """Return (hot_alphas, full_alphas, served_hot, served_full, dropped).

    hot_alphas   q_hot rows of the hot table to query (dummies are 0)
    full_alphas  q_full rows of the full table to query (dummies are 0)
    served_hot   for each hot query, the wanted index it retrieves, or None
    served_full  the same for the full queries
    dropped      wanted indices beyond their table's budget
    """
    hot_alphas, full_alphas, served_hot, served_full, dropped = [], [], [], [], []
    for x in indices:
        x = int(x)
        if x in hot_map:
            if len(hot_alphas) < q_hot:
                hot_alphas.append(int(hot_map[x]))
                served_hot.append(x)
            else:
                dropped.append(x)
        else:
            if len(full_alphas) < q_full:
                full_alphas.append(x)
                served_full.append(x)
            else:
                dropped.append(x)
    while len(hot_alphas) < q_hot:
        hot_alphas.append(0)
        served_hot.append(None)
    while len(full_alphas) < q_full:
        full_alphas.append(0)
        served_full.append(None)
    return hot_alphas, full_alphas, served_hot, served_full, dropped
