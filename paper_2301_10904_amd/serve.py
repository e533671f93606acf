"""Request loop of a PIR server: admit queries as they arrive, batch them by
table, answer each batch with one pir_answer_multi call, report latency.

The tables stay resident in HBM.  A table is admitted only while the resident
total stays within an HBM budget; a request is admitted only while its
table's queue is below a bound (beyond it the server is overloaded and the
request is rejected).  A batch takes up to `max_batch` queued requests of every
table (fewer for large tables, so that a batch holds at most about
`max_batch_leaves` leaves of work), copies their keys (already in pinned host memory, as if just received)
to the device, runs the answer and copies the answers back, all on one side
stream; several batches may be in flight.  Completion is observed by polling
HIP events, and the latency of a request is completion time minus arrival
time.  This module only marshals data and orders work; every step of the
answer runs in the library's kernels.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import pir


@dataclass
class ServeStats:
    offered: int = 0
    admitted: int = 0
    rejected: int = 0
    completed: int = 0
    batches: int = 0
    wall_s: float = 0.0
    latencies_ms: list = field(default_factory=list)

    def summary(self) -> dict:
        lat = np.asarray(self.latencies_ms, dtype=np.float64)
        return {
            "offered": self.offered,
            "admitted": self.admitted,
            "rejected": self.rejected,
            "reject_rate": round(self.rejected / max(1, self.offered), 4),
            "completed": self.completed,
            "batches": self.batches,
            "sustained_qps": round(self.completed / self.wall_s, 1) if self.wall_s else 0.0,
            "p50_ms": round(float(np.percentile(lat, 50)), 3) if lat.size else None,
            "p99_ms": round(float(np.percentile(lat, 99)), 3) if lat.size else None,
        }


class PirServer:
    """Resident tables plus a batching request loop on one GPU stream."""

    def __init__(self, hbm_budget_bytes: int, max_batch: int = 1024, max_queue: int = 4096,
                 max_inflight: int = 3, max_batch_leaves: int = 1 << 30, device="cuda:0",
                 prf=pir.PRF_AES128):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.budget = int(hbm_budget_bytes)
        self.max_batch = int(max_batch)
        self.max_queue = int(max_queue)
        self.max_inflight = int(max_inflight)
        # work cap of one batch, in leaves (keys x table rows): keys of large
        # tables enter in slices so a batch stays short and small tables keep
        # flowing under overload
        self.max_batch_leaves = int(max_batch_leaves)
        self.prf = pir.prf_id(prf)  # the PRF every served key uses
        self.tables = []  # (tensor, rows, dim, n)
        self.resident_bytes = 0
        self.stream = torch.cuda.Stream(device=self.device)

    # -- tables -----------------------------------------------------------------
    def admit_table(self, table) -> int:
        """Register a resident device table; returns its id or -1 if over budget.

        The table may still be being written by work queued on the caller's
        current stream: the server stream is made to wait for that work."""
        nbytes = table.numel() * table.element_size()
        if self.resident_bytes + nbytes > self.budget:
            return -1
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        self.resident_bytes += nbytes
        rows, dim = table.shape
        self.tables.append((table, rows, dim, pir.log_domain(rows)))
        return len(self.tables) - 1

    # -- loop ---------------------------------------------------------------------
    def run(self, arrivals_s: np.ndarray, table_ids: np.ndarray, key_pool: list,
            key_index: np.ndarray, stride: int, check=None) -> ServeStats:
        """Serve requests i (arrival arrivals_s[i], table table_ids[i], key
        key_pool[table_ids[i]][key_index[i]]) in real time.  `check(table,
        key_index, answer_row)` is called on a sample of completed requests
        after the run."""
        torch = self.torch
        # anything the caller queued before the run (tables, keys) comes first
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        T = len(self.tables)
        n_req = len(arrivals_s)
        st = ServeStats(offered=n_req)
        dims = [t[2] for t in self.tables]
        # all keys in one host array; request i uses row pool_row[i]
        pool = np.concatenate(key_pool)
        base = np.cumsum([0] + [len(k) for k in key_pool])[:-1]
        pool_row = base[table_ids] + key_index
        # per-table FIFO queues of request ids (array + head/tail)
        q_ids = [np.empty(self.max_queue, dtype=np.int64) for _ in range(T)]
        q_head = [0] * T
        q_len = [0] * T
        cap_keys = self.max_batch * T
        slots = []
        for _ in range(self.max_inflight):
            slots.append({
                "hkeys": torch.empty((cap_keys, stride), dtype=torch.uint8, pin_memory=True),
                "dkeys": torch.empty((cap_keys, stride), dtype=torch.uint8, device=self.device),
                "dout": torch.empty(cap_keys * max(dims), dtype=torch.int32, device=self.device),
                "hout": torch.empty(cap_keys * max(dims), dtype=torch.int32, pin_memory=True),
                "event": torch.cuda.Event(), "reqs": None, "counts": None,
            })
        free = deque(range(self.max_inflight))
        inflight = deque()
        samples = []
        lat_chunks = []
        nxt = 0
        t0 = time.perf_counter()
        while st.completed + st.rejected < n_req:
            now = time.perf_counter() - t0
            # admit everything that has arrived
            if nxt < n_req and arrivals_s[nxt] <= now:
                end = int(np.searchsorted(arrivals_s, now, side="right"))
                for i in range(nxt, end):
                    t = int(table_ids[i])
                    if q_len[t] < self.max_queue:
                        q_ids[t][(q_head[t] + q_len[t]) % self.max_queue] = i
                        q_len[t] += 1
                        st.admitted += 1
                    else:
                        st.rejected += 1
                nxt = end
            # retire finished batches
            while inflight and slots[inflight[0]]["event"].query():
                s = inflight.popleft()
                done = time.perf_counter() - t0
                slot = slots[s]
                reqs = slot["reqs"]
                lat_chunks.append((done - arrivals_s[reqs]) * 1e3)
                st.completed += len(reqs)
                if check is not None and len(samples) < 64:
                    hout = slot["hout"].numpy().view(np.uint32)
                    off, k = 0, 0
                    for t, c in enumerate(slot["counts"]):
                        if c:
                            samples.append((t, int(key_index[reqs[k]]), hout[off:off + dims[t]].copy()))
                        off += c * dims[t]
                        k += c
                free.append(s)
            # launch a batch if a slot is free and work is queued
            if free and any(q_len):
                s = free.popleft()
                slot = slots[s]
                parts, counts = [], []
                for t in range(T):
                    by_work = max(16, (self.max_batch_leaves >> self.tables[t][3]) // 16 * 16)
                    take = min(q_len[t], self.max_batch, by_work)
                    counts.append(take)
                    if take:
                        idx = (q_head[t] + np.arange(take)) % self.max_queue
                        parts.append(q_ids[t][idx])
                        q_head[t] = (q_head[t] + take) % self.max_queue
                        q_len[t] -= take
                reqs = np.concatenate(parts)
                nk = len(reqs)
                slot["hkeys"].numpy()[:nk] = pool[pool_row[reqs]]
                total_words = sum(c * d for c, d in zip(counts, dims))
                with torch.cuda.stream(self.stream):
                    slot["dkeys"][:nk].copy_(slot["hkeys"][:nk], non_blocking=True)
                    pir.answer_multi([t[0] for t in self.tables], counts, slot["dkeys"][:nk],
                                     out=slot["dout"][:total_words], stream=self.stream, prf=self.prf)
                    slot["hout"][:total_words].copy_(slot["dout"][:total_words], non_blocking=True)
                    slot["event"].record(self.stream)
                slot["reqs"], slot["counts"] = reqs, counts
                inflight.append(s)
                st.batches += 1
            elif not inflight and nxt < n_req:
                # idle until the next arrival
                wait = arrivals_s[nxt] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.001))
        self.stream.synchronize()
        st.wall_s = time.perf_counter() - t0
        st.latencies_ms = np.concatenate(lat_chunks).tolist() if lat_chunks else []
        if check is not None:
            for t, ki, row in samples:
                check(t, ki, row)
        return st
