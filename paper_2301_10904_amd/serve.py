"""Request loop of a PIR server: admit queries as they arrive, batch them by
table, answer each batch with one pir_answer_multi call, report latency.

The tables stay resident in HBM.  A table is admitted only while the resident
total stays within an HBM budget.  A request costs 2^n leaf evaluations on
its table (2^n >= rows); it is admitted only while the work already queued,
with it, can be answered within `queue_budget_s` at the service rate the
server has measured (leaves per second of GPU time, from the batches it has
completed), and while its table's queue has room (`max_queue`).  Otherwise the
server is overloaded and the request is rejected on arrival, so the latency of
admitted requests stays near the budget whatever the offered load.

A batch takes up to `max_batch` queued requests of every table (fewer for
large tables, so that a batch holds at most about `max_batch_leaves` leaves of
work per table), copies their keys (already in pinned host memory, as if just
received) to the device, runs the answer and copies the answers back, all on
one side stream; several batches may be in flight.  Completion is observed by
polling HIP events, and the latency of a request is completion time minus
arrival time.  This module only marshals data and orders work; every step of
the answer runs in the library's kernels.
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
    rate_leaves_per_s: float = 0.0
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
            "service_rate_gleaves_per_s": round(self.rate_leaves_per_s / 1e9, 2),
        }


class WorkQueues:
    """Per-table FIFO rings of request ids with a bound on the queued work.

    `cost[t]` is the work of one request on table t (its leaves).  `admit`
    takes the requests that arrived since the last call, in arrival order,
    and admits the longest prefix whose work fits under `work_limit` (the
    rest of the batch of arrivals is rejected: they arrived within one turn
    of the loop, when the queue was already full); a table whose ring is full
    rejects its excess.  Host-only bookkeeping, no GPU."""

    def __init__(self, cost, capacity: int):
        self.cost = np.asarray(cost, dtype=np.float64)
        self.cap = int(capacity)
        T = len(self.cost)
        self.ring = [np.empty(self.cap, dtype=np.int64) for _ in range(T)]
        self.head = [0] * T
        self.length = [0] * T
        self.work = 0.0  # queued leaves

    def admit(self, ids: np.ndarray, tids: np.ndarray, work_limit: float) -> int:
        """Queue what fits of requests `ids` (tables `tids`); returns how many were admitted."""
        if len(ids) == 0:
            return 0
        c = self.cost[tids]
        fits = np.cumsum(c) <= work_limit - self.work
        admitted = 0
        for t in range(len(self.cost)):
            mine = ids[fits & (tids == t)]
            mine = mine[: self.cap - self.length[t]]
            k = len(mine)
            if k:
                pos = (self.head[t] + self.length[t] + np.arange(k)) % self.cap
                self.ring[t][pos] = mine
                self.length[t] += k
                self.work += k * self.cost[t]
                admitted += k
        return admitted

    def take(self, t: int, k: int) -> np.ndarray:
        """Dequeue up to k requests of table t, oldest first."""
        k = min(k, self.length[t])
        idx = (self.head[t] + np.arange(k)) % self.cap
        out = self.ring[t][idx].copy()
        self.head[t] = (self.head[t] + k) % self.cap
        self.length[t] -= k
        self.work -= k * self.cost[t]
        return out

    def any(self) -> bool:
        return any(self.length)


class PirServer:
    """Resident tables plus a batching request loop on one GPU stream."""

    def __init__(self, hbm_budget_bytes: int, max_batch: int = 1024, max_queue: int = 4096,
                 max_inflight: int = 3, max_batch_leaves: int = 1 << 30, device="cuda:0",
                 prf=pir.PRF_AES128, queue_budget_s: float | None = 0.1):
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
        # admission bound: queued work drained within this many seconds at the
        # measured service rate (None: bounded by max_queue only)
        self.queue_budget_s = queue_budget_s
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
        table_ids = np.asarray(table_ids)
        st = ServeStats(offered=n_req)
        dims = [t[2] for t in self.tables]
        leaves = [float(1 << t[3]) for t in self.tables]
        # all keys in one host array; request i uses row pool_row[i]
        pool = np.concatenate(key_pool)
        base = np.cumsum([0] + [len(k) for k in key_pool])[:-1]
        pool_row = base[table_ids] + key_index
        queues = WorkQueues(leaves, self.max_queue)
        per_batch = [min(self.max_batch, max(16, (self.max_batch_leaves >> t[3]) // 16 * 16)) for t in self.tables]
        cap_keys = sum(per_batch)
        slots = []
        for _ in range(self.max_inflight):
            slots.append({
                "hkeys": torch.empty((cap_keys, stride), dtype=torch.uint8, pin_memory=True),
                "dkeys": torch.empty((cap_keys, stride), dtype=torch.uint8, device=self.device),
                "dout": torch.empty(cap_keys * max(dims), dtype=torch.int32, device=self.device),
                "hout": torch.empty(cap_keys * max(dims), dtype=torch.int32, pin_memory=True),
                "start": torch.cuda.Event(enable_timing=True), "event": torch.cuda.Event(enable_timing=True),
                "reqs": None, "counts": None, "leaves": 0.0,
            })
        free = deque(range(self.max_inflight))
        inflight = deque()
        samples = []
        lat_chunks = []
        rate = 0.0  # measured service rate, leaves per second of GPU time
        nxt = 0
        t0 = time.perf_counter()
        while st.completed + st.rejected < n_req:
            now = time.perf_counter() - t0
            # admit everything that has arrived
            if nxt < n_req and arrivals_s[nxt] <= now:
                end = int(np.searchsorted(arrivals_s, now, side="right"))
                ids = np.arange(nxt, end)
                limit = self.queue_budget_s * rate if (self.queue_budget_s and rate > 0) else np.inf
                k = queues.admit(ids, table_ids[ids], limit)
                st.admitted += k
                st.rejected += len(ids) - k
                nxt = end
            # retire finished batches
            while inflight and slots[inflight[0]]["event"].query():
                s = inflight.popleft()
                done = time.perf_counter() - t0
                slot = slots[s]
                reqs = slot["reqs"]
                lat_chunks.append((done - arrivals_s[reqs]) * 1e3)
                st.completed += len(reqs)
                gpu_s = slot["start"].elapsed_time(slot["event"]) * 1e-3
                if gpu_s > 0:
                    r = slot["leaves"] / gpu_s
                    rate = r if rate == 0 else 0.7 * rate + 0.3 * r
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
            if free and queues.any():
                s = free.popleft()
                slot = slots[s]
                parts = [queues.take(t, per_batch[t]) for t in range(T)]
                counts = [len(p) for p in parts]
                reqs = np.concatenate(parts)
                nk = len(reqs)
                slot["hkeys"].numpy()[:nk] = pool[pool_row[reqs]]
                total_words = sum(c * d for c, d in zip(counts, dims))
                with torch.cuda.stream(self.stream):
                    slot["start"].record(self.stream)
                    slot["dkeys"][:nk].copy_(slot["hkeys"][:nk], non_blocking=True)
                    pir.answer_multi([t[0] for t in self.tables], counts, slot["dkeys"][:nk],
                                     out=slot["dout"][:total_words], stream=self.stream, prf=self.prf)
                    slot["hout"][:total_words].copy_(slot["dout"][:total_words], non_blocking=True)
                    slot["event"].record(self.stream)
                slot["reqs"], slot["counts"] = reqs, counts
                slot["leaves"] = sum(c * lv for c, lv in zip(counts, leaves))
                inflight.append(s)
                st.batches += 1
            elif not inflight and nxt < n_req:
                # idle until the next arrival
                wait = arrivals_s[nxt] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.001))
        self.stream.synchronize()
        st.wall_s = time.perf_counter() - t0
        st.rate_leaves_per_s = rate
        st.latencies_ms = np.concatenate(lat_chunks).tolist() if lat_chunks else []
        if check is not None:
            for t, ki, row in samples:
                check(t, ki, row)
        return st
