"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds none of the method's arithmetic: it only draws the inputs
(embedding tables, query indices, per-query Gen seeds, batch sizes, arrival
times) that both the GPU path and the CPU oracle consume.

Tables are counter-based, so any row can be regenerated on its own (the
oracle checks samples of tables too large to copy to the host):
    T[j][k] = low 32 bits of splitmix64 at counter j*D + k under `seed`,
with splitmix64 as published by S. Vigna (state advanced by the golden-ratio
increment 0x9E3779B97F4A7C15, output mix with shifts 30/27/31 and multipliers
0xBF58476D1CE4E5B9 / 0x94D049BB133111EB).
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
M64 = (1 << 64) - 1


def _i64(x: int) -> int:
    x &= M64
    return x - (1 << 64) if x >> 63 else x


def _splitmix_torch(idx, seed: int):
    """splitmix64 output for counters `idx` (int64 tensor); wrapping int64 math."""
    import torch

    z = idx.add(1).mul_(_i64(GAMMA)).add_(_i64(seed))
    z = z.bitwise_xor_(torch.bitwise_and(z >> 30, (1 << 34) - 1)).mul_(_i64(MIX1))
    z = z.bitwise_xor_(torch.bitwise_and(z >> 27, (1 << 37) - 1)).mul_(_i64(MIX2))
    z = z.bitwise_xor_(torch.bitwise_and(z >> 31, (1 << 33) - 1))
    return z


def splitmix64_scalar(counter: int, seed: int) -> int:
    z = (seed + (counter + 1) * GAMMA) & M64
    z = ((z ^ (z >> 30)) * MIX1) & M64
    z = ((z ^ (z >> 27)) * MIX2) & M64
    return z ^ (z >> 31)


def make_table(rows: int, dim: int, seed: int, device="cpu", out=None, chunk_elems: int = 1 << 25):
    """int32 tensor [rows, dim] holding the uint32 table bits (see module doc)."""
    import torch

    if out is None:
        out = torch.empty((rows, dim), dtype=torch.int32, device=device)
    flat = out.view(-1)
    total = rows * dim
    for start in range(0, total, chunk_elems):
        end = min(total, start + chunk_elems)
        idx = torch.arange(start, end, dtype=torch.int64, device=out.device)
        z = _splitmix_torch(idx, seed) & 0xFFFFFFFF
        z = torch.where(z >= (1 << 31), z - (1 << 32), z)
        flat[start:end] = z.to(torch.int32)
        del idx, z
    return out


def table_rows_np(row_ids, dim: int, seed: int) -> np.ndarray:
    """Selected rows of make_table(..., seed) as uint32 [len(row_ids), dim] (CPU)."""
    import torch

    row_ids = np.asarray(row_ids, dtype=np.int64).reshape(-1)
    idx = (torch.from_numpy(row_ids)[:, None] * dim + torch.arange(dim, dtype=torch.int64)[None, :])
    z = _splitmix_torch(idx.reshape(-1), seed) & 0xFFFFFFFF
    return z.numpy().astype(np.uint32).reshape(len(row_ids), dim)


def uniform_indices(rows: int, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng([seed, 0x11])
    return rng.integers(0, rows, count, dtype=np.int64)


def zipf_indices(rows: int, count: int, seed: int, s: float = 1.05) -> np.ndarray:
    """Bounded Zipf over [0, rows): P(row r) proportional to (r + 1)^-s, by inverse CDF."""
    rng = np.random.default_rng([seed, 0x21])
    w = np.arange(1, rows + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    u = rng.random(count) * cdf[-1]
    return np.minimum(np.searchsorted(cdf, u, side="right"), rows - 1).astype(np.int64)


def row_permutation(rows: int, seed: int) -> np.ndarray:
    """A seeded permutation of [0, rows): maps popularity ranks to rows, so that
    popular rows are scattered over the table instead of leading it."""
    return np.random.default_rng([seed, 0x61]).permutation(rows).astype(np.int64)


def key_seeds(count: int, seed: int) -> np.ndarray:
    """One 16-byte Gen seed per query, [count, 16] uint8."""
    rng = np.random.default_rng([seed, 0x31])
    return rng.integers(0, 256, (count, 16), dtype=np.uint8)


def ragged_batch_sizes(n_tables: int, seed: int, lo: int = 32, hi: int = 1024) -> np.ndarray:
    rng = np.random.default_rng([seed, 0x41])
    return rng.integers(lo, hi + 1, n_tables, dtype=np.int64)


def poisson_arrivals(rate_per_s: float, count: int, seed: int) -> np.ndarray:
    """Arrival times in seconds of a Poisson process (exponential gaps)."""
    rng = np.random.default_rng([seed, 0x51])
    return np.cumsum(rng.exponential(1.0 / rate_per_s, count))
