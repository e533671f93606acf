"""CPU oracle for the two-server DPF-PIR server path.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(the HIP library and its Python binding) shares no code with it.

The arithmetic lives in plain C (``aes_ref.c``: FIPS-197 AES-128;
``chacha_ref.c``: RFC 8439 ChaCha20; ``dpf_ref.c``: Gen, the Eq. (p1)-(p3)
node recurrence of paper section 3.1 with either PRF, the answer T x Eval
mod 2^32 and the client's reconstruction).  This module
only builds that library with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SOURCES = ("aes_ref.c", "chacha_ref.c", "dpf_ref.c")
LIB_PATH = HERE / "liboracle.so"

_lib = None


def build(out: Path | None = None, src_dir: Path | None = None, extra=()) -> Path:
    """Compile the oracle with gcc into a shared library (C11, -O2)."""
    out = Path(out) if out else LIB_PATH
    src_dir = Path(src_dir) if src_dir else HERE
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-pthread", *extra, "-o", str(out)] + [str(src_dir / s) for s in SOURCES]
    subprocess.run(cmd, check=True)
    return out


def _bind(lib):
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    sig = {
        "or_aes128_sbox": (None, [u8p]),
        "or_aes128_expand": (None, [u8p, u8p]),
        "or_aes128": (None, [u8p, u8p, u8p]),
        "or_prf": (None, [u8p, ctypes.c_uint64, u8p]),
        "or_prf_chacha": (None, [u8p, ctypes.c_uint64, u8p]),
        "or_prf_by": (ctypes.c_int, [ctypes.c_uint32, u8p, ctypes.c_uint64, u8p]),
        "or_chacha20_quarter": (None, [u32p, u32p, u32p, u32p]),
        "or_chacha20_block": (None, [u8p, ctypes.c_uint32, u8p, u8p]),
        "or_drbg_block": (None, [u8p, ctypes.c_uint64, u8p]),
        "or_key_size": (ctypes.c_size_t, [ctypes.c_uint32]),
        "or_gen": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                                  u8p, u8p, u8p]),
        "or_gen_prf": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                                      u8p, ctypes.c_uint32, u8p, u8p]),
        "or_eval_point": (ctypes.c_uint32, [u8p, ctypes.c_uint64]),
        "or_eval_level": (ctypes.c_int, [u8p, ctypes.c_uint32, u8p]),
        "or_eval_full": (ctypes.c_int, [u8p, u32p]),
        "or_answer": (ctypes.c_int, [u8p, u32p, ctypes.c_uint64, ctypes.c_uint32, u32p]),
        "or_answer_slice": (ctypes.c_int, [u8p, ctypes.c_uint64, u32p, ctypes.c_uint64, ctypes.c_uint32,
                                           u32p]),
        "or_answer_batch": (ctypes.c_int, [u8p, ctypes.c_uint32, ctypes.c_size_t, u32p,
                                           ctypes.c_uint64, ctypes.c_uint32, u32p,
                                           ctypes.c_int]),
        "or_answer_bins": (ctypes.c_int, [u8p, ctypes.c_uint32, ctypes.c_size_t, u32p,
                                          ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, u32p,
                                          ctypes.c_int]),
        "or_reconstruct": (None, [u32p, u32p, ctypes.c_uint32, u32p]),
        "or_count_prf": (ctypes.c_uint64, []),
        "or_count_drbg": (ctypes.c_uint64, []),
        "or_reset_counts": (None, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def load(path: Path | None = None):
    """Load (building first if absent) and return the bound oracle library."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(str(path)))
    if _lib is None:
        if not LIB_PATH.exists():
            build()
        _lib = _bind(ctypes.CDLL(str(LIB_PATH)))
    return _lib


def _u8(a: np.ndarray):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _u32(a: np.ndarray):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


class Oracle:
    """numpy-facing wrapper around one loaded oracle library."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load()

    # --- AES-128 (FIPS-197) -------------------------------------------------
    def sbox(self) -> np.ndarray:
        out = np.zeros(256, np.uint8)
        self.lib.or_aes128_sbox(_u8(out))
        return out

    def expand_key(self, key: bytes) -> bytes:
        k = np.frombuffer(bytes(key), np.uint8).copy()
        w = np.zeros(176, np.uint8)
        self.lib.or_aes128_expand(_u8(k), _u8(w))
        return w.tobytes()

    def aes128(self, key: bytes, block: bytes) -> bytes:
        k = np.frombuffer(bytes(key), np.uint8).copy()
        b = np.frombuffer(bytes(block), np.uint8).copy()
        o = np.zeros(16, np.uint8)
        self.lib.or_aes128(_u8(k), _u8(b), _u8(o))
        return o.tobytes()

    def prf(self, s: bytes, x: int) -> bytes:
        k = np.frombuffer(bytes(s), np.uint8).copy()
        o = np.zeros(16, np.uint8)
        self.lib.or_prf(_u8(k), x, _u8(o))
        return o.tobytes()

    def prf_chacha(self, s: bytes, x: int) -> bytes:
        k = np.frombuffer(bytes(s), np.uint8).copy()
        o = np.zeros(16, np.uint8)
        self.lib.or_prf_chacha(_u8(k), x, _u8(o))
        return o.tobytes()

    def prf_by(self, prf_id: int, s: bytes, x: int) -> bytes:
        k = np.frombuffer(bytes(s), np.uint8).copy()
        o = np.zeros(16, np.uint8)
        if self.lib.or_prf_by(prf_id, _u8(k), x, _u8(o)):
            raise ValueError("unknown prf id")
        return o.tobytes()

    # --- ChaCha20 (RFC 8439) ----------------------------------------------------
    def chacha20_quarter(self, a: int, b: int, c: int, d: int):
        v = [ctypes.c_uint32(a), ctypes.c_uint32(b), ctypes.c_uint32(c), ctypes.c_uint32(d)]
        self.lib.or_chacha20_quarter(*[ctypes.pointer(x) for x in v])
        return tuple(int(x.value) for x in v)

    def chacha20_block(self, key: bytes, counter: int, nonce: bytes) -> bytes:
        k = np.frombuffer(bytes(key), np.uint8).copy()
        nc = np.frombuffer(bytes(nonce), np.uint8).copy()
        assert k.size == 32 and nc.size == 12
        o = np.zeros(64, np.uint8)
        self.lib.or_chacha20_block(_u8(k), counter, _u8(nc), _u8(o))
        return o.tobytes()

    def drbg(self, seed: bytes, i: int) -> bytes:
        k = np.frombuffer(bytes(seed), np.uint8).copy()
        o = np.zeros(16, np.uint8)
        self.lib.or_drbg_block(_u8(k), i, _u8(o))
        return o.tobytes()

    # --- DPF ------------------------------------------------------------------
    def key_size(self, n: int) -> int:
        return int(self.lib.or_key_size(n))

    def gen(self, n: int, alpha: int, beta: int, seed: bytes, prf_id: int = 0):
        """Return (key0, key1) as uint8 arrays, or raise ValueError."""
        ks = self.key_size(n)
        k0 = np.zeros(ks, np.uint8)
        k1 = np.zeros(ks, np.uint8)
        sd = np.frombuffer(bytes(seed), np.uint8).copy()
        if self.lib.or_gen_prf(n, alpha, beta & 0xFFFFFFFF, _u8(sd), prf_id, _u8(k0),
                               _u8(k1)):
            raise ValueError("or_gen rejected its arguments")
        return k0, k1

    def gen_batch(self, n: int, alphas, seeds, beta: int = 1, prf_id: int = 0):
        """Keys for a batch: returns (keys0, keys1), each [B, key_size] uint8."""
        ks = self.key_size(n)
        B = len(alphas)
        k0 = np.zeros((B, ks), np.uint8)
        k1 = np.zeros((B, ks), np.uint8)
        for q in range(B):
            a, b = self.gen(n, int(alphas[q]), beta, bytes(seeds[q]), prf_id)
            k0[q] = a
            k1[q] = b
        return k0, k1

    def eval_point(self, key: np.ndarray, j: int) -> int:
        return int(self.lib.or_eval_point(_u8(np.ascontiguousarray(key)), j))

    def eval_level(self, key: np.ndarray, d: int) -> np.ndarray:
        out = np.zeros((1 << d, 16), np.uint8)
        if self.lib.or_eval_level(_u8(np.ascontiguousarray(key)), d, _u8(out)):
            raise ValueError("or_eval_level rejected its arguments")
        return out

    def eval_full(self, key: np.ndarray) -> np.ndarray:
        n = int(key[2])
        out = np.zeros(1 << n, np.uint32)
        if self.lib.or_eval_full(_u8(np.ascontiguousarray(key)), _u32(out)):
            raise ValueError("or_eval_full rejected its key")
        return out

    def answer(self, key: np.ndarray, table: np.ndarray) -> np.ndarray:
        table = np.ascontiguousarray(table, dtype=np.uint32)
        rows, dim = table.shape
        out = np.zeros(dim, np.uint32)
        if self.lib.or_answer(_u8(np.ascontiguousarray(key)), _u32(table), rows, dim,
                              _u32(out)):
            raise ValueError("or_answer rejected its arguments")
        return out

    def answer_slice(self, key: np.ndarray, table: np.ndarray, row0: int) -> np.ndarray:
        """One GPU's share of a row-sharded table (section 3.2.7): table row i
        holds index row0 + i."""
        table = np.ascontiguousarray(table, dtype=np.uint32)
        rows, dim = table.shape
        out = np.zeros(dim, np.uint32)
        if self.lib.or_answer_slice(_u8(np.ascontiguousarray(key)), row0, _u32(table), rows, dim,
                                    _u32(out)):
            raise ValueError("or_answer_slice rejected its arguments")
        return out

    def answer_batch(self, keys: np.ndarray, table: np.ndarray,
                     nthreads: int | None = None) -> np.ndarray:
        keys = np.ascontiguousarray(keys, dtype=np.uint8)
        table = np.ascontiguousarray(table, dtype=np.uint32)
        rows, dim = table.shape
        B, stride = keys.shape
        out = np.zeros((B, dim), np.uint32)
        nt = nthreads or os.cpu_count() or 1
        if self.lib.or_answer_batch(_u8(keys), B, stride, _u32(table), rows, dim,
                                    _u32(out), nt):
            raise ValueError("or_answer_batch rejected its arguments")
        return out

    def answer_bins(self, keys: np.ndarray, table: np.ndarray, bin_log: int, n_clients: int,
                    nthreads: int | None = None) -> np.ndarray:
        """Partial batch retrieval, server side (section 4.1): keys [n_clients *
        n_bins, stride] ordered client-major; returns [n_clients, n_bins, dim]."""
        keys = np.ascontiguousarray(keys, dtype=np.uint8)
        table = np.ascontiguousarray(table, dtype=np.uint32)
        rows, dim = table.shape
        n_bins = -(-rows // (1 << bin_log))
        if keys.shape[0] != n_clients * n_bins:
            raise ValueError("keys must hold n_clients * n_bins rows")
        out = np.zeros((n_clients, n_bins, dim), np.uint32)
        nt = nthreads or os.cpu_count() or 1
        if self.lib.or_answer_bins(_u8(keys), n_clients, keys.shape[1], _u32(table), rows, dim,
                                   bin_log, _u32(out), nt):
            raise ValueError("or_answer_bins rejected its arguments")
        return out

    def reconstruct(self, a0: np.ndarray, a1: np.ndarray) -> np.ndarray:
        a0 = np.ascontiguousarray(a0, np.uint32)
        a1 = np.ascontiguousarray(a1, np.uint32)
        out = np.zeros_like(a0)
        self.lib.or_reconstruct(_u32(a0), _u32(a1), a0.size, _u32(out))
        return out

    # --- counters ---------------------------------------------------------------
    def reset_counts(self):
        self.lib.or_reset_counts()

    def counts(self):
        return int(self.lib.or_count_prf()), int(self.lib.or_count_drbg())
