"""Python binding of libpir.so (include/pir.h): argument marshalling only.

Every step of the server path runs in the library's HIP kernels; PyTorch
tensors only supply device memory (``data_ptr()``) and the HIP stream
(``torch.cuda.current_stream().cuda_stream``).  There is no fallback: if the
library is missing, ``load()`` raises.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

import numpy as np

PKG = Path(__file__).resolve().parent
LIB_PATH = PKG / "libpir.so"

PIR_OK, PIR_EINVAL, PIR_ENOMEM, PIR_EHIP, PIR_EKEY, PIR_ESTALL = 0, -1, -2, -3, -4, -5
MAX_DIM = 256
PRF_AES128, PRF_CHACHA20 = 0, 1  # key byte 3
PRFS = {"aes128": PRF_AES128, "chacha20": PRF_CHACHA20}

# the exported C ABI, as declared in include/pir.h
EXPORTS = ("dpf_key_size", "dpf_gen", "dpf_gen_prf", "pir_answer", "pir_answer_prf", "pir_answer_slice",
           "pir_answer_multi", "pir_answer_multi_prf", "pir_answer_bins", "pir_plan", "pir_plan_bins",
           "pir_reconstruct", "pir_workspace_size", "pir_set_workspace", "pir_workspace_status",
           "pir_check_status", "pir_strerror", "pir_last_hip_error", "pir_set_tuning", "pir_tuning_count",
           "pir_kernel_digest", "pir_set_wait_limit")
PLAN_MODEL, PLAN_TUNED = 0, 1
TUNE_MODEL = 0xFFFFFFFF
WORKSPACE_BYTES = 256
STATUS_BAD_KEY, STATUS_STALLED = 1, 2
WAIT_LIMIT_DEFAULT = 1 << 22
KERNEL_WAVES, KERNEL_SMALL_BATCH, KERNEL_STREAM = 1, 2, 3
BINS_MIN_LOG, BINS_MAX_DIM = 3, 128

_lib = None


class PirError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = _lib.pir_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} (status {status})")


class PirTable(ctypes.Structure):
    _fields_ = [("d_table", ctypes.c_void_p), ("rows", ctypes.c_uint64),
                ("dim", ctypes.c_uint32), ("n_keys", ctypes.c_uint32)]


class PirPlan(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_uint32), ("n", ctypes.c_uint32), ("items", ctypes.c_uint64),
                ("workgroups", ctypes.c_uint64), ("lanes_per_workgroup", ctypes.c_uint32),
                ("lds_bytes", ctypes.c_uint32), ("keys_per_item", ctypes.c_uint32),
                ("subtree_log", ctypes.c_uint32), ("rows_per_item", ctypes.c_uint64),
                ("descent_levels", ctypes.c_uint32), ("bfs_levels", ctypes.c_uint32),
                ("tail_keys", ctypes.c_uint32), ("source", ctypes.c_uint32)]


class PirTune(ctypes.Structure):
    _fields_ = [("prf_id", ctypes.c_uint32), ("n", ctypes.c_uint32), ("dim_lo", ctypes.c_uint32),
                ("dim_hi", ctypes.c_uint32), ("keys_lo", ctypes.c_uint32), ("keys_hi", ctypes.c_uint32),
                ("kernel", ctypes.c_uint32), ("subtree_log", ctypes.c_uint32),
                ("keys_per_item", ctypes.c_uint32), ("tail_keys", ctypes.c_uint32)]


class PirBins(ctypes.Structure):
    _fields_ = [("d_table", ctypes.c_void_p), ("rows", ctypes.c_uint64), ("dim", ctypes.c_uint32),
                ("n_clients", ctypes.c_uint32), ("bin_log", ctypes.c_uint32)]


def load(path: Path | None = None):
    """Load libpir.so (built by paper_2301_10904_amd.build); raise if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = Path(path) if path else LIB_PATH
    if not p.exists():
        raise ImportError(f"{p} is missing: build it with `python -m paper_2301_10904_amd.build` "
                          "(there is no fallback path)")
    # One HIP runtime per process: PyTorch's (it supplies the device memory
    # and streams) is loaded first, and the library binds to the same one.
    # Loaded the other way round, the two disagree about the devices.
    import torch  # noqa: F401
    lib = ctypes.CDLL(str(p))
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.dpf_key_size.restype = ctypes.c_size_t
    lib.dpf_key_size.argtypes = [ctypes.c_uint32]
    lib.dpf_gen.restype = ctypes.c_int
    lib.dpf_gen.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, u8p, u8p, u8p]
    lib.dpf_gen_prf.restype = ctypes.c_int
    lib.dpf_gen_prf.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, u8p,
                                ctypes.c_uint32, u8p, u8p]
    lib.pir_answer_prf.restype = ctypes.c_int
    lib.pir_answer_prf.argtypes = [ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p,
                                   ctypes.c_void_p]
    lib.pir_answer_slice.restype = ctypes.c_int
    lib.pir_answer_slice.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p,
                                     ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint64,
                                     ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
    lib.pir_answer_multi_prf.restype = ctypes.c_int
    lib.pir_answer_multi_prf.argtypes = [ctypes.c_uint32, ctypes.POINTER(PirTable), ctypes.c_uint32,
                                         ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                         ctypes.c_void_p]
    lib.pir_answer.restype = ctypes.c_int
    lib.pir_answer.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                               ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
    lib.pir_answer_multi.restype = ctypes.c_int
    lib.pir_answer_multi.argtypes = [ctypes.POINTER(PirTable), ctypes.c_uint32, ctypes.c_void_p,
                                     ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
    lib.pir_answer_bins.restype = ctypes.c_int
    lib.pir_answer_bins.argtypes = [ctypes.c_uint32, ctypes.POINTER(PirBins), ctypes.c_uint32,
                                    ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
    lib.pir_plan.restype = ctypes.c_int
    lib.pir_plan.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                             ctypes.POINTER(PirPlan)]
    lib.pir_plan_bins.restype = ctypes.c_int
    lib.pir_plan_bins.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_uint32, ctypes.POINTER(PirPlan)]
    lib.pir_workspace_size.restype = ctypes.c_size_t
    lib.pir_workspace_size.argtypes = []
    lib.pir_set_workspace.restype = ctypes.c_int
    lib.pir_set_workspace.argtypes = [ctypes.c_void_p, ctypes.c_size_t]
    lib.pir_workspace_status.restype = ctypes.c_int
    lib.pir_workspace_status.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.pir_set_tuning.restype = ctypes.c_int
    lib.pir_set_tuning.argtypes = [ctypes.POINTER(PirTune), ctypes.c_uint32]
    lib.pir_tuning_count.restype = ctypes.c_uint32
    lib.pir_tuning_count.argtypes = []
    lib.pir_kernel_digest.restype = ctypes.c_char_p
    lib.pir_kernel_digest.argtypes = []
    lib.pir_reconstruct.restype = ctypes.c_int
    lib.pir_reconstruct.argtypes = [u32p, u32p, ctypes.c_uint32, u32p]
    lib.pir_check_status.restype = ctypes.c_int
    lib.pir_check_status.argtypes = []
    lib.pir_strerror.restype = ctypes.c_char_p
    lib.pir_strerror.argtypes = [ctypes.c_int]
    lib.pir_last_hip_error.restype = ctypes.c_int
    lib.pir_last_hip_error.argtypes = []
    lib.pir_set_wait_limit.restype = ctypes.c_int
    lib.pir_set_wait_limit.argtypes = [ctypes.c_uint32]
    if path is None:
        _lib = lib
    return lib


def _check(status: int, what: str):
    if status != PIR_OK:
        raise PirError(status, what)


def _u8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _u32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def key_size(n: int) -> int:
    return int(load().dpf_key_size(n))


def log_domain(rows: int) -> int:
    """n = ceil(log2 rows), at least 1: the key domain for a table of `rows` rows."""
    return max(1, (int(rows) - 1).bit_length())


def prf_id(prf) -> int:
    """PRF id from an id or a name ("aes128", "chacha20")."""
    if isinstance(prf, str):
        if prf not in PRFS:
            raise ValueError(f"unknown PRF {prf!r}; known: {sorted(PRFS)}")
        return PRFS[prf]
    return int(prf)


def gen(n: int, alpha: int, beta: int = 1, seed: bytes | None = None, prf=PRF_AES128):
    """Client Gen: returns (key0, key1) as uint8 numpy arrays of key_size(n) bytes.
    `prf` picks the tree's PRF (id or name); the random draws do not depend on it."""
    lib = load()
    ks = key_size(n)
    if ks == 0:
        raise PirError(PIR_EINVAL, "dpf_gen")
    k0 = np.zeros(ks, np.uint8)
    k1 = np.zeros(ks, np.uint8)
    sd = None
    if seed is not None:
        sd = np.frombuffer(bytes(seed), np.uint8).copy()
        if sd.size != 16:
            raise ValueError("seed must be 16 bytes")
    _check(lib.dpf_gen_prf(n, alpha, beta & 0xFFFFFFFF, _u8(sd) if sd is not None else None,
                           prf_id(prf), _u8(k0), _u8(k1)), "dpf_gen")
    return k0, k1


def gen_batch(n: int, alphas, seeds=None, beta: int = 1, prf=PRF_AES128):
    """Keys for a batch of indices: (keys0, keys1), each uint8 [B, key_size(n)]."""
    B = len(alphas)
    ks = key_size(n)
    K0 = np.zeros((B, ks), np.uint8)
    K1 = np.zeros((B, ks), np.uint8)
    for q in range(B):
        K0[q], K1[q] = gen(n, int(alphas[q]), beta, None if seeds is None else seeds[q], prf)
    return K0, K1


def _stream_handle(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_dev(t, name, dtypes):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} has dtype {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def answer_slice(keys, table, n, row0, out=None, stream=None, prf=PRF_AES128):
    """One GPU's share of a row-sharded table (pir_answer_slice): keys of
    domain 2^n evaluated on the indices row0 .. row0 + rows - 1 only, table
    row i holding index row0 + i; summing the slices' outputs mod 2^32 gives
    answer() over the whole table.  Arguments otherwise as for answer()."""
    import torch

    lib = load()
    _check_dev(keys, "keys", (torch.uint8,))
    _check_dev(table, "table", (torch.int32, torch.uint32))
    B, stride = keys.shape
    rows, dim = table.shape
    if out is None:
        out = torch.empty((B, dim), dtype=torch.int32, device=table.device)
    _check_dev(out, "out", (torch.int32, torch.uint32))
    if tuple(out.shape) != (B, dim):
        raise ValueError("out must be [B, dim]")
    _check(lib.pir_answer_slice(prf_id(prf), n, row0, keys.data_ptr(), B, stride, table.data_ptr(), rows, dim,
                                out.data_ptr(), _stream_handle(stream)), "pir_answer_slice")
    return out


def answer(keys, table, out=None, stream=None, prf=PRF_AES128):
    """Server answer for one table: out[q] = sum_j Eval(keys[q], j) * table[j] mod 2^32.

    keys  : uint8 device tensor [B, stride] (stride a multiple of 16)
    table : int32/uint32 device tensor [rows, dim]
    out   : int32/uint32 device tensor [B, dim] (allocated if None)
    prf   : the keys' PRF (id or name); a key of another PRF answers zero and
            raises the flag of check_status()
    """
    import torch

    lib = load()
    _check_dev(keys, "keys", (torch.uint8,))
    _check_dev(table, "table", (torch.int32, torch.uint32))
    B, stride = keys.shape
    rows, dim = table.shape
    if out is None:
        out = torch.empty((B, dim), dtype=torch.int32, device=table.device)
    _check_dev(out, "out", (torch.int32, torch.uint32))
    if tuple(out.shape) != (B, dim):
        raise ValueError("out must be [B, dim]")
    _check(lib.pir_answer_prf(prf_id(prf), keys.data_ptr(), B, stride, table.data_ptr(), rows, dim,
                              out.data_ptr(), _stream_handle(stream)), "pir_answer")
    return out


def answer_multi(tables, key_counts, keys, out=None, stream=None, prf=PRF_AES128):
    """Server answer over several tables in one call.

    tables     : list of int32/uint32 device tensors [rows_t, dim_t]
    key_counts : keys per table; keys are grouped by table in this order
    keys       : uint8 device tensor [sum(key_counts), stride]
    out        : flat int32 device tensor of sum_t key_counts[t] * dim_t words
    Returns out and the list of per-table [n_t, dim_t] views into it.
    """
    import torch

    lib = load()
    _check_dev(keys, "keys", (torch.uint8,))
    if len(tables) != len(key_counts):
        raise ValueError("one key count per table")
    descs = (PirTable * max(1, len(tables)))()
    total = 0
    for i, (t, c) in enumerate(zip(tables, key_counts)):
        _check_dev(t, f"tables[{i}]", (torch.int32, torch.uint32))
        descs[i] = PirTable(t.data_ptr(), t.shape[0], t.shape[1], int(c))
        total += int(c) * t.shape[1]
    if keys.shape[0] != sum(int(c) for c in key_counts):
        raise ValueError("keys must hold sum(key_counts) rows")
    if out is None:
        out = torch.empty(total, dtype=torch.int32, device=keys.device)
    _check_dev(out, "out", (torch.int32, torch.uint32))
    if out.numel() != total:
        raise ValueError("out has the wrong size")
    _check(lib.pir_answer_multi_prf(prf_id(prf), descs, len(tables), keys.data_ptr(), keys.shape[1],
                                    out.data_ptr(), _stream_handle(stream)), "pir_answer_multi")
    views, off = [], 0
    for t, c in zip(tables, key_counts):
        n = int(c) * t.shape[1]
        views.append(out[off:off + n].view(int(c), t.shape[1]))
        off += n
    return out, views


def plan(n_keys: int, rows: int, dim: int, prf=PRF_AES128) -> dict:
    """The work plan pir_answer uses for one table (no GPU needed)."""
    p = PirPlan()
    _check(load().pir_plan(prf_id(prf), n_keys, rows, dim, ctypes.byref(p)), "pir_plan")
    return {name: getattr(p, name) for name, _ in PirPlan._fields_}


TUNE_FIELDS = tuple(name for name, _ in PirTune._fields_)


def set_tuning(entries) -> None:
    """Replace the library's tuned plan table (pir_set_tuning) with `entries`,
    a list of dicts with the fields of pir_tune_t (an empty list clears it)."""
    arr = (PirTune * max(1, len(entries)))()
    for i, e in enumerate(entries):
        arr[i] = PirTune(*[int(e[f]) for f in TUNE_FIELDS])
    _check(load().pir_set_tuning(arr, len(entries)), "pir_set_tuning")


def tuning_count() -> int:
    return int(load().pir_tuning_count())


def kernel_digest() -> str:
    """Fingerprint of the kernel sources the loaded library was built from."""
    return load().pir_kernel_digest().decode()


def plan_bins(rows: int, dim: int, n_clients: int, bin_log: int, prf=PRF_AES128) -> dict:
    """The work plan pir_answer_bins uses for one table (no GPU needed)."""
    p = PirPlan()
    _check(load().pir_plan_bins(prf_id(prf), rows, dim, n_clients, bin_log, ctypes.byref(p)), "pir_plan_bins")
    return {name: getattr(p, name) for name, _ in PirPlan._fields_}


def n_bins(rows: int, bin_log: int) -> int:
    """Bins of 2^bin_log rows over a table of `rows` rows (the last may be shorter)."""
    return (int(rows) + (1 << bin_log) - 1) >> bin_log


def answer_bins(tables, client_counts, bin_logs, keys, out=None, stream=None, prf=PRF_AES128):
    """Partial batch retrieval, server side (section 4.1), over one or more tables.

    tables        : list of int32/uint32 device tensors [rows_t, dim_t] (dim_t <= 128)
    client_counts : clients per table; each sends one key per bin of its table
    bin_logs      : bins of 2^bin_logs[t] rows per table
    keys          : uint8 device tensor, per table client-major: key (c, b) of
                    table t is row sum_{t'<t} clients_t' bins_t' + c bins_t + b
    Returns out and the list of per-table [clients_t, bins_t, dim_t] views.
    """
    import torch

    lib = load()
    _check_dev(keys, "keys", (torch.uint8,))
    if not (len(tables) == len(client_counts) == len(bin_logs)):
        raise ValueError("one client count and one bin size per table")
    descs = (PirBins * max(1, len(tables)))()
    total_keys, total = 0, 0
    shapes = []
    for i, (t, c, bl) in enumerate(zip(tables, client_counts, bin_logs)):
        _check_dev(t, f"tables[{i}]", (torch.int32, torch.uint32))
        nb = n_bins(t.shape[0], int(bl))
        descs[i] = PirBins(t.data_ptr(), t.shape[0], t.shape[1], int(c), int(bl))
        shapes.append((int(c), nb, t.shape[1]))
        total_keys += int(c) * nb
        total += int(c) * nb * t.shape[1]
    if keys.shape[0] != total_keys:
        raise ValueError(f"keys must hold {total_keys} rows (clients x bins per table)")
    if out is None:
        out = torch.empty(total, dtype=torch.int32, device=keys.device)
    _check_dev(out, "out", (torch.int32, torch.uint32))
    if out.numel() != total:
        raise ValueError("out has the wrong size")
    _check(lib.pir_answer_bins(prf_id(prf), descs, len(tables), keys.data_ptr(), keys.shape[1],
                               out.data_ptr(), _stream_handle(stream)), "pir_answer_bins")
    views, off = [], 0
    for c, nb, d in shapes:
        views.append(out[off:off + c * nb * d].view(c, nb, d))
        off += c * nb * d
    return out, views


def reconstruct(a0: np.ndarray, a1: np.ndarray) -> np.ndarray:
    """Client reconstruction a0 + a1 mod 2^32 (host arrays)."""
    lib = load()
    a0 = np.ascontiguousarray(a0).view(np.uint32).reshape(-1)
    a1 = np.ascontiguousarray(a1).view(np.uint32).reshape(-1)
    if a0.size != a1.size:
        raise ValueError("answers differ in length")
    out = np.zeros_like(a0)
    _check(lib.pir_reconstruct(_u32(a0), _u32(a1), a0.size, _u32(out)), "pir_reconstruct")
    return out


def check_status() -> int:
    """Status of the last call that used the library's own workspace on the
    current device (after the caller has synchronised): PIR_OK, PIR_EKEY if it
    saw a key with a bad header, PIR_ESTALL if a kernel gave up a bounded wait
    (its output is then not valid)."""
    return int(load().pir_check_status())


def set_wait_limit(tries: int) -> None:
    """Tries of a kernel's bounded wait before it gives up (0: the default,
    WAIT_LIMIT_DEFAULT); a small limit forces the stalled-wait path in tests."""
    _check(load().pir_set_wait_limit(int(tries)), "pir_set_wait_limit")


def workspace(device=None):
    """A status workspace (uint8 device tensor of pir_workspace_size() bytes)."""
    import torch

    return torch.zeros(int(load().pir_workspace_size()), dtype=torch.uint8,
                       device=device if device is not None else "cuda")


def set_workspace(ws) -> None:
    """Bind `ws` (from workspace(), or None to unbind) as the status workspace
    of the answer calls this thread makes from now on."""
    import torch

    lib = load()
    if ws is None:
        _check(lib.pir_set_workspace(None, 0), "pir_set_workspace")
        return
    _check_dev(ws, "workspace", (torch.uint8,))
    _check(lib.pir_set_workspace(ws.data_ptr(), ws.numel()), "pir_set_workspace")


def workspace_status(ws, stream=None) -> int:
    """Status of the last call that used workspace `ws`, read in the order of
    `stream` (waits for the calls enqueued on it): PIR_OK, PIR_EKEY or
    PIR_ESTALL, as check_status()."""
    import torch

    _check_dev(ws, "workspace", (torch.uint8,))
    return int(load().pir_workspace_status(ws.data_ptr(), _stream_handle(stream)))
