"""Autotuner of the single-table work plan (paper sections 3.2.1, 3.2.3 and
3.2.5: the batch size, the traversal's node budget K and the table size at
which one query is spread over the whole GPU are tuned by measurement).

For each shape -- PRF, aligned row height n (a table of 2^n rows), row width
and a bucket of batch sizes -- the tuner times the candidate plans of one
call on the GPU (which kernel, the wave kernel's per-lane subtree height, the
small-batch kernel's keys per workgroup, whether a ragged remainder gets a
launch of its own) and keeps the fastest.  The winners go to the library
through pir_set_tuning; pir_plan then reports PIR_PLAN_TUNED for the shapes
they cover and the cost model keeps every other shape.

A cache file holds the winners measured on one GPU architecture, ROCm
version and kernel build (the fingerprint pir_kernel_digest reports).
load() applies a file only when all three match the running system and
otherwise clears the table, so a changed kernel or another GPU falls back to
the model until it is tuned again:

    python -m paper_2301_10904_amd.autotune            # tune, write tuning/<arch>.json
    python -m paper_2301_10904_amd.autotune --quick    # a small grid (a check of the tuner)
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from pathlib import Path

import numpy as np

from . import pir

FORMAT = 1
TUNING_DIR = Path(__file__).resolve().parent / "tuning"
ALL_KEYS = 0xFFFFFFFF

# the shapes of the default grid: (n, dim), a table of 2^n rows of dim words
SHAPES = [(14, 16), (14, 64), (16, 64), (18, 64), (20, 16), (20, 32), (20, 64), (20, 128), (22, 64)]
# batch sizes tuned; the entry of size b covers the keys after the previous size up to b (the
# largest covers every larger batch)
BATCHES = [1, 2, 3, 4, 6, 8, 9, 12, 15, 16, 17, 20, 24, 32, 40, 48, 64, 100, 128, 200, 256, 512, 520, 1024]
QUICK_SHAPES = [(14, 16), (20, 64)]
QUICK_BATCHES = [1, 4, 16, 17, 64, 520]
PRFS = ("aes128", "chacha20")
# a candidate replaces the model's plan only if it is faster by more than this
MIN_GAIN = 0.02
HMAX = 9  # the wave kernel's largest per-lane subtree height


def default_path(arch: str) -> Path:
    return TUNING_DIR / f"{arch}.json"


def system_identity() -> dict:
    """The running system's identity: GPU architecture, ROCm (HIP) version and
    the kernel build of the loaded library."""
    import torch

    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    return {"arch": arch, "rocm": str(torch.version.hip), "kernel_digest": pir.kernel_digest()}


def mismatch(doc: dict, identity: dict) -> str | None:
    """Why a cache document does not apply to `identity` (None if it does)."""
    if doc.get("format") != FORMAT:
        return f"format {doc.get('format')} is not {FORMAT}"
    for k in ("arch", "rocm", "kernel_digest"):
        if doc.get(k) != identity.get(k):
            return f"{k} {doc.get(k)!r} differs from this system's {identity.get(k)!r}"
    return None


def entries_of(doc: dict) -> list[dict]:
    return [{f: int(e[f]) for f in pir.TUNE_FIELDS} for e in doc.get("entries", [])]


def apply(doc: dict, identity: dict) -> dict:
    """Hand the document's entries to the library if it was measured on this
    system; otherwise clear the library's table (the model plans everything)."""
    why = mismatch(doc, identity)
    if why:
        pir.set_tuning([])
        return {"applied": False, "entries": 0, "reason": why}
    ents = entries_of(doc)
    pir.set_tuning(ents)
    return {"applied": True, "entries": len(ents), "reason": None}


def load(path: Path | None = None, identity: dict | None = None) -> dict:
    """Apply the cache file for this system (default: tuning/<arch>.json)."""
    identity = identity or system_identity()
    p = Path(path) if path else default_path(identity["arch"])
    if not p.exists():
        pir.set_tuning([])
        return {"applied": False, "entries": 0, "reason": f"no cache file {p.name}", "path": str(p)}
    res = apply(json.loads(p.read_text()), identity)
    res["path"] = str(p)
    return res


def buckets(batches):
    """(keys_lo, keys_hi, representative) for each tuned batch size."""
    out, lo = [], 1
    for i, b in enumerate(batches):
        hi = ALL_KEYS if i == len(batches) - 1 else b
        out.append((lo, hi, b))
        lo = b + 1
    return out


def entry(prf_id, n, dim_lo, dim_hi, keys_lo, keys_hi, kernel=0, subtree_log=0, keys_per_item=0,
          tail_keys=pir.TUNE_MODEL) -> dict:
    return {"prf_id": prf_id, "n": n, "dim_lo": dim_lo, "dim_hi": dim_hi, "keys_lo": keys_lo, "keys_hi": keys_hi,
            "kernel": kernel, "subtree_log": subtree_log, "keys_per_item": keys_per_item, "tail_keys": tail_keys}


COLUMN_CLASSES = (16, 32, 64, 128, 256)  # row widths of one wave-kernel instantiation (and rows past 128 words)


def dim_range(dim: int, dims: list[int]) -> tuple[int, int]:
    """The row widths an entry measured at `dim` covers: from just past the
    next narrower tuned width of the same table height, up to `dim` itself, or
    for the widest tuned width to the end of its column class."""
    lo = max([d for d in dims if d < dim], default=0) + 1
    hi = dim if dim < max(dims) else min(c for c in COLUMN_CLASSES if c >= dim)
    return lo, hi


def kernel_candidates(n: int, dim: int, keys: int) -> list[dict]:
    """Kernel configurations worth timing for one call shape (fields of an
    entry; 0 leaves a field to the model)."""
    c = [dict(kernel=0, subtree_log=0, keys_per_item=0)]  # the model's plan
    if n >= 3 and dim <= 128:
        hmax = min(HMAX, n - 2)
        for h in range(hmax, max(2, hmax - 4), -1):
            c.append(dict(kernel=pir.KERNEL_WAVES, subtree_log=h, keys_per_item=0))
    if keys < 512:
        qmax = 16 if dim <= 64 else 8
        for q in (1, 2, 4, 8, 16):
            if q <= qmax and q <= 2 * keys:
                c.append(dict(kernel=pir.KERNEL_SMALL_BATCH, subtree_log=0, keys_per_item=q))
    return c


def tune(prfs=PRFS, shapes=SHAPES, batches=BATCHES, reps: int = 7, log=print) -> dict:
    """Measure the grid on the current GPU and return a cache document."""
    import torch

    from . import workloads as W

    identity = system_identity()
    dev = torch.device("cuda:0")
    decided: list[dict] = []
    records = []
    dims_at = {}
    for n, dim in shapes:
        dims_at.setdefault(n, []).append(dim)
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in ev:
            e0.record(stream)
            fn()
            e1.record(stream)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    def timed_pair(prep_a, prep_b, fn, rounds):
        """Medians of fn() under two tables, the calls alternating (so that a
        drift of the GPU's clocks affects both alike)."""
        ev = {0: [], 1: []}
        for prep in (prep_a, prep_b):
            prep()
            fn()
        torch.cuda.synchronize()
        for _ in range(rounds):
            for k, prep in ((0, prep_a), (1, prep_b)):
                prep()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                fn()
                e1.record(stream)
                ev[k].append((e0, e1))
        torch.cuda.synchronize()
        return tuple(float(np.median([a.elapsed_time(b) for a, b in ev[k]])) for k in (0, 1))

    t_start = time.time()
    for prf in prfs:
        pid = pir.prf_id(prf)
        for n, dim in shapes:
            rows = 1 << n
            T = W.make_table(rows, dim, 11, device=dev)
            most = max(batches)
            pairs = (most + 1) // 2
            alphas = W.uniform_indices(rows, pairs, 11)
            K0, K1 = pir.gen_batch(n, alphas, W.key_seeds(pairs, 11), prf=prf)
            allk = torch.from_numpy(np.concatenate([K0, K1])).to(dev)
            want = W.table_rows_np(alphas, dim, 11)
            dlo, dhi = dim_range(dim, dims_at[n])
            for lo, hi, B in buckets(batches):
                half = B // 2
                sel = list(range(half)) + list(range(pairs, pairs + half)) + ([half] if B % 2 else [])
                keys = allk[sel].contiguous()
                out = torch.empty((B, dim), dtype=torch.int32, device=dev)

                def run_with(fields):
                    e = entry(pid, n, dlo, dhi, lo, hi, **fields)
                    pir.set_tuning(decided + [e])
                    try:
                        return timed(lambda: pir.answer(keys, T, out, prf=prf))
                    except pir.PirError as err:
                        raise RuntimeError(f"{prf} 2^{n} x {dim}, {B} keys, entry {e}, plan "
                                           f"{pir.plan(B, rows, dim, prf=prf)}: {err}; hipError "
                                           f"{pir.load().pir_last_hip_error()}") from err

                seen = set()

                def plan_key(fields):
                    # candidates that come to the same plan are timed once
                    pir.set_tuning(decided + [entry(pid, n, dlo, dhi, lo, hi, **fields)])
                    return tuple(sorted((k, v) for k, v in pir.plan(B, rows, dim, prf=prf).items() if k != "source"))

                results = []

                def consider(fields):
                    k = plan_key(fields)
                    if k not in seen:
                        seen.add(k)
                        results.append((run_with(fields), fields))

                for kc in kernel_candidates(n, dim, B):
                    consider(dict(kc, tail_keys=pir.TUNE_MODEL))
                model_ms, model = results[0]
                best_ms, best = min(results, key=lambda r: r[0])
                rem = B % 16
                if B > 16 and 1 <= rem <= 8:
                    # the remainder split, both ways, with the best kernel configuration
                    for tail in (0, rem):
                        consider(dict(best, tail_keys=tail))
                    best_ms, best = min(results, key=lambda r: r[0])
                if best is not model and best_ms <= model_ms * (1 - MIN_GAIN):
                    # confirm against the model with the calls alternating
                    m_ms, b_ms = timed_pair(
                        lambda: pir.set_tuning(decided + [entry(pid, n, dlo, dhi, lo, hi, **model)]),
                        lambda: pir.set_tuning(decided + [entry(pid, n, dlo, dhi, lo, hi, **best)]),
                        lambda: pir.answer(keys, T, out, prf=prf), max(reps, 9))
                    if b_ms <= m_ms * (1 - MIN_GAIN):
                        model_ms, best_ms = m_ms, b_ms
                    else:
                        best_ms, best = model_ms, model
                else:
                    best_ms, best = model_ms, model
                e = entry(pid, n, dlo, dhi, lo, hi, **best)
                # the chosen plan answers exactly: every pair reconstructs
                pir.set_tuning(decided + [e])
                pir.answer(keys, T, out, prf=prf)
                torch.cuda.synchronize()
                got = out.cpu().numpy().view(np.uint32)
                ok = bool((((got[:half].astype(np.uint64) + got[half:2 * half]) & 0xFFFFFFFF)
                           .astype(np.uint32) == want[:half]).all())
                if not ok:
                    raise RuntimeError(f"tuned plan {e} answered wrongly on {prf} 2^{n} x {dim}, {B} keys")
                plan = pir.plan(B, rows, dim, prf=prf)
                decided.append(e)
                records.append({"prf": prf, "n": n, "dim": dim, "keys": B, "model_ms": round(model_ms, 4),
                                "tuned_ms": round(best_ms, 4), "candidates": len(results),
                                "kernel": plan["kernel"], "subtree_log": plan["subtree_log"],
                                "keys_per_item": plan["keys_per_item"], "tail_keys": plan["tail_keys"]})
                log(json.dumps(records[-1]))
            del T, allk
            torch.cuda.empty_cache()
    pir.set_tuning(decided)
    return {"format": FORMAT, **identity, "created": time.strftime("%Y-%m-%d %H:%M:%S"),
            "seconds": round(time.time() - t_start, 1), "reps": reps, "min_gain": MIN_GAIN,
            "entries": decided, "measurements": records}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", type=Path, help="cache file to write (default: tuning/<arch>.json)")
    ap.add_argument("--quick", action="store_true", help="a small grid, to check the tuner")
    ap.add_argument("--prf", choices=PRFS, action="append", help="tune this PRF only (repeatable)")
    ap.add_argument("--reps", type=int, default=7)
    args = ap.parse_args(argv)
    pir.load()
    doc = tune(prfs=tuple(args.prf or PRFS), shapes=QUICK_SHAPES if args.quick else SHAPES,
               batches=QUICK_BATCHES if args.quick else BATCHES, reps=args.reps,
               log=lambda s: print(s, flush=True))
    out = args.out or default_path(doc["arch"])
    out.parent.mkdir(parents=True, exist_ok=True)
    out.write_text(json.dumps(doc, indent=1) + "\n")
    print(f"wrote {len(doc['entries'])} entries to {out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
