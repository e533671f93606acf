"""The tuned plan table and the autotuner's cache, on the host (no GPU):
pir_set_tuning validation, how an entry changes pir_plan (and that every
other shape stays on the model), and the cache rules -- a file applies only
to the architecture, ROCm version and kernel build it was measured on."""
import json

import pytest

from paper_2301_10904_amd import autotune as A
from paper_2301_10904_amd import build
from paper_2301_10904_amd import pir


@pytest.fixture(autouse=True)
def clean_table():
    pir.set_tuning([])
    yield
    pir.set_tuning([])


def E(**kw):
    base = A.entry(pir.PRF_AES128, 20, 1, 64, 1, A.ALL_KEYS)
    base.update(kw)
    return base


def test_library_reports_the_digest_of_its_kernel_sources():
    assert pir.kernel_digest() == build.kernel_digest()


def test_entries_override_the_model_only_where_they_match():
    model = pir.plan(1024, 1 << 20, 64)
    assert model["source"] == pir.PLAN_MODEL and model["kernel"] == pir.KERNEL_WAVES
    pir.set_tuning([E(keys_lo=1000, keys_hi=1100, kernel=pir.KERNEL_SMALL_BATCH, keys_per_item=8)])
    assert pir.tuning_count() == 1
    p = pir.plan(1024, 1 << 20, 64)
    assert p["source"] == pir.PLAN_TUNED and p["kernel"] == pir.KERNEL_SMALL_BATCH and p["keys_per_item"] == 8
    # outside the entry: batch size, PRF, height, width
    assert pir.plan(512, 1 << 20, 64) == dict(model, items=pir.plan(512, 1 << 20, 64)["items"],
                                              workgroups=pir.plan(512, 1 << 20, 64)["workgroups"])
    assert pir.plan(1024, 1 << 20, 64, prf="chacha20")["source"] == pir.PLAN_MODEL
    assert pir.plan(1024, 1 << 21, 64)["source"] == pir.PLAN_MODEL
    assert pir.plan(1024, 1 << 20, 65)["source"] == pir.PLAN_MODEL


def test_wave_height_and_group_size():
    pir.set_tuning([E(kernel=pir.KERNEL_WAVES, subtree_log=5)])
    p = pir.plan(256, 1 << 20, 64)
    assert p["kernel"] == pir.KERNEL_WAVES and p["subtree_log"] == 5 and p["rows_per_item"] == 4 << 5
    assert p["items"] == (1 << 20) // (4 << 5) * 16
    # clamped to what the rows allow: 2^6 rows hold four subtrees of height 4 at most
    pir.set_tuning([E(n=6, kernel=pir.KERNEL_WAVES, subtree_log=9)])
    assert pir.plan(64, 64, 64)["subtree_log"] == 4
    # a wave-kernel entry on rows wider than 128 words falls back to the small-batch kernel
    pir.set_tuning([E(dim_hi=256, kernel=pir.KERNEL_WAVES, subtree_log=7)])
    assert pir.plan(64, 1 << 20, 200)["kernel"] == pir.KERNEL_SMALL_BATCH
    # keys per workgroup: a power of two within what the row width allows
    pir.set_tuning([E(kernel=pir.KERNEL_SMALL_BATCH, keys_per_item=4)])
    assert pir.plan(100, 1 << 20, 64)["keys_per_item"] == 4
    pir.set_tuning([E(dim_hi=128, kernel=pir.KERNEL_SMALL_BATCH, keys_per_item=16)])
    assert pir.plan(100, 1 << 20, 100)["keys_per_item"] == 8  # 16 keys do not fit rows of 65..128 words


def test_remainder_split():
    assert pir.plan(520, 1 << 20, 64)["tail_keys"] == 8  # the model splits 1..8 keys off
    pir.set_tuning([E(tail_keys=0)])
    assert pir.plan(520, 1 << 20, 64)["tail_keys"] == 0
    pir.set_tuning([E(tail_keys=4)])
    assert pir.plan(520, 1 << 20, 64)["tail_keys"] == 0
    assert pir.plan(516, 1 << 20, 64)["tail_keys"] == 4
    assert pir.plan(16, 1 << 20, 64)["tail_keys"] == 0


@pytest.mark.parametrize("bad", [dict(prf_id=2), dict(n=0), dict(n=33), dict(dim_lo=0), dict(dim_lo=9, dim_hi=8),
                                 dict(dim_hi=257), dict(keys_lo=0), dict(keys_lo=5, keys_hi=4), dict(kernel=3),
                                 dict(subtree_log=10), dict(keys_per_item=3), dict(keys_per_item=32),
                                 dict(tail_keys=9)])
def test_invalid_entries_are_rejected_and_leave_the_table(bad):
    pir.set_tuning([E(kernel=pir.KERNEL_WAVES)])
    with pytest.raises(pir.PirError):
        pir.set_tuning([E(), E(**bad)])
    assert pir.tuning_count() == 1


def test_buckets_cover_every_batch_size_once():
    b = A.buckets(A.BATCHES)
    assert b[0][0] == 1 and b[-1][1] == A.ALL_KEYS
    for (lo0, hi0, r0), (lo1, hi1, r1) in zip(b, b[1:]):
        assert hi0 + 1 == lo1 and lo0 <= r0 == hi0
    assert A.dim_range(16, [16, 32, 64, 128]) == (1, 16)
    assert A.dim_range(64, [16, 32, 64, 128]) == (33, 64)
    assert A.dim_range(128, [16, 32, 64, 128]) == (65, 128)
    assert A.dim_range(64, [16, 64]) == (17, 64)


def doc_for(identity, entries):
    return {"format": A.FORMAT, **identity, "entries": entries}


def test_cache_applies_only_to_its_own_system(tmp_path):
    ident = {"arch": "gfx950", "rocm": "7.0", "kernel_digest": pir.kernel_digest()}
    ents = [E(keys_lo=1, keys_hi=8, kernel=pir.KERNEL_SMALL_BATCH, keys_per_item=2)]
    f = tmp_path / "gfx950.json"
    f.write_text(json.dumps(doc_for(ident, ents)))
    r = A.load(f, identity=ident)
    assert r["applied"] and r["entries"] == 1 and pir.tuning_count() == 1
    assert pir.plan(8, 1 << 20, 64)["source"] == pir.PLAN_TUNED
    # another architecture, ROCm version or kernel build: the table is cleared
    for k, v in (("arch", "gfx942"), ("rocm", "6.4"), ("kernel_digest", "0" * 16)):
        r = A.load(f, identity=dict(ident, **{k: v}))
        assert not r["applied"] and k in r["reason"] and pir.tuning_count() == 0
        assert pir.plan(8, 1 << 20, 64)["source"] == pir.PLAN_MODEL
        A.load(f, identity=ident)
    # a stale format, or no file at all
    f.write_text(json.dumps(dict(doc_for(ident, ents), format=0)))
    assert not A.load(f, identity=ident)["applied"] and pir.tuning_count() == 0
    assert not A.load(tmp_path / "none.json", identity=ident)["applied"]


def test_committed_cache_is_well_formed():
    """The committed cache for gfx950 (if present) holds valid entries that
    the library accepts, and measurements for every entry."""
    f = A.default_path("gfx950")
    if not f.exists():
        pytest.skip("no committed cache")
    doc = json.loads(f.read_text())
    assert doc["format"] == A.FORMAT and doc["arch"] == "gfx950"
    ents = A.entries_of(doc)
    pir.set_tuning(ents)
    assert pir.tuning_count() == len(ents) == len(doc["measurements"])
    for m in doc["measurements"]:
        assert m["tuned_ms"] <= m["model_ms"] * (1 + 1e-9)
