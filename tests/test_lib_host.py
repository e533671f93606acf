"""Host-side checks of libpir.so that need no GPU.

  - the library loads and exports every function include/pir.h declares;
  - the library's Gen (its own AES, ChaCha20 and code) and the oracle's Gen
    produce byte-identical keys from the same 16-byte seed, for both PRFs;
  - argument validation returns PIR_EINVAL before anything is launched;
  - reconstruction and status strings.
"""
import ctypes
import re
from pathlib import Path

import numpy as np
import pytest

from paper_2301_10904_amd import pir

ROOT = Path(__file__).resolve().parent.parent


def declared_functions():
    text = (ROOT / "include" / "pir.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    return pir.load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert set(names) == set(pir.EXPORTS), names
    for name in names:
        assert hasattr(lib, name), name


def test_key_size(lib):
    assert pir.key_size(1) == 96
    assert pir.key_size(20) == 32 + 1280
    assert lib.dpf_key_size(0) == 0 and lib.dpf_key_size(33) == 0


@pytest.mark.parametrize("n", [1, 2, 3, 8, 14, 20, 25, 32])
def test_gen_matches_oracle_bytes(O, n):
    rng = np.random.default_rng(n)
    for trial in range(4):
        alpha = int(rng.integers(0, 1 << n))
        beta = int(rng.integers(0, 2**32)) if trial else 1
        seed = rng.integers(0, 256, 16, dtype=np.uint8).tobytes()
        k0, k1 = pir.gen(n, alpha, beta, seed)
        o0, o1 = O.gen(n, alpha, beta, seed)
        assert (k0 == o0).all() and (k1 == o1).all(), (n, alpha, beta)


@pytest.mark.parametrize("n", [1, 3, 9, 20, 32])
def test_gen_chacha_matches_oracle_bytes(O, n):
    rng = np.random.default_rng([n, 20])
    for trial in range(3):
        alpha = int(rng.integers(0, 1 << n))
        beta = int(rng.integers(0, 2**32)) if trial else 1
        seed = rng.integers(0, 256, 16, dtype=np.uint8).tobytes()
        k0, k1 = pir.gen(n, alpha, beta, seed, prf="chacha20")
        o0, o1 = O.gen(n, alpha, beta, seed, prf_id=1)
        assert k0[3] == pir.PRF_CHACHA20
        assert (k0 == o0).all() and (k1 == o1).all(), (n, alpha, beta)


def test_gen_rejects_unknown_prf(lib):
    with pytest.raises(pir.PirError) as e:
        pir.gen(5, 3, 1, bytes(16), prf=2)
    assert e.value.status == pir.PIR_EINVAL
    with pytest.raises(ValueError):
        pir.gen(5, 3, 1, bytes(16), prf="salsa20")


def test_gen_without_seed_is_random_and_correct(O):
    k0, k1 = pir.gen(6, 17)
    k0b, _ = pir.gen(6, 17)
    assert not (k0[16:] == k0b[16:]).all()
    s = (O.eval_full(k0) + O.eval_full(k1)).astype(np.uint32)
    want = np.zeros(64, np.uint32)
    want[17] = 1
    assert (s == want).all()


def test_gen_rejects_bad_arguments():
    for n, alpha in ((0, 0), (33, 0), (4, 16), (1, 2)):
        with pytest.raises(pir.PirError) as e:
            pir.gen(n, alpha, 1, bytes(16))
        assert e.value.status == pir.PIR_EINVAL


def test_reconstruct_wraps():
    a0 = np.array([1, 2**32 - 1, 5], np.uint32)
    a1 = np.array([2**32 - 1, 2, 7], np.uint32)
    assert (pir.reconstruct(a0, a1) == np.array([0, 1, 12], np.uint32)).all()


def test_strerror(lib):
    for st in (0, -1, -2, -3, -4, -5, 99):
        assert isinstance(lib.pir_strerror(st), bytes)
    msgs = {lib.pir_strerror(st) for st in (0, -1, -2, -3, -4, -5)}
    assert len(msgs) == 6 and lib.pir_strerror(99) not in msgs
    assert b"not valid" in lib.pir_strerror(pir.PIR_ESTALL)


def test_wait_limit_is_set_and_restored_without_gpu(lib):
    """The wait limit is host state (no HIP call): any value is accepted, 0
    restores the default."""
    for tries in (1, 7, 0, 2**32 - 1, 0):
        assert lib.pir_set_wait_limit(tries) == pir.PIR_OK
    pir.set_wait_limit(0)


def test_answer_validation_without_gpu(lib):
    """Every rejected call returns before touching the HIP runtime."""
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    ks = pir.key_size(10)
    cases = [
        (None, 1, ks, fake, 1024, 4, fake),        # null keys
        (fake, 1, ks, None, 1024, 4, fake),        # null table
        (fake, 1, ks, fake, 1024, 4, None),        # null out
        (fake, 1, ks, fake, 0, 4, fake),           # no rows
        (fake, 1, ks, fake, 1024, 0, fake),        # no columns
        (fake, 1, ks, fake, 1024, 257, fake),      # too many columns
        (fake, 1, ks, fake, 2**32 + 1, 4, fake),   # rows beyond 2^32
        (fake, 1, ks - 16, fake, 1024, 4, fake),   # stride below the key size
        (fake, 1, ks + 8, fake, 1024, 4, fake),    # stride not a multiple of 16
        (ctypes.c_void_p(0x1008), 1, ks, fake, 1024, 4, fake),  # misaligned keys
    ]
    for c in cases:
        assert lib.pir_answer(*c, None) == pir.PIR_EINVAL, c
        for prf in (pir.PRF_AES128, pir.PRF_CHACHA20):
            assert lib.pir_answer_prf(prf, *c, None) == pir.PIR_EINVAL, (prf, c)
    # zero keys is a no-op
    assert lib.pir_answer(None, 0, ks, None, 1024, 4, None, None) == pir.PIR_OK
    # an unknown PRF id is rejected even where the call is otherwise valid
    assert lib.pir_answer_prf(2, fake, 1, ks, fake, 1024, 4, fake, None) == pir.PIR_EINVAL


def test_answer_slice_validation_without_gpu(lib):
    """Row slices (one GPU's share of a row-sharded table): the slice must lie
    in one aligned subtree inside the keys' domain; every rejected call returns
    before touching the HIP runtime."""
    fake = ctypes.c_void_p(0x1000)
    ks = pir.key_size(20)
    ok = dict(n=20, row0=3 << 12, keys=fake, nk=1, ks=ks, table=fake, rows=1 << 12, dim=4, out=fake)

    def call(**kw):
        a = {**ok, **kw}
        return lib.pir_answer_slice(pir.PRF_AES128, a["n"], a["row0"], a["keys"], a["nk"], a["ks"], a["table"],
                                    a["rows"], a["dim"], a["out"], None)

    bad = [dict(n=0), dict(n=33),
           dict(rows=(1 << 20) + 1),                 # slice taller than the domain
           dict(row0=(3 << 12) + 1),                 # not on a 2^12 boundary
           dict(row0=1 << 11),                       # 2^11 is not a multiple of 2^12
           dict(row0=(1 << 20) - (1 << 12), rows=(1 << 12) + 1),  # past 2^n (and unaligned height)
           dict(row0=1 << 20),                       # starts past the domain
           dict(ks=pir.key_size(12)),                # stride for a 12-level key, the keys have 20
           dict(keys=None), dict(table=None), dict(out=None), dict(rows=0), dict(dim=0), dict(dim=257)]
    for b in bad:
        assert call(**b) == pir.PIR_EINVAL, b
    # rows = 1: the slice's subtree has height 1, so row0 must be even
    assert call(rows=1, row0=5) == pir.PIR_EINVAL
    assert call(nk=0) == pir.PIR_OK  # no keys: nothing to do
    assert lib.pir_answer_slice(2, 20, 0, fake, 1, ks, fake, 1 << 12, 4, fake, None) == pir.PIR_EINVAL


def test_answer_multi_validation_without_gpu(lib):
    fake = 0x1000
    ks = pir.key_size(12)
    T = (pir.PirTable * 2)(pir.PirTable(fake, 4096, 8, 3), pir.PirTable(fake, 0, 8, 2))
    assert lib.pir_answer_multi(T, 2, fake, ks, fake, None) == pir.PIR_EINVAL
    T = (pir.PirTable * 1)(pir.PirTable(fake, 4096, 300, 3))
    assert lib.pir_answer_multi(T, 1, fake, ks, fake, None) == pir.PIR_EINVAL
    T = (pir.PirTable * 1)(pir.PirTable(fake, 4096, 8, 0))
    assert lib.pir_answer_multi(T, 1, None, ks, None, None) == pir.PIR_OK
    assert lib.pir_answer_multi_prf(pir.PRF_CHACHA20, T, 1, None, ks, None, None) == pir.PIR_OK
    assert lib.pir_answer_multi_prf(5, T, 1, None, ks, None, None) == pir.PIR_EINVAL


def test_answer_bins_validation_without_gpu(lib):
    fake = 0x1000
    ks = pir.key_size(10)
    ok = pir.PirBins(fake, 1 << 14, 16, 4, 10)
    bad = [
        pir.PirBins(fake, 1 << 14, 129, 4, 10),     # rows wider than 128 words
        pir.PirBins(fake, 1 << 14, 16, 4, 2),       # bins below 8 rows
        pir.PirBins(fake, 0, 16, 4, 10),            # no rows
        pir.PirBins(None, 1 << 14, 16, 4, 10),      # null table
        pir.PirBins(fake, 1 << 14, 16, 4, 33),      # bins beyond 2^32 rows
    ]
    for d in bad:
        T = (pir.PirBins * 2)(ok, d)
        assert lib.pir_answer_bins(0, T, 2, fake, ks, fake, None) == pir.PIR_EINVAL, d.dim
    T = (pir.PirBins * 1)(ok)
    assert lib.pir_answer_bins(0, T, 1, fake, ks - 16, fake, None) == pir.PIR_EINVAL  # short stride
    assert lib.pir_answer_bins(0, T, 1, 0x1008, ks, fake, None) == pir.PIR_EINVAL    # misaligned keys
    assert lib.pir_answer_bins(7, T, 1, fake, ks, fake, None) == pir.PIR_EINVAL      # unknown PRF
    T = (pir.PirBins * 1)(pir.PirBins(fake, 1 << 14, 16, 0, 10))
    assert lib.pir_answer_bins(1, T, 1, None, ks, None, None) == pir.PIR_OK          # no clients


def test_client_plans_match_the_oracle():
    """The library's client plans (numpy) against the oracle's (plain loops)."""
    from oracle import client as oc
    from paper_2301_10904_amd import client as pc

    rng = np.random.default_rng(31)
    for trial in range(200):
        rows = int(rng.integers(8, 3000))
        bin_log = int(rng.integers(3, 12))
        wanted = rng.integers(0, rows, int(rng.integers(0, 60)))
        a, s, d = pc.pbr_plan(wanted, rows, bin_log)
        oa, os_, od = oc.pbr_plan(wanted, rows, bin_log)
        assert list(a) == oa and [None if x < 0 else int(x) for x in s] == os_ and list(d) == od
        hot = rng.choice(rows, min(rows, 20), replace=False)
        hot_of = np.full(rows, -1, np.int64)
        hot_of[hot] = np.arange(hot.size)
        q_hot, q_full = int(rng.integers(0, 6)), int(rng.integers(0, 6))
        got = pc.hot_full_plan(wanted, hot_of, q_hot, q_full)
        want = oc.hot_full_plan(wanted, {int(x): i for i, x in enumerate(hot)}, q_hot, q_full)
        assert list(got[0]) == want[0] and list(got[1]) == want[1]
        assert [None if x < 0 else int(x) for x in got[2]] == want[2]
        assert [None if x < 0 else int(x) for x in got[3]] == want[3]
        assert list(got[4]) == want[4]


def test_hot_rows_by_frequency():
    from paper_2301_10904_amd import client as pc

    counts = np.array([5, 9, 9, 1, 0, 9, 9])
    rows, hot_of = pc.hot_rows_by_frequency(counts, 3)
    assert list(rows) == [1, 2, 5]
    assert list(hot_of) == [-1, 0, 1, -1, -1, 2, -1]


def test_plan_batched_default_workload():
    p = pir.plan(1024, 1 << 20, 64)
    assert p["kernel"] == pir.KERNEL_WAVES and p["n"] == 20
    assert p["subtree_log"] == 9 and p["descent_levels"] == 11 and p["bfs_levels"] == 0
    assert p["keys_per_item"] == 16 and p["rows_per_item"] == 4 << 9
    assert p["items"] == 64 * ((1 << 20) // (4 << 9))  # 64 key groups x 512 row chunks
    assert p["workgroups"] == p["items"] // 8 and p["lanes_per_workgroup"] == 512
    assert p["lds_bytes"] == 65536
    assert pir.plan(1024, 1 << 20, 64, prf="chacha20")["lds_bytes"] == 0


def test_plan_single_key_spreads_over_every_cu():
    """One key: about two workgroups per CU of the 256, each covering its own
    rows; with AES-128 the stream kernel (256 tree lanes per workgroup: 8
    breadth-first levels) while its subtree height fits the path registers,
    otherwise, and with ChaCha20, the small-batch kernel."""
    for rows in (1 << 20, 1 << 22, 1 << 25, 1 << 32):
        for prf in ("aes128", "chacha20"):
            p = pir.plan(1, rows, 64, prf=prf)
            stream = prf == "aes128" and rows < 1 << 32
            assert p["kernel"] == (pir.KERNEL_STREAM if stream else pir.KERNEL_SMALL_BATCH), (rows, prf, p)
            assert p["bfs_levels"] == (8 if stream else 9)
            assert p["workgroups"] >= 2 * 256, (rows, p)
            assert p["workgroups"] * p["rows_per_item"] >= rows
            assert p["descent_levels"] + p["bfs_levels"] + p["subtree_log"] == p["n"]
    # rows of 16, 32 or 64 words stream, on small tables too (cached row reads
    # up to 256 MiB); wider rows, rows of a width not a multiple of 4 words,
    # tables of at most 256 rows (no subtree below 256 tree lanes), and two
    # keys do not
    for rows, dim in ((1 << 23, 16), (1 << 22, 32), (1 << 22, 16), (1 << 14, 16), (1 << 10, 64), (257, 4)):
        p = pir.plan(1, rows, dim)
        assert p["kernel"] == pir.KERNEL_STREAM and p["subtree_log"] >= 1, (rows, dim, p)
    for rows, dim in ((1 << 22, 100), (1 << 22, 63), (1 << 8, 64), (100, 16)):
        assert pir.plan(1, rows, dim)["kernel"] == pir.KERNEL_SMALL_BATCH, (rows, dim)
    assert pir.plan(2, 1 << 25, 64)["kernel"] == pir.KERNEL_SMALL_BATCH


def test_plan_tuned_one_key_per_group_over_several_keys_keeps_the_fused_kernel():
    """The stream kernel answers one key: a tuned plan of one key per
    workgroup over 3 keys on a table above 256 MiB stays on the small-batch
    kernel (one group per key); a tuned group of 2 over a single key does not
    stream either."""
    T = pir.TUNE_MODEL
    base = dict(prf_id=0, n=22, dim_lo=1, dim_hi=64, kernel=pir.KERNEL_SMALL_BATCH, subtree_log=0, tail_keys=T)
    try:
        pir.set_tuning([dict(base, keys_lo=3, keys_hi=3, keys_per_item=1),
                        dict(base, keys_lo=1, keys_hi=1, keys_per_item=2)])
        p = pir.plan(3, 1 << 22, 64)
        assert p["kernel"] == pir.KERNEL_SMALL_BATCH and p["keys_per_item"] == 1 and p["items"] % 3 == 0, p
        p = pir.plan(1, 1 << 22, 64)
        assert p["kernel"] == pir.KERNEL_SMALL_BATCH and p["keys_per_item"] == 2, p
    finally:
        pir.set_tuning([])
    assert pir.plan(1, 1 << 22, 64)["kernel"] == pir.KERNEL_STREAM


def test_plan_small_wave_batches_fill_the_gpu():
    """Few key groups: the subtree height drops below the register limit (9)
    until the items fill the GPU's 4096 wave slots, but not so far that the
    per-lane descent dominates; many groups keep the full height."""
    p = pir.plan(16, 1 << 21, 64)  # one key group
    assert p["kernel"] == pir.KERNEL_WAVES
    assert p["items"] == 4096 and p["subtree_log"] == 7
    assert p["descent_levels"] + p["subtree_log"] == 21
    p = pir.plan(32, 1 << 20, 64)  # two key groups
    assert p["items"] == 4096 and p["subtree_log"] == 7
    assert pir.plan(64, 1 << 20, 64)["subtree_log"] == 7
    assert pir.plan(128, 1 << 20, 64)["subtree_log"] == 8
    for keys in (256, 1024, 4096):
        assert pir.plan(keys, 1 << 20, 64)["subtree_log"] == 9
    for keys in (33, 40, 47, 100, 300, 5000):  # 33, 40, 100 and 5000: the first launch, past the remainder
        p = pir.plan(keys, 1 << 20, 64)
        assert p["kernel"] == pir.KERNEL_WAVES
        assert p["items"] >= 4096 and 3 <= p["subtree_log"] <= 9, (keys, p)


def test_plan_kernel_choice():
    assert pir.plan(1024, 1 << 20, 129)["kernel"] == pir.KERNEL_SMALL_BATCH  # rows wider than 128 words
    assert pir.plan(1024, 1 << 20, 65)["kernel"] == pir.KERNEL_WAVES
    assert pir.plan(1024, 1 << 20, 128)["kernel"] == pir.KERNEL_WAVES
    assert pir.plan(16, 1 << 20, 64)["kernel"] == pir.KERNEL_SMALL_BATCH     # AES-128, up to 2^20 rows: 16 keys
    assert pir.plan(31, 1 << 20, 64)["kernel"] == pir.KERNEL_SMALL_BATCH     # AES-128 on 2^20 rows: up to 31 keys
    assert pir.plan(32, 1 << 20, 64)["kernel"] == pir.KERNEL_WAVES
    assert pir.plan(127, 1 << 18, 64)["kernel"] == pir.KERNEL_SMALL_BATCH    # 2^18 rows: up to 127
    assert pir.plan(128, 1 << 18, 64)["kernel"] == pir.KERNEL_WAVES
    assert pir.plan(2047, 1 << 14, 64)["kernel"] == pir.KERNEL_SMALL_BATCH   # 2^14 rows: up to 2047
    assert pir.plan(2048, 1 << 14, 64)["kernel"] == pir.KERNEL_WAVES
    assert pir.plan(8, (1 << 20) + 1, 64)["kernel"] == pir.KERNEL_SMALL_BATCH  # larger domains: 8 keys
    assert pir.plan(9, (1 << 20) + 1, 64)["kernel"] == pir.KERNEL_WAVES
    assert pir.plan(16, 1 << 20, 64, prf="chacha20")["kernel"] == pir.KERNEL_SMALL_BATCH  # ChaCha20: 16
    assert pir.plan(255, 1 << 20, 64, prf="chacha20")["kernel"] == pir.KERNEL_SMALL_BATCH  # up to 255 on 2^20
    assert pir.plan(256, 1 << 20, 64, prf="chacha20")["kernel"] == pir.KERNEL_WAVES
    assert pir.plan(1024, 1 << 17, 64, prf="chacha20")["kernel"] == pir.KERNEL_SMALL_BATCH
    assert pir.plan(25, (1 << 20) + 1, 64, prf="chacha20")["kernel"] == pir.KERNEL_WAVES
    assert pir.plan(25, 1 << 20, 100, prf="chacha20")["kernel"] == pir.KERNEL_WAVES  # wider rows: from 17
    # ChaCha20 on rows of 65..128 words above 2^20 rows: the wave kernel from 9 keys
    assert pir.plan(9, (1 << 20) + 1, 100, prf="chacha20")["kernel"] == pir.KERNEL_WAVES
    assert pir.plan(8, (1 << 20) + 1, 100, prf="chacha20")["kernel"] == pir.KERNEL_SMALL_BATCH
    assert pir.plan(16, (1 << 20) + 1, 64, prf="chacha20")["kernel"] == pir.KERNEL_SMALL_BATCH
    assert pir.plan(16, 1 << 20, 128, prf="chacha20")["kernel"] == pir.KERNEL_SMALL_BATCH
    assert pir.plan(16, (1 << 20) + 1, 129, prf="chacha20")["kernel"] == pir.KERNEL_SMALL_BATCH
    # the small-batch kernel takes at most 8 keys per workgroup on rows of two column chunks
    assert pir.plan(16, 1 << 20, 64)["keys_per_item"] == 16
    assert pir.plan(16, 1 << 20, 65)["keys_per_item"] == 8
    assert pir.plan(16, 1 << 20, 128)["keys_per_item"] == 8
    assert pir.plan(5, 1 << 20, 128)["keys_per_item"] == 8
    assert pir.plan(16, 1 << 20, 129)["keys_per_item"] == 16
    # a remainder of 1..8 keys past whole groups of 16 runs as a second, small-batch launch
    p = pir.plan(17, 1 << 20, 64)
    assert p["tail_keys"] == 1 and p["kernel"] == pir.KERNEL_SMALL_BATCH and p["keys_per_item"] == 16
    p = pir.plan(40, 1 << 20, 64)
    assert p["tail_keys"] == 8 and p["kernel"] == pir.KERNEL_WAVES and p["items"] % 2 == 0
    assert pir.plan(41, 1 << 20, 64)["tail_keys"] == 0      # a remainder of 9 fills its group well enough
    assert pir.plan(32, 1 << 20, 64)["tail_keys"] == 0
    assert pir.plan(16, 1 << 20, 64)["tail_keys"] == 0
    assert pir.plan(20, 1 << 16, 64)["tail_keys"] == 0      # small domains stay one launch
    assert pir.plan(20, 1 << 17, 64)["tail_keys"] == 4
    assert pir.plan(40, 1 << 18, 64)["tail_keys"] == 0      # up to 64 keys below 2^19 rows: remainders of 1..4
    assert pir.plan(36, 1 << 18, 64)["tail_keys"] == 4
    assert pir.plan(24, 1 << 17, 64)["tail_keys"] == 0
    assert pir.plan(40, (1 << 18) + 1, 64)["tail_keys"] == 8
    assert pir.plan(70, 1 << 17, 64)["tail_keys"] == 6
    assert pir.plan(1 << 22, 4, 8)["kernel"] == pir.KERNEL_SMALL_BATCH       # n = 2: too small for waves
    assert pir.plan(1 << 22, 8, 8)["kernel"] == pir.KERNEL_WAVES             # n = 3: from 32 * 2^17 keys
    assert pir.plan(25, 1 << 17, 100)["kernel"] == pir.KERNEL_WAVES          # wider rows: from 17 keys
    assert pir.plan(255, 1 << 14, 100)["kernel"] == pir.KERNEL_SMALL_BATCH   # small domains: from 64 2^(16-n)
    assert pir.plan(256, 1 << 14, 100)["kernel"] == pir.KERNEL_WAVES
    assert pir.plan(511, 1 << 14, 100, prf="chacha20")["kernel"] == pir.KERNEL_SMALL_BATCH
    assert pir.plan(512, 1 << 14, 100, prf="chacha20")["kernel"] == pir.KERNEL_WAVES
    rng = np.random.default_rng(5)
    for _ in range(300):
        keys = int(rng.integers(1, 5000))
        rows = int(rng.integers(1, 1 << int(rng.integers(1, 33))))
        dim = int(rng.integers(1, 257))
        p = pir.plan(keys, rows, dim)
        n = max(1, (rows - 1).bit_length())
        assert p["n"] == n
        tail = p["tail_keys"]
        if tail:  # a remainder past whole groups of 16 goes to a second launch
            assert 1 <= tail <= 8 and keys > 16 and keys % 16 == tail and n >= 17
            assert not (n < 19 and keys <= 64 and tail > 4)
        else:
            assert keys <= 16 or keys % 16 == 0 or keys % 16 > 8 or n < 17 or (n < 19 and keys <= 64 and keys % 16 > 4)
        keys -= tail
        if dim > 64:
            wave_min = 9 if n > 20 else 17 if n > 16 else 64 << (16 - n)
        else:
            wave_min = 9 if n > 20 else 32 << (20 - n)
        assert (p["kernel"] == pir.KERNEL_WAVES) == (keys >= wave_min and dim <= 128 and n >= 3), (keys, rows, dim)
        if p["kernel"] == pir.KERNEL_WAVES:
            assert p["descent_levels"] + p["subtree_log"] == n
            chunks = -(-rows // p["rows_per_item"])
            if dim > 64:  # wave pairs take the chunks two at a time
                chunks = 2 * -(-chunks // 2)
            assert p["items"] == chunks * -(-keys // 16)
        else:
            assert p["descent_levels"] + p["bfs_levels"] + p["subtree_log"] == n
            chunks = -(-rows // p["rows_per_item"])
            assert p["workgroups"] == chunks * -(-keys // p["keys_per_item"])
            assert p["items"] == p["workgroups"]
            assert 1 <= p["subtree_log"] <= 10


def test_plan_rejects_bad_arguments(lib):
    out = pir.PirPlan()
    assert lib.pir_plan(0, 1, 1 << 10, 8, ctypes.byref(out)) == pir.PIR_OK
    for args in ((2, 1, 1 << 10, 8), (0, 0, 1 << 10, 8), (0, 1, 0, 8), (0, 1, 1 << 10, 0),
                 (0, 1, 1 << 10, 257), (0, 1, (1 << 32) + 1, 8)):
        assert lib.pir_plan(*args, ctypes.byref(out)) == pir.PIR_EINVAL, args
    assert lib.pir_plan(0, 1, 1 << 10, 8, None) == pir.PIR_EINVAL


def test_prf_engine_library_exports_and_rejects_bad_arguments():
    """The PRF-engine measurement kernel (bench.py's PRF ceiling) is a library
    of its own; bad arguments are refused before anything is launched."""
    import ctypes

    from paper_2301_10904_amd import build as pbuild

    if not pbuild.ENGINE_LIB.exists():
        pytest.skip("libpir_engine.so not built")
    eng = ctypes.CDLL(str(pbuild.ENGINE_LIB))
    eng.pir_prf_engine.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                   ctypes.c_void_p]
    eng.pir_prf_engine.restype = ctypes.c_int
    assert eng.pir_prf_engine(0, 1, 1, None, None) == -1        # no output buffer
    assert eng.pir_prf_engine(4, 1, 1, ctypes.c_void_p(16), None) == -1  # unknown engine
    assert eng.pir_prf_engine(0, 0, 1, ctypes.c_void_p(16), None) == -1  # no workgroups
    eng.pir_prf_engine_lanes.argtypes = [ctypes.c_uint32]
    eng.pir_prf_engine_lanes.restype = ctypes.c_uint32
    assert [eng.pir_prf_engine_lanes(k) for k in range(5)] == [512, 512, 512, 256, 0]
    f = eng.pir_prf_bitsliced_pairs
    f.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    assert f(None, 32, ctypes.c_void_p(16), None) == -1               # no seeds
    assert f(ctypes.c_void_p(16), 32, None, None) == -1               # no output
    assert f(ctypes.c_void_p(16), (1 << 26) + 1, ctypes.c_void_p(16), None) == -1  # too many seeds
    assert f(None, 0, None, None) == 0                                # nothing to do


def test_peak_probes_export_and_reject_bad_arguments():
    """The peak probes (bench.py's measured peaks) live in the same measurement
    library; bad arguments are refused before anything is launched."""
    import ctypes

    from paper_2301_10904_amd import build as pbuild

    if not pbuild.ENGINE_LIB.exists():
        pytest.skip("libpir_engine.so not built")
    eng = ctypes.CDLL(str(pbuild.ENGINE_LIB))
    f = eng.pir_peak_probe
    f.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint64,
                  ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    buf, out = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    assert f(0, 1, 1, buf, 1024, None, None) == -1                    # no output buffer
    assert f(5, 1, 1, buf, 1024, out, None) == -1                     # unknown probe
    assert f(1, 0, 1, buf, 1024, out, None) == -1                     # no workgroups
    assert f(0, 1, 1, None, 1024, out, None) == -1                    # read probe without input
    assert f(0, 1, 1, buf, 0, out, None) == -1                        # empty input
    assert f(0, 1, 1, buf, 1022, out, None) == -1                     # not whole 16-byte units
    assert f(0, 1, 1, ctypes.c_void_p(0x1004), 1024, out, None) == -1  # misaligned input
    assert f(0, 1 << 20, 1, buf, 1 << 46, out, None) == -1            # shares past 64-bit offsets


def test_too_much_work_is_refused_before_any_launch(lib):
    """16384 keys on a table of 2^32 rows would need 2^31 wave items: the plan
    and the call both return PIR_ENOMEM, and the call touches no device
    memory (placeholder pointers, no GPU here)."""
    import ctypes

    out = pir.PirPlan()
    assert lib.pir_plan(0, 16384, 1 << 32, 1, ctypes.byref(out)) == pir.PIR_ENOMEM
    assert lib.pir_plan(0, 16368, 1 << 32, 1, ctypes.byref(out)) == pir.PIR_OK  # 1023 groups of 16
    stride = (pir.key_size(32) + 15) // 16 * 16
    fake = ctypes.c_void_p(0x100000)
    assert lib.pir_answer(fake, 16384, stride, fake, 1 << 32, 1, fake, None) == pir.PIR_ENOMEM
    assert lib.pir_answer_prf(1, fake, 16384, stride, fake, 1 << 32, 1, fake, None) == pir.PIR_ENOMEM


def test_workspace_api_without_gpu(lib):
    """The status workspace: its size, and the binding rules (checked on the
    host; a bound workspace is only dereferenced by kernels)."""
    assert lib.pir_workspace_size() == pir.WORKSPACE_BYTES == 256
    fake = ctypes.c_void_p(0x10000)
    assert lib.pir_set_workspace(fake, 255) == pir.PIR_EINVAL                  # too short
    assert lib.pir_set_workspace(ctypes.c_void_p(0x10008), 256) == pir.PIR_EINVAL  # not 16-byte aligned
    assert lib.pir_set_workspace(fake, 256) == pir.PIR_OK
    assert lib.pir_set_workspace(fake, 4096) == pir.PIR_OK
    assert lib.pir_set_workspace(None, 0) == pir.PIR_OK                        # unbind
    assert lib.pir_workspace_status(None, None) == pir.PIR_EINVAL
    assert lib.pir_workspace_status(ctypes.c_void_p(0x10004), None) == pir.PIR_EINVAL
    # argument errors are still found before any device work, with or without a binding
    assert lib.pir_set_workspace(fake, 256) == pir.PIR_OK
    ks = pir.key_size(10)
    assert lib.pir_answer(fake, 1, ks, fake, 1024, 0, fake, None) == pir.PIR_EINVAL
    assert lib.pir_set_workspace(None, 0) == pir.PIR_OK


def test_workspace_binding_is_per_thread(lib):
    """A binding made by one thread does not change another's: a short buffer
    is rejected in every thread, and each thread's unbind leaves the others."""
    import threading

    res = {}

    def worker(i):
        res[i] = (lib.pir_set_workspace(ctypes.c_void_p(0x20000 + 256 * i), 256),
                  lib.pir_set_workspace(ctypes.c_void_p(0x20000), 16),
                  lib.pir_set_workspace(None, 0))

    ts = [threading.Thread(target=worker, args=(i,)) for i in range(4)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert all(r == (pir.PIR_OK, pir.PIR_EINVAL, pir.PIR_OK) for r in res.values())


def test_plan_wave_pairs_count_items_in_pairs():
    """Rows of 65..128 words run as wave pairs: two waves on adjacent chunks of
    a bin share a key group, so a plan counts a bin's chunks rounded up to an
    even number, and every launch's item count is even (both waves of a pair
    exist and leave together)."""
    for prf in ("aes128", "chacha20"):
        for rows in (9000, 5 * 2048 + 7, 1 << 20, (1 << 20) + 5):
            for dim in (65, 100, 128):
                for keys in (64, 1024):
                    p = pir.plan(keys, rows, dim, prf=prf)
                    if p["kernel"] != pir.KERNEL_WAVES:
                        continue
                    chunks = -(-rows // p["rows_per_item"])
                    assert p["items"] % 2 == 0
                    assert p["items"] == 2 * -(-chunks // 2) * -(-(keys - p["tail_keys"]) // 16), (rows, dim, keys, p)
        for rows, bin_log, clients in ((3000, 10, 17), (1 << 14, 12, 5), (5 * 2048 + 7, 13, 40)):
            p = pir.plan_bins(rows, 100, clients, bin_log, prf=prf)
            bin_rows = min(rows, 1 << bin_log)
            chunks = -(-bin_rows // p["rows_per_item"])
            assert p["items"] == pir.n_bins(rows, bin_log) * 2 * -(-chunks // 2) * -(-clients // 16), p


@pytest.mark.parametrize("rows", [1, 2, 3, 4, 5, 8, 9, 777, 1 << 14])
@pytest.mark.parametrize("bin_log", [3, 4, 10, 32])
def test_plan_bins_subtree_height_stays_in_the_bin(rows, bin_log):
    """Partial batch retrieval plans: the per-lane subtree height h satisfies
    1 <= h <= bin_log and never exceeds the aligned subtree holding a bin's rows
    (tables of 1..4 rows included), and the items cover every bin."""
    for prf in ("aes128", "chacha20"):
        for clients in (1, 16, 17):
            p = pir.plan_bins(rows, 16, clients, bin_log, prf=prf)
            bin_rows = min(rows, 1 << bin_log)
            m = max(1, (bin_rows - 1).bit_length())
            assert p["kernel"] == pir.KERNEL_WAVES and p["n"] == bin_log
            assert 1 <= p["subtree_log"] <= min(m, bin_log, 9), p
            assert p["descent_levels"] == bin_log - p["subtree_log"]
            assert p["rows_per_item"] == 4 << p["subtree_log"]
            chunks = -(-bin_rows // p["rows_per_item"])
            assert p["items"] == pir.n_bins(rows, bin_log) * chunks * (-(-clients // 16))


def test_plan_bins_rejects_what_answer_bins_rejects():
    for args in [(1 << 10, 129, 1, 5), (1 << 10, 16, 1, 2), (0, 16, 1, 5), (1 << 10, 16, 0, 5), (1 << 10, 16, 1, 33)]:
        with pytest.raises(pir.PirError):
            pir.plan_bins(*args)
