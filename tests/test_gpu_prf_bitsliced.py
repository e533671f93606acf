"""The bitsliced AES-128 PRF of the PRF-engine library (a measured alternative
to the T-table rounds; the PIR kernels do not use it) computes the PRF the
oracle defines: PRF_s(0) and PRF_s(1) of every seed, through the bit-plane
transposes and the quad's DPP exchanges, on full and ragged groups of 32
seeds.  The timed engine chains are checked too: with one step, every lane's
checksum is recomputed from the oracle's PRF outputs of the seeds the lane
started from."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

M32 = (1 << 32) - 1


@pytest.fixture(scope="module")
def eng(gpu_lib):
    from paper_2301_10904_amd import build as pbuild

    if not pbuild.ENGINE_LIB.exists():
        pytest.fail("libpir_engine.so is not built")
    lib = ctypes.CDLL(str(pbuild.ENGINE_LIB))
    lib.pir_prf_bitsliced_pairs.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
    lib.pir_prf_bitsliced_pairs.restype = ctypes.c_int
    lib.pir_prf_engine.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                   ctypes.c_void_p]
    lib.pir_prf_engine.restype = ctypes.c_int
    lib.pir_prf_engine_lanes.argtypes = [ctypes.c_uint32]
    lib.pir_prf_engine_lanes.restype = ctypes.c_uint32
    return lib


def stream_ptr():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def bitsliced_pairs(eng, seeds: np.ndarray) -> np.ndarray:
    import torch

    n = len(seeds)
    d_seeds = torch.from_numpy(np.ascontiguousarray(seeds).view(np.int32).reshape(-1).copy()).cuda()
    out = torch.full((n * 8,), -1, dtype=torch.int32, device="cuda")
    rc = eng.pir_prf_bitsliced_pairs(ctypes.c_void_p(d_seeds.data_ptr()), n, ctypes.c_void_p(out.data_ptr()),
                                     stream_ptr())
    assert rc == 0
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32).reshape(n, 8)


def oracle_words(O, seed: bytes, x: int) -> np.ndarray:
    return np.frombuffer(O.prf(seed, x), dtype="<u4")


@pytest.mark.parametrize("n", [1, 31, 32, 33, 1000, 4096 + 17])
def test_bitsliced_prf_matches_the_oracle(O, eng, n):
    rng = np.random.default_rng(1000 + n)
    seeds = rng.integers(0, 256, (n, 16), dtype=np.uint8)
    seeds[0] = 0
    if n > 2:
        seeds[1] = 0xFF
        seeds[2] = np.arange(16, dtype=np.uint8)
    got = bitsliced_pairs(eng, seeds)
    for i in range(n):
        s = seeds[i].tobytes()
        assert (got[i, :4] == oracle_words(O, s, 0)).all(), (i, "block 0")
        assert (got[i, 4:] == oracle_words(O, s, 1)).all(), (i, "block 1")


def test_bitsliced_prf_rejects_bad_arguments(eng):
    import torch

    buf = torch.zeros(64, dtype=torch.int32, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    assert eng.pir_prf_bitsliced_pairs(None, 4, p, stream_ptr()) == -1
    assert eng.pir_prf_bitsliced_pairs(p, 4, None, stream_ptr()) == -1
    assert eng.pir_prf_bitsliced_pairs(p, (1 << 26) + 1, p, stream_ptr()) == -1
    assert eng.pir_prf_bitsliced_pairs(None, 0, None, stream_ptr()) == 0


def run_engine(eng, kind, blocks, steps):
    import torch

    lanes = eng.pir_prf_engine_lanes(kind)
    out = torch.zeros(blocks * lanes, dtype=torch.int32, device="cuda")
    assert eng.pir_prf_engine(kind, blocks, steps, ctypes.c_void_p(out.data_ptr()), stream_ptr()) == 0
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


def test_engine_lanes_per_kind(eng):
    assert [eng.pir_prf_engine_lanes(k) for k in range(5)] == [512, 512, 512, 256, 0]


def test_bitsliced_engine_one_step(O, eng):
    """Lane q of quad j starts from 32 bit planes; transposed, they are word q
    of the quad's 32 seeds.  After one step its checksum is plane 0 of its
    column of PRF_s(0): bit i is bit 0 of word q of node i's block 0."""
    steps, lanes = 1, 256
    got = run_engine(eng, 3, 1, steps)
    gid = np.arange(lanes, dtype=np.uint64)
    planes = np.array([[(((g + 1) * 0x9E3779B9) ^ (i * 0x85EBCA6B) ^ steps) & M32 for i in range(32)]
                       for g in gid], dtype=np.uint64)
    for quad in range(0, lanes // 4, 7):  # every 7th quad: 10 quads, 320 nodes
        words = np.zeros((32, 4), dtype=np.uint32)
        for q in range(4):
            p = planes[4 * quad + q]
            for node in range(32):
                words[node, q] = sum(((int(p[b]) >> node) & 1) << b for b in range(32))
        for q in range(4):
            want = 0
            for node in range(32):
                a0 = oracle_words(O, words[node].astype("<u4").tobytes(), 0)
                want |= (int(a0[q]) & 1) << node
            assert int(got[4 * quad + q]) == want, (quad, q)


def test_ttable_full_node_engine_one_step(O, eng):
    """One step of the full-node T-table chain: the checksum is word 0 of
    PRF_s(0) for the lane's starting seed."""
    blocks, steps = 2, 1
    got = run_engine(eng, 2, blocks, steps)
    for g in range(0, blocks * 512, 37):
        s = np.array([g, (0x9E3779B9 * (g + 1)) & M32, steps, 0x7F4A7C15], dtype="<u4").tobytes()
        assert int(got[g]) == int(oracle_words(O, s, 0)[0]), g


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_engines_are_deterministic(eng, kind):
    a = run_engine(eng, kind, 3, 4)
    b = run_engine(eng, kind, 3, 4)
    assert (a == b).all() and a.any()
