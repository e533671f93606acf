"""The peak probes behind bench.py's measured peaks do the work they are
counted for: every lane's checksum is recomputed on the host from the probe's
definition (the HBM read sums the buffer, the VALU chains XOR a constant, the
LDS chains walk the table, the matrix-core accumulators add A B each
iteration).  Small launches; bit-exact uint32 comparisons."""
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
    lib.pir_peak_probe.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                   ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
    lib.pir_peak_probe.restype = ctypes.c_int
    return lib


def run(eng, kind, blocks, iters, lanes, buf=None):
    import torch

    out = torch.zeros(blocks * lanes, dtype=torch.int32, device="cuda")
    ptr = ctypes.c_void_p(buf.data_ptr()) if buf is not None else None
    words = buf.numel() if buf is not None else 0
    rc = eng.pir_peak_probe(kind, blocks, iters, ptr, words, ctypes.c_void_p(out.data_ptr()),
                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("blocks", [37, 256])
@pytest.mark.parametrize("words", [4, 4 * 1000, 4 * 777777])
def test_hbm_read_sums_the_buffer(eng, words, blocks):
    """Each workgroup's share sums to its lanes' checksums: the shares cover
    the buffer once, also when it splits unevenly or has fewer 16-byte units
    than there are workgroups."""
    import torch

    rng = np.random.default_rng(words)
    host = rng.integers(0, 1 << 32, words, dtype=np.uint64).astype(np.uint32)
    buf = torch.from_numpy(host.view(np.int32)).cuda()
    got = run(eng, 0, blocks, 0, 256, buf).reshape(blocks, 256).astype(np.uint64)
    n4 = words // 4
    for b in range(blocks):
        lo, hi = b * n4 // blocks, (b + 1) * n4 // blocks
        assert int(got[b].sum()) & M32 == int(host[4 * lo:4 * hi].astype(np.uint64).sum()) & M32, b


@pytest.mark.parametrize("iters", [1, 6, 101])
def test_valu_chains(eng, iters):
    blocks, k = 3, 0x6A09E667
    g = np.arange(blocks * 256, dtype=np.uint64)
    want = np.zeros(g.shape, np.uint64)
    for c in range(16):
        x = (g * 0x9E3779B9 + c) & M32
        want += x ^ (k if iters % 2 else 0)
    got = run(eng, 1, blocks, iters, 256)
    assert (got == (want & M32).astype(np.uint32)).all()


@pytest.mark.parametrize("iters", [1, 5, 64])
def test_lds_chains(eng, iters):
    i = np.arange(16384, dtype=np.uint64)
    tab = ((i * 0x9E3779B9) & M32) ^ (i >> 5)
    t = np.arange(1024, dtype=np.uint64)
    l4 = (t % 64 % 32) * 4
    acc = np.zeros(1024, np.uint64)
    for c in range(8):
        v = (t * 0x85EBCA6B + c) & M32
        for _ in range(iters):
            v = tab[((v & 0xFF80) | l4) >> 2]
        acc ^= v
    got = run(eng, 2, 2, iters, 1024)
    assert (got.reshape(2, 1024) == acc.astype(np.uint32)).all()


def lane_bytes(words):
    """The int8 K values a lane supplies: the bytes of its operand words, in order."""
    b = np.stack([(w >> (8 * j)) & 0xFF for w in words for j in range(4)], 1)
    return b.astype(np.uint8).view(np.int8).astype(np.int64)


@pytest.mark.parametrize("kind", [3, 4])
@pytest.mark.parametrize("iters", [1, 3, 1000])
def test_mfma_accumulators(eng, kind, iters):
    """Lane l of a wave holds A[l mod 16][K (l / 16) + j] and B[K (l / 16) + j][l mod 16]
    for j < K (K = 16 bytes for the 16x16x64 form, kind 3; 8 for 16x16x32, kind
    4); its accumulator registers i = 0..3 hold D[4 (l / 16) + i][l mod 16].
    Which K index a byte stands for does not change D as long as A and B use
    the same order, which the two operands' layouts do."""
    blocks = 2
    got = run(eng, kind, blocks, iters, 256)
    g = np.arange(blocks * 256, dtype=np.uint64)
    w0 = (g * 0x9E3779B9) & M32
    w1 = g ^ 0x5BD1E995
    if kind == 3:
        w2, w3 = w0 ^ 0x3C6EF372, w1 ^ 0xA54FF53A
        av = lane_bytes([w0, w1, w2, w3])
        bv = lane_bytes([w0 ^ 0x01234567, w1 ^ 0x89ABCDEF, w2 ^ 0x0F1E2D3C, w3 ^ 0x4B5A6978])
    else:
        av = lane_bytes([w0, w1])
        bv = lane_bytes([w0 ^ 0x01234567, w1 ^ 0x89ABCDEF])
    k = av.shape[1]
    for w in range(blocks * 4):
        A = np.zeros((16, 4 * k), np.int64)
        B = np.zeros((4 * k, 16), np.int64)
        for l in range(64):
            A[l % 16, k * (l // 16):k * (l // 16) + k] = av[64 * w + l]
            B[k * (l // 16):k * (l // 16) + k, l % 16] = bv[64 * w + l]
        D = A @ B
        for l in range(64):
            s = 8 * iters * int(D[4 * (l // 16):4 * (l // 16) + 4, l % 16].sum())
            assert int(got[64 * w + l]) == s & M32, (w, l)
