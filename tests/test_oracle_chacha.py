"""Pins for the oracle's ChaCha20 and for the DPF built on it (the alternative
PRF of paper section 3.2.6, Table 5).

Pinned against the vectors RFC 8439 prints (quarter round, block function),
against the host's OpenSSL command line tool as a library routine (skipped
when the tool is absent), and, for the DPF, against the same facts the
AES-keyed DPF is pinned to: the point-function identity by brute force, the
node structure at every depth, and the tree step of Eq. (p3) recomputed with
OpenSSL's ChaCha20 keystream as the PRF.
"""
import shutil
import subprocess

import numpy as np
import pytest

from conftest import read_golden
from test_oracle_dpf import BETAS, indicator, numpy_answer, seed_for, tbit

CHACHA = 1
openssl = shutil.which("openssl")


def _keystream(key32: bytes, nbytes: int, counter: int = 0, nonce: bytes = bytes(12)) -> bytes:
    """OpenSSL's ChaCha20: its 16-byte iv is the block counter (little-endian)
    followed by the 96-bit nonce."""
    iv = counter.to_bytes(4, "little") + nonce
    cmd = [openssl, "enc", "-chacha20", "-K", key32.hex(), "-iv", iv.hex()]
    return subprocess.run(cmd, input=bytes(nbytes), capture_output=True, check=True).stdout


def test_quarter_round_rfc8439(O):
    g = read_golden("rfc8439_chacha20.txt")
    inp = [int(w, 16) for w in g["qr_in"].split()]
    out = [int(w, 16) for w in g["qr_out"].split()]
    assert list(O.chacha20_quarter(*inp)) == out


@pytest.mark.parametrize("vec", ["block1", "block2", "block3"])
def test_block_function_rfc8439(O, vec):
    g = read_golden("rfc8439_chacha20.txt")
    got = O.chacha20_block(bytes.fromhex(g[f"{vec}_key"]), int(g[f"{vec}_counter"]),
                           bytes.fromhex(g[f"{vec}_nonce"]))
    assert got.hex() == g[f"{vec}_out"]


def test_quarter_round_is_a_permutation_step(O):
    """Every step of the quarter round is invertible (add, xor, rotate), so
    distinct inputs give distinct outputs; and it is not the identity."""
    rng = np.random.default_rng(11)
    seen = set()
    for _ in range(200):
        v = tuple(int(x) for x in rng.integers(0, 2**32, 4, dtype=np.uint64))
        o = O.chacha20_quarter(*v)
        assert o != v
        seen.add(o)
    assert len(seen) == 200


@pytest.mark.skipif(openssl is None, reason="openssl command line tool not installed")
def test_block_function_against_openssl(O):
    rng = np.random.default_rng(12)
    for _ in range(8):
        key = rng.integers(0, 256, 32, dtype=np.uint8).tobytes()
        nonce = rng.integers(0, 256, 12, dtype=np.uint8).tobytes()
        ctr = int(rng.integers(0, 2**32 - 4))
        ref = _keystream(key, 128, ctr, nonce)
        assert O.chacha20_block(key, ctr, nonce) + O.chacha20_block(key, ctr + 1, nonce) == ref


@pytest.mark.skipif(openssl is None, reason="openssl command line tool not installed")
def test_prf_is_keystream_under_doubled_seed(O):
    """PRF_s(x) = bytes [16x, 16x+16) of the keystream under key s || s,
    nonce 0, counter from 0; PRF_s(0) || PRF_s(1) is half of block 0."""
    rng = np.random.default_rng(13)
    for _ in range(10):
        s = rng.integers(0, 256, 16, dtype=np.uint8).tobytes()
        ref = _keystream(s + s, 128)
        assert b"".join(O.prf_chacha(s, x) for x in range(8)) == ref
        assert O.prf_by(CHACHA, s, 1) == ref[16:32]
        assert O.prf_by(0, s, 1) == O.prf(s, 1)


def test_unknown_prf_rejected(O):
    with pytest.raises(ValueError):
        O.prf_by(2, bytes(16), 0)
    with pytest.raises(ValueError):
        O.gen(4, 3, 1, bytes(16), prf_id=2)
    k0, _ = O.gen(4, 3, 1, bytes(16), prf_id=CHACHA)
    bad = k0.copy()
    bad[3] = 2
    with pytest.raises(ValueError):
        O.answer(bad, np.zeros((16, 2), np.uint32))


@pytest.mark.parametrize("n", range(1, 6))
def test_dpf_identity_every_alpha(O, n):
    for alpha in range(1 << n):
        beta = BETAS[alpha % len(BETAS)]
        k0, k1 = O.gen(n, alpha, beta, seed_for(n, alpha, 20), prf_id=CHACHA)
        assert k0[3] == CHACHA and k1[3] == CHACHA
        s = (O.eval_full(k0) + O.eval_full(k1)).astype(np.uint32)
        assert (s == indicator(n, alpha, beta)).all(), (n, alpha)


@pytest.mark.parametrize("n", [8, 11])
@pytest.mark.parametrize("beta", [1, 2**32 - 1, 0x9E3779B9])
def test_dpf_identity_random_alpha(O, n, beta):
    rng = np.random.default_rng([n, beta, 20])
    alpha = int(rng.integers(0, 1 << n))
    k0, k1 = O.gen(n, alpha, beta, seed_for(n, beta, 20), prf_id=CHACHA)
    s = (O.eval_full(k0) + O.eval_full(k1)).astype(np.uint32)
    assert (s == indicator(n, alpha, beta)).all()


def test_large_domain_point_identity(O):
    n, alpha = 32, 0x1234ABCD
    k0, k1 = O.gen(n, alpha, 9, seed_for(32, 20), prf_id=CHACHA)
    for j in (alpha, alpha - 1, alpha + 1, 0, 2**32 - 1):
        got = (O.eval_point(k0, j) + O.eval_point(k1, j)) & 0xFFFFFFFF
        assert got == (9 if j == alpha else 0)


@pytest.mark.parametrize("n,alpha,beta", [(6, 45, 1), (9, 511, 3)])
def test_node_invariants(O, n, alpha, beta):
    k0, k1 = O.gen(n, alpha, beta, seed_for(n, alpha, beta, 20), prf_id=CHACHA)
    for d in range(0, n + 1):
        L0, L1 = O.eval_level(k0, d), O.eval_level(k1, d)
        on = alpha >> (n - d)
        off = np.arange(1 << d) != on
        assert (L0[off] == L1[off]).all(), d
        if d < n:
            assert tbit(L0[on]) != tbit(L1[on]), d
        else:
            lo0 = int.from_bytes(L0[on][:4].tobytes(), "little")
            lo1 = int.from_bytes(L1[on][:4].tobytes(), "little")
            assert (lo0 - lo1) % 2**32 == beta


@pytest.mark.skipif(openssl is None, reason="openssl command line tool not installed")
def test_tree_step_uses_chacha_keystream(O):
    """Eq. (p3) with the PRF taken from OpenSSL: every node at depths 1..3 is
    the keystream of its parent's seed (key parent || parent), block half
    j mod 2, XOR the codeword selected by the parent's control bit."""
    n = 3
    k0, k1 = O.gen(n, 5, 1, seed_for(3, 20), prf_id=CHACHA)
    for key in (k0, k1):
        levels = [key[16:32][None, :]] + [O.eval_level(key, d) for d in range(1, n + 1)]
        for d in range(1, n + 1):
            for j in range(1 << d):
                parent = levels[d - 1][j // 2].tobytes()
                ks = _keystream(parent + parent, 32)
                c = j % 2
                off = 32 + 64 * (d - 1) + 32 * tbit(levels[d - 1][j // 2]) + 16 * c
                want = np.frombuffer(ks[16 * c:16 * c + 16], np.uint8) ^ key[off:off + 16]
                assert (levels[d][j] == want).all(), (d, j)


def test_answer_reconstruct_and_work_counts(O):
    rng = np.random.default_rng(21)
    rows, dim, n = 90, 9, 7
    T = rng.integers(0, 2**32, (rows, dim), dtype=np.uint64).astype(np.uint32)
    for alpha in (0, 44, 89):
        k0, k1 = O.gen(n, alpha, 1, seed_for(rows, alpha, 20), prf_id=CHACHA)
        a0, a1 = O.answer(k0, T), O.answer(k1, T)
        assert (a0 == numpy_answer(O.eval_full(k0), T)).all()
        assert (O.reconstruct(a0, a1) == T[alpha]).all()
    O.reset_counts()
    O.eval_full(k0)
    assert O.counts() == (2 * ((1 << n) - 1), 0)
    O.reset_counts()
    O.gen(n, 3, 1, seed_for(1), prf_id=CHACHA)
    assert O.counts() == (4 * n, 3 * n + 1)


def test_prf_choice_changes_keys_not_draws(O):
    """The random draws are the same for both PRFs: the roots and the first
    level's random codewords agree; the PRF-dependent codewords differ."""
    sd = seed_for(77)
    a0, _ = O.gen(10, 600, 1, sd, prf_id=0)
    c0, _ = O.gen(10, 600, 1, sd, prf_id=CHACHA)
    assert (a0[16:32] == c0[16:32]).all()
    tau = tbit(a0[16:32])
    lvl1 = slice(32 + 32 * tau, 64 + 32 * tau)  # C_tau[0, 1], C_tau[1, 1] = R, R'
    assert (a0[lvl1] == c0[lvl1]).all()
    assert not (a0[32:] == c0[32:]).all()
