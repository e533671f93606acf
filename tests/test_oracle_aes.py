"""Pins for the oracle's AES-128 and counter mode (the PRF of paper section 3.1).

Pinned against published values (FIPS-197, SP 800-38A), against algebraic
properties of the S-box, and against the host's OpenSSL command line tool as a
library routine (skipped when the tool is absent).
"""
import shutil
import subprocess

import numpy as np
import pytest

from conftest import read_golden


def test_fips197_vectors(O):
    g = read_golden("fips197_aes128.txt")
    for p in ("c1", "b"):
        ct = O.aes128(bytes.fromhex(g[f"{p}_key"]), bytes.fromhex(g[f"{p}_plaintext"]))
        assert ct.hex() == g[f"{p}_ciphertext"]
    w = O.expand_key(bytes.fromhex(g["b_key"]))
    assert w[16:32].hex() == g["a1_w4_w7"]
    assert w[160:176].hex() == g["a1_w40_w43"]
    # the first Nk words of the schedule are the key itself
    assert w[:16].hex() == g["b_key"]


def test_sbox_properties(O):
    g = read_golden("fips197_aes128.txt")
    s = O.sbox()
    assert s[0x53] == int(g["sbox_53"], 16)
    assert s[0x00] == int(g["sbox_00"], 16)
    assert sorted(s.tolist()) == list(range(256)), "S-box must be a permutation"
    assert all(s[x] != x for x in range(256)), "AES S-box has no fixed points"
    assert all(s[x] != (x ^ 0xFF) for x in range(256)), "nor opposite fixed points"


def test_ctr_mode_sp800_38a(O):
    """CTR block = AES_K(counter) XOR plaintext; our PRF takes counters 0, 1, ..."""
    g = read_golden("sp800_38a_ctr.txt")
    ks = O.aes128(bytes.fromhex(g["key"]), bytes.fromhex(g["counter"]))
    ct = bytes(a ^ b for a, b in zip(ks, bytes.fromhex(g["plaintext"])))
    assert ct.hex() == g["ciphertext"]


def test_prf_is_counter_block(O):
    """PRF_s(x) = AES_s(x as a 128-bit big-endian counter block)."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        s = rng.integers(0, 256, 16, dtype=np.uint8).tobytes()
        for x in (0, 1, 2, 255, 256, 2**40 + 3):
            assert O.prf(s, x) == O.aes128(s, x.to_bytes(16, "big"))


openssl = shutil.which("openssl")


def _ossl(mode, key: bytes, data: bytes, iv: bytes | None = None) -> bytes:
    cmd = [openssl, "enc", "-" + mode, "-nopad", "-K", key.hex()]
    if iv is not None:
        cmd += ["-iv", iv.hex()]
    return subprocess.run(cmd, input=data, capture_output=True, check=True).stdout


@pytest.mark.skipif(openssl is None, reason="openssl command line tool not installed")
def test_aes_against_openssl_ecb(O):
    rng = np.random.default_rng(2024)
    n = 1000
    keys = rng.integers(0, 256, (n, 16), dtype=np.uint8)
    # one openssl run per distinct key would be slow; use 20 keys x 50 blocks
    for i in range(20):
        key = keys[i].tobytes()
        blocks = rng.integers(0, 256, (50, 16), dtype=np.uint8).tobytes()
        ref = _ossl("aes-128-ecb", key, blocks)
        got = b"".join(O.aes128(key, blocks[16 * b:16 * b + 16]) for b in range(50))
        assert got == ref


@pytest.mark.skipif(openssl is None, reason="openssl command line tool not installed")
def test_prf_and_drbg_against_openssl_ctr(O):
    """PRF_s(0..3) and DRBG draws are the AES-128-CTR keystream from counter 0."""
    rng = np.random.default_rng(7)
    for _ in range(10):
        s = rng.integers(0, 256, 16, dtype=np.uint8).tobytes()
        ref = _ossl("aes-128-ctr", s, bytes(64), bytes(16))
        assert b"".join(O.prf(s, x) for x in range(4)) == ref
        assert b"".join(O.drbg(s, x) for x in range(4)) == ref
