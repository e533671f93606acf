"""AddressSanitizer and UndefinedBehaviorSanitizer on the host C/C++ code (CPU only).

  - The oracle is rebuilt with -fsanitize=address,undefined and its whole pin
    suite runs against that build (a sanitizer report aborts the run).
  - The library's host code (Gen with its own AES-128 and ChaCha20, the
    reconstruction, the status strings) is built the same way with g++ and its
    keys are checked byte for byte against the oracle's for n = 1..32 and both
    PRFs, under the sanitizers.
The device code is not built here: GPU sanitizers are not used.
"""
import os
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))
import oracle  # noqa: E402

SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-g"]


def runtime_env():
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not libasan or not Path(libasan).exists():
        pytest.skip("libasan not available")
    env = dict(os.environ)
    env["LD_PRELOAD"] = libasan
    # the Python interpreter is not instrumented: leak reports would be its own
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return env


def test_oracle_pins_under_sanitizers(tmp_path):
    lib = oracle.build(out=tmp_path / "liboracle_san.so", extra=tuple(SAN))
    env = runtime_env()
    env["ORACLE_LIB_PATH"] = str(lib)
    suites = [str(ROOT / "tests" / f) for f in
              ("test_oracle_aes.py", "test_oracle_dpf.py", "test_oracle_chacha.py", "test_oracle_batch.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider", *suites],
                       env=env, capture_output=True, text=True, timeout=900, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]


HOST_CHECK = r"""
import ctypes, sys
import numpy as np
sys.path.insert(0, sys.argv[2])
from oracle import Oracle
lib = ctypes.CDLL(sys.argv[1])
u8p = ctypes.POINTER(ctypes.c_uint8)
lib.dpf_gen_prf.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, u8p, ctypes.c_uint32, u8p, u8p]
lib.dpf_key_size.restype = ctypes.c_size_t
O = Oracle()
rng = np.random.default_rng(77)
p = lambda a: a.ctypes.data_as(u8p)
for prf in (0, 1):
    for n in range(1, 33):
        ks = lib.dpf_key_size(n)
        for trial in range(2):
            alpha = int(rng.integers(0, 1 << n)); beta = int(rng.integers(0, 2**32))
            seed = rng.integers(0, 256, 16, dtype=np.uint8)
            k0 = np.zeros(ks, np.uint8); k1 = np.zeros(ks, np.uint8)
            assert lib.dpf_gen_prf(n, alpha, beta, p(seed), prf, p(k0), p(k1)) == 0
            o0, o1 = O.gen(n, alpha, beta, seed.tobytes(), prf_id=prf)
            assert (k0 == o0).all() and (k1 == o1).all(), (prf, n)
        # rejected arguments return before touching the buffers
        assert lib.dpf_gen_prf(n, 1 << n, 1, p(seed), prf, p(k0), p(k1)) == -1
    assert lib.dpf_gen_prf(0, 0, 1, p(seed), prf, p(k0), p(k1)) == -1
# no seed: the operating system's randomness
k0 = np.zeros(lib.dpf_key_size(5), np.uint8); k1 = np.zeros_like(k0)
assert lib.dpf_gen_prf(5, 3, 1, None, 1, p(k0), p(k1)) == 0
lib.pir_strerror.restype = ctypes.c_char_p
for s in (0, -1, -2, -3, -4, 9):
    lib.pir_strerror(s)
a = np.arange(64, dtype=np.uint32); b = np.arange(64, dtype=np.uint32); o = np.zeros(64, np.uint32)
u32p = ctypes.POINTER(ctypes.c_uint32)
assert lib.pir_reconstruct(a.ctypes.data_as(u32p), b.ctypes.data_as(u32p), 64, o.ctypes.data_as(u32p)) == 0
assert (o == 2 * a).all()
print("host code clean")
"""


def test_library_host_code_under_sanitizers(tmp_path):
    csrc = ROOT / "paper_2301_10904_amd" / "csrc"
    lib = tmp_path / "libpirhost_san.so"
    subprocess.run(["g++", "-std=c++17", "-O1", "-fPIC", "-shared", *SAN, f"-I{ROOT / 'include'}", f"-I{csrc}",
                    str(csrc / "pir_host.cpp"), "-o", str(lib)], check=True)
    env = runtime_env()
    r = subprocess.run([sys.executable, "-c", HOST_CHECK, str(lib), str(ROOT)], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "host code clean" in r.stdout, r.stdout[-3000:] + r.stderr[-3000:]


def test_sanitizer_build_catches_a_planted_overflow(tmp_path):
    """Control: the same sanitized build of an oracle copy with an out-of-bounds
    read planted in the ChaCha20 PRF must abort the pin suite."""
    import shutil

    for s in oracle.SOURCES + ("oracle.h",):
        shutil.copy(oracle.HERE / s, tmp_path / s)
    src = (tmp_path / "dpf_ref.c").read_text()
    old = "memcpy(out, blk + 16 * (x % 4), 16);"
    assert src.count(old) == 1
    (tmp_path / "dpf_ref.c").write_text(src.replace(old, "memcpy(out, blk + 16 * (x % 4) + 56, 16);"))
    lib = oracle.build(out=tmp_path / "liboracle_bad.so", src_dir=tmp_path, extra=tuple(SAN) + ("-w",))
    env = runtime_env()
    env["ORACLE_LIB_PATH"] = str(lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider",
                        str(ROOT / "tests" / "test_oracle_chacha.py")],
                       env=env, capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode != 0
    assert "AddressSanitizer" in r.stdout + r.stderr, (r.stdout[-2000:], r.stderr[-2000:])
