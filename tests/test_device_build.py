"""Build-time checks of the HIP device code (CPU only: hipcc cross-compiles).

Every kernel that walks the tree with AES reads its tables from LDS; if the
compiler ever loses sight of those reads it may drop the table fill and the
LDS allocation (a kernel would then read unallocated LDS).  The assembled AES
kernels must each keep at least the 64 KiB table region; the ChaCha20 kernels
need no table.  No kernel may spill more than a few loop-invariant words to
scratch (64 bytes per lane).
"""
import re
import shutil
import subprocess

import pytest

from paper_2301_10904_amd import build as pbuild


@pytest.fixture(scope="module")
def device_asm(tmp_path_factory):
    hipcc = pbuild.hipcc()
    if not shutil.which(hipcc):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("asm") / "pir_device.s"
    flags = [f for f in pbuild.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    subprocess.run([hipcc, *flags, f"-I{pbuild.ROOT / 'include'}", f"-I{pbuild.CSRC}",
                    "--cuda-device-only", "-S", str(pbuild.CSRC / "pir_device.hip"), "-o", str(out)],
                   check=True, capture_output=True)
    return out.read_text()


def kernel_metadata(asm):
    meta = {}
    for block in re.split(r"\n\s*- \.", asm):
        name = re.search(r"\.name:\s+(\S+)", block)
        lds = re.search(r"\.group_segment_fixed_size:\s+(\d+)", block)
        scratch = re.search(r"\.private_segment_fixed_size:\s+(\d+)", block)
        if name and lds and scratch:
            meta[name.group(1)] = (int(lds.group(1)), int(scratch.group(1)))
    return meta


def test_tree_kernels_keep_their_lds_tables(device_asm):
    meta = kernel_metadata(device_asm)
    aes = {k: v for k, v in meta.items() if "k_pir_" in k and "AesPrf" in k}
    chacha = {k: v for k, v in meta.items() if "k_pir_" in k and "ChaChaPrf" in k}
    # every kernel has both PRFs, except the single-key stream kernel (AES-128 only)
    assert len(aes) >= 10 and len(chacha) == len(aes) - 2, sorted(meta)
    assert sum("k_pir_stream" in k for k in aes) == 2 and not any("k_pir_stream" in k for k in chacha)
    for name, (lds, scratch) in aes.items():
        assert lds >= 65536, f"{name}: LDS {lds} bytes, the AES tables need 65536"
        assert scratch <= 64, f"{name}: {scratch} bytes of scratch per lane"
    for name, (lds, scratch) in chacha.items():
        assert lds < 65536, f"{name}: LDS {lds} bytes; ChaCha20 needs no table"
        assert scratch <= 64, f"{name}: {scratch} bytes of scratch per lane"



def test_plans_report_the_wave_kernels_lds(device_asm):
    """pir_plan's lds_bytes for the wave kernel is the static LDS the assembled
    kernel allocates: the AES tables for rows of up to 64 words, and for the
    wave pairs of 65..128-word rows the tables plus the share ring."""
    from paper_2301_10904_amd import pir

    meta = kernel_metadata(device_asm)

    def lds_of(sub):
        found = {lds for name, (lds, _) in meta.items() if sub in name}
        assert len(found) == 1, (sub, found)
        return found.pop()

    pairs_aes = lds_of("k_pir_waves_pairsINS_6AesPrf")
    pairs_chacha = lds_of("k_pir_waves_pairsINS_9ChaChaPrf")
    assert pir.plan(1024, 1 << 20, 128)["lds_bytes"] == pairs_aes
    assert pir.plan(1024, 1 << 20, 100, prf="chacha20")["lds_bytes"] == pairs_chacha
    assert pir.plan_bins(1 << 20, 128, 64, 12)["lds_bytes"] == pairs_aes
    assert pir.plan(1024, 1 << 20, 64)["lds_bytes"] == lds_of("k_pir_wavesINS_6AesPrfELi4ELb1")

def test_bitsliced_prf_engine_builds_without_scratch():
    """The bitsliced AES-128 engine (measurement library) compiles, which runs
    its compile-time checks of the tower-field S-box circuit against the
    FIPS-197 S-box on all 256 bytes and of the bit transpose, and keeps its 96
    state planes in registers: no scratch and no LDS."""
    hipcc = pbuild.hipcc()
    if not shutil.which(hipcc):
        pytest.skip("hipcc not available")
    import tempfile
    from pathlib import Path

    flags = [f for f in pbuild.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    with tempfile.TemporaryDirectory() as d:
        out = Path(d) / "prf_engine.s"
        subprocess.run([hipcc, *flags, f"-I{pbuild.ROOT / 'include'}", f"-I{pbuild.CSRC}",
                        "--cuda-device-only", "-S", str(pbuild.CSRC / "prf_engine.hip"), "-o", str(out)],
                       check=True, capture_output=True)
        meta = kernel_metadata(out.read_text())
    bs = {k: v for k, v in meta.items() if "bitsliced" in k}
    assert len(bs) == 2, sorted(meta)
    for name, (lds, scratch) in bs.items():
        assert lds == 0 and scratch == 0, (name, lds, scratch)
