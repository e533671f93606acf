"""Build the HIP library libpir.so in-tree for gfx950 (hipcc, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
LIB = PKG / "libpir.so"
SOURCES = ["pir_device.hip", "pir_host.cpp"]
# measurement kernels (the PRF-engine ceiling, the peak probes), kept out of the PIR library
ENGINE_LIB = PKG / "libpir_engine.so"
ENGINE_SOURCES = ["prf_engine.hip", "peak_probes.hip"]

# the sources of the kernels' device code: their fingerprint is compiled into
# the library (pir_kernel_digest) and keys measurements taken on it
KERNEL_SOURCES = ["pir_kernels.h", "aes_gfx950.h", "aes_tables.h", "chacha_gfx950.h", "quad_gfx950.h"]


def kernel_digest() -> str:
    """Fingerprint of the kernel sources' code: comments and whitespace are
    dropped, so editing a comment keeps measurements taken on the kernels
    valid."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        text = (CSRC / f).read_text()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    "-Wall",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return str(Path(rocm) / "bin" / "hipcc")


def build_library(out: Path | None = None, extra: list[str] | None = None, verbose: bool = False,
                  sources: list[str] | None = None) -> Path:
    """Compile every HIP/C++ source of the library into one shared object."""
    out = Path(out) if out else LIB
    tmp = out.with_suffix(".so.tmp")
    cmd = [hipcc(), *HIPCC_FLAGS, f'-DPIR_KERNEL_DIGEST="{kernel_digest()}"', *(extra or []),
           f"-I{ROOT / 'include'}", f"-I{CSRC}",
           *[str(CSRC / s) for s in (sources or SOURCES)], "-o", str(tmp)]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{r.stderr[-6000:]}")
    os.replace(tmp, out)
    return out


def build_engine(verbose: bool = False) -> Path:
    """The PRF-engine measurement kernel (used by bench.py only)."""
    return build_library(ENGINE_LIB, verbose=verbose, sources=ENGINE_SOURCES)


if __name__ == "__main__":
    print(build_library(verbose=True))
    print(build_engine(verbose=True))
