"""Builds libphoton.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import hashlib
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "photon.hip")
OUT = os.path.join(HERE, "libphoton.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # no packed-FP32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]


SOURCES = [os.path.join(HERE, "csrc", f) for f in ("photon.hip", "photon_device.hpp", "photon_adjoint.hpp",
                                                   "photon_peaks.hpp")] + \
    [os.path.join(ROOT, "include", "photon.h")]


def source_hash() -> str:
    """SHA-256 (first 16 hex digits) of the library's sources; the library
    reports the hash it was built from in photon_version()."""
    h = hashlib.sha256()
    for f in SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build_library(extra=()) -> str:
    tmp = OUT + ".tmp"
    cmd = [HIPCC, *FLAGS, f"-DPHOTON_SOURCE_HASH=\"{source_hash()}\"", *extra, SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build_library())
