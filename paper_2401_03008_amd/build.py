"""Build libsrmhd.so (HIP, gfx950) in-tree with hipcc.

The library carries the identifier of the sources it was built from
(``source_id``: a sha256 prefix over the HIP sources and the C header),
returned by ``srmhd_build_id``; the binding refuses a library whose
identifier differs from the sources beside it.
"""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsrmhd.so")
SOURCES = ["srmhd_kernels.hip", "srmhd_api.hip", "srmhd_mlp.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def source_files(root: str = ROOT) -> list:
    """The files the library is built from: every HIP source and header of
    the package's csrc/ and the C header, in a fixed order."""
    csrc = os.path.join(root, "paper_2401_03008_amd", "csrc")
    files = sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp")))
    return files + [os.path.join(root, "include", "srmhd.h")]


def source_id(root: str = ROOT) -> str:
    """sha256[:16] over the names and contents of source_files(root)."""
    h = hashlib.sha256()
    for f in source_files(root):
        h.update(os.path.basename(f).encode() + b"\0")
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False) -> str:
    """Compile every HIP source of the package into ``libsrmhd.so``."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, f'-DSRMHD_BUILD_ID="{source_id()}"', "-o", tmp]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
