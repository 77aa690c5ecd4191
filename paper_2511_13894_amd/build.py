"""Build the gfx950 shared library libpdhg.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
OUT = PKG / "libpdhg.so"
BUILD = PKG / "_build"
SOURCES = ["pdhg_setup.hip", "pdhg_iter.hip", "pdhg_sell.hip", "pdhg_compact.hip", "pdhg_batch.hip", "pdhg_mlp.hip", "pdhg_learned.hip",
           "pdhg_capi.cpp", "pdhg_mlp_capi.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall",
    f"-I{ROOT / 'include'}", f"-I{CSRC}",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build_library(verbose: bool = False) -> Path:
    BUILD.mkdir(exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = BUILD / (src.rsplit(".", 1)[0] + ".o")
        objs.append(obj)
        cmd = [HIPCC, *FLAGS, "-c", str(CSRC / src), "-o", str(obj)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append(src)
        if out and (verbose or p.returncode != 0):
            print(out, file=sys.stderr)
    if failed:
        raise RuntimeError(f"hipcc failed on {failed}")
    tmp = OUT.with_suffix(".so.tmp")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
