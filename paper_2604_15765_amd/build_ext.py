"""Build the hermtile HIP library for gfx950 (and its host-side test helper).

    python paper_2604_15765_amd/build_ext.py      # or __graft_entry__.build()

Outputs, next to this file:
    libhermtile.so   the C-ABI library (include/hermtile.h)
    _hostcheck.so    test support: the conjugation lane body run on the CPU
    _probe.so        measurement tool: HBM streaming probe (stream_probe.py)
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(HERE, "_build")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          f"-I{os.path.join(ROOT, 'include')}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=fast"]

LIB_SOURCES = ["ht_conj.hip", "ht_native.hip", "ht_k3.hip", "ht_misc.hip", "ht_batch.hip", "ht_api.cpp",
               "ht_batch_api.cpp", "ht_circuit.cpp", "ht_batch_runner.cpp", "ht_autotune.cpp",
               "ht_fuse.cpp", "ht_server.cpp", "ht_prep.cpp", "ht_noalloc.hip",
               "ht_tune.cpp"]
LIB = os.path.join(HERE, "libhermtile.so")
HOSTCHECK = os.path.join(HERE, "_hostcheck.so")
PROBE = os.path.join(HERE, "_probe.so")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}")
    return r


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    # every source is HIP: the .cpp files use the HIP runtime API
    _run([HIPCC, "-x", "hip", *COMMON, *DEVICE, "-c", path, "-o", obj], verbose)
    return obj


def build(verbose: bool = False) -> None:
    """Compile every source and link the libraries (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), LIB_SOURCES))
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    # host-only helper: ht_geom.h compiled for the CPU, plus the op preparation
    tmp = HOSTCHECK + ".tmp"
    _run([HIPCC, "-x", "hip", "--offload-host-only", *COMMON, "-shared",
          os.path.join(CSRC, "ht_hostcheck.cpp"), "-x", "c++", os.path.join(CSRC, "ht_prep.cpp"),
          "-o", tmp], verbose)
    os.replace(tmp, HOSTCHECK)
    tmp = PROBE + ".tmp"
    _run([HIPCC, "-x", "hip", *COMMON, *DEVICE, "-shared", os.path.join(CSRC, "ht_probe.hip"), "-o", tmp],
         verbose)
    os.replace(tmp, PROBE)


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB, HOSTCHECK)
