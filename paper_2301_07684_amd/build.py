"""Build step of the package: the approximation tables and the HIP library for gfx950.

    python -m paper_2301_07684_amd.build

compiles csrc/sfq.hip into libsfq.so next to this file (hipcc, --offload-arch=gfx950),
csrc/mem_probe.hip into libsfq_probe.so (the benchmark's memory-only reference, not part of
the step's ABI) and (re)generates data/sfq_tables.bin when the table generator's source
changed.
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libsfq.so")
SOURCES = [os.path.join(HERE, "csrc", "sfq.hip")]
PROBE_LIB = os.path.join(HERE, "libsfq_probe.so")
PROBE_SOURCES = [os.path.join(HERE, "csrc", "mem_probe.hip")]
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _strip_comments(src: str) -> str:
    """C/C++ source without its comments and blank-space runs (string and character literals
    kept as they are), so that editing a comment does not change the hash below."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            i = src.find("\n", i)
            i = n if i < 0 else i
        elif src.startswith("/*", i):
            k = src.find("*/", i + 2)
            i = n if k < 0 else k + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    """Hash of the HIP sources and the ABI header without their comments (identifies the
    kernels a profile was taken of)."""
    h = hashlib.sha256()
    for f in (*SOURCES, os.path.join(HERE, "csrc", "sfq_device.h"),
              os.path.join(os.path.dirname(HERE), "include", "sfq.h")):
        with open(f, encoding="utf-8") as fh:
            h.update(_strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


def hipcc() -> str:
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _hipcc_shared(out: str, sources, verbose: bool) -> str:
    tmp = out + ".tmp"
    cmd = [hipcc(), *HIP_FLAGS, "-o", tmp, *sources]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, out)
    return out


def build_library(verbose: bool = True) -> str:
    return _hipcc_shared(LIB, SOURCES, verbose)


def build_probe(verbose: bool = True) -> str:
    return _hipcc_shared(PROBE_LIB, PROBE_SOURCES, verbose)


def build_tables(verbose: bool = True) -> str:
    from . import tablegen

    tablegen.main([tablegen.default_path()])
    return tablegen.default_path()


def build(verbose: bool = True):
    build_tables(verbose)
    build_library(verbose)
    build_probe(verbose)


if __name__ == "__main__":
    build()
