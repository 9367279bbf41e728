"""Build libevosort.so (HIP, gfx950) in-tree.

    python -m paper_2505_18681_amd.build        # or: python paper_2505_18681_amd/build.py

Every source is compiled by hipcc for gfx950 only; the radix pass kernel file
is compiled once per (key bytes, value bytes) pair so the instantiations build
in parallel.  Only the evosort_* C symbols are exported.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libevosort.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall", "-Wno-unused-function",
    # packed FP32 instructions stay off in every HIP object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]

UNITS = [
    ("radix_host.hip", "radix_host.o", []),
    ("small_sort.hip", "small_sort.o", []),
    ("merge.hip", "merge.o", []),
    ("segmented.hip", "segmented.o", []),
    ("capi.cpp", "capi.o", ["-x", "hip"]),
    ("server.cpp", "server.o", ["-x", "hip"]),
    ("noalloc.cpp", "noalloc.o", ["-x", "hip"]),
] + [
    ("radix_inst.hip", f"radix_k{kb}_v{vb}.o", [f"-DEVOSORT_KB={kb}", f"-DEVOSORT_VB={vb}"])
    for kb in (4, 8) for vb in (0, 4, 8)
] + [
    ("seg_block.hip", f"seg_block_k{kb}_v{vb}.o", [f"-DEVOSORT_KB={kb}", f"-DEVOSORT_VB={vb}"])
    for kb in (4, 8) for vb in (0, 4, 8)
]


def source_hash() -> str:
    """First 16 hex digits of SHA-256 over csrc/ and include/ (name order; path, NUL, bytes per file)."""
    h = hashlib.sha256()
    files = []
    for top, rel in ((CSRC, "csrc"), (INCLUDE, "include")):
        for name in os.listdir(top):
            path = os.path.join(top, name)
            if os.path.isfile(path):
                files.append((f"{rel}/{name}", path))
    for rel, path in sorted(files):
        h.update(rel.encode() + b"\0")
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _compile(unit, verbose, defines=()):
    src, obj, extra = unit
    out = os.path.join(BUILD, obj)
    cmd = [HIPCC] + COMMON + list(defines) + extra + ["-c", os.path.join(CSRC, src), "-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"  # the host pass does not know the feature; harmless
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{msgs}")
    if msgs and verbose:
        print(msgs, flush=True)
    return out


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(UNITS), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    defines = [f'-DEVOSORT_SOURCE_HASH="{source_hash()}"']
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose, defines), UNITS))
    vscript = os.path.join(BUILD, "exports.map")
    with open(vscript, "w") as f:
        f.write("{ global: evosort_*; local: *; };\n")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + [
        f"-Wl,--version-script={vscript}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    t = build(verbose="-v" in sys.argv)
    print(t)
