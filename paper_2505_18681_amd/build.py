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
import re
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

# Default tile shapes of the radix pass per (key bytes, value bytes) at 8-bit
# digits (radix_default_shape_c in csrc/radix_shapes.hpp): their kernels must
# not lose workgroups per CU to registers, and no radix pass may use scratch.
DEFAULT_PASS_SHAPES = {(4, 0): (768, 24), (4, 4): (768, 24), (4, 8): (512, 24),
                       (8, 0): (768, 12), (8, 4): (512, 24), (8, 8): (512, 16)}
LDS_PER_CU = 160 * 1024

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


def _resource_usage(text: str) -> dict:
    """Per kernel: the compiler's resource remarks (-Rpass-analysis=kernel-resource-usage)."""
    usage, name = {}, None
    for line in text.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            usage[name] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[[^\]]*\])?: (\d+)", line)
        if name and m:
            usage[name][m.group(1).strip()] = int(m.group(2))
    return usage


def _check_pass_kernels(usage: dict):
    """No radix pass kernel spills to scratch; the default shapes keep every workgroup LDS allows per CU."""
    bad = []
    for name, u in usage.items():
        m = re.search(r"radix_pass_kernelILi(\d+)ELi(\d+)ELi(\d+)ELi(\d+)ELi(\d+)E([jm])E", name)
        if not m:
            continue
        kb, vb, bits, threads, items = (int(m.group(i)) for i in range(1, 6))
        if u.get("ScratchSize", 0) > 0:
            bad.append(f"{name}: {u['ScratchSize']} bytes of scratch per lane")
        if bits == 8 and DEFAULT_PASS_SHAPES.get((kb, vb)) == (threads, items) and "LDS Size" in u:
            by_lds = LDS_PER_CU // max(u["LDS Size"], 1)
            waves = threads // 64
            by_regs = (4 * u.get("Occupancy", 0)) // waves
            if by_regs < min(by_lds, 8):
                bad.append(f"{name}: {u.get('VGPRs')} VGPRs allow {by_regs} workgroups per CU, LDS allows {by_lds}")
    if bad:
        raise RuntimeError("radix pass kernels lost occupancy or spill:\n  " + "\n  ".join(bad))


def _check_no_scratch(usage: dict, what: str):
    """No kernel of the unit uses scratch (spills or private arrays in memory)."""
    bad = [f"{name}: {u['ScratchSize']} bytes of scratch per lane" for name, u in usage.items()
           if u.get("ScratchSize", 0) > 0]
    if bad:
        raise RuntimeError(f"{what} kernels use scratch:\n  " + "\n  ".join(bad))


# Units whose kernels' resource usage is checked at build time.
CHECKED_UNITS = {"radix_inst.hip": _check_pass_kernels,
                 "merge.hip": lambda usage: _check_no_scratch(usage, "mergesort")}


def _compile(unit, verbose, defines=()):
    src, obj, extra = unit
    out = os.path.join(BUILD, obj)
    report = src in CHECKED_UNITS
    cmd = [HIPCC] + COMMON + list(defines) + extra + ["-c", os.path.join(CSRC, src), "-o", out]
    if report:
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"  # the host pass does not know the feature; harmless
    text = r.stdout + r.stderr
    msgs = "\n".join(l for l in text.splitlines()
                     if noise not in l and l.strip() and "kernel-resource-usage" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{msgs}")
    if msgs and verbose:
        print(msgs, flush=True)
    if report:
        CHECKED_UNITS[src](_resource_usage(text))
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
