"""Build libcapart.so (HIP for gfx950) in-tree with hipcc.

The kernels are split over several translation units (the heuristic launchers
once per part count, rank-mask width and policy), compiled to objects in
parallel under paper_2105_10312_amd/_build/ and linked into one library.
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libcapart.so")
OBJDIR = os.path.join(PKG, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I" + INCLUDE, "-I" + CSRC,
]


def units():
    """(object name, source, extra defines) of every translation unit."""
    u = [("kernels", "capart_kernels.hip", []), ("api", "capart_api.cpp", [])]
    for k in (4, 8):
        for mt in ("uint32_t", "uint64_t"):
            for pol in ("POL_FP", "POL_EDF"):
                name = f"heur_k{k}_{mt[4:6]}_{pol[4:].lower()}"
                u.append((name, "capart_launch_heur.hip",
                          [f"-DCAPART_I_K={k}", f"-DCAPART_I_MT={mt}", f"-DCAPART_I_POL={pol}"]))
    for pol in ("POL_FP", "POL_EDF"):
        u.append((f"wide_{pol[4:].lower()}", "capart_launch_wide.hip", [f"-DCAPART_I_POL={pol}"]))
        u.append((f"alg1_{pol[4:].lower()}", "capart_launch_alg1.hip", [f"-DCAPART_I_POL={pol}"]))
    u.append(("alg1_big", "capart_launch_alg1big.hip", []))
    return u


def source_hash() -> str:
    """sha256 (first 16 hex digits) over every source and header the library is built from."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp", ".h")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(INCLUDE, "capart.h"), "rb") as f:
        h.update(b"capart.h\0" + f.read())
    return h.hexdigest()[:16]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every translation unit and link paper_2105_10312_amd/libcapart.so
    (always recompiles).  The library carries the source hash it was built from
    (capart_build_hash), which the binding checks at load time."""
    os.makedirs(OBJDIR, exist_ok=True)
    digest = source_hash()
    hash_flag = f'-DCAPART_BUILD_HASH="{digest}"'
    jobs = jobs or min(16, os.cpu_count() or 1)
    cmds, objs = [], []
    for name, src, defs in units():
        obj = os.path.join(OBJDIR, name + ".o")
        objs.append(obj)
        cmds.append([HIPCC] + FLAGS + defs + [hash_flag, "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
