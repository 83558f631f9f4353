"""Build libdwt2.so (HIP, gfx950) in-tree.

    python -m paper_1605_00561_amd.build            # compile changed sources, link
    python -m paper_1605_00561_amd.build --force    # rebuild everything

Sources are compiled in parallel into _build/ at the repository root and
linked into paper_1605_00561_amd/libdwt2.so.  Packed FP32 instructions are
disabled (-Xclang -target-feature -Xclang -packed-fp32-ops).

A second, test-only variant, libdwt2_poison.so, is built from the same
sources with DWT2_POISON_LDS: every work-group fills its LDS with NaN before
its first LDS access, so a kernel that reads a cell it has not written shows
NaN or wrong values in the GPU tests that load it.  The binding never loads
it.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libdwt2.so")
POISON_LIB = os.path.join(PKG, "libdwt2_poison.so")
VARIANTS = {"": ([], LIB), "poison": (["-DDWT2_POISON_LDS"], POISON_LIB)}
ARCH = os.environ.get("DWT2_OFFLOAD_ARCH", "gfx950")

SOURCES = ["dwt2_api.cpp", "dwt2_server.cpp", "tile_kernels.hip", "fused_kernels.hip",
           "rowcol_kernels.hip"]
HEADERS = ["dwt2_internal.h", "server_plan.h"]

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CFLAGS = ["-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
          "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", INCLUDE, "-I", CSRC]


def _newest_dep_mtime() -> float:
    deps = [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(INCLUDE, "dwt2.h")]
    return max(os.path.getmtime(d) for d in deps)


def _compile(src: str, force: bool, variant: str = "") -> str:
    s = os.path.join(CSRC, src)
    o = os.path.join(BUILD, variant, src + ".o")
    if force or not os.path.exists(o) or os.path.getmtime(o) < max(os.path.getmtime(s),
                                                                    _newest_dep_mtime()):
        cmd = [HIPCC, *CFLAGS, *VARIANTS[variant][0], "-c", s, "-o", o]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        if r.stderr.strip():
            # the host pass warns that it does not know the packed-fp32 feature
            lines = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln
                     and "warning generated" not in ln and ln.strip()]
            if lines:
                sys.stderr.write("\n".join(lines) + "\n")
    return o


def _link(objs, lib: str) -> None:
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs,
           "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)


def build(force: bool = False, variants=("", "poison")) -> str:
    """Compile and link the library and (by default) its test-only variant;
    returns the library's path."""
    jobs = [(v, src) for v in variants for src in SOURCES]
    for v in variants:
        os.makedirs(os.path.join(BUILD, v), exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda j: (j[0], _compile(j[1], force, j[0])), jobs))
    for v in variants:
        _link([o for (vv, o) in objs if vv == v], VARIANTS[v][1])
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    args = ap.parse_args()
    print(build(force=args.force))
