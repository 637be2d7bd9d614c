"""Build the HIP library ``libmapa.so`` (gfx950) in-tree.

    python -m paper_2110_03214_amd.build

The library is the whole product path: the device units (kernels.hip: batch
front end, finalize and state kernels; fused.hip: the small-batch launch;
enum_*.hip: the enumeration kernel, one unit per pair-level variant) and the
host units (host.cpp: C ABI, validation, memory, launches; serve.cpp: the
serving loop; wide.hip / wide.cpp: servers of up to 32 accelerators and
patterns of up to 12 vertices; noalloc.hip: the allocation-free batch; simulate.hip /
simulate.cpp: the job-trace simulation; autotune.cpp: the autotuner), each compiled by hipcc for gfx950 only, in
parallel, then
linked into one shared object.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libmapa.so")
SOURCES = [os.path.join(CSRC, f) for f in (
    "enum_pair12_lds.hip", "enum_pair12_glb.hip", "enum_pair6.hip", "enum_plain.hip",
    "fused.hip", "kernels.hip", "wide.hip", "noalloc.hip", "simulate.hip", "host.cpp", "serve.cpp", "wide.cpp", "simulate.cpp",
    "autotune.cpp")]
ARCH = "gfx950"


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wall", "-Wno-unused-function"]


def compile_command(src: str, obj: str, extra=()) -> list[str]:
    return [hipcc(), f"--offload-arch={ARCH}", *FLAGS, f"-I{INCLUDE}", f"-I{CSRC}", *extra,
            "-c", "-o", obj, src]


def link_command(objs, out: str) -> list[str]:
    return [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out, *objs]


def build(verbose: bool = False, extra=()) -> str:
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory(prefix="mapa_build_") as d:
        objs = [os.path.join(d, os.path.basename(s) + ".o") for s in SOURCES]
        cmds = [compile_command(s, o, extra) for s, o in zip(SOURCES, objs)]

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            return subprocess.run(cmd, capture_output=True, text=True)

        jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(jobs) as ex:
            done = list(ex.map(run, cmds))
        for cmd, r in zip(cmds, done):
            sys.stderr.write(r.stderr)
            if r.returncode:
                raise subprocess.CalledProcessError(r.returncode, cmd, r.stdout, r.stderr)
        link = link_command(objs, tmp)
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
    sys.exit(0)
