"""Build the HIP library libpetto.so for gfx950 in-tree.

Usage: python -m paper_2509_06971_amd.build   (or call build()).
Every call recompiles; objects go to a temporary folder, the shared library to
paper_2509_06971_amd/libpetto.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libpetto.so")
PROBE = os.path.join(PKG, "stream_probe")
SOURCES = ["petto.hip", "el2d.hip", "el2d_tb.hip", "el3d.hip", "el3d_stream.hip", "heat2d.hip", "heat2d_tb.hip", "control.hip", "phase.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def _compile(src, obj, verbose):
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{p.stderr}")
    if verbose:
        errs = [ln for ln in p.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if errs:
            print("\n".join(errs), file=sys.stderr)
    return obj


def build(verbose: bool = False) -> str:
    tmp = tempfile.mkdtemp(prefix="petto_build_")
    try:
        objs = [os.path.join(tmp, s.replace(".hip", ".o")) for s in SOURCES]
        with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1, 8)) as ex:
            list(ex.map(lambda a: _compile(a[0], a[1], verbose), zip(SOURCES, objs)))
        out_tmp = LIB + ".tmp"
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out_tmp] + objs
        p = subprocess.run(cmd, capture_output=True, text=True)
        if p.returncode != 0:
            raise RuntimeError(f"link failed:\n{p.stderr}")
        os.replace(out_tmp, LIB)
        # the streaming bandwidth probe: a standalone program, not linked into the library
        probe_tmp = PROBE + ".tmp"
        cmd = [HIPCC] + FLAGS + [os.path.join(CSRC, "stream_probe.hip"), "-o", probe_tmp]
        p = subprocess.run(cmd, capture_output=True, text=True)
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed on stream_probe.hip:\n{p.stderr}")
        os.replace(probe_tmp, PROBE)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
