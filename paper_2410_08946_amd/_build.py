"""Compiles the HIP sources of libws for gfx950 into paper_2410_08946_amd/libws.so.

Every source is compiled to an object of its own (in parallel), then the
objects are linked into one shared library.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libws.so")
SOURCES = ["api.hip", "watershed.hip", "waterfall.hip", "gradient.hip", "rag.hip", "pixel.hip"]
# ws_shape.hip is compiled once per watershed tile shape id (TileShape in ws_device.h)
SHAPES = [2, 12, 22, 32, 3, 13, 23, 33]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _jobs() -> int:
    n = os.cpu_count() or 1
    return max(1, min(len(SOURCES) + len(SHAPES), n, int(os.environ.get("MAX_JOBS", n))))


def build(verbose: bool = False) -> str:
    """Always recompiles (the build check must exercise the compiler)."""
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    objs, cmds = [], []
    units = [(s, os.path.splitext(s)[0], []) for s in SOURCES]
    units += [("ws_shape.hip", "ws_shape_%d" % sh, ["-DWS_SHAPE=%d" % sh]) for sh in SHAPES]
    for s, stem, defs in units:
        o = os.path.join(OBJ, stem + ".o")
        objs.append(o)
        cmds.append([cc] + FLAGS + defs + inc + ["-c", "-o", o, os.path.join(CSRC, s)])
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    with cf.ThreadPoolExecutor(max_workers=_jobs()) as ex:
        futs = [ex.submit(subprocess.run, c, check=False) for c in cmds]
        rcs = [f.result().returncode for f in futs]
    for c, rc in zip(cmds, rcs):
        if rc != 0:
            raise subprocess.CalledProcessError(rc, c)
    tmp = LIB + ".tmp%d" % os.getpid()
    link = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
