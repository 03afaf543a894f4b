"""CPU oracle for the watershed / waterfall hot path -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of `bench.py`
may import this package. The HIP library and its Python binding never do.

The arithmetic lives in `ws_oracle.c` (plain sequential C, double precision for
the gradient). This module compiles it with gcc when no built library is
present and wraps it with ctypes. Every function takes and returns numpy
arrays in C order with x fastest ((ny, nx) or (nz, ny, nx)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ws_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ws_oracle.c into liboracle.so (plain -O2, single thread)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64, i32, ptr, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_double
        lib.or_set_progress.argtypes = [i32]
        lib.or_set_progress.restype = None
        lib.or_step1.argtypes = [ptr, i64, i64, i64, i32, ptr, ptr]
        lib.or_watershed.argtypes = [ptr, i64, i64, i64, i32, i32, i64, ptr, ptr, ptr, ptr, ptr]
        lib.or_waterfall_g1.argtypes = [ptr, ptr, i64, i64, i64, i32, i32, ptr, ptr]
        lib.or_waterfall_recon.argtypes = [ptr, i64, i64, i64, i32, i32, ptr, ptr]
        lib.or_gradient.argtypes = [ptr, i64, i64, i64, dbl, i32, ptr, ptr]
        for f in (lib.or_step1, lib.or_watershed, lib.or_waterfall_g1, lib.or_waterfall_recon,
                  lib.or_gradient):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def set_progress(on: bool) -> None:
    """Progress lines on stderr after each step of the watershed (for runs
    over hundreds of millions of pixels)."""
    _load().or_set_progress(1 if on else 0)


def _dims(shape):
    if len(shape) == 1:
        return shape[0], 1, 1
    if len(shape) == 2:
        return shape[1], shape[0], 1
    if len(shape) == 3:
        return shape[2], shape[1], shape[0]
    raise ValueError("1D, 2D or 3D arrays only")


def _grey(img):
    a = np.ascontiguousarray(img)
    if a.dtype not in (np.uint8, np.uint16):
        raise TypeError("grey image must be uint8 or uint16")
    return np.ascontiguousarray(a, dtype=np.uint16)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError("%s failed with code %d" % (what, rc))


def step1(img, conn):
    """Step I: (state, label) arrays (Eq. (1) and the four states)."""
    I = _grey(img)
    nx, ny, nz = _dims(I.shape)
    S = np.empty(I.shape, np.int32)
    L = np.empty(I.shape, np.int32)
    _check(_load().or_step1(_p(I), nx, ny, nz, conn, _p(S), _p(L)), "or_step1")
    return S, L


def watershed(img, conn, RR=6, max_step2_sweeps=-1, full=False):
    """Canonical watershed labels (int32, same shape as img).

    With full=True also returns a dict with the Step I states ("state1"), the
    balanced Step II encoding ("bal": -distance for resolved plateau pixels,
    else the state), the arrows after Step II ("arrow") and the counters
    ("sweeps" of Step II incl. the final unchanged one, "syncs" of Step III
    that changed labels, "nbasins").
    """
    I = _grey(img)
    nx, ny, nz = _dims(I.shape)
    lab = np.empty(I.shape, np.int32)
    if full:
        s1 = np.empty(I.shape, np.int32)
        bal = np.empty(I.shape, np.int32)
        arr = np.empty(I.shape, np.int32)
        ptrs = (_p(s1), _p(bal), _p(arr))
    else:
        ptrs = (None, None, None)
    st = np.zeros(3, np.int64)
    _check(_load().or_watershed(_p(I), nx, ny, nz, conn, RR, max_step2_sweeps, _p(lab), *ptrs, _p(st)),
           "or_watershed")
    if not full:
        return lab
    return lab, dict(state1=s1, bal=bal, arrow=arr, sweeps=int(st[0]), syncs=int(st[1]),
                     nbasins=int(st[2]))


def waterfall_g1(labels0, img, conn, NL):
    """(out, nregions): NL layers of the graph waterfall starting at labels0."""
    I = _grey(img)
    L0 = np.ascontiguousarray(labels0, dtype=np.int32)
    if L0.shape != I.shape:
        raise ValueError("labels and image shapes differ")
    nx, ny, nz = _dims(I.shape)
    out = np.empty((NL,) + I.shape, np.int32)
    nreg = np.zeros(NL, np.int64)
    _check(_load().or_waterfall_g1(_p(L0), _p(I), nx, ny, nz, conn, NL, _p(out), _p(nreg)),
           "or_waterfall_g1")
    return out, nreg


def waterfall_recon(img, conn, NL):
    """(out, nregions): NL layers of the reconstruction waterfall (Alg. 4 + 5)."""
    I = _grey(img)
    nx, ny, nz = _dims(I.shape)
    out = np.empty((NL,) + I.shape, np.int32)
    nreg = np.zeros(NL, np.int64)
    _check(_load().or_waterfall_recon(_p(I), nx, ny, nz, conn, NL, _p(out), _p(nreg)),
           "or_waterfall_recon")
    return out, nreg


def gradient(img, sigma, dtype="u8", return_mag=False):
    """Quantised gradient magnitude (uint8 or uint16) of a float image."""
    f = np.ascontiguousarray(img, dtype=np.float32)
    nx, ny, nz = _dims(f.shape)
    Q = 255 if dtype == "u8" else 65535
    q = np.empty(f.shape, np.uint16)
    mag = np.empty(f.shape, np.float64) if return_mag else None
    _check(_load().or_gradient(_p(f), nx, ny, nz, float(sigma), Q, _p(mag) if mag is not None else None,
                               _p(q)), "or_gradient")
    q = q.astype(np.uint8) if dtype == "u8" else q
    return (q, mag) if return_mag else q
