"""ctypes access to the host build of the library's kernel arithmetic
(``cans_emu.cpp``), for the CPU tests.  Built with hipcc as host-only code."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "cans_emu.cpp")
LIB = os.path.join(HERE, "libcans_emu.so")
CSRC = os.path.join(ROOT, "paper_2001_05234_amd", "csrc")
HEADERS = [os.path.join(CSRC, h) for h in ("xform_core.h", "zsolve_core.h", "tables.h")]


def build(force: bool = False) -> None:
    newest = max(os.path.getmtime(p) for p in [SRC] + HEADERS)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
        subprocess.check_call([os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "-x", "hip", "--cuda-host-only",
                               "-O2", "-std=c++17", "-fPIC", "-shared", "-I", os.path.join(ROOT, "include"),
                               "-I", CSRC, SRC, "-o", LIB + ".tmp"])
        os.replace(LIB + ".tmp", LIB)


_lib = None
dp = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        i, d = ctypes.c_int, ctypes.c_double
        ip = ctypes.POINTER(ctypes.c_int)
        L.emu_xform.argtypes = [i, i, i, i, i, i, i, dp, dp]
        L.emu_xform_geom.argtypes = [i, i, i, i, i, i, i, i, i, dp, dp]
        L.emu_zsolve.argtypes = [i, i, i, ip, d, d, dp, dp, dp]
        L.emu_zsolve_part.argtypes = [i, i, i, ip, d, d, dp, dp, dp]
        L.emu_solve.argtypes = [i, i, i, ip, d, d, dp, i, d, dp, dp, dp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(dp)


def xform(field, kind, fwd, axis, prec=64):
    f = np.ascontiguousarray(field, dtype=np.float64)
    nz, ny, nx = f.shape
    out = np.zeros_like(f)
    rc = lib().emu_xform(kind, int(fwd), axis, prec, nx, ny, nz, _p(f), _p(out))
    assert rc == 0
    return out


def xform_geom(field, kind, fwd, axis, prec, L, rmax):
    """As xform with an explicit tile geometry; None if the geometry is invalid."""
    f = np.ascontiguousarray(field, dtype=np.float64)
    nz, ny, nx = f.shape
    out = np.zeros_like(f)
    rc = lib().emu_xform_geom(kind, int(fwd), axis, prec, nx, ny, nz, L, rmax, _p(f), _p(out))
    if rc == -2:
        return None
    assert rc == 0
    return out


def zsolve(fhat, bc, dx, dy, dzf):
    d = np.array(fhat, dtype=np.float64, copy=True)
    nz, ny, nx = d.shape
    dzf = np.ascontiguousarray(dzf, dtype=np.float64)
    rem = ctypes.c_double(0)
    rc = lib().emu_zsolve(nx, ny, nz, (ctypes.c_int * 6)(*bc), dx, dy, _p(dzf), _p(d), ctypes.pointer(rem))
    assert rc == 0
    return d, rem.value


def zsolve_part(fhat, bc, dx, dy, dzf):
    """The partitioned (register-resident) z kernel; None where it does not apply."""
    d = np.array(fhat, dtype=np.float64, copy=True)
    nz, ny, nx = d.shape
    dzf = np.ascontiguousarray(dzf, dtype=np.float64)
    rem = ctypes.c_double(0)
    rc = lib().emu_zsolve_part(nx, ny, nz, (ctypes.c_int * 6)(*bc), dx, dy, _p(dzf), _p(d), ctypes.pointer(rem))
    if rc == -2:
        return None
    assert rc == 0
    return d, rem.value


def solve(f, bc, dx, dy, dzf, max_iter=-1, tol=1e-10):
    """max_iter < 0: FP64 pipeline; else FP32 transforms + FP64 refinement.
    Returns (p, info) with info = [removed, corrections, converged, last, hist...]."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    nz, ny, nx = f.shape
    dzf = np.ascontiguousarray(dzf, dtype=np.float64)
    p = np.zeros_like(f)
    info = np.full(4 + 32, -1.0)
    rc = lib().emu_solve(nx, ny, nz, (ctypes.c_int * 6)(*bc), dx, dy, _p(dzf), max_iter, tol, _p(f), _p(p), _p(info))
    assert rc == 0
    return p, info
