"""ctypes binding of the C ABI in ``include/cans_poisson.h``.

Argument marshalling only: every step of a solve runs in the HIP library
``libcans_poisson.so`` (built by ``paper_2001_05234_amd.build``).  If the
library is missing, importing the solver raises; there is no fallback.

Device arrays are passed as torch CUDA tensors (float64, contiguous, shape
(nz, ny, nx)) or raw integer device addresses; the stream defaults to torch's
current stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcans_poisson.so")

CANS_OK = 0
STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported problem", -3: "allocation failed",
          -4: "HIP runtime error", -5: "rhs and p alias",
          -6: "problem exceeds the fixed scratch of the no-allocation solve"}
PREC_FP64, PREC_FP32_REFINE = 0, 1
XFORM_AUTO, XFORM_FFT, XFORM_DENSE = 0, 1, 2
BC_PERIODIC, BC_NEUMANN, BC_DIRICHLET, BC_DIRICHLET_FACE, BC_NEUMANN_FACE = 0, 1, 2, 3, 4
HISTORY = 17


def z_widths(nz: int, bc) -> int:
    """z widths a problem takes: nz cells, or the nz+1 cells around a
    face-located z field (BC_DIRICHLET_FACE)."""
    return nz + 1 if int(bc[4]) == BC_DIRICHLET_FACE else nz

# every symbol the header declares
EXPORTS = ["cans_default_opts", "cans_poisson_plan", "cans_poisson_plan_ex", "cans_poisson_solve",
           "cans_poisson_get_info", "cans_poisson_destroy", "cans_status_string",
           "cans_poisson_workspace_bytes", "cans_poisson_debug_stage", "cans_poisson_plan_batched",
           "cans_poisson_solve_batched", "cans_poisson_get_info_batched", "cans_poisson_project",
           "cans_poisson_project_ex", "cans_poisson_solve_noalloc", "cans_poisson_xform_mode"]


class CansOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("xform_x", ctypes.c_int), ("xform_y", ctypes.c_int),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("autotune", ctypes.c_int),
                ("graph", ctypes.c_int), ("shift", ctypes.c_double)]


class CansInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("residual", ctypes.c_double),
                ("history", ctypes.c_double * HISTORY), ("removed_mean", ctypes.c_double),
                ("residual_inf", ctypes.c_double)]


class CansDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("bc", ctypes.c_int * 6),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.POINTER(ctypes.c_double))]


class CansError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {STATUS.get(code, 'unknown status')} ({code})")


_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2001_05234_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    pp = ctypes.POINTER(vp)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    sig = {
        "cans_default_opts": ([ctypes.POINTER(CansOpts)], None),
        "cans_poisson_plan": ([pp, i, i, i, ip, d, d, dp], i),
        "cans_poisson_plan_ex": ([pp, i, i, i, ip, d, d, dp, ctypes.POINTER(CansOpts)], i),
        "cans_poisson_solve": ([vp, vp, vp, vp], i),
        "cans_poisson_solve_noalloc": ([vp, vp, vp, vp], i),
        "cans_poisson_project": ([vp, vp, vp, vp, vp, d, vp], i),
        "cans_poisson_project_ex": ([vp, vp, vp, vp, vp, d, d, d, vp, vp], i),
        "cans_poisson_get_info": ([vp, ctypes.POINTER(CansInfo)], i),
        "cans_poisson_destroy": ([vp], None),
        "cans_status_string": ([i], ctypes.c_char_p),
        "cans_poisson_workspace_bytes": ([vp], ctypes.c_size_t),
        "cans_poisson_xform_mode": ([vp, i], i),
        "cans_poisson_debug_stage": ([vp, i, vp, vp, vp], i),
        "cans_poisson_plan_batched": ([pp, i, ctypes.POINTER(CansDesc), ctypes.POINTER(CansOpts)], i),
        "cans_poisson_solve_batched": ([vp, pp, pp, vp], i),
        "cans_poisson_get_info_batched": ([vp, i, ctypes.POINTER(CansInfo)], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(code: int, what: str) -> None:
    if code != CANS_OK:
        raise CansError(code, what)


def _addr(x, numel: int = -1, device: int = -1) -> int:
    """Device address of `x`.  A torch tensor must be a contiguous float64
    CUDA tensor; with numel / device given it must hold exactly that many
    elements on that device (the kernels read and write the plan's full grid,
    so a smaller array or one on another device would be accessed out of
    bounds).  A raw integer address is passed through unchecked."""
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        import torch
        if not x.is_cuda or x.dtype != torch.float64 or not x.is_contiguous():
            raise ValueError("device arrays must be contiguous float64 CUDA tensors")
        if numel >= 0 and x.numel() != numel:
            raise ValueError(f"device array holds {x.numel()} elements, the plan's grid {numel}")
        if device >= 0 and x.device.index != device:
            raise ValueError(f"device array is on cuda:{x.device.index}, the plan on cuda:{device}")
        return x.data_ptr()
    raise TypeError("expected a torch CUDA tensor or a device address")


def _current_device() -> int:
    import torch
    return torch.cuda.current_device()


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def default_opts() -> CansOpts:
    o = CansOpts()
    load().cans_default_opts(ctypes.byref(o))
    return o


def _info(ci: CansInfo) -> dict:
    hist = [h for h in ci.history if h >= 0]
    return {"iterations": ci.iterations, "converged": bool(ci.converged), "residual": ci.residual,
            "history": hist, "removed_mean": ci.removed_mean, "residual_inf": ci.residual_inf}


class Plan:
    """One planned problem: ``cans_poisson_plan_ex``; ``solve`` enqueues
    ``cans_poisson_solve`` on a stream without host synchronisation."""

    def __init__(self, nx: int, ny: int, nz: int, bc, dx: float, dy: float, dzf,
                 precision: str = "fp64", tol: float = 1e-10, max_iter: int = 4, xform_x: str = "auto",
                 autotune: bool = False, graph: bool = False, shift: float = 0.0):
        lib = load()
        self._lib = lib
        self.shape = (nz, ny, nx)
        self.precision = precision
        o = default_opts()
        o.precision = PREC_FP64 if precision == "fp64" else PREC_FP32_REFINE
        o.tol = tol
        o.max_iter = max_iter
        o.xform_x = {"auto": XFORM_AUTO, "fft": XFORM_FFT, "dense": XFORM_DENSE}[xform_x]
        o.autotune = int(bool(autotune))
        o.graph = int(bool(graph))
        o.shift = float(shift)
        dz = np.ascontiguousarray(np.asarray(dzf, dtype=np.float64))
        if dz.shape != (z_widths(nz, bc),):
            raise ValueError("dzf must hold nz cell widths (nz+1 for a face-located z)")
        bca = (ctypes.c_int * 6)(*[int(b) for b in bc])
        h = ctypes.c_void_p()
        _check(lib.cans_poisson_plan_ex(ctypes.byref(h), nx, ny, nz, bca, float(dx), float(dy),
                                        dz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(o)),
               "cans_poisson_plan_ex")
        self._h = h
        self.numel = nx * ny * nz
        self.device = _current_device()

    def _a(self, x) -> int:
        return _addr(x, self.numel, self.device)

    def solve(self, rhs, p, stream=None) -> None:
        _check(self._lib.cans_poisson_solve(self._h, self._a(rhs), self._a(p), _stream(stream)), "cans_poisson_solve")

    def solve_noalloc(self, rhs, p, stream=None) -> None:
        """cans_poisson_solve_noalloc: the same solve on the library's fixed
        scratch (no device allocation)."""
        _check(self._lib.cans_poisson_solve_noalloc(self._h, self._a(rhs), self._a(p), _stream(stream)),
               "cans_poisson_solve_noalloc")

    def project(self, u, v, w, p, gdt: float, stream=None) -> None:
        """One projection step (``cans_poisson_project``): u, v, w -= gdt G Phi,
        p += Phi with L_h Phi = D u / gdt; FP64 plans with periodic or wall
        boundaries."""
        _check(self._lib.cans_poisson_project(self._h, self._a(u), self._a(v), self._a(w), self._a(p), float(gdt),
                                              _stream(stream)), "cans_poisson_project")

    def project_ex(self, u, v, w, p, gdt: float, alpha: float = 0.0, nu: float = 0.0, dt_max=None,
                   stream=None) -> None:
        """``cans_poisson_project_ex``: the projection step with the pressure
        update p += Phi - alpha L_h Phi (implicit diffusion) and, when
        `dt_max` (a one-element float64 CUDA tensor) is given, the bound of
        eq. (dt) on the corrected velocity written into it."""
        dt_addr = None
        if dt_max is not None:
            dt_addr = _addr(dt_max, 1, self.device)
        _check(self._lib.cans_poisson_project_ex(self._h, self._a(u), self._a(v), self._a(w), self._a(p),
                                                 float(gdt), float(alpha), float(nu), dt_addr, _stream(stream)),
               "cans_poisson_project_ex")

    def debug_stage(self, stage: int, inp, out, stream=None) -> None:
        _check(self._lib.cans_poisson_debug_stage(self._h, stage, self._a(inp), self._a(out), _stream(stream)),
               "cans_poisson_debug_stage")

    def info(self) -> dict:
        ci = CansInfo()
        _check(self._lib.cans_poisson_get_info(self._h, ctypes.byref(ci)), "cans_poisson_get_info")
        return _info(ci)

    @property
    def workspace_bytes(self) -> int:
        return int(self._lib.cans_poisson_workspace_bytes(self._h))

    def xform_mode(self, axis: int) -> str:
        """Form of the transform along axis 0 (x) or 1 (y) the plan uses:
        "fft" or "dense" (``cans_poisson_xform_mode``)."""
        m = int(self._lib.cans_poisson_xform_mode(self._h, int(axis)))
        if m < 0:
            raise CansError(m, "cans_poisson_xform_mode")
        return {XFORM_FFT: "fft", XFORM_DENSE: "dense"}[m]

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.cans_poisson_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedPlan:
    """Many independent problems in one plan (``cans_poisson_plan_batched``)."""

    def __init__(self, problems, precision: str = "fp32_refine", tol: float = 1e-10, max_iter: int = 4,
                 autotune: bool = False, shift: float = 0.0):
        lib = load()
        self._lib = lib
        o = default_opts()
        o.precision = PREC_FP64 if precision == "fp64" else PREC_FP32_REFINE
        o.tol = tol
        o.max_iter = max_iter
        o.autotune = int(bool(autotune))
        o.shift = float(shift)
        self._dz = []
        descs = (CansDesc * len(problems))()
        for d, pr in zip(descs, problems):
            dz = np.ascontiguousarray(np.asarray(pr.dzf, dtype=np.float64))
            if dz.shape != (z_widths(pr.nz, pr.bc),):
                raise ValueError("dzf must hold nz cell widths (nz+1 for a face-located z)")
            self._dz.append(dz)
            d.nx, d.ny, d.nz = pr.nx, pr.ny, pr.nz
            for k in range(6):
                d.bc[k] = int(pr.bc[k])
            d.dx, d.dy = float(pr.dx), float(pr.dy)
            d.dz = dz.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        h = ctypes.c_void_p()
        _check(lib.cans_poisson_plan_batched(ctypes.byref(h), len(problems), descs, ctypes.byref(o)),
               "cans_poisson_plan_batched")
        self._h = h
        self.count = len(problems)
        self.numels = [pr.nx * pr.ny * pr.nz for pr in problems]
        self.device = _current_device()

    def solve(self, rhs_list, p_list, stream=None) -> None:
        n = self.count
        if len(rhs_list) != n or len(p_list) != n:
            raise ValueError(f"the plan holds {n} problems: {len(rhs_list)} rhs and {len(p_list)} p arrays given")
        ra = (ctypes.c_void_p * n)(*[_addr(r, m, self.device) for r, m in zip(rhs_list, self.numels)])
        pa = (ctypes.c_void_p * n)(*[_addr(p, m, self.device) for p, m in zip(p_list, self.numels)])
        _check(self._lib.cans_poisson_solve_batched(self._h, ra, pa, _stream(stream)), "cans_poisson_solve_batched")

    def info(self, index: int) -> dict:
        ci = CansInfo()
        _check(self._lib.cans_poisson_get_info_batched(self._h, index, ctypes.byref(ci)),
               "cans_poisson_get_info_batched")
        return _info(ci)

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.cans_poisson_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
