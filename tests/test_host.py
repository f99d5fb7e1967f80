"""Host-only checks of the HIP library (no GPU, no compute calls): it loads,
exports every function the public header declares, and rejects invalid or
unsupported problems before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2001_05234_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\**\s*(cans_[a-z_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_header_symbol():
    lib = capi.load()
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(capi.EXPORTS) == names


def test_status_strings():
    lib = capi.load()
    for code, text in capi.STATUS.items():
        assert lib.cans_status_string(code).decode() == text


def _plan(nx, ny, nz, bc, dx=1.0, dy=1.0, dz=None, opts=None):
    lib = capi.load()
    h = ctypes.c_void_p()
    dz = np.full(max(nz, 1), 0.5) if dz is None else np.asarray(dz, dtype=np.float64)
    rc = lib.cans_poisson_plan_ex(ctypes.byref(h), nx, ny, nz, (ctypes.c_int * 6)(*bc), dx, dy,
                                  dz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.byref(opts) if opts is not None else None)
    return rc


@pytest.mark.parametrize("args,code", [
    ((8, 8, 8, (0, 1, 0, 0, 1, 1)), -1),      # periodic paired with Neumann
    ((8, 8, 8, (0, 0, 0, 0, 3, 1)), -1),      # face-located z paired with Neumann
    ((8, 8, 8, (3, 1, 0, 0, 1, 1)), -1),      # a face code paired with a cell code
    ((8, 8, 8, (0, 0, 4, 2, 1, 1)), -1),
    ((8, 8, 8, (0, 0, 0, 0, 4, 4)), -1),      # z takes only the Dirichlet face pair
    ((8, 8, 8, (0, 0, 0, 0, 3, 4)), -1),
    ((8, 8, 8, (0, 0, 0, 0, 5, 5)), -1),      # unknown boundary code
    ((6, 8, 8, (3, 3, 0, 0, 1, 1)), -2),      # DST-I of 6: extended line of 14 (7 is no radix)
    ((8, 8, 8, (4, 4, 0, 0, 2, 2)), -2),      # DCT-I of 8: extended line of 14
    ((7, 8, 8, (3, 4, 0, 0, 1, 1)), -2),      # type-III face pair of odd length
    ((9, 8, 8, (4, 4, 0, 0, 1, 1)), -2),      # a (4,4) axis in an otherwise singular problem
    ((4096, 8, 4, (3, 3, 0, 0, 1, 1)), -2),   # extended line longer than 4096
    ((0, 8, 8, (0, 0, 0, 0, 1, 1)), -1),      # empty axis
    ((8, 8, 0, (0, 0, 0, 0, 1, 1)), -1),
    ((7, 8, 8, (0, 0, 0, 0, 1, 1)), -2),      # odd length
    ((8, 14, 8, (0, 0, 0, 0, 1, 1)), -2),     # 7 is not a supported radix
    ((8, 8, 2, (0, 0, 0, 0, 0, 0)), -2),      # periodic z shorter than 3
    ((8192, 8, 4, (0, 0, 0, 0, 1, 1)), -2),   # longer than one LDS tile
])
def test_plan_validation(args, code):
    assert _plan(*args) == code


def test_plan_validation_spacing():
    assert _plan(8, 8, 4, (0, 0, 0, 0, 1, 1), dx=0.0) == -1
    assert _plan(8, 8, 4, (0, 0, 0, 0, 1, 1), dy=-1.0) == -1
    assert _plan(8, 8, 4, (0, 0, 0, 0, 1, 1), dz=[0.1, 0.2, -0.1, 0.3]) == -1
    assert _plan(8, 8, 4, (0, 0, 0, 0, 1, 1), dz=[0.1, 0.2, np.nan, 0.3]) == -1
    # periodic z must be uniform
    assert _plan(8, 8, 4, (0, 0, 0, 0, 0, 0), dz=[0.1, 0.2, 0.1, 0.3]) == -2
    # a face-located z reads nz+1 widths: the last one is checked too
    assert _plan(8, 8, 4, (0, 0, 0, 0, 3, 3), dz=[0.1, 0.2, 0.1, 0.3, -0.2]) == -1
    with pytest.raises(ValueError):
        capi.Plan(8, 8, 4, (0, 0, 0, 0, 3, 3), 1.0, 1.0, np.full(4, 0.5))


def test_options_validation():
    o = capi.default_opts()
    assert o.precision == 0 and o.tol == 1e-10 and o.max_iter == 4 and o.autotune == 0 and o.graph == 0 and o.shift == 0.0
    o.max_iter = 99
    assert _plan(8, 8, 4, (0, 0, 0, 0, 1, 1), opts=o) == -1
    o = capi.default_opts(); o.precision = 7
    assert _plan(8, 8, 4, (0, 0, 0, 0, 1, 1), opts=o) == -1
    o = capi.default_opts(); o.tol = -1.0
    assert _plan(8, 8, 4, (0, 0, 0, 0, 1, 1), opts=o) == -1
    o = capi.default_opts(); o.autotune = 2
    assert _plan(8, 8, 4, (0, 0, 0, 0, 1, 1), opts=o) == -1
    o = capi.default_opts(); o.graph = 2
    assert _plan(8, 8, 4, (0, 0, 0, 0, 1, 1), opts=o) == -1
    o = capi.default_opts(); o.shift = float("nan")
    assert _plan(8, 8, 4, (0, 0, 0, 0, 1, 1), opts=o) == -1
    o = capi.default_opts(); o.shift = 0.5  # indefinite Helmholtz form
    assert _plan(8, 8, 4, (0, 0, 0, 0, 1, 1), opts=o) == -2
    o = capi.default_opts(); o.xform_y = 2
    assert _plan(128, 8, 4, (0, 0, 0, 0, 1, 1), opts=o) == -2


def test_project_rejects_null_plan():
    lib = capi.load()
    assert lib.cans_poisson_project(None, None, None, None, None, 1.0, None) == -1
    assert lib.cans_poisson_project_ex(None, None, None, None, None, 1.0, 0.0, 0.0, None, None) == -1


def test_null_arguments():
    lib = capi.load()
    assert lib.cans_poisson_solve(None, None, None, None) == -1
    assert lib.cans_poisson_get_info(None, None) == -1
    assert lib.cans_poisson_debug_stage(None, 1, None, None, None) == -1
    assert lib.cans_poisson_workspace_bytes(None) == 0
    lib.cans_poisson_destroy(None)


def test_product_path_has_no_oracle_dependency():
    """The library and its binding never import, include or load the oracle."""
    pkg = os.path.join(ROOT, "paper_2001_05234_amd")
    pat = re.compile(r"(^\s*(import|from)\s+oracle)|(#include\s+.*oracle)|(liboracle)", re.M)
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert not pat.search(text), fn


def _struct_fields(header: str, name: str):
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), header, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in body.split(";"):
        if not decl.strip():
            continue
        for part in decl.split(","):  # "int nx, ny, nz" declares three fields
            names.append(re.search(r"(\w+)\s*(\[\w+\])?\s*$", part.strip()).group(1))
    return names


def test_binding_structs_match_header():
    """The ctypes structures list the header's fields in the header's order."""
    with open(os.path.join(ROOT, "include", "cans_poisson.h")) as fh:
        header = fh.read()
    for cname, cls in [("cans_opts", capi.CansOpts), ("cans_info", capi.CansInfo), ("cans_desc", capi.CansDesc)]:
        assert _struct_fields(header, cname) == [f[0] for f in cls._fields_], cname


class _FakeTensor:
    """Stands in for a CUDA tensor in the binding's argument checks (no GPU here)."""

    def __init__(self, numel, device=0, dtype=None, contiguous=True):
        import torch
        self.is_cuda = True
        self.dtype = torch.float64 if dtype is None else dtype
        self._numel = numel
        self.device = type("Dev", (), {"index": device})()
        self._contiguous = contiguous

    def is_contiguous(self):
        return self._contiguous

    def numel(self):
        return self._numel

    def data_ptr(self):
        return 0x1000


def test_binding_checks_array_size_and_device():
    """Arrays that do not hold the plan's nx*ny*nz doubles on the plan's device
    are refused before any call into the library (the kernels would access
    them out of bounds)."""
    import torch
    assert capi._addr(_FakeTensor(60), 60, 0) == 0x1000
    with pytest.raises(ValueError, match="elements"):
        capi._addr(_FakeTensor(59), 60, 0)
    with pytest.raises(ValueError, match="cuda:1"):
        capi._addr(_FakeTensor(60, device=1), 60, 0)
    with pytest.raises(ValueError, match="float64"):
        capi._addr(_FakeTensor(60, dtype=torch.float32), 60, 0)
    with pytest.raises(ValueError, match="contiguous"):
        capi._addr(_FakeTensor(60, contiguous=False), 60, 0)
    assert capi._addr(0x2000, 60, 0) == 0x2000  # raw addresses pass unchecked
