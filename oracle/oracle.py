"""ctypes wrapper around the FP64 CPU oracle (``cans_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  It shares no
code with the GPU path.

The oracle computes the direct solution of the staggered 7-point Poisson
problem, eq. (poi) of Section 2 (z in conservative form for a stretched grid),
by eigenfunction expansion, eq. (poi_reduced): O(N^2) transform matrices along
x and y, Gauss elimination (Thomas) along z, inverse transforms.

Fields are numpy float64 arrays of shape (nz, ny, nx) (x fastest).
Boundary codes: 0 periodic, 1 Neumann, 2 Dirichlet; bc = (x-, x+, y-, y+, z-, z+).
Codes 3 and 4 (at both ends of an axis) put the field on the faces of that
axis: 3 Dirichlet on the boundary face (zero there, not an unknown), 4 Neumann
on the boundary face (an unknown, mirrored about it).  Along x and y any pair
of 3 and 4 (uniform spacing; the unknowns are the C-1, C+1 or C faces of C
cells); along z only (3, 3), the nz interior faces of an (nz+1)-cell grid
whose nz+1 widths dzf holds.
Axis kinds: 0 P, 1 NN, 2 DD, 3 ND, 4 DN (cell-centred); 5 (3,3) DST-I,
6 (4,4) DCT-I, 7 (3,4), 8 (4,3) (face-located).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cans_oracle.c")
_LIBS = {False: os.path.join(_HERE, "liboracle.so"), True: os.path.join(_HERE, "liboracle_ld.so")}

P, N, D, DF, NF = 0, 1, 2, 3, 4
K_P, K_NN, K_DD, K_ND, K_DN, K_FD, K_FN, K_FDN, K_FND = 0, 1, 2, 3, 4, 5, 6, 7, 8


def n_dz(bc, nz: int) -> int:
    """Length of the z spacing array: nz cell widths, or nz+1 for a
    face-located z field (code 3)."""
    return nz + 1 if bc[4] == DF else nz


def build(force: bool = False) -> None:
    """Compile the oracle (double and long-double variants) with gcc."""
    for ld, path in _LIBS.items():
        if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                   _SRC, "-o", path + ".tmp", "-lm"]
            if ld:
                cmd.insert(1, "-DORACLE_LONG_DOUBLE")
            subprocess.check_call(cmd)
            os.replace(path + ".tmp", path)


_handles: dict = {}


def _lib(ld: bool = False):
    if ld not in _handles:
        if not os.path.exists(_LIBS[ld]):
            build()
        lib = ctypes.CDLL(_LIBS[ld])
        sfx = "_ld" if ld else ""
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i, d = ctypes.c_int, ctypes.c_double
        sig = {
            "oracle_axis_kind": ([i, i], i),
            "oracle_eigen": ([i, i, dp, dp], None),
            "oracle_zcoef": ([i, i, i, dp, dp, dp, dp], i),
            "oracle_tridiag": ([i, dp, dp, dp, dp, dp, i], None),
            "oracle_transform": ([i, i, i, i, i, i, dp, dp], None),
            "oracle_spectral_solve": ([i, i, i, ip, d, d, dp, d, dp, dp, dp], i),
            "oracle_solve": ([i, i, i, ip, d, d, dp, d, dp, dp, dp], i),
            "oracle_apply_L": ([i, i, i, ip, d, d, dp, d, dp, dp], None),
            "oracle_set_threads": ([i], None),
            "oracle_threads": ([], i),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name + sfx)
            fn.argtypes = args
            fn.restype = res
            setattr(lib, name, fn)
        _handles[ld] = lib
    return _handles[ld]


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _bc(bc):
    arr = (ctypes.c_int * 6)(*[int(b) for b in bc])
    return arr


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    """OpenMP threads used by the oracle's loops (timing runs)."""
    _lib().oracle_set_threads(int(n))


def threads() -> int:
    """Threads a parallel loop of the oracle uses now."""
    return int(_lib().oracle_threads())


def axis_kind(lo: int, hi: int) -> int:
    return _lib().oracle_axis_kind(lo, hi)


def eigen(kind: int, n: int, ld: bool = False):
    """Transform rows T (n x n, T[q, i]) and eigenvalues mu (n,) of one axis
    (T A = diag(mu) T for the axis's 1-D operator A)."""
    T = np.zeros((n, n)); mu = np.zeros(n)
    _lib(ld).oracle_eigen(kind, n, _dp(T), _dp(mu))
    return T, mu


def zcoef(nz: int, lo: int, hi: int, dzf):
    dzf = _f64(dzf)
    assert dzf.shape == (nz + 1 if lo == DF else nz,)
    a, b, c = np.zeros(nz), np.zeros(nz), np.zeros(nz)
    rc = _lib().oracle_zcoef(nz, lo, hi, _dp(dzf), _dp(a), _dp(b), _dp(c))
    if rc:
        raise ValueError("invalid z boundary pair")
    return a, b, c


def tridiag(a, b, c, d, cyclic: bool = False, ld: bool = False) -> np.ndarray:
    a, b, c, d = (_f64(v) for v in (a, b, c, d))
    x = np.zeros_like(d)
    _lib(ld).oracle_tridiag(len(d), _dp(a), _dp(b), _dp(c), _dp(d), _dp(x), int(cyclic))
    return x


def transform(field, axis: int, kind: int, inverse: bool = False, ld: bool = False) -> np.ndarray:
    """Apply T (or T^{-1}) of `kind` along axis 0=x, 1=y, 2=z of a (nz,ny,nx) field."""
    f = _f64(field)
    nz, ny, nx = f.shape
    out = np.zeros_like(f)
    _lib(ld).oracle_transform(axis, int(inverse), kind, nx, ny, nz, _dp(f), _dp(out))
    return out


def spectral_solve(fhat, bc, dx: float, dy: float, dzf, ld: bool = False, shift: float = 0.0):
    """Column-wise tridiagonal solves of eq. (poi_reduced) on a spectral field
    (shift: added to every column's diagonal, the Helmholtz form).

    Returns (phat, removed) where removed is the dzf-weighted mean taken out of
    the singular column (spectral units) or 0."""
    f = _f64(fhat); dzf = _f64(dzf)
    nz, ny, nx = f.shape
    assert dzf.shape == (n_dz(bc, nz),)
    out = np.zeros_like(f); rem = ctypes.c_double(0.0)
    rc = _lib(ld).oracle_spectral_solve(nx, ny, nz, _bc(bc), dx, dy, _dp(dzf), float(shift), _dp(f), _dp(out),
                                        ctypes.pointer(rem))
    if rc:
        raise ValueError("invalid boundary conditions")
    return out, rem.value


def solve(f, bc, dx: float, dy: float, dzf, ld: bool = False, shift: float = 0.0):
    """Direct solve of (L_h + shift) p = f (shift <= 0; 0 is eq. (poi)).
    Returns (p, removed_mean).

    For singular problems (every axis P or NN, shift 0) f is projected by its
    dzf-weighted mean, which is returned, and p has zero weighted mean.  A
    problem that a face-located (4, 4) axis would make singular is not
    defined (ValueError), nor is code 4 with a single unknown."""
    f = _f64(f); dzf = _f64(dzf)
    nz, ny, nx = f.shape
    assert dzf.shape == (n_dz(bc, nz),)
    p = np.zeros_like(f); info = np.zeros(4)
    rc = _lib(ld).oracle_solve(nx, ny, nz, _bc(bc), dx, dy, _dp(dzf), float(shift), _dp(f), _dp(p), _dp(info))
    if rc:
        raise ValueError("invalid boundary conditions")
    return p, float(info[0])


def apply_L(p, bc, dx: float, dy: float, dzf, shift: float = 0.0) -> np.ndarray:
    """The discrete operator L_h of eq. (poi), z in conservative form, plus
    shift times p."""
    p = _f64(p); dzf = _f64(dzf)
    nz, ny, nx = p.shape
    assert dzf.shape == (n_dz(bc, nz),)
    out = np.zeros_like(p)
    _lib().oracle_apply_L(nx, ny, nz, _bc(bc), dx, dy, _dp(dzf), float(shift), _dp(p), _dp(out))
    return out


def is_singular(bc, shift: float = 0.0) -> bool:
    return shift == 0.0 and all(axis_kind(bc[2 * a], bc[2 * a + 1]) in (K_P, K_NN) for a in range(3))


def weighted_mean(p, dzf) -> float:
    p = np.asarray(p, dtype=np.float64)
    w = np.asarray(dzf, dtype=np.float64)
    return float((p.sum(axis=(1, 2)) * w).sum() / (w.sum() * p.shape[1] * p.shape[2]))


def residual(p, f, bc, dx, dy, dzf, shift: float = 0.0):
    """Relative residual ||Pi f - (L_h + shift) p||_2 / ||Pi f||_2 (Pi =
    projection removing the weighted mean when the problem is singular)."""
    f = _f64(f)
    if is_singular(bc, shift):
        f = f - weighted_mean(f, dzf)
    r = f - apply_L(p, bc, dx, dy, dzf, shift)
    return float(np.linalg.norm(r) / np.linalg.norm(f))


def residual_inf(p, f, bc, dx, dy, dzf, shift: float = 0.0):
    """Max-norm form of `residual`: max|Pi f - (L_h + shift) p| / max|Pi f|."""
    f = _f64(f)
    if is_singular(bc, shift):
        f = f - weighted_mean(f, dzf)
    r = f - apply_L(p, bc, dx, dy, dzf, shift)
    return float(np.abs(r).max() / np.abs(f).max())


# --------------------------------------------------------------------------- #
# Pressure-correction (projection) step around the solve, the equations that
# follow eq. (up): Phi solves L_h Phi = D u* / (gamma dt), then
# u = u* - gamma dt G Phi and p = p + Phi.  Staggered velocity: u on the +x
# face of each cell, v on the +y face, w on the +z face (arrays (nz, ny, nx),
# x fastest).  Every axis is periodic or bounded by walls (pressure Neumann):
# there the normal velocity below the first cell is zero and the entries on
# the last (wall) face are boundary values, left as given.

def _axis_periodic(bc, axis: int) -> bool:
    lo, hi = bc[2 * axis], bc[2 * axis + 1]
    assert (lo, hi) in ((P, P), (N, N)), "projection needs periodic or wall (Neumann) pressure boundaries"
    return lo == P


def _face_below(a, arr_axis: int, periodic: bool):
    """Value on the face below each cell: the previous face, wrapping when
    periodic, zero at a wall."""
    if periodic:
        return np.roll(a, 1, arr_axis)
    out = np.zeros_like(a)
    dst = [slice(None)] * 3; src = [slice(None)] * 3
    dst[arr_axis] = slice(1, None); src[arr_axis] = slice(0, -1)
    out[tuple(dst)] = a[tuple(src)]
    return out


def divergence(u, v, w, bc, dx: float, dy: float, dzf):
    """D u at the cell centres: (u - u_below)/dx + (v - v_below)/dy +
    (w - w_below)/dzf_k."""
    u, v, w = _f64(u), _f64(v), _f64(w)
    dzf = _f64(dzf)
    px, py, pz = (_axis_periodic(bc, a) for a in range(3))
    return ((u - _face_below(u, 2, px)) / dx + (v - _face_below(v, 1, py)) / dy
            + (w - _face_below(w, 0, pz)) / dzf[:, None, None])


def gradient(phi, bc, dx: float, dy: float, dzf):
    """G Phi on the +faces: (Phi_next - Phi) over the centre distance (dx,
    dy, dzc_k = (dzf_k + dzf_{k+1})/2); the next cell wraps across a periodic
    boundary, and the gradient is zero on a wall face."""
    phi = _f64(phi)
    dzf = _f64(dzf)
    nz = phi.shape[0]
    px, py, pz = (_axis_periodic(bc, a) for a in range(3))
    gx = (np.roll(phi, -1, 2) - phi) / dx
    gy = (np.roll(phi, -1, 1) - phi) / dy
    dzc = 0.5 * (dzf + np.roll(dzf, -1))
    gz = (np.roll(phi, -1, 0) - phi) / dzc[:, None, None]
    if not px:
        gx[:, :, -1] = 0.0
    if not py:
        gy[:, -1, :] = 0.0
    if not pz:
        gz[nz - 1] = 0.0
    return gx, gy, gz


def project(u, v, w, p, bc, dx: float, dy: float, dzf, gdt: float, alpha: float = 0.0):
    """One projection step with gdt = gamma dt: returns (u, v, w, p, Phi)
    after Phi = L_h^{-1} (D u / gdt) (zero weighted mean), u -= gdt G Phi and
    the pressure update p += Phi - alpha L_h Phi.  alpha = gamma nu dt / 2
    with implicit diffusion (the update after eq. (poi_ns_id)), 0 with
    explicit diffusion (the update after eq. (poi_ns))."""
    f = divergence(u, v, w, bc, dx, dy, dzf) / gdt
    phi, _ = solve(f, bc, dx, dy, dzf)
    gx, gy, gz = gradient(phi, bc, dx, dy, dzf)
    pn = _f64(p) + phi
    if alpha != 0.0:
        pn = pn - alpha * apply_L(phi, bc, dx, dy, dzf)
    return (_f64(u) - gdt * gx, _f64(v) - gdt * gy, _f64(w) - gdt * gz, pn, phi)


# --------------------------------------------------------------------------- #
# Time-step criterion, eq. (dt): dt < min(1.65 dl^2 / nu, sqrt(3) dl / max(|u|
# + |v| + |w|)), dl the smallest spacing.  The advective part is evaluated as
# the Listing of Section 3 does: at the +x, +y and +z face of every cell, the
# face-normal component is taken as it is and the two others as the
# magnitude of the mean of their four nearest values; each is divided by the
# spacing of its direction (dzf_k at x and y faces, the centre distance dzc_k
# at z faces), and the sum is the local rate.  sqrt(3) over the largest rate
# is the advective bound.  Neighbour rules (same layout as the projection
# step): along a periodic axis indices wrap; at walls the normal component on
# the face below the first cell is zero, and a tangential component beyond
# the last cell is the no-slip mirror (the negative of the last cell's).

def _shift_normal_below(a, arr_axis: int, periodic: bool):
    """Normal component on the face below (index - 1 along its own axis)."""
    return _face_below(a, arr_axis, periodic)


def _shift_tangential_above(a, arr_axis: int, periodic: bool):
    """Tangential component at index + 1 across an axis: wraps, or beyond a
    wall the no-slip mirror -a of the last cell."""
    if periodic:
        return np.roll(a, -1, arr_axis)
    out = np.empty_like(a)
    dst = [slice(None)] * 3; src = [slice(None)] * 3
    dst[arr_axis] = slice(0, -1); src[arr_axis] = slice(1, None)
    out[tuple(dst)] = a[tuple(src)]
    dst[arr_axis] = slice(-1, None); src[arr_axis] = slice(-1, None)
    out[tuple(dst)] = -a[tuple(src)]
    return out


def dt_rates(u, v, w, bc, dx: float, dy: float, dzf):
    """Advective rates (rx, ry, rz) at the +x, +y and +z face of every cell,
    arrays (nz, ny, nx), as defined above."""
    u, v, w, dzf = _f64(u), _f64(v), _f64(w), _f64(dzf)
    px, py, pz = (_axis_periodic(bc, a) for a in range(3))
    # array axes: 2 = x, 1 = y, 0 = z
    v_s = _shift_normal_below(v, 1, py)
    w_b = _shift_normal_below(w, 0, pz)
    u_w = _shift_normal_below(u, 2, px)
    # x face (i+1/2, j, k): v at (i|i+1, j-1|j), w at (i|i+1, k-1|k)
    vx = 0.25 * np.abs(v + v_s + _shift_tangential_above(v, 2, px) + _shift_tangential_above(v_s, 2, px))
    wx = 0.25 * np.abs(w + w_b + _shift_tangential_above(w, 2, px) + _shift_tangential_above(w_b, 2, px))
    idzf = (1.0 / dzf)[:, None, None]
    rx = np.abs(u) / dx + vx / dy + wx * idzf
    # y face (i, j+1/2, k): u at (i-1|i, j|j+1), w at (j|j+1, k-1|k)
    uy = 0.25 * np.abs(u + u_w + _shift_tangential_above(u, 1, py) + _shift_tangential_above(u_w, 1, py))
    wy = 0.25 * np.abs(w + w_b + _shift_tangential_above(w, 1, py) + _shift_tangential_above(w_b, 1, py))
    ry = uy / dx + np.abs(v) / dy + wy * idzf
    # z face (i, j, k+1/2): u at (i-1|i, k|k+1), v at (j-1|j, k|k+1)
    uz = 0.25 * np.abs(u + u_w + _shift_tangential_above(u, 0, pz) + _shift_tangential_above(u_w, 0, pz))
    vz = 0.25 * np.abs(v + v_s + _shift_tangential_above(v, 0, pz) + _shift_tangential_above(v_s, 0, pz))
    nz = dzf.shape[0]
    dzc = np.empty(nz)
    dzc[:-1] = 0.5 * (dzf[:-1] + dzf[1:])
    dzc[-1] = 0.5 * (dzf[-1] + dzf[0]) if pz else dzf[-1]   # wall face: mirror ghost cell
    rz = uz / dx + vz / dy + np.abs(w) / dzc[:, None, None]
    return rx, ry, rz


def max_dt(u, v, w, bc, dx: float, dy: float, dzf, nu: float = 0.0) -> float:
    """The bound of eq. (dt): min(sqrt(3) / max rate, 1.65 dl^2 / nu) with dl
    = min(dx, dy, min dzf); nu = 0 omits the viscous bound (implicit
    diffusion).  A field at rest with nu = 0 gives +inf."""
    rx, ry, rz = dt_rates(u, v, w, bc, dx, dy, dzf)
    rate = max(float(rx.max()), float(ry.max()), float(rz.max()))
    dt = np.sqrt(3.0) / rate if rate > 0 else np.inf
    if nu > 0:
        dl = min(dx, dy, float(np.min(_f64(dzf))))
        dt = min(dt, 1.65 * dl * dl / nu)
    return float(dt)
