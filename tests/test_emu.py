"""The library's kernel arithmetic, built for the host and run serially
(tests/emu), against the oracle -- index math of every transform family,
radix, tile shape and the z solve, checked without a GPU."""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_2001_05234_amd import inputs
from tests.emu import emu

P, N, D = 0, 1, 2
PAIRS = [(P, P), (N, N), (D, D), (N, D), (D, N)]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def scale(kind, n):
    return n // 2 if kind in (O.K_ND, O.K_DN) else n


@pytest.mark.parametrize("shape", [(3, 8, 12), (2, 6, 16), (2, 48, 72), (1, 10, 2), (2, 40, 30),
                                   (1, 4, 256), (1, 256, 4), (2, 18, 20)])
@pytest.mark.parametrize("kind", range(5))
def test_transforms_fp64(shape, kind):
    """Forward T and inverse B (B T = s I) along x and y, every family;
    lengths cover radices 2, 3, 4, 5, 8, n = 2 and ragged tiles."""
    rng = np.random.default_rng(sum(shape) + kind)
    f = rng.standard_normal(shape)
    nz, ny, nx = shape
    for axis, n in ((0, nx), (1, ny)):
        T = O.transform(f, axis, kind)
        assert rel(emu.xform(f, kind, True, axis), T) < 1e-13
        Bi = scale(kind, n) * O.transform(f, axis, kind, inverse=True)
        assert rel(emu.xform(f, kind, False, axis), Bi) < 1e-13
        assert rel(emu.xform(f, kind, True, axis, prec=32), T) < 2e-6


@pytest.mark.parametrize("n", [2, 6, 16, 20, 48, 72, 128, 144, 512, 1024])
def test_transforms_every_tuned_geometry(n):
    """Every tile geometry the plan-time tuner may choose (lines per tile from
    a quarter to four times the default, radix-8 or radix-4 first) gives the
    same transform, along x and y, FP64 and FP32."""
    rng = np.random.default_rng(n)
    f = rng.standard_normal((2, 3, n)) if n > 128 else rng.standard_normal((2, 40, n))
    g = np.ascontiguousarray(np.swapaxes(f, 1, 2))
    tried = 0
    for kind in range(5):
        for fwd in (True, False):
            ref_x = O.transform(f, 0, kind) if fwd else scale(kind, n) * O.transform(f, 0, kind, inverse=True)
            ref_y = O.transform(g, 1, kind) if fwd else scale(kind, n) * O.transform(g, 1, kind, inverse=True)
            for L in (1, 2, 4, 8, 16, 32, 64):
                for rmax in (8, 4):
                    for prec, tol in ((64, 1e-13), (32, 3e-6)):
                        out = emu.xform_geom(f, kind, fwd, 0, prec, L, rmax)
                        if out is not None:
                            tried += 1
                            assert rel(out, ref_x) < tol, (n, kind, fwd, L, rmax, prec)
                        out = emu.xform_geom(g, kind, fwd, 1, prec, L, rmax)
                        if out is not None:
                            tried += 1
                            assert rel(out, ref_y) < tol, (n, kind, fwd, L, rmax, prec, "y")
    assert tried > 0


@pytest.mark.parametrize("zp", PAIRS)
@pytest.mark.parametrize("yp", PAIRS)
@pytest.mark.parametrize("xp", PAIRS)
def test_solve_every_bc(xp, yp, zp):
    bc = xp + yp + zp
    nx, ny, nz = 12, 10, 7
    dzf = np.full(nz, 0.3) if zp == (P, P) else inputs.tanh_dzf(nz, 1.5, 2.0)
    rng = np.random.default_rng(sum(bc))
    f = rng.standard_normal((nz, ny, nx))
    po, mo = O.solve(f, bc, 0.3, 0.4, dzf)
    pe, info = emu.solve(f, bc, 0.3, 0.4, dzf)
    assert rel(pe, po) < 1e-12
    assert abs(info[0] - mo) < 1e-12 * max(1, abs(mo))
    pr, info = emu.solve(f, bc, 0.3, 0.4, dzf, max_iter=6, tol=1e-12)
    if O.is_singular(bc):
        pr = pr - O.weighted_mean(pr, dzf)
        assert abs(info[0] - mo) < 1e-13 * max(1, abs(mo))
    assert info[2] == 1 and info[3] <= 1e-12
    assert rel(pr, po) < 1e-10


@pytest.mark.parametrize("xy", [(P, P, P, P), (N, N, D, N), (D, D, N, D)])
def test_solve_face_located_z(xy):
    """z-face-located field (code 3): the library's plan tables, z solve
    and residual stencil against the oracle, stretched, with and without a
    Helmholtz shift in the oracle (the emulated solve takes none)."""
    bc = xy + (3, 3)
    nx, ny, nz = 12, 10, 9
    cells = inputs.tanh_dzf(nz + 1, 1.5, 2.0)
    f = np.random.default_rng(sum(bc) + 40).standard_normal((nz, ny, nx))
    po, mo = O.solve(f, bc, 0.3, 0.4, cells)
    assert mo == 0.0
    pe, info = emu.solve(f, bc, 0.3, 0.4, cells)
    assert rel(pe, po) < 1e-12 and info[0] == 0.0
    pr, info = emu.solve(f, bc, 0.3, 0.4, cells, max_iter=6, tol=1e-12)
    assert info[2] == 1 and info[3] <= 1e-12
    assert rel(pr, po) < 1e-10


def test_zsolve_stage():
    rng = np.random.default_rng(4)
    for bc in [(P, P, N, N, N, N), (D, N, P, P, D, D), (P, P, P, P, P, P), (N, N, N, N, N, D)]:
        nz, ny, nx = 9, 6, 8
        dzf = np.full(nz, 0.2) if bc[4] == P else inputs.tanh_dzf(nz, 1.5, 2.0)
        fh = rng.standard_normal((nz, ny, nx))
        ph, rem = O.spectral_solve(fh, bc, 0.3, 0.5, dzf)
        kx, ky = O.axis_kind(bc[0], bc[1]), O.axis_kind(bc[2], bc[3])
        pe, reme = emu.zsolve(fh, bc, 0.3, 0.5, dzf)
        s = scale(kx, nx) * scale(ky, ny)
        assert rel(pe * s, ph) < 1e-12
        assert abs(reme * s - rem) < 1e-12 * max(1, abs(rem))


@pytest.mark.parametrize("nz", [1, 2, 5, 8, 9, 16, 17, 31, 64, 96, 100, 128, 129, 256, 257, 300, 384, 512])
def test_zsolve_partitioned(nz):
    """Register-resident partitioned z solve (segments per wave, reduced
    interface system) against the oracle's column solves, including the
    singular column and ragged column blocks.  For 128 < nz <= 384 on a
    non-periodic z this is the persistent pipelined kernel's arithmetic
    (single-sweep reduction, interface from both ends, padded levels)."""
    rng = np.random.default_rng(nz)
    for bc in [(P, P, N, N, N, N), (D, N, P, P, D, D), (N, N, N, N, N, D), (P, P, P, P, D, N)]:
        ny, nx = 6, 22
        dzf = inputs.tanh_dzf(nz, 1.5, 2.0)
        fh = rng.standard_normal((nz, ny, nx))
        ph, rem = O.spectral_solve(fh, bc, 0.3, 0.5, dzf)
        kx, ky = O.axis_kind(bc[0], bc[1]), O.axis_kind(bc[2], bc[3])
        res = emu.zsolve_part(fh, bc, 0.3, 0.5, dzf)
        assert res is not None
        pe, reme = res
        s = scale(kx, nx) * scale(ky, ny)
        e = rel(pe * s, ph)
        if e >= 1e-12:  # conditioning: compare both FP64 results with long double
            phl, _ = O.spectral_solve(fh, bc, 0.3, 0.5, dzf, ld=True)
            assert rel(pe * s, phl) < 2 * rel(ph, phl), (nz, bc, e)
        assert abs(reme * s - rem) < 1e-12 * max(1, abs(rem))
    # periodic z: the cyclic (Sherman-Morrison) form of the same kernel, uniform
    # z, nz <= 128 (deeper periodic columns use the plain elimination)
    if 3 <= nz <= 128:
        for bc in [(P, P, N, N, P, P), (P, P, P, P, P, P), (D, N, D, D, P, P)]:
            dzf = np.full(nz, 2.0 / nz)
            fh = rng.standard_normal((nz, 6, 22))
            ph, rem = O.spectral_solve(fh, bc, 0.3, 0.5, dzf)
            kx, ky = O.axis_kind(bc[0], bc[1]), O.axis_kind(bc[2], bc[3])
            res = emu.zsolve_part(fh, bc, 0.3, 0.5, dzf)
            assert res is not None
            pe, reme = res
            s = scale(kx, 22) * scale(ky, 6)
            e = rel(pe * s, ph)
            if e >= 1e-12:
                phl, _ = O.spectral_solve(fh, bc, 0.3, 0.5, dzf, ld=True)
                assert rel(pe * s, phl) < 2 * rel(ph, phl), (nz, bc, e)
            assert abs(reme * s - rem) < 1e-12 * max(1, abs(rem))
    if nz > 128:
        assert emu.zsolve_part(fh, (P, P, N, N, P, P), 0.3, 0.5, np.full(nz, 0.1)) is None


def test_c1_refine_converges():
    pr = inputs.config("c1")
    f = pr.rhs()
    po, _ = O.solve(f, pr.bc, pr.dx, pr.dy, pr.dzf)
    p, info = emu.solve(f, pr.bc, pr.dx, pr.dy, pr.dzf, max_iter=4, tol=1e-10)
    assert info[2] == 1 and info[1] == 1
    assert rel(p - O.weighted_mean(p, pr.dzf), po) < 1e-11
    # the update keeps the weighted mean pinned to FP64 accuracy
    assert abs(O.weighted_mean(p, pr.dzf)) < 1e-14 * np.abs(po).max()


# --------------------------------------------------------------------------- #
# Fields on the faces of x or y (codes 3 and 4): DST-I and DCT-I through the
# odd / even extension of each line, the type-III face pairs as the DD / NN
# transforms run the other way round.  The kernels' forward transform is
# twice the oracle's T (its rows carry the factor 2 of the unnormalised
# type-1 and type-3 forms) and B T = s I with s = 2(n+1), 2(n-1) or n.
DF, NF = 3, 4
FACE_SIZES = {O.K_FD: [1, 2, 4, 7, 11, 15, 47, 63, 127], O.K_FN: [2, 3, 4, 5, 9, 13, 17, 49, 65, 129],
              O.K_FDN: [2, 4, 6, 8, 10, 16, 24, 48, 128], O.K_FND: [2, 4, 6, 8, 10, 16, 24, 48, 128]}
FACE_BC = {O.K_FD: (DF, DF), O.K_FN: (NF, NF), O.K_FDN: (DF, NF), O.K_FND: (NF, DF)}


def face_scale(kind, n):
    return {O.K_FD: 2 * (n + 1), O.K_FN: 2 * (n - 1)}.get(kind, n)


@pytest.mark.parametrize("kind,n", [(k, n) for k, ns in FACE_SIZES.items() for n in ns])
def test_face_transforms(kind, n):
    """Forward and inverse face transforms along x and y against the oracle,
    FP64 and FP32, over every tile geometry the tuner may pick."""
    rng = np.random.default_rng(10 * kind + n)
    for axis in (0, 1):
        f = rng.standard_normal((2, 5, n) if axis == 0 else (2, n, 7))
        T = 2.0 * O.transform(f, axis, kind)
        Bi = 0.5 * face_scale(kind, n) * O.transform(f, axis, kind, inverse=True)
        assert rel(emu.xform(f, kind, True, axis), T) < 1e-13, axis
        assert rel(emu.xform(f, kind, False, axis), Bi) < 1e-13, axis
        assert rel(emu.xform(f, kind, True, axis, prec=32), T) < 3e-6, axis
        tried = 0
        for L in (1, 2, 4, 8, 16, 32, 64):
            for rmax in (8, 4):
                for fwd, ref in ((True, T), (False, Bi)):
                    out = emu.xform_geom(f, kind, fwd, axis, 64, L, rmax)
                    if out is not None:
                        tried += 1
                        assert rel(out, ref) < 1e-13, (axis, L, rmax, fwd)
        assert tried > 0


@pytest.mark.parametrize("yp", [(P, P), (D, N), (DF, DF), (NF, DF), (DF, NF)])
@pytest.mark.parametrize("xp", [(DF, DF), (NF, NF), (DF, NF), (NF, DF)])
def test_solve_face_located_xy(xp, yp):
    """Face-located x (and y) fields: the library's tables, transforms, z
    solve and residual stencil (refinement) against the oracle."""
    nx = {(DF, DF): 15, (NF, NF): 17, (DF, NF): 16, (NF, DF): 16}[xp]
    ny = {(P, P): 10, (D, N): 10, (DF, DF): 11, (NF, DF): 12, (DF, NF): 12}[yp]
    nz = 7
    zp = (D, N) if xp == (NF, NF) and yp == (P, P) else (N, N)
    bc = xp + yp + zp
    dzf = inputs.tanh_dzf(nz, 1.5, 2.0)
    f = np.random.default_rng(sum(bc) + 60).standard_normal((nz, ny, nx))
    po, mo = O.solve(f, bc, 0.3, 0.4, dzf)
    assert mo == 0.0
    pe, info = emu.solve(f, bc, 0.3, 0.4, dzf)
    assert rel(pe, po) < 1e-12 and info[0] == 0.0
    pr, info = emu.solve(f, bc, 0.3, 0.4, dzf, max_iter=6, tol=1e-12)
    assert info[2] == 1 and info[3] <= 1e-12
    assert rel(pr, po) < 1e-10
