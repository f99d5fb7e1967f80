"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws numbers and builds grids; it holds none of the
solver's arithmetic.  Every array is numpy float64, C order, shape
(nz, ny, nx) (x fastest), generated with numpy's PCG64 from an explicit seed
so the oracle and the GPU library see the same bytes.

Workload shapes follow the channel-flow case of Section 4 (periodic x and y,
walls in z, z clustered at the walls by the tanh map given there).  The
paper's own flow fields and reference statistics are not available; the
divergence of a random staggered velocity stands in for the right-hand side
D u* / (gamma dt) of eq. (poi_ns).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

P, N, D = 0, 1, 2


def tanh_faces(nz: int, a: float, lz: float) -> np.ndarray:
    """Face positions z_f(k), k = 0..nz, clustered at both walls.

    The paper gives the centre positions z_k = Lz/2 (1 + tanh(a(Z_k - 1/2)) /
    tanh(a/2)) with Z_k = (k - 1/2)/Nz (Section 4).  Faces use the same map
    at Z = k/nz, so the walls sit exactly at 0 and Lz."""
    k = np.arange(nz + 1, dtype=np.float64)
    z = 0.5 * lz * (1.0 + np.tanh(a * (k / nz - 0.5)) / math.tanh(0.5 * a))
    z[0], z[-1] = 0.0, lz
    return z


def tanh_dzf(nz: int, a: float = 1.5, lz: float = 2.0) -> np.ndarray:
    """Cell widths dzf of the tanh-clustered grid."""
    return np.diff(tanh_faces(nz, a, lz))


def uniform_dzf(nz: int, lz: float = 1.0) -> np.ndarray:
    return np.full(nz, lz / nz, dtype=np.float64)


def uniform_rhs(shape, seed: int, subtract_mean: bool = False) -> np.ndarray:
    """i.i.d. U[-1, 1] right-hand side; optionally minus its plain mean."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = rng.uniform(-1.0, 1.0, size=shape)
    if subtract_mean:
        f -= f.mean()
    return f


def divergence_rhs(nx: int, ny: int, nz: int, dx: float, dy: float, dzf: np.ndarray,
                   seed: int) -> np.ndarray:
    """Discrete divergence of a seeded random staggered velocity field.

    u, v of shape (nz, ny, nx) and w of shape (nz+1, ny, nx) are drawn N(0, 1)
    in that order; w vanishes on the two wall faces (no penetration).  With u
    on the +x face and v on the +y face of each cell, periodic in x and y:
        f = (u_i - u_{i-1})/dx + (v_j - v_{j-1})/dy + (w_{k+1} - w_k)/dzf_k.
    Its dzf-weighted sum is zero, so the singular problem is compatible."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.standard_normal((nz, ny, nx))
    f = (u - np.roll(u, 1, axis=2)) * (1.0 / dx)
    del u
    v = rng.standard_normal((nz, ny, nx))
    f += (v - np.roll(v, 1, axis=1)) * (1.0 / dy)
    del v
    w = rng.standard_normal((nz + 1, ny, nx))
    w[0] = 0.0
    w[nz] = 0.0
    f += (w[1:] - w[:-1]) / np.asarray(dzf, dtype=np.float64)[:, None, None]
    return f


@dataclass
class Problem:
    nx: int
    ny: int
    nz: int
    bc: tuple
    dx: float
    dy: float
    dzf: np.ndarray = field(repr=False)
    seed: int = 0
    rhs_kind: str = "uniform"

    @property
    def npts(self) -> int:
        return self.nx * self.ny * self.nz

    def rhs(self) -> np.ndarray:
        if self.rhs_kind == "divergence":
            return divergence_rhs(self.nx, self.ny, self.nz, self.dx, self.dy, self.dzf, self.seed)
        f = uniform_rhs((self.nz, self.ny, self.nx), self.seed)
        if _is_singular(self.bc):
            f = weighted_project(f, self.dzf)
        return f


def _axis_kind(lo, hi):
    if lo == P or hi == P:
        return "P" if lo == hi == P else None
    # codes 3 and 4: a field on the faces of the axis (Dirichlet / Neumann face)
    return {(N, N): "NN", (D, D): "DD", (N, D): "ND", (D, N): "DN", (3, 3): "FD", (4, 4): "FN",
            (3, 4): "FDN", (4, 3): "FND"}.get((lo, hi))


def _is_singular(bc) -> bool:
    return all(_axis_kind(bc[2 * a], bc[2 * a + 1]) in ("P", "NN") for a in range(3))


def config(name: str) -> Problem:
    """The named workloads: c1 .. c4 (c5 is `batch_c5`)."""
    if name == "c1":
        # 32^3 unit cube, periodic x and y, Neumann z, uniform; U[-1,1] minus mean
        n = 32
        return Problem(n, n, n, (P, P, P, P, N, N), 1.0 / n, 1.0 / n, uniform_dzf(n), 1, "uniform")
    if name == "c2":
        # 256^3 channel: Lx = 2 pi, Ly = pi, Lz = 2, tanh a = 1.5
        n = 256
        return Problem(n, n, n, (P, P, P, P, N, N), 2 * math.pi / n, math.pi / n,
                       tanh_dzf(n, 1.5, 2.0), 2, "divergence")
    if name == "c3":
        # one GPU's slab of a large channel, same boundary conditions and stretching
        nx, ny, nz = 1024, 512, 384
        return Problem(nx, ny, nz, (P, P, P, P, N, N), 2 * math.pi / nx, math.pi / ny,
                       tanh_dzf(nz, 1.5, 2.0), 3, "divergence")
    if name == "c4":
        # mixed: Dirichlet-Neumann x, periodic y, Dirichlet-Dirichlet z, unit lengths
        nx, ny, nz = 512, 256, 256
        return Problem(nx, ny, nz, (D, N, P, P, D, D), 1.0 / nx, 1.0 / ny, uniform_dzf(nz), 4, "uniform")
    raise KeyError(name)


# 3-smooth lengths {2^a 3^b, a >= 3} within the instance size range, like the
# paper's grid (1536 = 2^9 3, 768 = 2^8 3, 576 = 2^6 3^2)
SMOOTH = [32, 48, 64, 72, 96, 128, 144, 192, 216, 256]


def batch_c5(count: int = 64, seed: int = 5):
    """Uneven batch of independent problems drawn from `seed`.

    nx from SMOOTH within [32, 256], ny within [32, 128], nz a multiple of 8 in
    [32, 96]; each axis draws its boundary pair uniformly from
    {P, NN, DD, mixed (ND or DN with equal odds)}; z is tanh-stretched
    (a = 1.5, Lz = 2) with probability 1/2 unless periodic; other lengths are 1.
    Instance i draws its RHS U[-1, 1] from seed 500 + i (minus its
    dzf-weighted mean when singular)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sx = [s for s in SMOOTH if s <= 256]
    sy = [s for s in SMOOTH if s <= 128]
    sz = list(range(32, 97, 8))
    probs = []
    for i in range(count):
        nx = int(rng.choice(sx)); ny = int(rng.choice(sy)); nz = int(rng.choice(sz))
        bcs = []
        for _ in range(3):
            t = int(rng.integers(4))
            if t == 0:
                bcs += [P, P]
            elif t == 1:
                bcs += [N, N]
            elif t == 2:
                bcs += [D, D]
            else:
                bcs += [N, D] if rng.integers(2) == 0 else [D, N]
        stretched = bool(rng.integers(2)) and bcs[4] != P
        dzf = tanh_dzf(nz, 1.5, 2.0) if stretched else uniform_dzf(nz, 1.0)
        probs.append(Problem(nx, ny, nz, tuple(bcs), 1.0 / nx, 1.0 / ny, dzf, 500 + i, "uniform"))
    return probs


def weighted_project(f: np.ndarray, dzf: np.ndarray) -> np.ndarray:
    """f minus its dzf-weighted mean (input preparation for singular cases)."""
    w = np.asarray(dzf, dtype=np.float64)
    m = (f.sum(axis=(1, 2)) * w).sum() / (w.sum() * f.shape[1] * f.shape[2])
    return f - m
