"""The x transform as a dense split-bf16 matrix product on the matrix cores
(refinement path) against the oracle, through the C ABI."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2001_05234_amd import capi, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
P, N, D = 0, 1, 2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dense_solve(f, bc, dx, dy, dzf, max_iter=6, shift=0.0):
    nz, ny, nx = f.shape
    plan = capi.Plan(nx, ny, nz, bc, dx, dy, dzf, precision="fp32_refine", tol=1e-10, max_iter=max_iter,
                     xform_x="dense", shift=shift)
    fd = torch.from_numpy(f).cuda()
    pd = torch.zeros_like(fd)
    plan.solve(fd, pd)
    torch.cuda.synchronize()
    out, info = pd.cpu().numpy(), plan.info()
    plan.close()
    return out, info


@pytest.mark.parametrize("nx", [128, 256, 384, 512])
@pytest.mark.parametrize("xp", [(P, P), (N, N), (D, D), (N, D), (D, N)])
def test_dense_x_every_kind(nx, xp):
    """Every x boundary pair through the dense form (ragged last block of 32
    lines when ny*nz is not a multiple of 32)."""
    ny, nz = 12, 7
    bc = xp + (P, P, N, D)
    dzf = inputs.tanh_dzf(nz, 1.5, 2.0)
    rng = np.random.default_rng(nx + sum(xp))
    f = rng.standard_normal((nz, ny, nx))
    say("dense", nx, bc)
    po, _ = O.solve(f, bc, 1 / nx, 1 / ny, dzf)
    pg, info = dense_solve(f, bc, 1 / nx, 1 / ny, dzf)
    assert info["converged"] and info["residual"] <= 1e-10, info
    assert rel(pg, po) < 1e-8
    # the first residual shows the dense form's accuracy: split bf16 products
    # carry ~16 significant bits, amplified by the operator to ~1e-3
    assert info["history"][0] < 1e-2 and info["iterations"] <= 4


@pytest.mark.parametrize("bc,s", [((D, N, P, P, 3, 3), 0.0), ((D, N, P, P, 3, 3), -25.0),
                                  ((N, N, P, P, N, N), -25.0)])
def test_dense_x_helmholtz_and_face_z(bc, s):
    """The dense x form with a Helmholtz shift and with a z-face-located
    field (the residual fused into the dense transform uses the halved wall
    couplings)."""
    nx, ny, nz = 256, 12, 9
    cells = inputs.tanh_dzf(nz + 1 if bc[4] == 3 else nz, 1.5, 2.0)
    f = np.random.default_rng(7 + sum(bc)).standard_normal((nz, ny, nx))
    say("dense", bc, s)
    po, mo = O.solve(f, bc, 1 / nx, 1 / ny, cells, shift=s)
    assert mo == 0.0
    pg, info = dense_solve(f, bc, 1 / nx, 1 / ny, cells, shift=s)
    assert info["converged"] and info["residual"] <= 1e-10, info
    assert O.residual(pg, f, bc, 1 / nx, 1 / ny, cells, shift=s) <= 1.5e-10
    assert rel(pg, po) < 1e-8


def test_dense_c4_full_size():
    """512x256x256, Dirichlet-Neumann x (DST-IV as a dense product), periodic
    y, Dirichlet z: refined to 1e-10, against the full oracle solve."""
    pr = inputs.config("c4")
    f = pr.rhs()
    say("c4 dense")
    pg, info = dense_solve(f, pr.bc, pr.dx, pr.dy, pr.dzf)
    say("  info", info)
    assert info["converged"] and info["residual"] <= 1e-10
    po, _ = O.solve(f, pr.bc, pr.dx, pr.dy, pr.dzf)
    assert rel(pg, po) < 1e-8


def test_dense_rejected_where_unsupported():
    with pytest.raises(capi.CansError) as e:
        capi.Plan(100, 8, 8, (P, P, P, P, N, N), 0.1, 0.1, np.full(8, 0.1), precision="fp32_refine",
                  xform_x="dense")
    assert e.value.code == -2
    with pytest.raises(capi.CansError) as e:
        capi.Plan(128, 8, 8, (P, P, P, P, N, N), 0.1, 0.1, np.full(8, 0.1), precision="fp64", xform_x="dense")
    assert e.value.code == -2
