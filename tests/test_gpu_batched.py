"""Batched solves (one graph launch for many uneven problems) against the
oracle, through the C ABI.  Same tolerances as tests/test_gpu_parity.py."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2001_05234_amd import capi, inputs
from tests.parity_checks import check_fp64, demean, rel, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c5():
    assert torch.cuda.is_available()
    probs = inputs.batch_c5()
    rhs = [pr.rhs() for pr in probs]
    return probs, rhs


def test_c5_batched_refine(c5):
    """64 uneven problems (sizes, boundary sets, stretching drawn from a seed),
    FP32 transforms + FP64 refinement, one graph launch."""
    probs, rhs = c5
    say("c5 plan", sum(p.npts for p in probs), "points")
    plan = capi.BatchedPlan(probs, precision="fp32_refine", tol=1e-10, max_iter=4, autotune=True)
    fs = [torch.from_numpy(f).cuda() for f in rhs]
    ps = [torch.zeros_like(f) for f in fs]
    say("c5 solve")
    plan.solve(fs, ps)
    torch.cuda.synchronize()
    for i, (pr, f) in enumerate(zip(probs, rhs)):
        info = plan.info(i)
        assert info["converged"] and info["residual"] <= 1e-10, (i, pr, info)
        po, mo = O.solve(f, pr.bc, pr.dx, pr.dy, pr.dzf)
        pg = ps[i].cpu().numpy()
        e = rel(demean(pg, pr.bc, pr.dzf), po)
        assert e < 1e-8, (i, pr.nx, pr.ny, pr.nz, pr.bc, e)
        assert O.residual(pg, f, pr.bc, pr.dx, pr.dy, pr.dzf) <= 1.5e-10
    plan.close()


def test_c5_graph_replays_exact(c5):
    """Replays of the captured graph, with unrelated eager GPU work and host
    synchronisations between them, reproduce the first result bitwise; new
    array addresses trigger a new capture that is also exact."""
    probs, rhs = c5
    probs, rhs = probs[:12], rhs[:12]
    plan = capi.BatchedPlan(probs, precision="fp32_refine")
    fs = [torch.from_numpy(f).cuda() for f in rhs]
    ps = [torch.zeros_like(f) for f in fs]
    plan.solve(fs, ps)
    torch.cuda.synchronize()
    ref = [p.cpu().numpy() for p in ps]
    for rep in range(3):
        say("replay", rep)
        for p in ps:
            p.zero_()
        junk = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")
        torch.cuda.synchronize()
        plan.solve(fs, ps)
        torch.cuda.synchronize()
        for a, p in zip(ref, ps):
            assert np.array_equal(a, p.cpu().numpy())
        del junk
    ps2 = [torch.zeros_like(f) for f in fs]
    plan.solve(fs, ps2)
    torch.cuda.synchronize()
    for a, p in zip(ref, ps2):
        assert np.array_equal(a, p.cpu().numpy())
    for i in range(len(probs)):
        assert plan.info(i)["converged"]
    plan.close()


def test_batched_fp64(c5):
    probs, rhs = c5
    probs, rhs = probs[:16], rhs[:16]
    plan = capi.BatchedPlan(probs, precision="fp64")
    fs = [torch.from_numpy(f).cuda() for f in rhs]
    ps = [torch.zeros_like(f) for f in fs]
    plan.solve(fs, ps)
    torch.cuda.synchronize()
    for i, (pr, f) in enumerate(zip(probs, rhs)):
        po, mo = O.solve(f, pr.bc, pr.dx, pr.dy, pr.dzf)
        pg = ps[i].cpu().numpy()
        check_fp64(pg, f, pr.bc, pr.dx, pr.dy, pr.dzf, po, case=f"batched fp64 member {i}")
        assert abs(plan.info(i)["removed_mean"] - mo) < 1e-12
    plan.close()


def test_batched_face_located_z():
    """Face-located z fields (code 3, nz+1 cell widths) batched with
    cell-centred ones and with each other, FP64 and FP32 + refinement."""
    P, N, D, DF = 0, 1, 2, 3
    shapes = [(32, 24, 17, (P, P, P, P, DF, DF)), (48, 32, 40, (N, N, D, N, DF, DF)),
              (24, 16, 12, (P, P, P, P, N, N)), (40, 20, 70, (D, D, P, P, DF, DF))]
    probs, rhs = [], []
    for i, (nx, ny, nz, bc) in enumerate(shapes):
        nw = nz + 1 if bc[4] == DF else nz
        probs.append(inputs.Problem(nx, ny, nz, bc, 1.0 / nx, 2.0 / ny, inputs.tanh_dzf(nw, 1.5, 2.0)))
        f = np.random.default_rng(70 + i).standard_normal((nz, ny, nx))
        if O.is_singular(bc):
            f -= O.weighted_mean(f, probs[-1].dzf)
        rhs.append(f)
    for precision in ("fp64", "fp32_refine"):
        say("batched face-located z", precision)
        plan = capi.BatchedPlan(probs, precision=precision, tol=1e-10, max_iter=6)
        fs = [torch.from_numpy(f).cuda() for f in rhs]
        ps = [torch.zeros_like(f) for f in fs]
        plan.solve(fs, ps)
        torch.cuda.synchronize()
        for i, (pr, f) in enumerate(zip(probs, rhs)):
            po, _ = O.solve(f, pr.bc, pr.dx, pr.dy, pr.dzf)
            pg = demean(ps[i].cpu().numpy(), pr.bc, pr.dzf)
            if precision == "fp64":
                assert rel(pg, po) < 1e-12, (i, rel(pg, po))
            else:
                info = plan.info(i)
                assert info["converged"] and info["residual"] <= 1e-10, (i, info)
                assert rel(pg, po) < 1e-8, (i, rel(pg, po))
        plan.close()


def test_batched_helmholtz():
    """A batch with a Helmholtz shift (one shift for the plan): cell-centred
    and face-located members, FP64 and FP32 + refinement; nothing removed."""
    P, N, D, DF = 0, 1, 2, 3
    s = -40.0
    shapes = [(32, 24, 16, (P, P, P, P, N, N)), (48, 16, 23, (N, N, D, N, DF, DF)), (24, 32, 12, (P, P, N, N, P, P))]
    probs, rhs = [], []
    for i, (nx, ny, nz, bc) in enumerate(shapes):
        nw = nz + 1 if bc[4] == DF else nz
        dzf = np.full(nw, 2.0 / nw) if bc[4] == P else inputs.tanh_dzf(nw, 1.5, 2.0)
        probs.append(inputs.Problem(nx, ny, nz, bc, 1.0 / nx, 2.0 / ny, dzf))
        rhs.append(np.random.default_rng(90 + i).standard_normal((nz, ny, nx)))
    for precision in ("fp64", "fp32_refine"):
        say("batched helmholtz", precision)
        plan = capi.BatchedPlan(probs, precision=precision, tol=1e-10, max_iter=6, shift=s)
        fs = [torch.from_numpy(f).cuda() for f in rhs]
        ps = [torch.zeros_like(f) for f in fs]
        plan.solve(fs, ps)
        torch.cuda.synchronize()
        for i, (pr, f) in enumerate(zip(probs, rhs)):
            po, mo = O.solve(f, pr.bc, pr.dx, pr.dy, pr.dzf, shift=s)
            assert mo == 0.0
            pg = ps[i].cpu().numpy()
            info = plan.info(i)
            assert info["removed_mean"] == 0.0
            if precision == "fp64":
                assert rel(pg, po) < 1e-12, (i, rel(pg, po))
            else:
                assert info["converged"] and info["residual"] <= 1e-10, (i, info)
                assert rel(pg, po) < 1e-8, (i, rel(pg, po))
        plan.close()


def test_batched_velocity_components():
    """The three Helmholtz solves of an implicit diffusion substep (eq.
    (up_id_2)) in a closed duct of 48 x 32 x 24 cells, one batch: u on the x
    faces (DST-I along x), v on the y faces (DST-I along y), w on the z
    faces, every tangential direction a no-slip wall (Dirichlet cells),
    stretched z; FP64 and FP32 + refinement against the oracle."""
    D, DF = 2, 3
    cx, cy, cz = 48, 32, 24
    dx, dy = 1.0 / cx, 0.75 / cy
    cells = inputs.tanh_dzf(cz, 1.5, 2.0)
    s = -2.0 / (8.0 / 15.0 * 1e-3 * 2e-3)   # -2 / (gamma_1 nu dt)
    probs = [inputs.Problem(cx - 1, cy, cz, (DF, DF, D, D, D, D), dx, dy, cells),
             inputs.Problem(cx, cy - 1, cz, (D, D, DF, DF, D, D), dx, dy, cells),
             inputs.Problem(cx, cy, cz - 1, (D, D, D, D, DF, DF), dx, dy, cells)]
    rhs = [np.random.default_rng(110 + i).standard_normal((pr.nz, pr.ny, pr.nx)) for i, pr in enumerate(probs)]
    for precision in ("fp64", "fp32_refine"):
        say("batched velocity components", precision)
        plan = capi.BatchedPlan(probs, precision=precision, tol=1e-10, max_iter=6, shift=s)
        fs = [torch.from_numpy(f).cuda() for f in rhs]
        ps = [torch.zeros_like(f) for f in fs]
        plan.solve(fs, ps)
        torch.cuda.synchronize()
        for i, (pr, f) in enumerate(zip(probs, rhs)):
            po, mo = O.solve(f, pr.bc, pr.dx, pr.dy, pr.dzf, shift=s)
            pg = ps[i].cpu().numpy()
            info = plan.info(i)
            assert info["removed_mean"] == 0.0
            if precision == "fp64":
                assert rel(pg, po) < 1e-12, (i, rel(pg, po))
            else:
                assert info["converged"] and info["residual"] <= 1e-10, (i, info)
                assert rel(pg, po) < 1e-8, (i, rel(pg, po))
        plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_grouped_batch_matches_single_solves(c5, precision):
    """The batch runs each step as one launch per kernel variant over all its
    problems (grouped launches).  Each member's result and info equal, bit
    for bit, the same problem solved by a single-problem plan with direct
    launches: C5 members of every transform kind, periodic and bounded z of
    several depths in one grouped z launch, and members whose z solve runs on
    its own (the pipelined solve at nz = 200, the plain one at nz = 600)."""
    P, N, D = 0, 1, 2
    probs, rhs = list(c5[0][:10]), list(c5[1][:10])
    for nx, ny, nz, bc in [(64, 48, 200, (P, P, N, N, N, D)), (32, 24, 600, (D, N, P, P, N, N)),
                           (40, 32, 40, (N, D, D, D, P, P)), (24, 40, 72, (P, P, P, P, P, P))]:
        dzf = np.full(nz, 2.0 / nz) if bc[4] == P else inputs.tanh_dzf(nz, 1.5, 2.0)
        probs.append(inputs.Problem(nx, ny, nz, bc, 1.0 / nx, 2.0 / ny, dzf))
        f = np.random.default_rng(nz + nx).standard_normal((nz, ny, nx))
        if O.is_singular(bc):
            f -= O.weighted_mean(f, dzf)
        rhs.append(f)
    say("grouped batch", precision, len(probs), "problems")
    plan = capi.BatchedPlan(probs, precision=precision, tol=1e-10, max_iter=4)
    fs = [torch.from_numpy(f).cuda() for f in rhs]
    ps = [torch.zeros_like(f) for f in fs]
    plan.solve(fs, ps)
    torch.cuda.synchronize()
    for i, pr in enumerate(probs):
        single = capi.Plan(pr.nx, pr.ny, pr.nz, pr.bc, pr.dx, pr.dy, pr.dzf, precision=precision, tol=1e-10,
                           max_iter=4)
        p1 = torch.zeros_like(fs[i])
        single.solve(fs[i], p1)
        torch.cuda.synchronize()
        assert torch.equal(p1, ps[i]), (i, pr.nx, pr.ny, pr.nz, pr.bc)
        assert single.info() == plan.info(i), (i, single.info(), plan.info(i))
        single.close()
    plan.close()
