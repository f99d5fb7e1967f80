"""GPU parity of the HIP library against the FP64 CPU oracle, through the C ABI.

Tolerances: FP64 path ||p - p_oracle|| / ||p_oracle|| <= 1e-12; FP32 transforms
with FP64 refinement: relative residual <= 1e-10 (the convergence target) and
parity <= 1e-8 (error/residual ratio measured about 1-10 on these grids).
Singular problems are compared after removing the dzf-weighted mean of both
fields (their solution is unique up to a constant).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2001_05234_amd import capi, inputs
from tests.parity_checks import TOL64, TOL_REF, check_fp64, demean, rel, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P, N, D = 0, 1, 2
PAIRS = [(P, P), (N, N), (D, D), (N, D), (D, N)]


def gpu_solve(f, bc, dx, dy, dzf, precision="fp64", tol=1e-10, max_iter=4, inplace=False, autotune=False):
    nz, ny, nx = f.shape
    plan = capi.Plan(nx, ny, nz, bc, dx, dy, dzf, precision=precision, tol=tol, max_iter=max_iter,
                     autotune=autotune)
    fd = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    if inplace:
        plan.solve(fd, fd)
        pd = fd
    else:
        pd = torch.zeros_like(fd)
        plan.solve(fd, pd)
    torch.cuda.synchronize()
    out = pd.cpu().numpy()
    info = plan.info()
    plan.close()
    return out, info


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    capi.load()
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("bc", [(P, P, P, P, N, N), (D, N, P, P, D, D), (N, D, N, N, N, D),
                                (D, D, D, N, P, P), (N, N, D, D, D, N)])
def test_stage_parity(bc):
    """Each stage of the FP64 pipeline against the oracle's stage."""
    nx, ny, nz = 24, 20, 10
    dzf = np.full(nz, 0.1) if bc[4] == P else inputs.tanh_dzf(nz, 1.5, 2.0)
    dx, dy = 0.25, 0.3
    rng = np.random.default_rng(3)
    f = rng.standard_normal((nz, ny, nx))
    kx, ky = O.axis_kind(bc[0], bc[1]), O.axis_kind(bc[2], bc[3])
    sx = nx // 2 if kx in (O.K_ND, O.K_DN) else nx
    sy = ny // 2 if ky in (O.K_ND, O.K_DN) else ny
    say("stage parity", bc)
    plan = capi.Plan(nx, ny, nz, bc, dx, dy, dzf)
    a = torch.from_numpy(f).cuda()
    b = torch.zeros_like(a)

    def stage(s, x):
        plan.debug_stage(s, torch.from_numpy(np.ascontiguousarray(x)).cuda(), b)
        torch.cuda.synchronize()
        return b.cpu().numpy()

    s1 = O.transform(f, 0, kx)
    assert rel(stage(1, f), s1) < 1e-13
    s2 = O.transform(s1, 1, ky)
    assert rel(stage(2, s1), s2) < 1e-13
    s3, _ = O.spectral_solve(s2, bc, dx, dy, dzf)
    assert rel(stage(3, s2) * (sx * sy), s3) < 1e-12
    s4 = O.transform(s3, 1, ky, inverse=True)
    assert rel(stage(4, s3), sy * s4) < 1e-13
    s5 = O.transform(s4, 0, kx, inverse=True)
    assert rel(stage(5, s4), sx * s5) < 1e-13
    plan.close()
    del a


@pytest.mark.parametrize("zp", PAIRS)
@pytest.mark.parametrize("yp", PAIRS)
@pytest.mark.parametrize("xp", PAIRS)
def test_fp64_every_bc(xp, yp, zp):
    """All 125 boundary combinations, uniform and stretched z."""
    bc = xp + yp + zp
    nx, ny, nz = 16, 12, 10
    rng = np.random.default_rng(sum(bc) + 7)
    f = rng.standard_normal((nz, ny, nx))
    for dzf in ([np.full(nz, 0.1)] + ([] if zp == (P, P) else [inputs.tanh_dzf(nz, 1.5, 2.0)])):
        say("fp64 bc", bc, "stretched" if dzf[0] != dzf[1] else "uniform")
        po, mo = O.solve(f, bc, 0.2, 0.3, dzf)
        pg, info = gpu_solve(f, bc, 0.2, 0.3, dzf)
        check_fp64(pg, f, bc, 0.2, 0.3, dzf, po)
        assert abs(info["removed_mean"] - mo) < 1e-12 * max(1.0, abs(mo))


@pytest.mark.parametrize("shape", [(1, 2, 2), (1, 2, 4), (5, 6, 10), (3, 40, 72), (2, 2, 512), (4, 512, 2),
                                   (7, 30, 50), (1, 96, 128), (3, 24, 1024)])
def test_fp64_shapes(shape):
    """Degenerate, ragged-tile and long-line shapes (radices 2..8, 3, 5)."""
    nz, ny, nx = shape
    rng = np.random.default_rng(nx + ny + nz)
    f = rng.standard_normal(shape)
    for bc in [(P, P, N, N, N, N), (D, N, P, P, D, D), (N, D, D, D, N, D)]:
        dzf = inputs.tanh_dzf(nz, 1.2, 1.0)
        say("fp64 shape", shape, bc)
        pg, _ = gpu_solve(f, bc, 0.3, 0.7, dzf)
        check_fp64(pg, f, bc, 0.3, 0.7, dzf)


@pytest.mark.parametrize("nz", [3, 12, 64, 97, 128, 200])
def test_periodic_z_cyclic(nz):
    """Periodic z: the cyclic (Sherman-Morrison) partitioned kernel up to 128
    levels (full and ragged segments, partial column blocks), the plain
    elimination beyond; singular and nonsingular columns; refinement too."""
    rng = np.random.default_rng(9 + nz)
    dzf = np.full(nz, 1.0 / nz)
    for bc in [(D, D, N, D, P, P), (P, P, P, P, P, P), (N, N, P, P, P, P)]:
        f = rng.standard_normal((nz, 10, 12))
        say("cyclic z", nz, bc)
        pg, _ = gpu_solve(f, bc, 0.3, 0.2, dzf)
        check_fp64(pg, f, bc, 0.3, 0.2, dzf)
    bc = (P, P, N, N, P, P)
    f = rng.standard_normal((nz, 10, 12))
    po, _ = O.solve(f, bc, 0.3, 0.2, dzf)
    pg, info = gpu_solve(f, bc, 0.3, 0.2, dzf, precision="fp32_refine", tol=1e-10, max_iter=6)
    assert info["converged"] and info["residual"] <= 1e-10, info
    assert rel(demean(pg, bc, dzf), po) < TOL_REF


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_fp64_config_full(name):
    pr = inputs.config(name)
    f = pr.rhs()
    say("fp64 config", name)
    po, mo = O.solve(f, pr.bc, pr.dx, pr.dy, pr.dzf)
    pg, info = gpu_solve(f, pr.bc, pr.dx, pr.dy, pr.dzf)
    assert rel(pg, po) < TOL64
    assert abs(info["removed_mean"] - mo) < 1e-13
    assert abs(O.weighted_mean(pg, pr.dzf)) < 1e-14 * np.abs(po).max()
    assert O.residual(pg, f, pr.bc, pr.dx, pr.dy, pr.dzf) < 1e-12


def test_fp64_inplace_and_deterministic():
    pr = inputs.config("c1")
    f = pr.rhs()
    say("fp64 in place")
    p1, _ = gpu_solve(f, pr.bc, pr.dx, pr.dy, pr.dzf)
    p2, _ = gpu_solve(f, pr.bc, pr.dx, pr.dy, pr.dzf, inplace=True)
    assert np.array_equal(p1, p2)


@pytest.mark.parametrize("zp", PAIRS)
@pytest.mark.parametrize("xp", PAIRS)
def test_refine_bc(xp, zp):
    """FP32 transforms + FP64 refinement, the boundary pairs in x and z (y
    runs through the same kernels as x)."""
    for yp in ((P, P), (D, N)):
        bc = xp + yp + zp
        nx, ny, nz = 32, 24, 16
        dzf = np.full(nz, 1 / nz) if zp == (P, P) else inputs.tanh_dzf(nz, 1.5, 2.0)
        rng = np.random.default_rng(sum(bc) + 11)
        f = rng.standard_normal((nz, ny, nx))
        say("refine bc", bc)
        po, mo = O.solve(f, bc, 1 / nx, 1 / ny, dzf)
        pg, info = gpu_solve(f, bc, 1 / nx, 1 / ny, dzf, precision="fp32_refine", tol=1e-10, max_iter=6)
        assert info["converged"] and info["residual"] <= 1e-10, info
        ro = O.residual(pg, f, bc, 1 / nx, 1 / ny, dzf)
        assert ro <= 1.5e-10
        # the reported residuals are the device's norms of the returned p
        assert abs(info["residual"] - ro) <= 1e-3 * ro + 1e-16
        ri = O.residual_inf(pg, f, bc, 1 / nx, 1 / ny, dzf)
        assert abs(info["residual_inf"] - ri) <= 1e-3 * ri + 1e-16
        assert rel(demean(pg, bc, dzf), po) < TOL_REF
        assert abs(info["removed_mean"] - mo) < 1e-13 * max(1, abs(mo))


@pytest.mark.parametrize("shape,bc", [((200, 30, 70), (D, N, P, P, N, D)), ((150, 6, 97), (P, P, N, N, N, N)),
                                      ((90, 54, 33), (N, D, D, D, D, N))])
def test_refine_ragged_tiles(shape, bc):
    """Refinement on grids that leave partial tiles everywhere: x not a
    multiple of 64, y not a multiple of 4, z chunks cut short; the reported
    residual must be the oracle's residual of the returned p."""
    nx, ny, nz = shape
    dzf = inputs.tanh_dzf(nz, 1.5, 2.0)
    rng = np.random.default_rng(nx + ny + nz)
    f = rng.standard_normal((nz, ny, nx))
    say("refine ragged", shape, bc)
    po, mo = O.solve(f, bc, 1 / nx, 1 / ny, dzf)
    pg, info = gpu_solve(f, bc, 1 / nx, 1 / ny, dzf, precision="fp32_refine", tol=1e-10, max_iter=6)
    assert info["converged"] and info["residual"] <= 1e-10, info
    ro = O.residual(pg, f, bc, 1 / nx, 1 / ny, dzf)
    assert abs(info["residual"] - ro) <= 1e-3 * ro + 1e-16
    ri = O.residual_inf(pg, f, bc, 1 / nx, 1 / ny, dzf)
    assert abs(info["residual_inf"] - ri) <= 1e-3 * ri + 1e-16
    assert rel(demean(pg, bc, dzf), po) < TOL_REF


def test_refine_alias_rejected():
    pr = inputs.config("c1")
    plan = capi.Plan(pr.nx, pr.ny, pr.nz, pr.bc, pr.dx, pr.dy, pr.dzf, precision="fp32_refine")
    a = torch.zeros(pr.nz, pr.ny, pr.nx, dtype=torch.float64, device="cuda")
    with pytest.raises(capi.CansError) as e:
        plan.solve(a, a)
    assert e.value.code == -5
    plan.close()


def test_refine_not_converged_reported():
    """max_iter = 0 and an unreachable tolerance: reported, not raised."""
    pr = inputs.config("c1")
    f = pr.rhs()
    say("refine not converged")
    pg, info = gpu_solve(f, pr.bc, pr.dx, pr.dy, pr.dzf, precision="fp32_refine", tol=1e-30, max_iter=0)
    assert not info["converged"] and info["iterations"] == 0
    assert 1e-9 < info["residual"] < 1e-5
    pg, info = gpu_solve(f, pr.bc, pr.dx, pr.dy, pr.dzf, precision="fp32_refine", tol=1e-30, max_iter=2)
    assert not info["converged"] and info["iterations"] == 2 and len(info["history"]) == 3


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_refine_config_full(name):
    pr = inputs.config(name)
    f = pr.rhs()
    say("refine config", name)
    po, _ = O.solve(f, pr.bc, pr.dx, pr.dy, pr.dzf)
    pg, info = gpu_solve(f, pr.bc, pr.dx, pr.dy, pr.dzf, precision="fp32_refine")
    say("  info", info)
    assert info["converged"] and info["residual"] <= 1e-10
    assert O.residual(pg, f, pr.bc, pr.dx, pr.dy, pr.dzf) <= 1.5e-10
    assert rel(demean(pg, pr.bc, pr.dzf), po) < TOL_REF
    # the refinement keeps the zero mode pinned in FP64
    assert abs(O.weighted_mean(pg, pr.dzf)) < 1e-13 * np.abs(po).max()


def test_c4_full_size():
    """512x256x256, Dirichlet-Neumann x (DST-IV), periodic y, Dirichlet z:
    both paths against the full oracle solve."""
    pr = inputs.config("c4")
    f = pr.rhs()
    say("c4 oracle")
    po, _ = O.solve(f, pr.bc, pr.dx, pr.dy, pr.dzf)
    say("c4 fp64")
    pg, _ = gpu_solve(f, pr.bc, pr.dx, pr.dy, pr.dzf)
    check_fp64(pg, f, pr.bc, pr.dx, pr.dy, pr.dzf, po)
    say("c4 refine")
    pr32, info = gpu_solve(f, pr.bc, pr.dx, pr.dy, pr.dzf, precision="fp32_refine")
    say("  info", info)
    assert info["converged"] and info["residual"] <= 1e-10
    assert rel(pr32, po) < TOL_REF


@pytest.mark.timeout(900)
def test_c3_full_size():
    """1024x512x384 channel slab at full size, element by element against the
    full oracle solve of the same rhs (about 15 s on 16 host threads): the
    FP64 path at 1e-12, the refined path at 1e-8 (both have zero weighted
    mean, as the oracle's solution does), plus the refined residual measured
    with the oracle's operator and the reported removed means."""
    pr = inputs.config("c3")
    say("c3 rhs")
    f = pr.rhs()
    say("c3 oracle")
    po, mo = O.solve(f, pr.bc, pr.dx, pr.dy, pr.dzf)
    say("c3 fp64")
    p64, info64 = gpu_solve(f, pr.bc, pr.dx, pr.dy, pr.dzf)
    e64 = check_fp64(demean(p64, pr.bc, pr.dzf), f, pr.bc, pr.dx, pr.dy, pr.dzf, po, case="c3 fp64")
    say("  fp64 vs oracle", e64)
    say("c3 refine")
    p32, info = gpu_solve(f, pr.bc, pr.dx, pr.dy, pr.dzf, precision="fp32_refine")
    say("  info", info)
    assert info["converged"] and info["residual"] <= 1e-10
    e32 = rel(demean(p32, pr.bc, pr.dzf), po)
    say("  refine vs oracle", e32)
    assert e32 < TOL_REF
    r32 = O.residual(p32, f, pr.bc, pr.dx, pr.dy, pr.dzf)
    say("  refine residual (oracle operator)", r32)
    assert r32 <= 1.5e-10 and abs(info["residual"] - r32) <= 1e-3 * r32
    scale = np.abs(po).max()
    assert abs(O.weighted_mean(p64, pr.dzf)) < 1e-13 * scale
    assert abs(O.weighted_mean(p32, pr.dzf)) < 1e-13 * scale
    assert abs(info["removed_mean"] - mo) < 1e-12 and abs(info64["removed_mean"] - mo) < 1e-12


@pytest.mark.parametrize("nz", [288, 320, 352, 384])
def test_zsolve_deep_columns(nz):
    """z depths 288..384: the partitioned z kernel with two 32-column
    segments per wave, 16-level segments and 576..768 threads a block (the
    kernel the 1024x512x384 slab runs), element by element against the
    oracle on a 64x48 plane, stretched z, FP64 and refined; the wall pairs
    NN, DN and ND, and a periodic z (plain elimination) beside them."""
    nx, ny = 64, 48
    rng = np.random.default_rng(nz)
    for bc in [(P, P, P, P, N, N), (D, N, P, P, D, N), (P, P, N, D, N, D), (N, N, D, D, P, P)]:
        dzf = np.full(nz, 2.0 / nz) if bc[4] == P else inputs.tanh_dzf(nz, 1.5, 2.0)
        dx, dy = 2 * np.pi / nx, np.pi / ny
        f = rng.standard_normal((nz, ny, nx))
        say("deep z", nz, bc)
        po, mo = O.solve(f, bc, dx, dy, dzf)
        pg, info = gpu_solve(f, bc, dx, dy, dzf)
        check_fp64(pg, f, bc, dx, dy, dzf, po, case=f"deep z nz {nz} {bc}")
        assert abs(info["removed_mean"] - mo) < 1e-12 * max(1.0, abs(mo))
        pg, info = gpu_solve(f, bc, dx, dy, dzf, precision="fp32_refine", tol=1e-10, max_iter=6)
        assert info["converged"] and info["residual"] <= 1e-10, info
        assert rel(demean(pg, bc, dzf), po) < TOL_REF


@pytest.mark.parametrize("name", ["c2", "c4"])
def test_autotuned_plans(name):
    """Plans whose transform tiles were picked by the plan-time tuner give the
    same results (FP64 and refined)."""
    pr = inputs.config(name)
    f = pr.rhs()
    say("autotune", name)
    po, _ = O.solve(f, pr.bc, pr.dx, pr.dy, pr.dzf)
    pg, _ = gpu_solve(f, pr.bc, pr.dx, pr.dy, pr.dzf, autotune=True)
    check_fp64(pg, f, pr.bc, pr.dx, pr.dy, pr.dzf, po)
    pg, info = gpu_solve(f, pr.bc, pr.dx, pr.dy, pr.dzf, precision="fp32_refine", autotune=True)
    assert info["converged"] and info["residual"] <= 1e-10
    assert rel(demean(pg, pr.bc, pr.dzf), po) < TOL_REF


def test_autotune_x_form_choice():
    """xform_x AUTO with autotune on a refinement plan whose x axis the dense
    form takes: the plan times whole refined solves with either x form, keeps
    one, reports it, and solves to the oracle with it; fixed forms report
    themselves."""
    nx, ny, nz = 512, 48, 32
    bc = (D, N, P, P, D, D)
    dz = np.full(nz, 1.0 / nz)
    f = np.random.default_rng(23).uniform(-1, 1, (nz, ny, nx))
    po, _ = O.solve(f, bc, 1.0 / nx, 1.0 / ny, dz)
    fd = torch.from_numpy(f).cuda()
    for xf, want in (("auto", None), ("dense", "dense"), ("fft", "fft")):
        plan = capi.Plan(nx, ny, nz, bc, 1.0 / nx, 1.0 / ny, dz, precision="fp32_refine", tol=1e-10,
                         max_iter=6, xform_x=xf, autotune=xf == "auto")
        mode = plan.xform_mode(0)
        say("x form", xf, "->", mode)
        assert mode == want if want else mode in ("fft", "dense")
        assert plan.xform_mode(1) == "fft"
        pd = torch.zeros_like(fd)
        plan.solve(fd, pd)
        torch.cuda.synchronize()
        info = plan.info()
        plan.close()
        assert info["converged"] and info["residual"] <= 1e-10, (xf, info)
        assert rel(pd.cpu().numpy(), po) < TOL_REF
    plan = capi.Plan(nx, ny, nz, bc, 1.0 / nx, 1.0 / ny, dz, autotune=True)
    assert plan.xform_mode(0) == "fft"
    with pytest.raises(capi.CansError):
        plan.xform_mode(2)
    plan.close()


def test_graph_mode_matches_direct_launches():
    """opts.graph: the first solve with a (rhs, p) pair records the kernel
    sequence into a HIP graph and later solves replay it.  Replays (with
    unrelated eager work and host synchronisations between them), a new
    recording for new arrays, and the in-place FP64 form all give the bits of
    direct launches."""
    nx, ny, nz = 96, 64, 40
    bc = (P, P, N, N, N, D)
    dzf = inputs.tanh_dzf(nz, 1.5, 2.0)
    f = np.random.default_rng(17).standard_normal((nz, ny, nx))
    fd = torch.from_numpy(f).cuda()
    for precision in ("fp64", "fp32_refine"):
        say("graph mode", precision)
        direct = capi.Plan(nx, ny, nz, bc, 1 / nx, 1 / ny, dzf, precision=precision)
        graph = capi.Plan(nx, ny, nz, bc, 1 / nx, 1 / ny, dzf, precision=precision, graph=True)
        p0 = torch.zeros_like(fd)
        direct.solve(fd, p0)
        torch.cuda.synchronize()
        ref, ref_info = p0.cpu().numpy(), direct.info()
        pg = torch.zeros_like(fd)
        for rep in range(3):
            pg.zero_()
            junk = torch.randn(256, 256, device="cuda") @ torch.randn(256, 256, device="cuda")
            torch.cuda.synchronize()
            graph.solve(fd, pg)
            torch.cuda.synchronize()
            assert np.array_equal(pg.cpu().numpy(), ref), (precision, rep)
            assert graph.info() == ref_info
            del junk
        pg2 = torch.zeros_like(fd)
        graph.solve(fd, pg2)
        torch.cuda.synchronize()
        assert np.array_equal(pg2.cpu().numpy(), ref)
        if precision == "fp64":
            x = fd.clone()
            graph.solve(x, x)
            torch.cuda.synchronize()
            assert np.array_equal(x.cpu().numpy(), ref)
        po, _ = O.solve(f, bc, 1 / nx, 1 / ny, dzf)
        assert rel(ref, po) < (1e-12 if precision == "fp64" else TOL_REF)
        direct.close()
        graph.close()


@pytest.mark.parametrize("bc", [(P, P, P, P, N, N), (P, P, P, P, P, P), (D, N, P, P, D, D), (N, N, D, D, N, D)])
def test_helmholtz(bc):
    """(L_h + s) p = f with s < 0 (implicit diffusion of a cell-centred
    quantity): FP64 and FP32 + refinement against the oracle's shifted solve;
    boundary sets that are singular for s = 0 are regular here."""
    nx, ny, nz = 48, 40, 36
    dzf = np.full(nz, 2.0 / nz) if bc[4] == P else inputs.tanh_dzf(nz, 1.5, 2.0)
    s = -25.0
    rng = np.random.default_rng(31 + sum(bc))
    f = rng.standard_normal((nz, ny, nx))
    say("helmholtz", bc)
    po, mo = O.solve(f, bc, 1 / nx, 1 / ny, dzf, shift=s)
    assert mo == 0.0
    nz_, ny_, nx_ = f.shape
    for precision in ("fp64", "fp32_refine"):
        plan = capi.Plan(nx, ny, nz, bc, 1 / nx, 1 / ny, dzf, precision=precision, tol=1e-10, max_iter=6, shift=s)
        fd = torch.from_numpy(f).cuda()
        pd = torch.zeros_like(fd)
        plan.solve(fd, pd)
        torch.cuda.synchronize()
        pg, info = pd.cpu().numpy(), plan.info()
        plan.close()
        assert info["removed_mean"] == 0.0
        if precision == "fp64":
            check_fp64(pg, f, bc, 1 / nx, 1 / ny, dzf, po, shift=s, case=f"helmholtz {bc}")
            assert O.residual(pg, f, bc, 1 / nx, 1 / ny, dzf, shift=s) < 1e-12
        else:
            assert info["converged"] and info["residual"] <= 1e-10, info
            ro = O.residual(pg, f, bc, 1 / nx, 1 / ny, dzf, shift=s)
            assert ro <= 1.5e-10 and abs(info["residual"] - ro) <= 1e-3 * ro + 1e-16
            assert rel(pg, po) < TOL_REF


@pytest.mark.parametrize("nz,bc", [(7, (P, P, P, P, 3, 3)), (40, (N, N, P, P, 3, 3)), (200, (D, N, N, D, 3, 3)),
                                   (300, (P, P, N, N, 3, 3)), (600, (P, P, P, P, 3, 3))])
def test_face_located_z(nz, bc):
    """A field on the z faces with zero on the wall faces (the wall-normal
    velocity of the implicit diffusion steps): nz interior faces of a
    stretched (nz+1)-cell grid, Poisson and Helmholtz, FP64 and FP32 +
    refinement, through every z-solve form (partitioned segments of 8 and 16
    levels, two segments per wave, and the plain elimination beyond 512)."""
    nx, ny = (48, 40) if nz <= 200 else (24, 20)
    cells = inputs.tanh_dzf(nz + 1, 1.5, 2.0)
    dx, dy = 2 * np.pi / nx, np.pi / ny
    rng = np.random.default_rng(nz + sum(bc))
    f = rng.standard_normal((nz, ny, nx))
    for s in (0.0, -25.0):
        say("face-located z", nz, bc, "shift", s)
        po, mo = O.solve(f, bc, dx, dy, cells, shift=s)
        assert mo == 0.0
        for precision in ("fp64", "fp32_refine"):
            plan = capi.Plan(nx, ny, nz, bc, dx, dy, cells, precision=precision, tol=1e-10, max_iter=6, shift=s)
            fd = torch.from_numpy(f).cuda()
            pd = torch.zeros_like(fd)
            plan.solve(fd, pd)
            torch.cuda.synchronize()
            pg, info = pd.cpu().numpy(), plan.info()
            plan.close()
            assert info["removed_mean"] == 0.0
            if precision == "fp64":
                check_fp64(pg, f, bc, dx, dy, cells, po, shift=s, case=f"face-located z nz {nz} {bc} shift {s}")
                assert O.residual(pg, f, bc, dx, dy, cells, shift=s) < 1e-12
            else:
                assert info["converged"] and info["residual"] <= 1e-10, info
                ro = O.residual(pg, f, bc, dx, dy, cells, shift=s)
                assert ro <= 1.5e-10 and abs(info["residual"] - ro) <= 1e-3 * ro + 1e-16
                assert rel(pg, po) < TOL_REF


DF, NF = 3, 4


@pytest.mark.timeout(600)
@pytest.mark.parametrize("shape,bc", [
    ((63, 40, 24), (DF, DF, P, P, N, N)),       # DST-I along x (extended line of 128)
    ((65, 48, 20), (NF, NF, D, D, N, N)),       # DCT-I along x
    ((64, 47, 30), (DF, NF, DF, DF, D, N)),     # (3,4) along x, DST-I along y
    ((96, 49, 16), (NF, DF, NF, NF, N, D)),     # (4,3) along x, DCT-I along y
    ((90, 36, 50), (P, P, DF, NF, DF, DF)),     # (3,4) along y, face-located z too
    ((1023, 64, 32), (DF, DF, P, P, N, N)),     # DST-I over 1024-point FFTs, many tiles
    ((1025, 24, 40), (NF, NF, P, P, D, N)),     # DCT-I over 1024-point FFTs
])
def test_face_located_xy(shape, bc):
    """Fields on the faces of x or y (DST-I, DCT-I and the type-III face
    pairs), FP64 and FP32 + refinement, Poisson and Helmholtz, element by
    element against the oracle."""
    nx, ny, nz = shape
    dz = inputs.tanh_dzf(nz + 1 if bc[4] == DF else nz, 1.5, 2.0)
    dx, dy = 2 * np.pi / (nx + 1), np.pi / (ny + 1)
    rng = np.random.default_rng(nx + 3 * ny + nz)
    f = rng.standard_normal((nz, ny, nx))
    for s in (0.0, -25.0):
        say("face-located x/y", shape, bc, "shift", s)
        po, mo = O.solve(f, bc, dx, dy, dz, shift=s)
        assert mo == 0.0
        for precision in ("fp64", "fp32_refine"):
            plan = capi.Plan(nx, ny, nz, bc, dx, dy, dz, precision=precision, tol=1e-10, max_iter=6, shift=s)
            fd = torch.from_numpy(f).cuda()
            pd = torch.zeros_like(fd)
            plan.solve(fd, pd)
            torch.cuda.synchronize()
            pg, info = pd.cpu().numpy(), plan.info()
            plan.close()
            assert info["removed_mean"] == 0.0
            if precision == "fp64":
                check_fp64(pg, f, bc, dx, dy, dz, po, shift=s, case=f"face-located x/y {shape} {bc} shift {s}")
            else:
                assert info["converged"] and info["residual"] <= 1e-10, info
                ro = O.residual(pg, f, bc, dx, dy, dz, shift=s)
                assert ro <= 1.5e-10 and abs(info["residual"] - ro) <= 1e-3 * ro + 1e-16
                assert rel(pg, po) < TOL_REF


def test_face_located_xy_rejections():
    """What the face-located x/y pairs do not take: a (4,4) axis in an
    otherwise singular problem, the dense transform, the projection step."""
    dz = np.full(8, 0.1)
    for kw in ({}, {"precision": "fp32_refine", "xform_x": "dense"}):
        bc = (NF, NF, P, P, N, N) if not kw else (DF, NF, P, P, N, N)
        nx = 65 if not kw else 128
        with pytest.raises(capi.CansError) as e:
            capi.Plan(nx, 32, 8, bc, 0.1, 0.1, dz, **kw)
        assert e.value.code == -2
    capi.Plan(65, 32, 8, (NF, NF, P, P, N, N), 0.1, 0.1, dz, shift=-1.0).close()
    plan = capi.Plan(63, 32, 8, (DF, DF, P, P, N, N), 0.1, 0.1, dz)
    a = [torch.zeros((8, 32, 63), dtype=torch.float64, device="cuda") for _ in range(4)]
    with pytest.raises(capi.CansError) as e:
        plan.project(*a, 0.1)
    assert e.value.code == -2
    plan.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("shape,bc", [((48, 40, 36), (P, P, P, P, N, N)), ((50, 24, 30), (N, N, P, P, N, N)),
                                      ((40, 30, 24), (P, P, N, N, P, P)), ((30, 20, 17), (N, N, N, N, N, N)),
                                      ((1024, 512, 384), (P, P, P, P, N, N))])
def test_projection_step(shape, bc):
    """cans_poisson_project against the oracle's projection step: Phi (the
    change of p), the velocity increments, a divergence-free result, wall
    faces kept; a second call reuses the plan's Phi field."""
    nx, ny, nz = shape
    dx, dy = 2 * np.pi / nx, np.pi / ny
    dzf = np.full(nz, 2.0 / nz) if bc[4] == P else inputs.tanh_dzf(nz, 1.5, 2.0)
    rng = np.random.default_rng(nx + ny + nz + sum(bc))
    u, v, w, p = (rng.standard_normal((nz, ny, nx)) for _ in range(4))
    if bc[0] == N:
        u[:, :, -1] = 0
    if bc[2] == N:
        v[:, -1, :] = 0
    if bc[4] == N:
        w[-1] = 0
    gdt = 0.8 * 2e-3
    say("projection", shape, bc)
    full = nx * ny * nz > 1e7
    plan = capi.Plan(nx, ny, nz, bc, dx, dy, dzf, precision="fp64", autotune=full)
    dev = [torch.from_numpy(a.copy()).cuda() for a in (u, v, w, p)]
    plan.project(*dev, gdt)
    torch.cuda.synchronize()
    ug, vg, wg, pg = (a.cpu().numpy() for a in dev)
    d0 = np.abs(O.divergence(u, v, w, bc, dx, dy, dzf)).max()
    d1 = np.abs(O.divergence(ug, vg, wg, bc, dx, dy, dzf)).max()
    assert d1 < 1e-10 * d0, (d1, d0)
    if bc[0] == N:
        assert np.array_equal(ug[:, :, -1], u[:, :, -1])
    if bc[4] == N:
        assert np.array_equal(wg[-1], w[-1])
    # element by element against the oracle's step, at every size (the
    # 1024x512x384 slab too: one oracle solve of about 15 s)
    uo, vo, wo, po, phi = O.project(u, v, w, p, bc, dx, dy, dzf, gdt)
    say("  phi vs oracle", rel(pg - p, phi))
    assert rel(pg - p, phi) < TOL64, rel(pg - p, phi)
    for g_, o_, a_ in ((ug, uo, u), (vg, vo, v), (wg, wo, w)):
        assert rel(g_ - a_, o_ - a_) < 1e-11, rel(g_ - a_, o_ - a_)
    del uo, vo, wo, po, phi
    # a second step on a divergence-free field changes it by rounding only
    plan.project(*dev, gdt)
    torch.cuda.synchronize()
    u2 = dev[0].cpu().numpy()
    assert np.abs(u2 - ug).max() < 1e-9 * np.abs(ug).max()
    plan.close()


@pytest.mark.parametrize("shape,bc", [((32, 24, 20), (P, P, P, P, N, N)), ((24, 16, 18), (N, N, P, P, N, N)),
                                      ((16, 20, 12), (P, P, N, N, P, P)), ((18, 12, 10), (N, N, N, N, N, N)),
                                      ((90, 40, 50), (P, P, P, P, N, N))])
def test_projection_implicit_update_and_dt(shape, bc):
    """cans_poisson_project_ex against the oracle: the implicit-diffusion
    pressure update p += Phi - alpha L_h Phi (1e-12 on the change of p) and
    the time-step bound of eq. (dt) on the corrected velocity (1e-14; with and
    without the viscous bound), for periodic and walled axes and a ragged
    grid; velocities equal those of the explicit form."""
    nx, ny, nz = shape
    dx, dy = 2 * np.pi / nx, np.pi / ny
    dzf = np.full(nz, 2.0 / nz) if bc[4] == P else inputs.tanh_dzf(nz, 1.5, 2.0)
    rng = np.random.default_rng(nx * ny + nz + sum(bc))
    u, v, w, p = (rng.standard_normal((nz, ny, nx)) for _ in range(4))
    if bc[0] == N:
        u[:, :, -1] = 0
    if bc[2] == N:
        v[:, -1, :] = 0
    if bc[4] == N:
        w[-1] = 0
    gdt, alpha = 1.6e-3, 0.8 * 2e-4 * 1.6e-3 / 2
    say("projection ex", shape, bc)
    plan = capi.Plan(nx, ny, nz, bc, dx, dy, dzf, precision="fp64")
    uo, vo, wo, po, phi = O.project(u, v, w, p, bc, dx, dy, dzf, gdt, alpha=alpha)
    for nu in (0.0, 5e-2):
        dev = [torch.from_numpy(a.copy()).cuda() for a in (u, v, w, p)]
        dt = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        plan.project_ex(*dev, gdt, alpha=alpha, nu=nu, dt_max=dt)
        torch.cuda.synchronize()
        ug, vg, wg, pg = (a.cpu().numpy() for a in dev)
        assert rel(pg - p, po - p) < TOL64, rel(pg - p, po - p)
        for g_, o_, a_ in ((ug, uo, u), (vg, vo, v), (wg, wo, w)):
            assert rel(g_ - a_, o_ - a_) < 1e-11, rel(g_ - a_, o_ - a_)
        # the bound on the velocity the GPU returned (rates are local sums)
        dto = O.max_dt(ug, vg, wg, bc, dx, dy, dzf, nu=nu)
        say("  dt", float(dt.item()), dto)
        assert abs(dt.item() - dto) <= 1e-14 * dto
        # explicit form: same velocity, p += Phi only
        dev2 = [torch.from_numpy(a.copy()).cuda() for a in (u, v, w, p)]
        plan.project(*dev2, gdt)
        torch.cuda.synchronize()
        for a_, b_ in zip(dev[:3], dev2[:3]):
            assert torch.equal(a_, b_)
        pe = dev2[3].cpu().numpy()
        # the implicit term -alpha L_h Phi alone
        assert rel(pg - pe, po - p - phi) < 1e-10, rel(pg - pe, po - p - phi)
    # without dt_max nothing is written
    dt = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    dev = [torch.from_numpy(a.copy()).cuda() for a in (u, v, w, p)]
    plan.project_ex(*dev, gdt, alpha=alpha)
    torch.cuda.synchronize()
    assert dt.item() == -1.0
    plan.close()


def test_projection_ex_rejections_and_rest():
    nx, ny, nz = 16, 12, 8
    a = [torch.zeros((nz, ny, nx), dtype=torch.float64, device="cuda") for _ in range(4)]
    plan = capi.Plan(nx, ny, nz, (P, P, P, P, N, N), 0.1, 0.1, np.full(nz, 0.1), precision="fp64")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    for kw in ({"alpha": -1.0}, {"nu": -1.0}, {"alpha": float("nan")}, {"nu": float("inf")}):
        with pytest.raises(capi.CansError) as e:
            plan.project_ex(*a, 0.1, dt_max=dt, **kw)
        assert e.value.code == -1
    # a field at rest: +inf without viscosity, the viscous bound with it
    plan.project_ex(*a, 0.1, dt_max=dt)
    torch.cuda.synchronize()
    assert dt.item() == float("inf")
    plan.project_ex(*a, 0.1, nu=1e-3, dt_max=dt)
    torch.cuda.synchronize()
    assert dt.item() == pytest.approx(1.65 * 0.1 ** 2 / 1e-3, rel=1e-15)
    plan.close()


def test_projection_rejections():
    nx, ny, nz = 16, 12, 8
    a = [torch.zeros((nz, ny, nx), dtype=torch.float64, device="cuda") for _ in range(4)]
    ok = capi.Plan(nx, ny, nz, (P, P, P, P, N, N), 0.1, 0.1, np.full(nz, 0.1), precision="fp64")
    with pytest.raises(capi.CansError) as e:
        ok.project(a[0], a[0], a[2], a[3], 0.1)
    assert e.value.code == -5
    with pytest.raises(capi.CansError) as e:
        ok.project(*a, 0.0)
    assert e.value.code == -1
    ok.close()
    for bc, prec in (((P, P, P, P, D, D), "fp64"), ((P, P, N, D, N, N), "fp64"), ((P, P, P, P, N, N), "fp32_refine")):
        plan = capi.Plan(nx, ny, nz, bc, 0.1, 0.1, np.full(nz, 0.1), precision=prec)
        with pytest.raises(capi.CansError) as e:
            plan.project(*a, 0.1)
        assert e.value.code == -2
        plan.close()
