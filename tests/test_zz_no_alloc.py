"""cans_poisson_solve_noalloc -- the solve for callers that cannot allocate,
on the library's fixed scratch array -- against cans_poisson_solve on the same
plan and rhs, through the C ABI.

Two calls in a row, the second with a smaller problem (so the scratch holds the
first call's contents), in FP64 and FP32 + refinement: the results must equal
the allocating entry point's element by element (the same kernels in the same
order, so bit for bit) and match the oracle at the FP64 (1e-12) / refined
(1e-8, residual 1e-10) tolerances; the reported info must be the same.  A deep
z (plain elimination with multipliers in the scratch) and the size limit are
checked too."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2001_05234_amd import capi, inputs
from tests.parity_checks import TOL_REF, check_fp64, demean, rel, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P, N, D = 0, 1, 2


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    capi.load()
    yield
    torch.cuda.synchronize()


def both(f, bc, dx, dy, dzf, precision):
    """(result, info) of cans_poisson_solve and of cans_poisson_solve_noalloc."""
    nz, ny, nx = f.shape
    plan = capi.Plan(nx, ny, nz, bc, dx, dy, dzf, precision=precision, tol=1e-10, max_iter=4)
    fd = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    pa, pb = torch.zeros_like(fd), torch.full_like(fd, 7.0)
    plan.solve(fd, pa)
    torch.cuda.synchronize()
    ia = plan.info()
    plan.solve_noalloc(fd, pb)
    torch.cuda.synchronize()
    ib = plan.info()
    plan.close()
    return pa.cpu().numpy(), ia, pb.cpu().numpy(), ib


# the first problem is the larger: the second call finds the scratch holding
# the first call's contents
CASES = [((96, 64, 200), (P, P, P, P, N, N), "stretched"),   # pipelined z, padded levels, singular
         ((48, 32, 40), (D, N, P, P, D, D), "uniform"),      # partitioned z, smaller
         ((16, 8, 600), (N, N, P, P, N, D), "stretched")]    # plain elimination, multipliers in scratch


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_noalloc_matches_solve(precision):
    rng = np.random.default_rng(77)
    for (nx, ny, nz), bc, grid in CASES:
        dzf = inputs.tanh_dzf(nz, 1.5, 2.0) if grid == "stretched" else np.full(nz, 1.0 / nz)
        dx, dy = 2 * np.pi / nx, np.pi / ny
        f = rng.standard_normal((nz, ny, nx))
        say("noalloc", precision, (nx, ny, nz), bc)
        pa, ia, pb, ib = both(f, bc, dx, dy, dzf, precision)
        assert np.array_equal(pa, pb), float(np.abs(pa - pb).max())
        assert ia == ib, (ia, ib)
        po, mo = O.solve(f, bc, dx, dy, dzf)
        if precision == "fp64":
            check_fp64(demean(pb, bc, dzf), f, bc, dx, dy, dzf, po, case=f"noalloc {(nx, ny, nz)} {bc}")
        else:
            assert ib["converged"] and ib["residual"] <= 1e-10, ib
            assert rel(demean(pb, bc, dzf), po) < TOL_REF
        assert abs(ib["removed_mean"] - mo) < 1e-12 * max(1.0, abs(mo))


def test_noalloc_size_limit():
    """A refined problem whose FP32 field alone exceeds the scratch is refused
    with CANS_ERR_TOO_LARGE; the same plan still solves through the
    allocating entry point."""
    nx, ny, nz = 256, 256, 384   # 25.2 M points: 100 MB of FP32 field
    dzf = np.full(nz, 1.0 / nz)
    plan = capi.Plan(nx, ny, nz, (P, P, P, P, N, N), 1.0 / nx, 1.0 / ny, dzf, precision="fp32_refine")
    fd = torch.zeros((nz, ny, nx), dtype=torch.float64, device="cuda")
    pd = torch.empty_like(fd)
    with pytest.raises(capi.CansError) as e:
        plan.solve_noalloc(fd, pd)
    assert e.value.code == -6
    plan.solve(fd, pd)
    torch.cuda.synchronize()
    assert float(pd.abs().max()) == 0.0
    plan.close()
