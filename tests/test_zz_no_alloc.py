"""The allocation-free CG entry point against the allocating one (needs an MI355X).

sdmm_solve_interface_noalloc runs the same kernels with the CG workspace in
the library's fixed per-GPU scratch array, so on the same inputs it must give
the same lambda, iteration counts, residuals and status as
sdmm_solve_interface.  Two calls in a row, the second with a smaller batch,
check that nothing the first call leaves in the shared array reaches the
second.  A batch larger than the array is refused before any work.
"""
import numpy as np
import pytest

from workloads import problem

from gpu_helpers import gpu_ctx, gpu_solve

pytestmark = pytest.mark.gpu


def _noalloc(ctx, idx, rtol):
    import torch
    M = ctx.sizes()["M"]
    n = len(idx)
    g = torch.tensor(np.asarray(idx, dtype=np.int64), device="cuda")
    lam = torch.full((n, M), np.nan, dtype=torch.float64, device="cuda")
    it = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    rr = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    st = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    ctx.solve_interface_noalloc(g, lam, rtol=rtol, iters=it, relres=rr, status=st)
    torch.cuda.synchronize()
    return lam.cpu().numpy(), it.cpu().numpy(), rr.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("name,first,second", [
    ("cfg0", list(range(16)), [3, 9, 1]),
    ("cfg1", list(range(0, 361, 2)), [5, 200, 17, 360, 44]),
])
def test_noalloc_matches_allocating_path(name, first, second):
    print("case: noalloc vs allocating", name, flush=True)
    ctx = gpu_ctx(problem(name), "fp64")
    for idx in (first, second):
        _, lam_a, it_a, rr_a, st_a, _ = gpu_solve(ctx, idx, rtol=1e-10)
        lam_b, it_b, rr_b, st_b = _noalloc(ctx, idx, 1e-10)
        lam_a = lam_a.cpu().numpy()
        assert (st_b == 0).all() and (st_a == 0).all()
        assert (it_a == it_b).all()
        # the same kernels and the same fixed summation orders: bit-identical
        assert np.array_equal(lam_a, lam_b), np.abs(lam_a - lam_b).max()
        assert np.array_equal(rr_a, rr_b)
    ctx.close()


def test_noalloc_feti_layout_and_size_limit():
    print("case: noalloc on the small floating-Stokes layout and its size limit", flush=True)
    import torch
    from paper_1802_06263_amd import sdmm
    p = problem("cfg2", stokes_mesh=(8, 8), darcy_mesh=(4, 4), mortar={"degree": 1, "elements": 2})
    ctx = gpu_ctx(p, "fp64")
    for idx in ([0, 17, 4000, 6560, 1234, 99], [6560, 3]):
        _, lam_a, it_a, _, st_a, _ = gpu_solve(ctx, idx, rtol=1e-10)
        lam_b, it_b, _, st_b = _noalloc(ctx, idx, 1e-10)
        assert (it_a == it_b).all() and (st_b == 0).all()
        assert np.array_equal(lam_a.cpu().numpy(), lam_b)
    # 40,000 realizations of this layout need about 400 MB of CG workspace
    M = ctx.sizes()["M"]
    big = 40000
    assert big * 8 * 2 * M > ctx.noalloc_scratch_bytes()
    g = torch.zeros(big, dtype=torch.int64, device="cuda")
    lam = torch.zeros((big, M), dtype=torch.float64, device="cuda")
    with pytest.raises(sdmm.SdmmError) as e:
        ctx.solve_interface_noalloc(g, lam, rtol=1e-8)
    assert e.value.code == sdmm.EINVAL and "scratch" in str(e.value)
    ctx.close()
