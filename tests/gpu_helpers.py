"""Shared helpers of the GPU parity tests (they compare the HIP path with the oracle)."""
import numpy as np


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def gpu_ctx(prob, precision="fp64"):
    import torch  # noqa: F401
    from paper_1802_06263_amd import sdmm
    ctx = sdmm.Context(0)
    ctx.set_problem(prob)
    ctx.build_flux_basis(precision)
    return ctx


def gpu_solve(ctx, idx, rtol=1e-12, max_iter=None, allow_notconv=False):
    import torch
    M = ctx.sizes()["M"]
    n = len(idx)
    g = torch.tensor(np.asarray(idx, dtype=np.int64), device="cuda")
    lam = torch.zeros((n, M), dtype=torch.float64, device="cuda")
    it = torch.zeros(n, dtype=torch.int32, device="cuda")
    rr = torch.zeros(n, dtype=torch.float64, device="cuda")
    st = torch.zeros(n, dtype=torch.int32, device="cuda")
    rc = ctx.solve_interface(g, lam, rtol=rtol, max_iter=max_iter, iters=it, relres=rr, status=st,
                             allow_notconv=allow_notconv)
    torch.cuda.synchronize()
    return g, lam, it.cpu().numpy(), rr.cpu().numpy(), st.cpu().numpy(), rc
