"""Write tests/golden/cfg2_reference.npz from the oracle alone.

The full-size 4x2 Stokes over 8x4 Darcy layout (64x64 meshes, P1 mortars with
8 elements, 3^8 tensor collocation) is too slow for the oracle inside a GPU
test, so its reference values are computed here once, by the FP64 oracle
only (no part of the GPU library is imported):

  * every Stokes S_{H,i} (Section 5.1, eqs. starSproblem1-2), the floating
    subdomains included, and the interface data g_H (eqs. barSproblem1-2)
    and G (the rigid-motion traces of the FETI coarse problem);
  * 24 seeded global collocation points with seeded positive weights,
    taken through Method S3 (Section 5.4) at CG rtol 1e-12: lambda of each
    point, and the weighted moments (Section 2: mean and E[u^2] - E[u]^2)
    of every field, stored on a seeded sample of 4096 entries per field
    together with the largest |mean| and |var| over the whole field.

Run:  python tests/golden/make_cfg2_reference.py   (about ten minutes on 8 cores)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.methods import FIELDS, Oracle  # noqa: E402
from workloads import problem  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg2_reference.npz")
N_POINTS = 24
N_SAMPLE = 4096
RTOL = 1e-12


def main():
    t0 = time.time()
    prob = problem("cfg2")
    o = Oracle(prob, threads=int(os.environ.get("ORACLE_THREADS", "8")))
    print("oracle set-up %.1f s" % (time.time() - t0), flush=True)
    stokes_S = o.stokes_basis()
    print("stokes bases %.1f s" % (time.time() - t0), flush=True)
    rng = np.random.default_rng(2024)
    idx = np.sort(rng.choice(o.grid.nreal, N_POINTS, replace=False))
    w = rng.uniform(0.5, 1.5, N_POINTS)
    w /= w.sum()
    mom, info = o.run("S3", indices=[int(l) for l in idx], weights=w, rtol=RTOL)
    print("S3 loop %.1f s" % (time.time() - t0), flush=True)
    out = {
        "idx": idx.astype(np.int64),
        "weights": w,
        "rtol": np.array(RTOL),
        "g": o.g_stokes,
        "G": o.G.T.copy(),  # n_kernel x M, the layout of sdmm_get_interface_data
        "lambda": np.stack([d["lambda"] for d in info]),
        "iters": np.array([d["iters"] for d in info], dtype=np.int64),
        "stokes_ids": np.array(o.stokes_ids, dtype=np.int64),
    }
    for i, S in stokes_S.items():
        out["S_stokes_%d" % i] = S
    srng = np.random.default_rng(7)
    for f in FIELDS:
        mean, var = mom[f]
        n = mean.size
        sel = np.sort(srng.choice(n, min(N_SAMPLE, n), replace=False))
        out["sel_" + f] = sel.astype(np.int64)
        out["mean_" + f] = mean[sel]
        out["var_" + f] = var[sel]
        out["maxmean_" + f] = np.array(np.abs(mean).max())
        out["maxvar_" + f] = np.array(np.abs(var).max())
        out["size_" + f] = np.array(n)
    np.savez_compressed(OUT, **out)
    print("wrote %s (%.1f s)" % (OUT, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
