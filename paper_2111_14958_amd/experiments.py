"""The paper's two tuning / scaling studies (arXiv 2111.14958, Sec. 3.1) on MI355X.

    python -m paper_2111_14958_amd.experiments fig1   # whole-CG time vs block size

Fig. 1 of the paper times the whole CG at 14^4 while varying the SYCL
workgroup size with the number of compute units fixed; here the block size of
every CG kernel is swept (64, 128, 256 threads) through wd_shape_set, using the
single-field FP64 CG of the paper's algorithm (plain CG on D D^dagger,
true-residual check at 1e-10) on seeded synthetic fields (links exp(i 0.5 H),
Gaussian source, m0 = 0.05).  Prints one JSON line per point.
"""
from __future__ import annotations

import json
import sys
import time


def _setup(dims=(14, 14, 14, 14), m0=0.05):
    import torch

    import paper_2111_14958_amd as wd
    import wdgen
    U = wdgen.gauge_field(dims, 0.5, 1002)
    src = wdgen.gaussian_source(dims, 1, 2002)
    g = wd.Gauge(torch.from_numpy(U).cuda(), dims)
    dsrc = torch.from_numpy(src).cuda()
    return wd, torch, g, dsrc, m0


def _time_solve(wd, torch, g, dsrc, m0, params, reps=3):
    sol = torch.zeros_like(dsrc)
    ws = torch.empty(wd.cg_workspace_bytes(g, 1, params), dtype=torch.uint8, device="cuda")
    wd.cg_solve_batch(g, m0, dsrc, sol=sol, params=params, ws=ws)   # warm (graph capture)
    torch.cuda.synchronize()
    best, rep = 1e30, None
    for _ in range(reps):
        t0 = time.perf_counter()
        _, reps_, rc = wd.cg_solve_batch(g, m0, dsrc, sol=sol, params=params, ws=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if dt < best:
            best, rep = dt, reps_[0]
    return best, rep


def fig1(blocks=(64, 128, 256)):
    wd, torch, g, dsrc, m0 = _setup()
    p = wd.cg_default_params(inner=wd.F64, reliable_every=0)
    for blk in blocks:
        for fam, dag in ((wd.FAMILY_CG_A, True), (wd.FAMILY_CG_B, False), (wd.FAMILY_CG_R, False)):
            wd.shape_set(g, wd.F64, 1, dag, fam, blk, rhs_per_thread=1)
        t, rep = _time_solve(wd, torch, g, dsrc, m0, p)
        print(json.dumps({"figure": 1, "lattice": "14^4", "block": blk, "seconds": t,
                          "iters": rep["iters"], "true_rel_res": rep["true_rel_res"],
                          "gflops": 2 * 1368.0 * 14 ** 4 * rep["iters"] / t / 1e9}), flush=True)


if __name__ == "__main__":
    {"fig1": fig1}[sys.argv[1]]()
