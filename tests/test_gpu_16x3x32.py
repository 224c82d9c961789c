"""The 16^3 x 32 mixed-precision workload: FP16 storage with per-site FP32
norms, FP32 arithmetic, FP64 reliable updates every 50 iterations, m0 = 0.02,
12 spin-colour point sources at the origin, tol 1e-10.

The oracle's own operator checks the true residual of every solution.  A full
oracle CG at this volume takes hours, so the error against the FP64 solution
is bounded instead: both the FP16N and the FP64 GPU solutions have true
residual <= tol, hence |x16 - x64| / |x64| <= kappa(D) 2 tol with
kappa(D) <= (8 + m0) / m0, which is asserted (and printed).
"""
import numpy as np
import pytest

import oracle
import paper_2111_14958_amd as wd
import wdgen
from gpu_util import dev, host, rel, say

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def test_16x3x32_fp16n_against_fp64():
    cfg = wdgen.CONFIGS["lat16x3x32_12rhs"]
    dims, m0 = cfg["dims"], cfg["m0"]
    U = wdgen.gauge_field(dims, cfg["eps"], cfg["gauge_seed"])
    eta = wdgen.point_sources(dims)
    say("16^3x32 f16n + f64")
    g = wd.Gauge(dev(U), dims)
    deta = dev(eta)
    p16 = wd.cg_default_params(inner=wd.F16N, reliable_every=50)
    x16, r16, rc = wd.cg_solve_batch(g, m0, deta, params=p16)
    assert rc == wd.WD_OK, r16
    p64 = wd.cg_default_params(inner=wd.F64, reliable_every=0)
    x64, r64, rc = wd.cg_solve_batch(g, m0, deta, params=p64)
    assert rc == wd.WD_OK, r64
    x16, x64 = host(x16), host(x64)
    res = oracle.true_residual(U, eta, x16, dims, m0)
    assert np.all(res <= TOL * 1.0000001), res
    res64 = oracle.true_residual(U, eta, x64, dims, m0)
    assert np.all(res64 <= TOL * 1.0000001), res64
    kappa = (8.0 + m0) / m0
    errs = [rel(x16[i], x64[i]) for i in range(eta.shape[0])]
    print("16^3x32 iters f16n", [r["iters"] for r in r16], "f64", [r["iters"] for r in r64],
          "max err f16n vs f64", max(errs), flush=True)
    assert max(errs) <= kappa * 2 * TOL
