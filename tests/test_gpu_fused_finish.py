"""The fused finish against the three-launch iteration.

With the fused finish a CG iteration is two launches: phase A completes the
previous iteration's finish itself (every block sums the partials in the
finish's fixed order and applies the same scalar update) and a trailing finish
closes each chunk.  It performs exactly the arithmetic of the three-launch
iteration (phase A, phase B, one-block finish), so solutions, iteration
counts and residuals must agree bit for bit.  WD_CG_UNFUSED=1 selects the
three-launch iteration (it is part of the chunk graph's key, so both run in
one process).  Each solution is also checked by the oracle's operator."""
import os

import numpy as np
import pytest

import oracle
import paper_2111_14958_amd as wd
import wdgen
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _solve(g, m0, eta, p, unfused):
    if unfused:
        os.environ["WD_CG_UNFUSED"] = "1"
    try:
        x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
    finally:
        os.environ.pop("WD_CG_UNFUSED", None)
    assert rc == wd.WD_OK, reps
    return host(x), reps


CASES = [((8, 8, 8, 8), 5, 0.05), ((6, 6, 4, 8), 3, 0.1)]   # plane blocks (64-site planes), site blocks


@pytest.mark.parametrize("dims,nrhs,m0", CASES, ids=[str(c[0]) for c in CASES])
@pytest.mark.parametrize("inner", [wd.F64, wd.F32, wd.F16N], ids=["f64", "f32", "f16n"])
def test_fused_finish_is_bitwise_the_three_launch_iteration(dims, nrhs, m0, inner):
    U = wdgen.gauge_field(dims, 0.5, 1200 + sum(dims))
    eta = wdgen.mixed_sources(dims, nrhs - 2, 2, 1300 + sum(dims))
    g = wd.Gauge(dev(U), dims, -1, recon12=True)
    # chunk 7 (odd): the trailing finish reads the second record array
    for chunk in (0, 7):
        p = wd.cg_default_params(inner=inner, reliable_every=0 if inner == wd.F64 else 20, chunk=chunk)
        say("fused vs three-launch", dims, nrhs, inner, "chunk", chunk)
        xf, rf = _solve(g, m0, eta, p, unfused=False)
        xu, ru = _solve(g, m0, eta, p, unfused=True)
        assert np.array_equal(xf.view(np.uint64), xu.view(np.uint64))
        assert [r["iters"] for r in rf] == [r["iters"] for r in ru]
        assert [r["reliable_updates"] for r in rf] == [r["reliable_updates"] for r in ru]
        assert [r["true_rel_res"] for r in rf] == [r["true_rel_res"] for r in ru]
        res = oracle.true_residual(U, eta, xf, dims, m0, -1)
        assert np.all(res <= 1e-10 * 1.0000001), res
    g.close()


def test_fused_finish_in_profiling_mode():
    """The profiling mode launches the same kernel sequence one by one."""
    dims, nrhs, m0 = (8, 8, 8, 8), 4, 0.05
    U = wdgen.gauge_field(dims, 0.5, 1401)
    eta = wdgen.mixed_sources(dims, 2, 2, 1402)
    g = wd.Gauge(dev(U), dims, -1, recon12=True)
    p = wd.cg_default_params(inner=wd.F32, reliable_every=50)
    xg, rg = _solve(g, m0, eta, p, unfused=False)
    wd.profile_reset()
    wd.profile_enable(True)
    try:
        say("fused finish, profiling mode")
        xp, rp = _solve(g, m0, eta, p, unfused=False)
    finally:
        wd.profile_enable(False)
    prof = wd.profile_read()
    assert prof["cg_phaseA"]["launches"] > 0 and prof["cg_phaseB"]["launches"] > 0
    assert np.array_equal(xg.view(np.uint64), xp.view(np.uint64))
    assert [r["iters"] for r in rg] == [r["iters"] for r in rp]
    g.close()


def test_fused_finish_in_the_server():
    """Grouped launches of the server: the same requests give bitwise the same
    results with the fused finish and with the three-launch iteration."""
    from test_gpu_serve import _requests, _run
    reqs = [r for r in _requests() if not r["eo"]]   # even-odd requests keep three launches
    say("serve fused vs three-launch", len(reqs))
    xf, rf, _ = _run(reqs, 256 << 20)
    os.environ["WD_CG_UNFUSED"] = "1"
    try:
        xu, ru, _ = _run(reqs, 256 << 20)
    finally:
        os.environ.pop("WD_CG_UNFUSED", None)
    for a, b, ea, eb in zip(xf, xu, rf, ru):
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
        assert [e["iters"] for e in ea] == [e["iters"] for e in eb]
