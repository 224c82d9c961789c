"""GPU even-odd preconditioned CG (precondition = WD_PRECOND_EO) against the oracle.

The GPU solves the Schur complement system on the even sites and rebuilds the
odd half.  Every returned solution is checked by the oracle's full operator:
true relative residual <= tol.  Against the oracle's even-odd CG and the dense
or plain-CG solutions the error is bounded by kappa(D) (tol_gpu + tol_oracle),
kappa(D) <= (8 + m0) / m0.  In FP64 without intermediate reliable updates the
GPU iterates the oracle's recurrence, so the iteration counts agree.
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


def kappa(m0):
    return (8.0 + m0) / m0


def _params(inner, **kw):
    kw.setdefault("reliable_every", 0 if inner == wd.F64 else 50)
    return wd.cg_default_params(inner=inner, precondition=wd.PRECOND_EO, **kw)


def _check_solution(U, eta, x, dims, m0):
    res = oracle.true_residual(U, eta, x, dims, m0)
    assert np.all(res <= TOL * 1.0000001), f"true residuals {res}"
    return res


@pytest.mark.parametrize("inner", [wd.F64, wd.F32, wd.F16N], ids=["f64", "f32", "f16n"])
def test_lat4x4_1rhs(inner):
    cfg = wdgen.CONFIGS["lat4x4_1rhs"]
    dims, m0 = cfg["dims"], cfg["m0"]
    U = wdgen.gauge_field(dims, cfg["eps"], cfg["gauge_seed"])
    eta = wdgen.gaussian_source(dims, 1, cfg["src_seed"])
    say("eo c1", inner)
    g = wd.Gauge(dev(U), dims)
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=_params(inner))
    x = host(x)
    assert rc == wd.WD_OK, reps
    res = _check_solution(U, eta, x, dims, m0)
    assert abs(reps[0]["true_rel_res"] - res[0]) <= 1e-3 * TOL + 1e-6 * res[0]
    D = oracle.dense(U, dims, m0)
    xs = np.linalg.solve(D, eta.ravel())
    assert rel(x.ravel(), xs) <= kappa(m0) * TOL
    xo, it, ro, st = oracle.cg_eo(U, eta, dims, m0, tol=TOL)
    assert st[0] == 0 and rel(x, xo) <= kappa(m0) * 2 * TOL
    if inner == wd.F64:
        assert abs(reps[0]["iters"] - it[0]) <= 1, (reps[0]["iters"], it[0])


@pytest.mark.parametrize("inner", [wd.F64, wd.F32, wd.F16N], ids=["f64", "f32", "f16n"])
def test_batch_mixed_sources_8x4(inner):
    dims, m0 = (8, 8, 8, 8), 0.05
    U = wdgen.gauge_field(dims, 0.5, 1003)
    eta = wdgen.mixed_sources(dims, 12, 4, 2003)
    say("eo batch 16 rhs", inner)
    g = wd.Gauge(dev(U), dims)
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=_params(inner))
    assert rc == wd.WD_OK, reps
    x = host(x)
    _check_solution(U, eta, x, dims, m0)
    for i in (0, 13):
        xo, it, ro, st = oracle.cg_eo(U, eta[i:i + 1], dims, m0, tol=TOL)
        assert st[0] == 0 and rel(x[i], xo[0]) <= kappa(m0) * 2 * TOL, i
        if inner == wd.F64:
            assert abs(reps[i]["iters"] - it[0]) <= 1, (i, reps[i]["iters"], it[0])
    # the unpreconditioned GPU solve reaches the same solution in more iterations
    xp, repp, rcp = wd.cg_solve_batch(g, m0, dev(eta), params=wd.cg_default_params(
        inner=inner, reliable_every=0 if inner == wd.F64 else 50))
    assert rcp == wd.WD_OK
    assert rel(host(xp), x) <= kappa(m0) * 2 * TOL
    assert max(r["iters"] for r in reps) < min(r["iters"] for r in repp)


def test_paper_volume_14x4_f32():
    dims, m0 = (14, 14, 14, 14), 0.05
    U = wdgen.gauge_field(dims, 0.5, 1002)
    eta = wdgen.gaussian_source(dims, 1, 2002)
    say("eo 14^4 f32")
    g = wd.Gauge(dev(U), dims)
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=_params(wd.F32))
    assert rc == wd.WD_OK, reps
    _check_solution(U, eta, host(x), dims, m0)


def test_initial_guess_zero_source_periodic_and_errors():
    dims, m0 = (4, 6, 4, 4), 0.1
    U = wdgen.gauge_field(dims, 0.5, 21)
    eta = wdgen.gaussian_source(dims, 2, 22)
    eta[1] = 0
    say("eo x0 / zero source / periodic / errors")
    g = wd.Gauge(dev(U), dims)
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=_params(wd.F64))
    assert rc == wd.WD_OK
    x = host(x)
    assert np.all(x[1] == 0) and reps[1]["iters"] == 0
    _check_solution(U, eta[:1], x[:1], dims, m0)
    x2, reps2, rc = wd.cg_solve_batch(g, m0, dev(eta), sol=dev(x), params=_params(wd.F64, use_x0=1))
    assert rc == wd.WD_OK and reps2[0]["iters"] == 0
    # periodic time direction: the boundary sign is carried by the packed links
    gp = wd.Gauge(dev(U), dims, t_sign=1)
    xp, repp, rc = wd.cg_solve_batch(gp, m0, dev(eta[:1]), params=_params(wd.F32))
    assert rc == wd.WD_OK
    assert np.all(oracle.true_residual(U, eta[:1], host(xp), dims, m0, t_sign=1) <= TOL * 1.0000001)
    # an odd Lx has no two-site parity pairs: rejected
    do = (5, 4, 4, 4)
    Uo = wdgen.gauge_field(do, 0.5, 23)
    go = wd.Gauge(dev(Uo), do)
    eo_src = dev(wdgen.gaussian_source(do, 1, 24))
    _, _, rc = wd.cg_solve_batch(go, m0, eo_src, params=_params(wd.F32), raise_on_error=False)
    assert rc == wd.WD_EINVAL


@pytest.mark.parametrize("inner", [wd.F64, wd.F32, wd.F16N], ids=["f64", "f32", "f16n"])
@pytest.mark.parametrize("dims", [(14, 14, 4, 4), (16, 8, 4, 6), (12, 12, 2, 6)], ids=["14x14", "16x8", "12x12"])
def test_half_plane_blocks(inner, dims):
    """The phases' half-lattice hops on half-plane blocks (the Lx Ly / 2 sites
    of one parity on an xy-plane, 98, 64 and 72 here: x and y neighbours from
    LDS, hop order 5; FP32 on the reconstruct-12 links) against site blocks
    (hop order 1, complete links): both solutions pass the oracle's residual
    check and agree within kappa(D) (2 tol); in FP64 without reliable updates
    both iterate the same recurrence, so the iteration counts agree to
    rounding."""
    m0 = 0.1
    U = wdgen.gauge_field(dims, 0.5, 1301)
    eta = wdgen.mixed_sources(dims, 3, 2, 1302)
    nrhs = eta.shape[0]
    sols, iters = {}, {}
    for xy in (1, 0):
        say("eo half-plane blocks", dims, inner, xy)
        g = wd.Gauge(dev(U), dims, recon12=bool(xy) and inner == wd.F32)
        for fam, dag in ((wd.FAMILY_CG_A, True), (wd.FAMILY_CG_B, False)):
            wd.shape_set(g, inner, nrhs, dag, fam, 256, 1, 1, 5 if xy else 1, 1, 0, 0, xy)
        x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=_params(inner))
        assert rc == wd.WD_OK, (xy, reps)
        sols[xy] = host(x)
        iters[xy] = [r["iters"] for r in reps]
        _check_solution(U, eta, sols[xy], dims, m0)
    for i in range(nrhs):
        assert rel(sols[1][i], sols[0][i]) <= kappa(m0) * 2 * TOL, i
        if inner == wd.F64:
            assert abs(iters[1][i] - iters[0][i]) <= 2, (iters, i)
