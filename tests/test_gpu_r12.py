"""Reconstruct-12 links (WD_GAUGE_RECON12): the FP32 operator, phases A and B
of CG with FP32 inner iterations (also their even-odd half-lattice hops) and
BiCGSTAB's plane-blocked stencils read a two-row FP32 copy of the links and
rebuild the third row from the first two.

The operator on such a gauge matches the oracle's D and D^dagger in every launch
shape (plane and site blocks, one or two fields per thread, both hop orders,
both time boundaries, a 288-site plane); its result differs in the last
bits from the one on the complete FP32 links, which shows the rebuilt row was
used.

The oracle's FP64 operator recomputes the true residual of every solution.
The solution agrees with the solve on the complete links within kappa(D) (2 tol).
The profiling mode's byte count shows that the two-row copy was read: a phase-B
launch moves exactly 4 x 6 complex numbers fewer per site.  Links that are not
SU(3) are refused.
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


def _phase_b_bytes(g, m0, eta, p):
    wd.profile_reset()
    wd.profile_enable(True)
    try:
        wd.cg_solve_batch(g, m0, dev(eta), params=p)
    finally:
        wd.profile_enable(False)
    st = wd.profile_read()["cg_phaseB"]
    return st["bytes_total"], st["launches"]


@pytest.mark.parametrize("inner", [wd.F32], ids=["f32"])
@pytest.mark.parametrize("dims,t_sign", [((8, 8, 4, 6), -1), ((8, 8, 4, 6), 1), ((6, 5, 4, 6), -1),
                                         ((14, 14, 6, 4), -1)],
                         ids=["8x8x4x6-anti", "8x8x4x6-peri", "6x5x4x6-site", "14x14x6x4"])
def test_r12_cg_matches_oracle(inner, dims, t_sign):
    m0 = 0.1
    U = wdgen.gauge_field(dims, 0.5, 501)
    eta = wdgen.mixed_sources(dims, 3, 2, 502)
    V = wdgen.volume(dims)
    p = wd.cg_default_params(inner=inner, reliable_every=50)
    say("r12 cg", dims, t_sign, inner)
    g12 = wd.Gauge(dev(U), dims, t_sign, recon12=True)
    x, reps, rc = wd.cg_solve_batch(g12, m0, dev(eta), params=p)
    assert rc == wd.WD_OK, reps
    x = host(x)
    res = oracle.true_residual(U, eta, x, dims, m0, t_sign=t_sign)
    assert np.all(res <= TOL * 1.0000001), res
    g = wd.Gauge(dev(U), dims, t_sign)
    x0, reps0, rc0 = wd.cg_solve_batch(g, m0, dev(eta), params=p)
    assert rc0 == wd.WD_OK
    assert rel(x, host(x0)) <= kappa(m0) * 2 * TOL
    # the phase-B kernel read the two-row copy: per launch with work (one field, so every
    # such launch has one active field), 4 links x 3 complex numbers of 8 bytes fewer per site
    b12, n12 = _phase_b_bytes(g12, m0, eta[:1], p)
    b, n = _phase_b_bytes(g, m0, eta[:1], p)
    assert n12 > 0 and n > 0
    assert abs(b / n - b12 / n12 - 4 * 3 * 8 * V) <= 1e-6 * b / n, (b / n, b12 / n12)


@pytest.mark.parametrize("dims,t_sign", [((8, 8, 4, 6), -1), ((8, 8, 4, 6), 1), ((6, 5, 4, 6), -1),
                                         ((18, 16, 2, 4), -1)],
                         ids=["8x8x4x6-anti", "8x8x4x6-peri", "6x5x4x6", "18x16x2x4-plane288"])
def test_r12_operator_matches_oracle(dims, t_sign):
    m0 = 0.1
    U = wdgen.gauge_field(dims, 0.5, 531)
    eta = wdgen.mixed_sources(dims, 2, 1, 532)   # 3 fields: a ragged pair with 2 per thread
    g12 = wd.Gauge(dev(U), dims, t_sign, recon12=True)
    g = wd.Gauge(dev(U), dims, t_sign)
    for dag in (False, True):
        want = oracle.dirac(U, eta, dims, m0, t_sign, dagger=dag)
        # planes of more than 256 sites take the site-blocked kernel only
        for xy in ((1, 0) if dims[0] * dims[1] <= 256 else (0,)):
            for nr in (1, 2):
                for order in (1, 3):
                    say("r12 operator", dims, t_sign, "dag", dag, "xy", xy, "nr", nr, "order", order)
                    for gg in (g12, g):
                        wd.shape_set(gg, wd.F32, eta.shape[0], dag, wd.FAMILY_DSLASH, 256, nr, 1, order, 1,
                                     0, 0, xy)
                    got12 = host(wd.dslash(g12, m0, dev(eta), wd.F32, dagger=dag))
                    got = host(wd.dslash(g, m0, dev(eta), wd.F32, dagger=dag))
                    for i in range(eta.shape[0]):
                        assert rel(got12[i], want[i]) <= 1e-6, (dag, xy, nr, order, i)
                    assert np.any(got12 != got), (dag, xy, nr, order)


def test_r12_gauge_serves_every_solver():
    """Every solver takes a reconstruct-12 gauge: kernels without a two-row
    variant (FP16 storage) keep reading its complete copies; BiCGSTAB's
    plane-blocked stencils (8 x 8 planes here), the even-odd half-lattice hops
    and the persistent kernel's phases read the two-row links."""
    dims, m0 = (8, 8, 4, 6), 0.1
    U = wdgen.gauge_field(dims, 0.5, 511)
    eta = wdgen.mixed_sources(dims, 2, 1, 512)
    g12 = wd.Gauge(dev(U), dims, recon12=True)
    for kw in ({"precondition": wd.PRECOND_EO}, {"method": wd.METHOD_BICGSTAB}, {"persistent": 1},
               {"inner": wd.F16N}):
        say("r12 gauge", kw)
        kw = {"inner": wd.F32, **kw}
        x, reps, rc = wd.cg_solve_batch(g12, m0, dev(eta), params=wd.cg_default_params(**kw))
        assert rc == wd.WD_OK, (kw, reps)
        assert np.all(oracle.true_residual(U, eta, host(x), dims, m0) <= TOL * 1.0000001), kw
    say("r12 gauge operator")
    got = host(wd.dslash(g12, m0, dev(eta), wd.F32))
    assert rel(got, oracle.dirac(U, eta, dims, m0, -1)) <= 1e-6


@pytest.mark.parametrize("t_sign", [-1, 1], ids=["antiperiodic", "periodic"])
def test_r12_even_odd_solve(t_sign):
    """Even-odd CG with FP32 inner iterations on a reconstruct-12 gauge: the
    half-lattice hops of phases A and B (both halves of each) read the two-row
    links.  The oracle's operator checks the solution; it agrees with the
    solve on the complete links within kappa(D) (2 tol) and is not bitwise
    that solve's (the rebuilt third rows round differently), which shows the
    two-row copy was read."""
    dims, m0 = (8, 6, 4, 6), 0.1   # even Lx
    U = wdgen.gauge_field(dims, 0.5, 531)
    eta = wdgen.mixed_sources(dims, 3, 2, 532)
    say("r12 even-odd", t_sign)
    p = wd.cg_default_params(inner=wd.F32, precondition=wd.PRECOND_EO)
    sols = []
    for r12 in (True, False):
        g = wd.Gauge(dev(U), dims, recon12=r12, t_sign=t_sign)
        x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
        assert rc == wd.WD_OK, (r12, reps)
        sols.append(host(x))
        assert np.all(oracle.true_residual(U, eta, sols[-1], dims, m0, t_sign) <= TOL * 1.0000001), r12
    for i in range(eta.shape[0]):
        assert rel(sols[0][i], sols[1][i]) <= kappa(m0) * 2 * TOL, i
    assert np.any(sols[0] != sols[1])


def test_r12_persistent_kernel():
    """The persistent kernel (FP32 inner, one 1024-thread block per compute
    unit) reads the two-row links of a reconstruct-12 gauge: the oracle checks
    the solution, it agrees with the persistent solve on the complete links
    within kappa(D) (2 tol) and is not bitwise that one, and confining the
    launch to 5 compute units gives the same bits."""
    dims, m0 = (8, 8, 4, 6), 0.1
    U = wdgen.gauge_field(dims, 0.5, 541)
    eta = wdgen.mixed_sources(dims, 2, 2, 542)
    say("r12 persistent")
    sols = {}
    for r12, n in ((True, 0), (True, 5), (False, 0)):
        g = wd.Gauge(dev(U), dims, recon12=r12)
        p = wd.cg_default_params(inner=wd.F32, reliable_every=50, persistent=1, max_cus=n)
        x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
        assert rc == wd.WD_OK, (r12, n, reps)
        sols[r12, n] = host(x)
        assert np.all(oracle.true_residual(U, eta, sols[r12, n], dims, m0) <= TOL * 1.0000001), (r12, n)
    assert np.array_equal(sols[True, 0], sols[True, 5])
    for i in range(eta.shape[0]):
        assert rel(sols[True, 0][i], sols[False, 0][i]) <= kappa(m0) * 2 * TOL, i
    assert np.any(sols[True, 0] != sols[False, 0])


def test_r12_refuses_links_outside_su3():
    dims = (4, 4, 4, 4)
    U = wdgen.gauge_field(dims, 0.5, 521)
    U[1, 2, 3, 0, 2] *= np.exp(0.3j)   # one link of U(3) with det e^{0.9 i}
    say("r12 refuses a U(3) link")
    with pytest.raises(wd.WDError) as e:
        wd.Gauge(dev(U), dims, recon12=True)
    assert e.value.code == wd.WD_EINVAL
    wd.Gauge(dev(U), dims)   # the complete copies take any links
