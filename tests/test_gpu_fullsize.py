"""Full-size parity and the right-hand-side limits.

* The benchmark workload (14^4, 16 fields: 12 spin-colour point sources and 4
  Gaussian sources, m0 0.05, links exp(i 0.5 H)) in the launch configuration
  the benchmark times, i.e. the default launch shapes:
  - the operator D and D^dagger on all 16 fields, in each storage precision,
    against the oracle's operator over the whole lattice;
  - the mixed-precision CG (FP32 inner, FP64 reliable updates every 50; with
    the reconstruct-12 link copies, as the benchmark, and without them): the
    oracle's FP64 operator recomputes every solution's true residual, which must
    be <= tol and agree with the residual the library reports; the solution
    agrees with the FP64 CG solution within kappa(D) (2 tol), the bound on the
    error of two solutions that both meet tol.
* The same 16 fields solved in one persistent launch per chunk (grid barriers,
  every block sweeping several tiles per phase), FP32 inner and FP64, with the
  default phase shapes and with site blocks of 4 (FP32) or 2 (FP64) right-hand
  sides per thread: oracle residuals, and agreement with the kernel-per-phase
  solution.
* 64 right-hand sides, the most one call takes, solve like single fields; 65
  are refused.
"""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2111_14958_amd as wd
import wdgen
from gpu_util import dev, host, rel, say
from test_gpu_dslash import check_per_site

pytestmark = pytest.mark.gpu
TOL = 1e-10
OP_TOL = {wd.F64: 1e-13, wd.F32: 1e-6, wd.F16N: 2e-3}


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


@pytest.fixture(scope="module")
def bench_fields():
    cfg = wdgen.CONFIGS["lat14x4_16rhs"]
    dims = cfg["dims"]
    U = wdgen.gauge_field(dims, cfg["eps"], cfg["gauge_seed"])
    src = wdgen.mixed_sources(dims, cfg["n_point"], cfg["n_gauss"], cfg["src_seed"])
    return cfg, U, src


def kappa(m0):
    return (8.0 + m0) / m0


@pytest.mark.parametrize("prec", [wd.F64, wd.F32, wd.F16N], ids=["f64", "f32", "f16n"])
def test_bench_operator_16_fields(bench_fields, prec):
    cfg, U, src = bench_fields
    dims, m0 = cfg["dims"], cfg["m0"]
    g = wd.Gauge(dev(U), dims)
    for dag in (False, True):
        say("full-size operator 14^4 x 16", prec, "dagger", dag)
        got = host(wd.dslash(g, m0, dev(src), prec, dagger=dag))
        want = oracle.dirac(U, src, dims, m0, -1, dagger=dag)
        # every field on its own, so the point sources count as much as the Gaussian ones
        for i in range(src.shape[0]):
            err = rel(got[i], want[i])
            assert err <= OP_TOL[prec], (prec, dag, i, err)
        # and every site of every field against the oracle on the GPU-held inputs
        check_per_site(got, U, src, dims, m0, -1, dag, prec, f"14^4 x 16 prec {prec} dagger {dag}")


@pytest.mark.parametrize("recon12", [True, False], ids=["recon12", "complete-links"])
def test_bench_cg_workload(bench_fields, recon12):
    cfg, U, src = bench_fields
    dims, m0, tol = cfg["dims"], cfg["m0"], cfg["tol"]
    g = wd.Gauge(dev(U), dims, recon12=recon12)
    say("full-size mixed CG 14^4 x 16", "recon12" if recon12 else "complete links")
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(src), params=wd.cg_default_params(tol=tol, inner=wd.F32,
                                                                                  reliable_every=50))
    assert rc == wd.WD_OK, reps
    x = host(x)
    res = oracle.true_residual(U, src, x, dims, m0)
    assert np.all(res <= tol * 1.0000001), res
    for r, o in zip(reps, res):
        assert r["status"] == 0
        assert abs(r["true_rel_res"] - o) <= 1e-3 * tol + 1e-6 * o, (r["true_rel_res"], o)
    say("full-size FP64 CG 14^4 x 16")
    x64, reps64, rc64 = wd.cg_solve_batch(g, m0, dev(src), params=wd.cg_default_params(tol=tol, inner=wd.F64,
                                                                                       reliable_every=0))
    assert rc64 == wd.WD_OK, reps64
    x64 = host(x64)
    assert np.all(oracle.true_residual(U, src, x64, dims, m0) <= tol * 1.0000001)
    for i in range(src.shape[0]):
        assert rel(x[i], x64[i]) <= kappa(m0) * 2 * tol, i


_PER_PHASE = {}


def _shape_raw(g, prec, nrhs, dag, fam):
    r = wd.TuneResult()
    assert wd.lib().wd_shape_get(g.handle, prec, nrhs, dag, fam, ctypes.byref(r)) == 0
    return r


@pytest.mark.parametrize("inner,nr", [(wd.F32, 0), (wd.F32, 4), (wd.F64, 0), (wd.F64, 2)],
                         ids=["f32-default", "f32-4rhs", "f64-default", "f64-2rhs"])
def test_persistent_kernel_benchmark_workload(bench_fields, inner, nr):
    cfg, U, src = bench_fields
    dims, m0, tol = cfg["dims"], cfg["m0"], cfg["tol"]
    nrhs = src.shape[0]
    g = wd.Gauge(dev(U), dims, recon12=True)
    ru = 0 if inner == wd.F64 else 50
    if inner not in _PER_PHASE:
        say("per-phase reference 14^4 x 16", inner)
        x0, _, rc0 = wd.cg_solve_batch(g, m0, dev(src), params=wd.cg_default_params(
            tol=tol, inner=inner, reliable_every=ru, persistent=0))
        assert rc0 == wd.WD_OK
        _PER_PHASE[inner] = host(x0)
    keep = [(dag, fam, _shape_raw(g, inner, nrhs, dag, fam)) for dag, fam in ((1, wd.FAMILY_CG_A),
                                                                             (0, wd.FAMILY_CG_B))]
    try:
        if nr:
            for dag, fam, _ in keep:
                wd.shape_set(g, inner, nrhs, bool(dag), fam, 256, rhs_per_thread=nr, hop_order=1, strip=4)
        say("persistent 14^4 x 16", inner, "rhs per thread", nr or "default")
        x, reps, rc = wd.cg_solve_batch(g, m0, dev(src), params=wd.cg_default_params(
            tol=tol, inner=inner, reliable_every=ru, persistent=1))
    finally:
        for dag, fam, r in keep:
            assert wd.lib().wd_shape_set(g.handle, inner, nrhs, dag, fam, ctypes.byref(r)) == 0
    assert rc == wd.WD_OK, reps
    x = host(x)
    res = oracle.true_residual(U, src, x, dims, m0)
    assert np.all(res <= tol * 1.0000001), res
    for r, o in zip(reps, res):
        assert abs(r["true_rel_res"] - o) <= 1e-3 * tol + 1e-6 * o, (r["true_rel_res"], o)
    for i in range(nrhs):
        assert rel(x[i], _PER_PHASE[inner][i]) <= kappa(m0) * 2 * tol, i


def test_rhs_count_limits():
    dims, m0 = (8, 8, 4, 4), 0.1   # 64-site planes: the plane-blocked kernels run
    U = wdgen.gauge_field(dims, 0.5, 91)
    eta = wdgen.gaussian_source(dims, 64, 92)
    g = wd.Gauge(dev(U), dims)
    p = wd.cg_default_params(inner=wd.F32, reliable_every=50)
    say("cg 64 rhs")
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
    assert rc == wd.WD_OK, reps
    x = host(x)
    assert np.all(oracle.true_residual(U, eta, x, dims, m0) <= TOL * 1.0000001)
    for i in (0, 37, 63):
        xi, ri, rci = wd.cg_solve(g, m0, dev(eta[i]), params=p)
        assert rci == wd.WD_OK
        assert rel(host(xi), x[i]) <= kappa(m0) * 2 * TOL, i
    say("operator 64 rhs")
    got = host(wd.dslash(g, m0, dev(eta), wd.F64))
    assert rel(got, oracle.dirac(U, eta, dims, m0, -1)) <= OP_TOL[wd.F64]
    # one field more than a call takes
    eta65 = wdgen.gaussian_source(dims, 65, 93)
    say("65 rhs refused")
    _, _, rc = wd.cg_solve_batch(g, m0, dev(eta65), params=p, raise_on_error=False)
    assert rc == wd.WD_EINVAL
    with pytest.raises(wd.WDError) as e:
        wd.dslash(g, m0, dev(eta65), wd.F32)
    assert e.value.code == wd.WD_EINVAL
    assert wd.cg_workspace_bytes(g, 65, p) == 0
