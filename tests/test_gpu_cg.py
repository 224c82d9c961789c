"""GPU solver parity: wd_cg_solve / wd_cg_solve_batch against the FP64 oracle.

Every returned solution is checked by the oracle's own operator: its true
relative residual |eta - D x| / |eta| must be <= tol = 1e-10.  Against the
oracle's CG solution the error is bounded by kappa(D) (tol_gpu + tol_oracle)
with kappa(D) <= (8 + m0) / m0 (|D| <= 8 + m0, sigma_min(D) >= m0); the
measured error is asserted below that bound.
"""
import numpy as np
import pytest

import oracle
import paper_2111_14958_amd as wd
import pins
import wdgen
from gpu_util import dev, host, rel, say, field_set

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def kappa(m0):
    return (8.0 + m0) / m0


def _check_solution(U, eta, x, dims, m0, t_sign=-1):
    res = oracle.true_residual(U, eta, x, dims, m0, t_sign)
    assert np.all(res <= TOL * 1.0000001), f"true residuals {res}"
    return res


@pytest.mark.parametrize("inner", [wd.F64, wd.F32, wd.F16N], ids=["f64", "f32", "f16n"])
def test_lat4x4_1rhs(inner):
    cfg = wdgen.CONFIGS["lat4x4_1rhs"]
    dims, m0 = cfg["dims"], cfg["m0"]
    U = wdgen.gauge_field(dims, cfg["eps"], cfg["gauge_seed"])
    eta = wdgen.gaussian_source(dims, 1, cfg["src_seed"])
    say("cg c1", inner)
    g = wd.Gauge(dev(U), dims)
    p = wd.cg_default_params(inner=inner, reliable_every=0 if inner == wd.F64 else 50)
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
    x = host(x)
    assert rc == wd.WD_OK, reps
    assert reps[0]["status"] == 0 and reps[0]["true_rel_res"] <= TOL
    res = _check_solution(U, eta, x, dims, m0)
    # the library's own FP64 true residual agrees with the oracle's
    assert abs(reps[0]["true_rel_res"] - res[0]) <= 1e-3 * TOL + 1e-6 * res[0]
    xo, it, ro, st = oracle.cg(U, eta, dims, m0, tol=TOL)
    assert rel(x, xo) <= kappa(m0) * 2 * TOL
    # and against the dense LAPACK solution of the 4^4 system
    D = oracle.dense(U, dims, m0)
    xs = np.linalg.solve(D, eta.ravel())
    assert rel(x.ravel(), xs) <= kappa(m0) * TOL


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (12, 12, 12, 12), (14, 14, 14, 14)],
                         ids=["8^4", "12^4", "14^4"])
@pytest.mark.parametrize("inner", [wd.F64, wd.F32], ids=["f64", "f32"])
def test_single_rhs_volumes(dims, inner):
    m0, eps = 0.05, 0.5
    U = wdgen.gauge_field(dims, eps, 1002)
    eta = wdgen.gaussian_source(dims, 1, 2002)
    say("cg c2", dims, inner)
    g = wd.Gauge(dev(U), dims)
    p = wd.cg_default_params(inner=inner, reliable_every=0 if inner == wd.F64 else 50)
    x, reps, rc = wd.cg_solve(g, m0, dev(eta[0]), params=p)
    assert rc == wd.WD_OK, reps
    x = host(x)[None]
    _check_solution(U, eta, x, dims, m0)
    if dims == (8, 8, 8, 8):
        xo = oracle.cg(U, eta, dims, m0, tol=TOL)[0]
        assert rel(x, xo) <= kappa(m0) * 2 * TOL


def test_free_field_matches_fft_solution():
    dims, m0 = (8, 8, 8, 8), 0.05
    U = wdgen.unit_gauge(dims)
    eta = wdgen.gaussian_source(dims, 1, 5)
    say("cg free field")
    g = wd.Gauge(dev(U), dims)
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=wd.cg_default_params(inner=wd.F32))
    assert rc == wd.WD_OK
    gam = [oracle.gamma(mu) for mu in range(4)]
    xs = pins.free_solve_fft(eta[0], dims, m0, -1, gam)
    assert rel(host(x)[0], xs) <= kappa(m0) * TOL


def test_pure_gauge_matches_rotated_free_solution():
    dims, m0 = (4, 4, 4, 8), 0.1
    Om = wdgen.site_matrices(dims, 2.0, 61)
    U = wdgen.pure_gauge(Om)
    eta = wdgen.gaussian_source(dims, 1, 62)
    say("cg pure gauge")
    g = wd.Gauge(dev(U), dims)
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=wd.cg_default_params(inner=wd.F64))
    assert rc == wd.WD_OK
    gam = [oracle.gamma(mu) for mu in range(4)]
    xs = wdgen.apply_site_matrix(
        Om, pins.free_solve_fft(wdgen.apply_site_matrix(Om, eta[0], dagger=True), dims, m0, -1, gam))
    assert rel(host(x)[0], xs) <= kappa(m0) * TOL


@pytest.mark.parametrize("inner", [wd.F64, wd.F32, wd.F16N], ids=["f64", "f32", "f16n"])
def test_batch_mixed_sources_8x4(inner):
    """12 point sources + 4 Gaussian ones sharing one gauge field (smaller volume)."""
    dims, m0 = (8, 8, 8, 8), 0.05
    U = wdgen.gauge_field(dims, 0.5, 1003)
    eta = wdgen.mixed_sources(dims, 12, 4, 2003)
    say("cg batch 16 rhs", inner)
    g = wd.Gauge(dev(U), dims)
    p = wd.cg_default_params(inner=inner, reliable_every=0 if inner == wd.F64 else 50)
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
    assert rc == wd.WD_OK, reps
    assert all(r["status"] == 0 for r in reps)
    x = host(x)
    _check_solution(U, eta, x, dims, m0)
    # each field agrees with the oracle's CG solution of that field
    for i in (0, 7, 13):
        xo = oracle.cg(U, eta[i:i + 1], dims, m0, tol=TOL)[0]
        assert rel(x[i:i + 1], xo) <= kappa(m0) * 2 * TOL


def test_batch_equals_single_solves():
    dims, m0 = (6, 6, 6, 6), 0.1
    U = wdgen.gauge_field(dims, 0.5, 71)
    eta = wdgen.gaussian_source(dims, 3, 72)
    g = wd.Gauge(dev(U), dims)
    p = wd.cg_default_params(inner=wd.F32)
    say("batch vs single")
    xb, rb, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
    assert rc == wd.WD_OK
    xb = host(xb)
    for i in range(3):
        xi, ri, rc = wd.cg_solve(g, m0, dev(eta[i]), params=p)
        assert rc == wd.WD_OK
        # same kernels, same per-field arithmetic and reduction order
        assert rel(host(xi), xb[i]) <= kappa(m0) * 2 * TOL
        assert ri["iters"] == rb[i]["iters"]


def test_initial_guess_zero_source_and_max_iter():
    dims, m0 = (4, 4, 4, 4), 0.1
    U = wdgen.gauge_field(dims, 0.3, 1001)
    eta = wdgen.gaussian_source(dims, 2, 2001)
    eta[1] = 0.0
    g = wd.Gauge(dev(U), dims)
    say("cg edge cases")
    p = wd.cg_default_params(inner=wd.F64, reliable_every=0)
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
    assert rc == wd.WD_OK
    assert reps[1]["iters"] == 0 and reps[1]["true_rel_res"] == 0.0
    assert not np.any(host(x)[1])
    # warm start from the solution: done without an iteration
    p.use_x0 = 1
    x2, reps2, rc = wd.cg_solve_batch(g, m0, dev(eta), sol=x.clone(), params=p)
    assert rc == wd.WD_OK and reps2[0]["iters"] == 0 and reps2[0]["reliable_updates"] == 1
    # too few iterations
    p = wd.cg_default_params(inner=wd.F64, reliable_every=0, max_iter=5)
    x3, reps3, rc = wd.cg_solve_batch(g, m0, dev(eta[:1]), params=p, raise_on_error=False)
    assert rc == wd.WD_ENOTCONV and reps3[0]["status"] == wd.WD_ENOTCONV
    assert reps3[0]["iters"] == 5 and reps3[0]["true_rel_res"] > TOL


@pytest.mark.parametrize("inner", [wd.F64, wd.F32, wd.F16N], ids=["f64", "f32", "f16n"])
def test_first_residual_without_stencil_is_bitwise_the_same(inner):
    """Without an initial guess the first residual is r = eta, formed without
    the FP64 stencil; an explicit zero initial guess runs the stencil on x = 0.
    Both give bitwise the same solutions and reports."""
    dims, m0 = (8, 8, 6, 6), 0.1
    U, eta = field_set(dims, 0.5, 1501, 3, 1502)
    g = wd.Gauge(dev(U), dims, -1, recon12=True)
    p = wd.cg_default_params(inner=inner, reliable_every=0 if inner == wd.F64 else 50)
    say("first residual", inner)
    x0, r0, rc0 = wd.cg_solve_batch(g, m0, dev(eta), params=p)
    p.use_x0 = 1
    x1, r1, rc1 = wd.cg_solve_batch(g, m0, dev(eta), sol=torch_zeros_like(dev(eta)), params=p)
    assert rc0 == rc1 == wd.WD_OK
    assert np.array_equal(host(x0), host(x1))
    for a, b in zip(r0, r1):
        assert a["iters"] == b["iters"] and a["true_rel_res"] == b["true_rel_res"]


def torch_zeros_like(t):
    import torch
    return torch.zeros_like(t)


def test_nan_source_breaks_down():
    dims, m0 = (4, 4, 4, 4), 0.1
    U = wdgen.gauge_field(dims, 0.3, 1001)
    eta = wdgen.gaussian_source(dims, 2, 2001)
    eta[0, 0, 0, 0, 0, 0, 0] = np.nan
    g = wd.Gauge(dev(U), dims)
    say("cg nan source")
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=wd.cg_default_params(), raise_on_error=False)
    assert rc == wd.WD_EBREAKDOWN
    assert reps[0]["status"] == wd.WD_EBREAKDOWN and reps[1]["status"] == wd.WD_OK


def test_graph_cache_keys_on_the_hop_order():
    """A solve whose phase kernels differ only in the hop order captures a graph
    of its own on the same workspace (the old order's graph is not replayed),
    and going back replays the cached one."""
    import torch
    dims, m0, nrhs = (8, 8, 8, 8), 0.05, 2
    U = wdgen.gauge_field(dims, 0.5, 1021)
    eta = wdgen.gaussian_source(dims, nrhs, 2021)
    g = wd.Gauge(dev(U), dims)
    p = wd.cg_default_params(inner=wd.F32, reliable_every=50)
    ws = torch.empty(wd.cg_workspace_bytes(g, nrhs, p), dtype=torch.uint8, device="cuda")
    base = {fam: wd.shape_get(g, wd.F32, nrhs, fam == wd.FAMILY_CG_A, fam)
            for fam in (wd.FAMILY_CG_A, wd.FAMILY_CG_B)}
    sols = {}
    try:
        for order in (3, 1, 3):
            for fam, sh in base.items():
                wd.shape_set(g, wd.F32, nrhs, fam == wd.FAMILY_CG_A, fam, sh["block"],
                             rhs_per_thread=sh["rhs_per_thread"], xcd_remap=sh["xcd_remap"], hop_order=order,
                             strip=sh["strip"], xy_lds=sh["xy_lds"])
            say("graph key hop order", order)
            before = wd.cg_graph_stats()[0]
            x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p, ws=ws)
            assert rc == wd.WD_OK
            built = wd.cg_graph_stats()[0] - before
            sols.setdefault(order, []).append((host(x), built))
    finally:
        for fam, sh in base.items():
            wd.shape_set(g, wd.F32, nrhs, fam == wd.FAMILY_CG_A, fam, sh["block"],
                         rhs_per_thread=sh["rhs_per_thread"], xcd_remap=sh["xcd_remap"],
                         hop_order=sh["hop_order"], strip=sh["strip"], xy_lds=sh["xy_lds"])
    # the new hop order captured its own graphs (one per chunk length the solve used)
    assert sols[1][0][1] == sols[3][0][1] >= 1
    assert sols[3][1][1] == 0                 # back to order 3: the cached graphs are replayed
    assert np.array_equal(sols[3][0][0], sols[3][1][0])
    _check_solution(U, eta, sols[1][0][0], dims, m0)


@pytest.mark.parametrize("inner", [wd.F64, wd.F32], ids=["f64", "f32"])
def test_adaptive_chunk_lengths_are_bitwise_neutral(inner):
    """With the library's chunk length (chunk = 0) the last replays are cut to
    the iterations the fields are estimated to need; the solutions and reports
    are bitwise those of fixed chunks of 50 and of 7 iterations, and the solve
    captured a shorter graph than 50."""
    import torch
    dims, m0, nrhs = (8, 8, 8, 8), 0.05, 4
    U, eta = field_set(dims, 0.5, 1601, nrhs, 1602)
    g = wd.Gauge(dev(U), dims, -1, recon12=True)
    ru = 0 if inner == wd.F64 else 50
    out = {}
    for chunk in (0, 50, 7):
        p = wd.cg_default_params(inner=inner, reliable_every=ru, chunk=chunk)
        ws = torch.empty(wd.cg_workspace_bytes(g, nrhs, p), dtype=torch.uint8, device="cuda")
        say("chunk length", chunk, inner)
        before = wd.cg_graph_stats()[0]
        x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p, ws=ws)
        assert rc == wd.WD_OK, reps
        out[chunk] = (host(x), [(r["iters"], r["true_rel_res"], r["reliable_updates"]) for r in reps],
                      wd.cg_graph_stats()[0] - before)
    assert max(r[0] for r in out[0][1]) > 50          # more than one chunk
    assert out[0][2] >= 2                              # a length of 50 and a shorter one
    for chunk in (50, 7):
        assert np.array_equal(out[0][0], out[chunk][0]), chunk
        assert out[0][1] == out[chunk][1], chunk
    _check_solution(U, eta, out[0][0], dims, m0)


def test_workspace_too_small():
    dims = (4, 4, 4, 4)
    U = wdgen.gauge_field(dims, 0.3, 1001)
    eta = wdgen.gaussian_source(dims, 1, 2001)
    g = wd.Gauge(dev(U), dims)
    import torch
    say("cg small workspace")
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    sol = torch.zeros_like(dev(eta))
    rep = (wd.CGReport * 1)()
    p = wd.cg_default_params()
    import ctypes
    rc = wd.lib().wd_cg_solve_batch(g.handle, 0.1, ctypes.c_void_p(dev(eta).data_ptr()),
                                    ctypes.c_void_p(sol.data_ptr()), 1, ctypes.byref(p),
                                    ctypes.c_void_p(ws.data_ptr()), 1024, rep, None)
    assert rc == wd.WD_ENOMEM


@pytest.mark.parametrize("inner", [wd.F64, wd.F32, wd.F16N], ids=["f64", "f32", "f16n"])
def test_persistent_kernel_matches_oracle(inner):
    """One persistent launch per chunk (grid barriers) gives a converged solution
    that the oracle accepts, agreeing with the kernel-per-phase path."""
    dims, m0 = (8, 8, 8, 8), 0.05
    U = wdgen.gauge_field(dims, 0.5, 1003)
    eta = wdgen.mixed_sources(dims, 3, 2, 2003)
    say("cg persistent", inner)
    g = wd.Gauge(dev(U), dims)
    ru = 0 if inner == wd.F64 else 50
    p = wd.cg_default_params(inner=inner, reliable_every=ru, persistent=1)
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
    assert rc == wd.WD_OK, reps
    x = host(x)
    _check_solution(U, eta, x, dims, m0)
    p0 = wd.cg_default_params(inner=inner, reliable_every=ru, persistent=0)
    x0, reps0, rc0 = wd.cg_solve_batch(g, m0, dev(eta), params=p0)
    assert rc0 == wd.WD_OK
    assert rel(x, host(x0)) <= kappa(m0) * 2 * TOL


@pytest.mark.parametrize("inner", [wd.F32, wd.F16N], ids=["f32", "f16n"])
def test_compute_unit_limited_persistent_kernel(inner):
    """The persistent kernel confined to n compute units (one 1024-thread block
    each) gives the same bits for every n, including grids that are not whole
    XCD rounds and n above the device's compute units, and so does the default
    persistent launch (that kernel on every compute unit); the oracle accepts
    the solution and it agrees with the kernel-per-phase path."""
    dims, m0 = (8, 8, 8, 12), 0.05   # 6144 sites: 6 site blocks of 1024 per rhs
    U = wdgen.gauge_field(dims, 0.5, 1013)
    eta = wdgen.mixed_sources(dims, 2, 1, 2013)
    g = wd.Gauge(dev(U), dims)
    sols = {}
    for n in (1, 3, 8, 40, 100000):
        say("cg compute-unit-limited", inner, n)
        p = wd.cg_default_params(inner=inner, reliable_every=50, persistent=1, max_cus=n)
        x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
        assert rc == wd.WD_OK, reps
        sols[n] = host(x)
        assert np.array_equal(sols[n], sols[1]), n
    # without max_cus the persistent kernel takes the same launch on every compute unit
    say("cg persistent default launch", inner)
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=wd.cg_default_params(
        inner=inner, reliable_every=50, persistent=1))
    assert rc == wd.WD_OK, reps
    assert np.array_equal(host(x), sols[1])
    _check_solution(U, eta, sols[1], dims, m0)
    x0, _, rc0 = wd.cg_solve_batch(g, m0, dev(eta), params=wd.cg_default_params(inner=inner, reliable_every=50))
    assert rc0 == wd.WD_OK
    assert rel(sols[1], host(x0)) <= kappa(m0) * 2 * TOL
    # max_cus needs the persistent kernel, a lower-precision inner iteration, n >= 0
    for kw in ({"max_cus": 4}, {"max_cus": 4, "persistent": 1, "inner": wd.F64},
               {"max_cus": -1, "persistent": 1}, {"max_cus": 4, "persistent": 1, "method": wd.METHOD_BICGSTAB}):
        _, _, rc = wd.cg_solve_batch(g, m0, dev(eta), params=wd.cg_default_params(**kw), raise_on_error=False)
        assert rc == wd.WD_EINVAL, kw


@pytest.mark.parametrize("inner", [wd.F64, wd.F32, wd.F16N], ids=["f64", "f32", "f16n"])
@pytest.mark.parametrize("dims", [(8, 8, 4, 6), (14, 14, 6, 4), (4, 8, 4, 6)],
                         ids=["8x8x4x6", "14x14x6x4", "4x8x4x6"])
def test_plane_blocked_phase_kernels(inner, dims):
    """Phases A and B with one xy-plane per block (x/y neighbours from LDS) and
    the site-blocked kernels reach the oracle-checked solution; the per-site
    arithmetic is the same, so the solutions agree to the solver tolerance.
    A plane of fewer than 64 sites (4x8) falls back to site blocks (the
    partial-sum buffer holds one entry per 64 sites)."""
    m0 = 0.1
    U = wdgen.gauge_field(dims, 0.5, 401)
    eta = wdgen.mixed_sources(dims, 3, 2, 402)
    nrhs = eta.shape[0]
    say("cg plane-blocked phases", dims, inner)
    g = wd.Gauge(dev(U), dims)
    p = wd.cg_default_params(inner=inner, reliable_every=0 if inner == wd.F64 else 50)
    sols = {}
    for xy in (0, 1, 2):
        for fam, dag in ((wd.FAMILY_CG_A, True), (wd.FAMILY_CG_B, False)):
            wd.shape_set(g, inner, nrhs, dag, fam, 256, 2, 1, 3, 1, 4, 0, xy)
            got = wd.shape_get(g, inner, nrhs, dag, fam)
            assert got["xy_lds"] == xy and got["strip"] == 4
        x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
        assert rc == wd.WD_OK, reps
        sols[xy] = host(x)
    _check_solution(U, eta, sols[1], dims, m0)
    _check_solution(U, eta, sols[2], dims, m0)
    assert rel(sols[1], sols[0]) <= kappa(m0) * 2 * TOL
    assert rel(sols[2], sols[0]) <= kappa(m0) * 2 * TOL


@pytest.mark.parametrize("inner", [wd.F32, wd.F16N], ids=["f32", "f16n"])
@pytest.mark.parametrize("block", [64, 256])
def test_four_rhs_per_thread_phase_kernels(inner, block):
    """Site-blocked phases A and B with four right-hand sides per thread (the
    most the FP32/FP16 kernels take), over 6 fields: one full group of four and
    a ragged one of two.  Phase B completes phase A's reduction for all four
    fields of its tile (waves 0..3 of a 256-thread block, or one wave for all
    four in a 64-thread block)."""
    dims, m0 = (8, 8, 4, 6), 0.1
    U = wdgen.gauge_field(dims, 0.5, 421)
    eta = wdgen.mixed_sources(dims, 4, 2, 422)
    nrhs = eta.shape[0]
    g = wd.Gauge(dev(U), dims)
    p = wd.cg_default_params(inner=inner, reliable_every=50)
    say("cg 4 rhs per thread", inner, block)
    x0, _, rc0 = wd.cg_solve_batch(g, m0, dev(eta), params=p)
    assert rc0 == wd.WD_OK
    for fam, dag in ((wd.FAMILY_CG_A, True), (wd.FAMILY_CG_B, False)):
        wd.shape_set(g, inner, nrhs, dag, fam, block, 4, 1, 3, 1, 4, 0, 0)
        assert wd.shape_get(g, inner, nrhs, dag, fam)["rhs_per_thread"] == 4
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
    assert rc == wd.WD_OK, reps
    x = host(x)
    _check_solution(U, eta, x, dims, m0)
    assert rel(x, host(x0)) <= kappa(m0) * 2 * TOL


@pytest.mark.parametrize("inner", [wd.F64, wd.F32], ids=["f64", "f32"])
@pytest.mark.parametrize("xy,block", [(1, 256), (0, 64)], ids=["planes", "sites"])
def test_rhs_pass_tile_order_is_bitwise_neutral(inner, xy, block):
    """Walking each eighth of the site blocks in passes of a few rhs groups
    (rhs_pass) only reorders the tiles: every tile forms the same partial sums,
    which the finish adds in site-block order, so the solution is bitwise the
    one of the default order.  30 site blocks (30 planes, or 30 blocks of 64
    sites) make chunks of 4 with a short last one; 5 fields in passes of 2 or 3
    leave a short last pass."""
    dims, m0 = (8, 8, 5, 6), 0.1
    U = wdgen.gauge_field(dims, 0.5, 411)
    eta = wdgen.mixed_sources(dims, 3, 2, 412)
    nrhs = eta.shape[0]
    g = wd.Gauge(dev(U), dims)
    p = wd.cg_default_params(inner=inner, reliable_every=0 if inner == wd.F64 else 50)
    sols = {}
    for fp in (0, 1, 2, 3):
        say("cg rhs passes", inner, "xy", xy, "pass", fp)
        for fam, dag in ((wd.FAMILY_CG_A, True), (wd.FAMILY_CG_B, False)):
            wd.shape_set(g, inner, nrhs, dag, fam, block, 1, 1, 3, 1, 0, 0, xy, 0, fp)
            assert wd.shape_get(g, inner, nrhs, dag, fam)["rhs_pass"] == fp
        x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
        assert rc == wd.WD_OK, reps
        sols[fp] = host(x)
    _check_solution(U, eta, sols[0], dims, m0)
    for fp in (1, 2, 3):
        assert np.array_equal(sols[fp], sols[0]), fp
    # passes are a CG phase A/B order only
    with pytest.raises(wd.WDError) as e:
        wd.shape_set(g, inner, nrhs, False, wd.FAMILY_DSLASH, 256, 1, 1, 1, 1, 0, 0, 0, 0, 2)
    assert e.value.code == wd.WD_EINVAL


@pytest.mark.parametrize("inner", [wd.F32, wd.F16N], ids=["f32", "f16n"])
@pytest.mark.parametrize("dims,chunks", [((8, 8, 6, 6), (1, 2, 3, 6, 0)), ((16, 8, 5, 4), (1, 2, 5, 0)),
                                         ((8, 16, 2, 6), (1, 2)), ((14, 14, 14, 4), (4, 7))],
                         ids=["8x8x6x6", "16x8x5x4", "8x16x2x6", "14x14x14x4"])
def test_z_marching_phase_kernels(inner, dims, chunks):
    """Phases A and B walking columns of xy-planes along z (two planes in LDS,
    the backward z hop carried from the previous plane): for every z-chunk
    count, from whole columns to one plane per chunk (0 = automatic), and for
    odd Lz and Lz = 2, the solution passes the oracle and agrees with the
    site-blocked kernels to the solver tolerance."""
    m0 = 0.1
    U = wdgen.gauge_field(dims, 0.5, 411)
    eta = wdgen.mixed_sources(dims, 2, 2, 412)
    nrhs = eta.shape[0]
    g = wd.Gauge(dev(U), dims)
    p = wd.cg_default_params(inner=inner, reliable_every=50)
    for fam, dag in ((wd.FAMILY_CG_A, True), (wd.FAMILY_CG_B, False)):
        wd.shape_set(g, inner, nrhs, dag, fam, 256, 1, 1, 3, 1, 0, 0, 0)
    say("cg site-blocked reference", dims, inner)
    x0, reps0, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
    assert rc == wd.WD_OK, reps0
    x0 = host(x0)
    for nzc in chunks:
        for fam, dag in ((wd.FAMILY_CG_A, True), (wd.FAMILY_CG_B, False)):
            wd.shape_set(g, inner, nrhs, dag, fam, 256, 1, 1, 3, 1, nzc, 0, 2)
            assert wd.shape_get(g, inner, nrhs, dag, fam)["xy_lds"] == 2
        say("cg z-marching", dims, inner, "chunks", nzc)
        x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
        assert rc == wd.WD_OK, reps
        x = host(x)
        _check_solution(U, eta, x, dims, m0)
        assert rel(x, x0) <= kappa(m0) * 2 * TOL, nzc


@pytest.mark.parametrize("inner", [wd.F32, wd.F64], ids=["f32", "f64"])
def test_cg_autotuner(inner):
    """wd_tune_cg times the CG phase shapes on a short run, stores the fastest
    for phases A and B, and the solve with it still passes the oracle."""
    dims, m0 = (8, 8, 6, 6), 0.1   # 64-site planes: plane and site blocks compete
    U = wdgen.gauge_field(dims, 0.5, 421)
    eta = wdgen.mixed_sources(dims, 2, 2, 422)
    g = wd.Gauge(dev(U), dims)
    say("cg autotune", inner)
    best = wd.tune_cg(g, m0, inner, dev(eta), iters=20)
    assert best["block"] == 256 and best["rhs_per_thread"] in (1, 2) and best["hop_order"] in (1, 3, 5)
    assert best["strip"] in (0, 2, 4) and best["us"] > 0
    for fam, dag in ((wd.FAMILY_CG_A, True), (wd.FAMILY_CG_B, False)):
        got = wd.shape_get(g, inner, eta.shape[0], dag, fam)
        assert (got["rhs_per_thread"], got["hop_order"], got["strip"], got["xy_lds"]) == \
            (best["rhs_per_thread"], best["hop_order"], best["strip"], best["xy_lds"])
    p = wd.cg_default_params(inner=inner, reliable_every=0 if inner == wd.F64 else 50)
    x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
    assert rc == wd.WD_OK, reps
    _check_solution(U, eta, host(x), dims, m0)
    with pytest.raises(wd.WDError) as e:
        wd.tune_cg(g, m0, inner, dev(eta), iters=0)
    assert e.value.code == wd.WD_EINVAL
