"""Launch shapes of the stencil kernels against the FP64 oracle (Eq. (1)).

* The z-marching operator kernel: a block walks a column of xy-planes along z
  (even chunks upward, odd chunks downward), the z hop from the far side
  carried in registers.  Every tile order and chunk count, D and D^dagger,
  FP32 on complete and reconstruct-12 links and FP16N storage, on lattices
  that include extent 2 (forward and backward neighbours coincide), odd
  extents, one-plane chunks and planes that are not a multiple of 64 sites.
  Each site is checked on its own (sitecheck) with the oracle given the links
  and fields the GPU holds.
* Hop orders 1, 3 and 5 (5: the hops that read memory before the ones that
  read LDS) of the plane-blocked operator, every precision.
* CG with phases A and B in hop orders 1, 3 and 5: oracle true residual.
* Several z-adjacent xy-planes per block (xy_planes 2..4) for the operator
  (the z neighbours inside the block read from LDS) and for CG phases A and
  B, every precision (FP64, and shapes where k planes do not fit, fall back
  to one plane), against the oracle site by site and against one plane per
  block; shape_set refuses the combinations the kernels do not have.
"""
import numpy as np
import pytest

import oracle
import paper_2111_14958_amd as wd
import sitecheck
from gpu_util import dev, host, rel, say, field_set

pytestmark = pytest.mark.gpu

NAMES = {wd.F64: "f64", wd.F32: "f32", wd.F16N: "f16n"}
TOL = {wd.F64: 1e-13, wd.F32: 1e-6, wd.F16N: 2e-3}
SITE_BOUND = {wd.F64: sitecheck.F64_BOUND, wd.F32: sitecheck.F32_BOUND, wd.F16N: sitecheck.F16N_BOUND}


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _held(U, psi, prec):
    """links and field as the GPU holds them in `prec` (complete link copies)"""
    if prec == wd.F64:
        return U, psi
    if prec == wd.F32:
        return sitecheck.links_f32(U), oracle.round_f32(psi)
    c, n = oracle.fp16n_encode(psi.reshape(psi.shape[0], -1, 4, 3).astype(np.complex64))
    return sitecheck.links_f16(U), oracle.fp16n_decode(c, n).astype(np.complex128).reshape(psi.shape)


def _check(got, U, psi, dims, m0, dag, prec, what, cache):
    key = (prec, dag)
    if key not in cache:
        Uh, ph = _held(U, psi, prec)
        cache[key] = (ph, oracle.dirac(Uh, ph, dims, m0, -1, dagger=dag), oracle.dirac(U, psi, dims, m0, -1, dagger=dag))
    ph, want_held, want = cache[key]
    assert rel(got, want) <= TOL[prec], f"{what}: global rel err {rel(got, want):.3e}"
    sitecheck.assert_sites(got, want_held, ph, m0, SITE_BOUND[prec], what)


ZM_CASES = [
    ((2, 2, 2, 2), 2, 0.1),      # extent 2 everywhere: one-plane chunks, coinciding neighbours
    ((3, 5, 4, 6), 3, 0.05),     # odd extents, 15-site planes
    ((4, 4, 6, 6), 2, 0.1),      # 3-plane chunks with 2 chunks, one-plane-ish with 6
    ((14, 14, 14, 14), 16, 0.05),  # the benchmark volume: 196-site planes, 16 rhs
]


@pytest.mark.parametrize("dims,nrhs,m0", ZM_CASES, ids=[str(c[0]) for c in ZM_CASES])
def test_z_marching_operator_matches_oracle(dims, nrhs, m0):
    U, psi = field_set(dims, 0.5, 600 + sum(dims), nrhs, 700 + sum(dims))
    Lz = dims[2]
    chunk_counts = sorted({2, min(4, Lz - Lz % 2), Lz - Lz % 2})
    cache = {}
    for r12, prec in ((False, wd.F32), (True, wd.F32), (False, wd.F16N)):
        g = wd.Gauge(dev(U), dims, -1, recon12=r12)
        x = dev(psi)
        for gm in (0, 1):
            for nch in chunk_counts:
                for remap in (1, 0):
                    for dag in (False, True):
                        wd.shape_set(g, prec, nrhs, dag, wd.FAMILY_DSLASH, dims[0] * dims[1], xcd_remap=remap,
                                     hop_order=3, strip=nch, group_major=gm, xy_lds=2)
                    for dag in (False, True):
                        what = f"z-march {NAMES[prec]} r12={r12} order={gm} chunks={nch} remap={remap} dag={dag}"
                        say(what, dims, nrhs)
                        got = host(wd.dslash(g, m0, x, prec, dagger=dag))
                        _check(got, U, psi, dims, m0, dag, prec, what, cache)
        g.close()


def test_z_marching_equals_itself_across_orders_bitwise():
    """The tile order and XCD remapping only move work between blocks: each
    site's arithmetic is the same, so the output is bitwise the same."""
    dims, nrhs, m0 = (8, 8, 8, 8), 5, 0.05
    U, psi = field_set(dims, 0.5, 801, nrhs, 802)
    g = wd.Gauge(dev(U), dims, -1)
    x = dev(psi)
    outs = []
    for gm in (0, 1):
        for remap in (0, 1):
            wd.shape_set(g, wd.F32, nrhs, False, wd.FAMILY_DSLASH, 64, xcd_remap=remap, hop_order=3, strip=4,
                         group_major=gm, xy_lds=2)
            say("z-march order", gm, "remap", remap)
            outs.append(host(wd.dslash(g, m0, x, wd.F32)))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


HOP_CASES = [((3, 5, 4, 6), 3, 0.05), ((8, 8, 8, 8), 4, 0.05), ((14, 14, 14, 14), 16, 0.05)]


@pytest.mark.parametrize("dims,nrhs,m0", HOP_CASES, ids=[str(c[0]) for c in HOP_CASES])
def test_plane_operator_hop_orders_match_oracle(dims, nrhs, m0):
    U, psi = field_set(dims, 0.5, 900 + sum(dims), nrhs, 950 + sum(dims))
    cache = {}
    for prec in (wd.F64, wd.F32, wd.F16N):
        g = wd.Gauge(dev(U), dims, -1)
        x = dev(psi)
        for ho in (1, 3, 5):
            for dag in (False, True):
                wd.shape_set(g, prec, nrhs, dag, wd.FAMILY_DSLASH, dims[0] * dims[1], hop_order=ho, strip=2,
                             xy_lds=1)
            for dag in (False, True):
                what = f"plane operator {NAMES[prec]} hop order {ho} dag={dag}"
                say(what, dims, nrhs)
                got = host(wd.dslash(g, m0, x, prec, dagger=dag))
                _check(got, U, psi, dims, m0, dag, prec, what, cache)
        g.close()


@pytest.mark.parametrize("inner", [wd.F64, wd.F32], ids=["f64", "f32"])
def test_cg_phase_hop_orders(inner):
    """Phases A and B in hop orders 1, 3 and 5 (plane blocks, one rhs per
    thread) reach solutions whose true residual, recomputed by the oracle, is
    <= 1e-10, and agree with each other to the solver tolerance."""
    dims, m0 = (8, 8, 6, 6), 0.1
    U, eta = field_set(dims, 0.5, 1001, 4, 1002)
    g = wd.Gauge(dev(U), dims, -1, recon12=True)
    p = wd.cg_default_params(inner=inner, reliable_every=0 if inner == wd.F64 else 50)
    sols = []
    for ho in (1, 3, 5):
        for fam, dag in ((wd.FAMILY_CG_A, True), (wd.FAMILY_CG_B, False)):
            wd.shape_set(g, inner, 4, dag, fam, 256, 1, 1, ho, 1, 2, 0, 1)
            assert wd.shape_get(g, inner, 4, dag, fam)["hop_order"] == ho
        say("cg hop order", ho, NAMES[inner])
        x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
        assert rc == wd.WD_OK, reps
        res = oracle.true_residual(U, eta, host(x), dims, m0, -1)
        assert np.all(res <= 1e-10 * 1.0000001), res
        sols.append(host(x))
    kappa = (8.0 + m0) / m0
    for s in sols[1:]:
        assert rel(s, sols[0]) <= kappa * 2e-10


MP_CASES = [((3, 5, 4, 6), 3, 0.05),        # 15-site planes; Lz 4 takes 2 and 4 planes
            ((8, 8, 6, 6), 4, 0.05),        # 64-site planes; Lz 6 takes 2 and 3 planes
            ((14, 14, 14, 14), 16, 0.05)]   # the benchmark volume: 2 planes of 196 sites


@pytest.mark.parametrize("dims,nrhs,m0", MP_CASES, ids=[str(c[0]) for c in MP_CASES])
def test_multi_plane_operator_matches_oracle(dims, nrhs, m0):
    U, psi = field_set(dims, 0.5, 1100 + sum(dims), nrhs, 1150 + sum(dims))
    np_ = dims[0] * dims[1]
    ks = [k for k in (2, 3, 4) if k * np_ <= 512] + ([3] if 3 * np_ > 512 else [])   # 3 at 14^4: falls back
    # processing orders (strip, XCD remap, group-major); the benchmark volume takes the default one
    orders = ((0, 1, 0), (2, 1, 0), (4, 1, 0), (2, 0, 1)) if np_ * dims[2] * dims[3] <= 8 ** 4 else ((4, 1, 0),)
    cache = {}
    for r12, prec in ((False, wd.F64), (False, wd.F32), (True, wd.F32), (False, wd.F16N)):
        g = wd.Gauge(dev(U), dims, -1, recon12=r12)
        x = dev(psi)
        one = {}
        for dag in (False, True):   # one plane per block, the same strip and hop order
            wd.shape_set(g, prec, nrhs, dag, wd.FAMILY_DSLASH, np_, hop_order=5, strip=0, xy_lds=1)
            one[dag] = host(wd.dslash(g, m0, x, prec, dagger=dag))
        for k in ks:
            for strip, remap, gm in orders:
                for ho in (3, 5):
                    for dag in (False, True):
                        wd.shape_set(g, prec, nrhs, dag, wd.FAMILY_DSLASH, k * np_, xcd_remap=remap, hop_order=ho,
                                     strip=strip, group_major=gm, xy_lds=1, xy_planes=k)
                        assert wd.shape_get(g, prec, nrhs, dag, wd.FAMILY_DSLASH)["xy_planes"] == k
                    for dag in (False, True):
                        what = (f"{k} planes {NAMES[prec]} r12={r12} strip={strip} remap={remap} group-major={gm} "
                                f"hop order {ho} dag={dag}")
                        say(what, dims, nrhs)
                        got = host(wd.dslash(g, m0, x, prec, dagger=dag))
                        _check(got, U, psi, dims, m0, dag, prec, what, cache)
                        # the same sums per site as one plane per block, up to rounding
                        assert rel(got, one[dag]) <= {wd.F64: 1e-14, wd.F32: 2e-6, wd.F16N: 2e-3}[prec], what
        g.close()


def test_multi_plane_shapes_refused():
    dims = (8, 8, 6, 6)
    U, _ = field_set(dims, 0.5, 1201, 1, 1202)
    g = wd.Gauge(dev(U), dims, -1)
    bad = [dict(family=wd.FAMILY_DSLASH, block=128, hop_order=5, strip=0, xy_lds=0, xy_planes=2),   # site blocks
           dict(family=wd.FAMILY_DSLASH, block=128, rhs_per_thread=2, hop_order=3, xy_lds=1, xy_planes=2),
           dict(family=wd.FAMILY_DSLASH, block=128, hop_order=1, xy_lds=1, xy_planes=2),
           dict(family=wd.FAMILY_DSLASH, block=128, hop_order=3, xy_lds=2, xy_planes=2),   # z-marching
           dict(family=wd.FAMILY_DSLASH, block=320, hop_order=5, xy_lds=1, xy_planes=5),
           dict(family=wd.FAMILY_CG_R, block=128, hop_order=3, xy_lds=1, xy_planes=2),
           dict(family=wd.FAMILY_CG_B, block=128, hop_order=3, xy_lds=1, xy_planes=2),   # CG: hop order 5 only
           dict(family=wd.FAMILY_DSLASH, block=128, hop_order=0, xy_lds=1, xy_planes=2)]
    for kw in bad:
        fam = kw.pop("family")
        with pytest.raises(RuntimeError):
            wd.shape_set(g, wd.F32, 4, False, fam, **kw)
    g.close()


MP_CG_CASES = [((8, 8, 6, 6), 1301),     # 64-site planes: blocks of 64, 128 and 192 threads
               ((10, 10, 6, 4), 1401)]   # 100-site planes: 200 and 300 sites in blocks of 256 and 320
                                         # threads (the idle lanes of the last wave hold no site)


@pytest.mark.parametrize("inner", [wd.F64, wd.F32, wd.F16N], ids=["f64", "f32", "f16n"])
@pytest.mark.parametrize("dims,seed", MP_CG_CASES, ids=[str(c[0]) for c in MP_CG_CASES])
def test_cg_phase_multi_plane(inner, dims, seed):
    """Phases A and B with 1, 2 and 3 z-adjacent planes per block (hop order 5;
    FP64 falls back to one plane): oracle true residual <= 1e-10, and the
    solutions agree with each other to the solver tolerance."""
    m0 = 0.1
    U, eta = field_set(dims, 0.5, seed, 4, seed + 1)
    g = wd.Gauge(dev(U), dims, -1, recon12=True)
    p = wd.cg_default_params(inner=inner, reliable_every=0 if inner == wd.F64 else 50)
    sols = []
    for k in (1, 2, 3):
        for fam, dag in ((wd.FAMILY_CG_A, True), (wd.FAMILY_CG_B, False)):
            wd.shape_set(g, inner, 4, dag, fam, 256, 1, 1, 5, 1, 0, 0, 1, xy_planes=k)
            assert wd.shape_get(g, inner, 4, dag, fam)["xy_planes"] == k
        say("cg planes", k, NAMES[inner])
        x, reps, rc = wd.cg_solve_batch(g, m0, dev(eta), params=p)
        assert rc == wd.WD_OK, reps
        res = oracle.true_residual(U, eta, host(x), dims, m0, -1)
        assert np.all(res <= 1e-10 * 1.0000001), res
        sols.append(host(x))
    kappa = (8.0 + m0) / m0
    for s_ in sols[1:]:
        assert rel(s_, sols[0]) <= kappa * 2e-10
    g.close()
