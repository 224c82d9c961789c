"""GPU operator parity: wd_dslash / wd_dslash_dag against the FP64 CPU oracle.

Two checks per case:
* global |GPU - oracle| / |oracle| against the unrounded FP64 inputs: FP64 1e-13,
  FP32 1e-6, FP16N 2e-3 (half storage carries 11 significant bits, unit roundoff
  4.9e-4; the bound allows a few roundings of the inputs and the output);
* every site on its own (sitecheck), with the oracle fed the links and fields the
  GPU holds (FP32- or FP16-rounded), so a single wrong component anywhere fails.
Packing is checked bit for bit.
"""
import numpy as np
import pytest

import oracle
import paper_2111_14958_amd as wd
import wdgen
from gpu_util import dev, host, rel, say, field_set
import sitecheck

pytestmark = pytest.mark.gpu

TOL = {wd.F64: 1e-13, wd.F32: 1e-6, wd.F16N: 2e-3}
NAMES = {wd.F64: "f64", wd.F32: "f32", wd.F16N: "f16n"}
SITE_BOUND = {wd.F64: sitecheck.F64_BOUND, wd.F32: sitecheck.F32_BOUND, wd.F16N: sitecheck.F16N_BOUND}


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    arch, ncu = wd.device_info(0)
    assert arch.startswith("gfx950")


def _oracle_input(psi, prec):
    """The field the GPU actually receives after rounding to `prec` storage."""
    if prec == wd.F64:
        return psi
    if prec == wd.F32:
        return oracle.round_f32(psi)
    c, n = oracle.fp16n_encode(psi.reshape(psi.shape[0], -1, 4, 3).astype(np.complex64))
    return oracle.fp16n_decode(c, n).astype(np.complex128).reshape(psi.shape)


def _oracle_links(U, prec):
    """The links the GPU reads in `prec` (the complete copy of a gauge made without
    reconstruct-12)."""
    return {wd.F64: lambda u: u, wd.F32: sitecheck.links_f32, wd.F16N: sitecheck.links_f16}[prec](U)


def check_per_site(got, U, psi, dims, m0, t_sign, dag, prec, what):
    """every site of got against the oracle on the GPU-held inputs"""
    pin = _oracle_input(psi, prec)
    want = oracle.dirac(_oracle_links(U, prec), pin, dims, m0, t_sign, dagger=dag)
    return sitecheck.assert_sites(got, want, pin, m0, SITE_BOUND[prec], what)


CASES = [
    ((2, 2, 2, 2), 0.1, 0.5, 1),       # extent 2: forward and backward neighbours coincide
    ((4, 4, 4, 4), 0.1, 0.3, 1),
    ((3, 5, 4, 6), 0.05, 0.7, 3),      # 360 sites: ragged last block, odd extents
    ((8, 8, 8, 8), 0.05, 0.5, 2),
    ((14, 14, 14, 14), 0.05, 0.5, 1),  # full benchmark volume
    ((16, 16, 16, 32), 0.02, 0.5, 1),
]


@pytest.mark.parametrize("prec", [wd.F64, wd.F32, wd.F16N], ids=["f64", "f32", "f16n"])
@pytest.mark.parametrize("dims,m0,eps,nrhs", CASES, ids=[str(c[0]) for c in CASES])
def test_dslash_matches_oracle(dims, m0, eps, nrhs, prec):
    U, psi = field_set(dims, eps, 100 + sum(dims), nrhs, 200 + sum(dims))
    for t_sign in (-1, +1) if dims == (3, 5, 4, 6) else (-1,):
        say("dslash", dims, NAMES[prec], nrhs, t_sign)
        g = wd.Gauge(dev(U), dims, t_sign)
        for dag in (False, True):
            got = host(wd.dslash(g, m0, dev(psi), prec, dagger=dag))
            want = oracle.dirac(U, psi, dims, m0, t_sign, dagger=dag)
            err = rel(got, want)
            assert err <= TOL[prec], f"{NAMES[prec]} dag={dag} t_sign={t_sign}: rel err {err:.3e}"
            check_per_site(got, U, psi, dims, m0, t_sign, dag, prec, f"{NAMES[prec]} dag={dag} t_sign={t_sign}")
        g.close()


def test_dslash_fp32_against_rounded_inputs_is_tighter():
    """With the FP32-rounded links and field as oracle input the only error left is
    FP32 arithmetic: a few ulps relative to the hopping sum."""
    dims, m0 = (8, 8, 8, 8), 0.05
    U, psi = field_set(dims, 0.5, 7, 1, 8)
    say("dslash f32 rounded inputs", dims)
    g = wd.Gauge(dev(U), dims)
    got = host(wd.dslash(g, m0, dev(psi), wd.F32))
    want = oracle.dirac(oracle.round_f32(U), oracle.round_f32(psi), dims, m0)
    assert rel(got, want) <= 3e-7


def test_multi_rhs_equals_single_rhs_bitwise():
    dims, m0 = (6, 6, 6, 8), 0.1
    U, psi = field_set(dims, 0.5, 11, 7, 12)
    g = wd.Gauge(dev(U), dims)
    for prec in (wd.F64, wd.F32, wd.F16N):
        say("multi-rhs", NAMES[prec])
        many = host(wd.dslash(g, m0, dev(psi), prec))
        for i in range(7):
            one = host(wd.dslash(g, m0, dev(psi[i:i + 1]), prec))
            assert np.array_equal(one[0], many[i])


def test_pack_unpack_bit_exact():
    import torch
    dims = (4, 6, 4, 5)
    V = wdgen.volume(dims)
    U, psi = field_set(dims, 0.5, 3, 3, 4)
    psi[1, 0, 0, 0, 0] = 0.0          # an all-zero site
    # a site of norm 3 whose values v give a product v * float32(1/3) that
    # rounds to a different half directly than through FP32 (the encoding
    # rounds to FP32 first, then to half)
    rng = np.random.default_rng(41)
    inv3 = np.float32(1) / np.float32(3)
    cand = rng.uniform(-3, 3, 2_000_000).astype(np.float32)
    direct = (cand.astype(np.float64) * np.float64(inv3)).astype(np.float16)
    twice = (cand * inv3).astype(np.float32).astype(np.float16)
    tricky = cand[direct.view(np.uint16) != twice.view(np.uint16)][:23]
    assert len(tricky) == 23
    site = np.concatenate([[np.float32(3)], tricky]).astype(np.float64)
    psi[2, 1, 0, 0, 0] = (site[0::2] + 1j * site[1::2]).reshape(4, 3)
    # a site whose norm is an FP32 subnormal with an overflowing reciprocal
    # (codes from the quotient), and one just above that range
    psi[2, 2, 0, 0, 0] = 0.0
    psi[2, 2, 0, 0, 0, 0, 0] = -2.0 ** -140 + 1j * 3 * 2.0 ** -143
    psi[2, 2, 0, 0, 0, 1, 2] = 2.0 ** -141 - 1j * 2.0 ** -145
    psi[2, 3, 0, 0, 0] = psi[2, 1, 0, 0, 0] * 2.0 ** -128
    g = wd.Gauge(dev(U), dims)
    say("pack f64/f32/f16n")
    # FP64: exact round trip
    b = wd.pack_spinor(g, dev(psi), wd.F64)
    assert np.array_equal(host(wd.unpack_spinor(g, b, wd.F64, 3)), psi)
    # FP64 packed layout: double2 [rhs][12][V]
    raw = host(b).view(np.complex128).reshape(3, 12, V)
    assert np.array_equal(raw, psi.reshape(3, V, 12).transpose(0, 2, 1))
    # FP32: round to nearest even
    b = wd.pack_spinor(g, dev(psi), wd.F32)
    assert np.array_equal(host(wd.unpack_spinor(g, b, wd.F32, 3)), oracle.round_f32(psi))
    raw = host(b).view(np.complex64).reshape(3, 6, V, 2)
    want = psi.astype(np.complex64).reshape(3, V, 6, 2).transpose(0, 2, 1, 3)
    assert np.array_equal(raw, want)
    # FP16N: codes and norms identical to the oracle's encoding, bit for bit
    b = host(wd.pack_spinor(g, dev(psi), wd.F16N))
    codes = b[: 3 * V * 48].view(np.float16).reshape(3, 3, V, 8).transpose(0, 2, 1, 3).reshape(3, V, 24)
    norms = b[3 * V * 48:].view(np.float32).reshape(3, V)
    oc, on = oracle.fp16n_encode(psi.reshape(3, V, 4, 3).astype(np.complex64))
    assert np.array_equal(norms, on)
    assert np.array_equal(codes.view(np.uint16), oc.view(np.uint16))
    dec = host(wd.unpack_spinor(g, torch.from_numpy(b).cuda(), wd.F16N, 3))
    assert np.array_equal(dec.reshape(3, V, 4, 3),
                          oracle.fp16n_decode(oc, on).astype(np.complex128))


def test_adjoint_identity_on_gpu():
    dims, m0 = (8, 8, 8, 8), 0.05
    U, psi = field_set(dims, 0.5, 21, 2, 22)
    g = wd.Gauge(dev(U), dims)
    say("adjoint identity")
    x, y = psi[0:1], psi[1:2]
    Dx = host(wd.dslash(g, m0, dev(x), wd.F64))
    Ddy = host(wd.dslash(g, m0, dev(y), wd.F64, dagger=True))
    lhs, rhs = np.vdot(x, Ddy), np.vdot(Dx, y)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(x) * np.linalg.norm(y) * 10
    g5 = np.array([1, 1, -1, -1])[:, None]
    g5Dg5y = g5 * host(wd.dslash(g, m0, dev(g5 * y), wd.F64))
    assert rel(Ddy, g5Dg5y) <= 1e-15


def test_gauge_covariance_on_gpu():
    dims, m0 = (4, 4, 6, 8), 0.1
    U, psi = field_set(dims, 0.7, 31, 1, 32)
    Om = wdgen.site_matrices(dims, 2.0, 33)
    say("gauge covariance")
    g = wd.Gauge(dev(U), dims)
    gt = wd.Gauge(dev(wdgen.transform_gauge(U, Om)), dims)
    lhs = host(wd.dslash(gt, m0, dev(wdgen.apply_site_matrix(Om, psi)), wd.F64))
    rhs = wdgen.apply_site_matrix(Om, host(wd.dslash(g, m0, dev(psi), wd.F64)))
    assert rel(lhs, rhs) <= 1e-14


def test_packed_mode_matches_canonical():
    dims, m0 = (8, 8, 8, 8), 0.05
    U, psi = field_set(dims, 0.5, 41, 4, 42)
    g = wd.Gauge(dev(U), dims)
    for prec in (wd.F64, wd.F32, wd.F16N):
        say("packed mode", NAMES[prec])
        canon = host(wd.dslash(g, m0, dev(psi), prec))
        pin = wd.pack_spinor(g, dev(psi), prec)
        pout = wd.dslash(g, m0, pin, prec, packed=True, nrhs=4)
        assert np.array_equal(host(wd.unpack_spinor(g, pout, prec, 4)), canon)


def test_autotuner_keeps_results_to_rounding():
    dims, m0 = (8, 8, 8, 12), 0.05
    U, psi = field_set(dims, 0.5, 51, 5, 52)
    g = wd.Gauge(dev(U), dims)
    for prec in (wd.F32, wd.F64):
        say("autotune", NAMES[prec])
        before = host(wd.dslash(g, m0, dev(psi), prec))
        best = wd.tune_dslash(g, prec, 5)
        assert best["block"] in (64, 128, 256) and best["rhs_per_thread"] in (1, 2, 4)
        assert best["us"] > 0 and best["gbps"] > 0
        assert wd.tune_lookup(g, prec, 5) == {**best, "us": 0.0, "gbps": 0.0}
        after = host(wd.dslash(g, m0, dev(psi), prec))
        # the tuned shape may sum the hops in another order than the default
        # (hop order 5 takes the memory hops first): equal to rounding, and
        # deterministic once chosen
        assert rel(after, before) <= TOL[prec]
        assert np.array_equal(after, host(wd.dslash(g, m0, dev(psi), prec)))


def test_dslash_argument_errors():
    dims = (4, 4, 4, 4)
    U, psi = field_set(dims, 0.3, 1, 1, 2)
    g = wd.Gauge(dev(U), dims, precs=(wd.F64,))
    say("dslash errors")
    with pytest.raises(wd.WDError) as e:
        wd.dslash(g, 0.1, dev(psi), wd.F32)     # no FP32 links in this handle
    assert e.value.code == wd.WD_EINVAL
