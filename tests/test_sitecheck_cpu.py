"""The per-site comparator of the operator parity tests (tests/sitecheck.py), on
the CPU: it accepts outputs that differ from the oracle only by the storage
rounding of their precision, and rejects a single wrong component that a
global relative norm lets through."""
import numpy as np

import oracle
import sitecheck
import wdgen


def _fields(dims=(4, 4, 4, 6), nrhs=3, m0=0.05):
    U = wdgen.gauge_field(dims, 0.5, 77)
    psi = wdgen.gaussian_source(dims, nrhs, 78)
    want = oracle.dirac(U, psi, dims, m0, -1)
    return U, psi, want, m0


def _fp16n_store(v):
    c, n = oracle.fp16n_encode(v.reshape(v.shape[0], -1, 4, 3).astype(np.complex64))
    return oracle.fp16n_decode(c, n).astype(np.complex128).reshape(v.shape)


def test_rounded_outputs_pass():
    U, psi, want, m0 = _fields()
    assert sitecheck.assert_sites(_fp16n_store(want), want, psi, m0, sitecheck.F16N_BOUND) <= 0.5
    assert sitecheck.assert_sites(oracle.round_f32(want), want, psi, m0, sitecheck.F32_BOUND) <= 0.1
    assert sitecheck.assert_sites(want.copy(), want, psi, m0, sitecheck.F64_BOUND) == 0.0


def _perturb_one(got, want, psi, m0, bound, factor):
    """got with one component moved by `factor` times that site's bound"""
    q, a = bound
    idx = (1, 2, 3, 1, 0, 2, 1)   # rhs, t, z, y, x, spin, colour
    site = idx[:5]
    lim = q * sitecheck._site_max(want)[site] + a * sitecheck.term_scale(psi, m0)[site]
    bad = got.copy()
    bad[idx] += factor * lim
    return bad


def test_single_wrong_component_fails_per_site_but_not_globally():
    U, psi, want, m0 = _fields()
    for bound, store, gtol in ((sitecheck.F16N_BOUND, _fp16n_store, 2e-3),
                               (sitecheck.F32_BOUND, oracle.round_f32, 1e-6)):
        got = store(want)
        bad = _perturb_one(got, want, psi, m0, bound, 3.0)
        # the global relative norm the earlier tests used lets it through ...
        assert np.linalg.norm(bad - want) / np.linalg.norm(want) <= gtol
        # ... the per-site bound does not, and names the site
        try:
            sitecheck.assert_sites(bad, want, psi, m0, bound, "planted")
        except AssertionError as e:
            assert "(1, 2, 3, 1, 0)" in str(e)
        else:
            raise AssertionError("a wrong component passed the per-site check")


def test_term_scale_counts_every_neighbour():
    """s(x) = (4 + m0) a(x) + the 8 neighbours' a(y), periodic; an extent-2 axis
    counts its one neighbour twice (both hops reach it)."""
    dims = (2, 3, 4, 5)
    psi = np.zeros((1, 5, 4, 3, 2, 4, 3), dtype=np.complex128)
    psi[0, 0, 0, 0, 0, 0, 0] = 2.0 - 1.0j            # a = 2 at the origin only
    s = sitecheck.term_scale(psi, 0.5)
    assert s[0, 0, 0, 0, 0] == 4.5 * 2.0
    assert s[0, 0, 0, 0, 1] == 2 * 2.0                # x extent 2: forward and backward neighbour
    for site in ((0, 0, 1, 0), (0, 0, 2, 0), (0, 1, 0, 0), (0, 3, 0, 0), (1, 0, 0, 0), (4, 0, 0, 0)):
        assert s[(0,) + site] == 2.0, site
    assert s[0, 2, 2, 1, 0] == 0.0
    assert np.count_nonzero(s) == 1 + 1 + 6
