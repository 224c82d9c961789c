"""Per-site comparison of an operator output with the oracle's.

A global relative norm lets one wrong component out of 12 V pass at large
volumes (one component of unit size in 14^4 x 12 complex numbers moves the norm
by about 1e-3).  These helpers bound the error of every site on its own:

    max_k |got_k(x) - want_k(x)|  <=  q * m(x)  +  a * s(x)

* m(x): the largest |re| or |im| of want at site x -- the scale of an output
  stored in FP16 with a per-site norm (its codes carry 11 significant bits, so
  rounding moves a component by at most 2^-12 m(x); q = 2^-11 allows twice that),
* s(x): (4 + m0) a(x) + sum over the 8 neighbours y of a(y), with a(y) the
  largest |re| or |im| of the input at y -- the magnitude of the terms that the
  operator adds at x (Eq. (1)), which sets the size of the arithmetic rounding.

The oracle is given the inputs the GPU actually holds (rounded links and
fields), so what is left is arithmetic and output rounding only.  Everything
here is index bookkeeping and norms; none of the operator's arithmetic.
"""
import numpy as np

# the bound's coefficients per storage precision: (q, a)
F64_BOUND = (0.0, 1e-14)
F32_BOUND = (0.0, 1e-6)
F16N_BOUND = (2.0 ** -11, 2e-6)


def _site_max(f):
    """largest |re| or |im| per (rhs, site): f is [nrhs, Lt, Lz, Ly, Lx, 4, 3] complex"""
    f = np.ascontiguousarray(f)
    r = np.abs(f.view(np.float64) if np.iscomplexobj(f) else f)
    return r.reshape(r.shape[:5] + (-1,)).max(axis=-1)


def term_scale(psi, m0):
    """s(x) of the module docstring for every (rhs, site) of psi"""
    a = _site_max(psi)
    s = (4.0 + m0) * a
    for ax in (1, 2, 3, 4):          # t, z, y, x
        s = s + np.roll(a, 1, axis=ax) + np.roll(a, -1, axis=ax)
    return s


def site_errors(got, want, psi, m0, bound):
    """ratio of each site's largest component error to its bound ([nrhs, sites])"""
    q, a = bound
    got = np.asarray(got).reshape(np.asarray(psi).shape)
    want = np.asarray(want).reshape(got.shape)
    err = _site_max(got - want)
    lim = q * _site_max(want) + a * term_scale(psi, m0)
    lim = np.maximum(lim, 1e-300)
    return err / lim


def assert_sites(got, want, psi, m0, bound, what=""):
    """fail with the worst site when any site exceeds its bound"""
    r = site_errors(got, want, psi, m0, bound)
    worst = float(r.max())
    if worst > 1.0:
        idx = tuple(int(i) for i in np.unravel_index(int(r.argmax()), r.shape))
        raise AssertionError(f"{what}: site {idx} (rhs, t, z, y, x) error is {worst:.3g} x its bound")
    return worst


def links_f32(U):
    """links as the FP32 copy holds them (round to nearest even)"""
    return np.asarray(U).astype(np.complex64).astype(np.complex128)


def links_f16(U):
    """links as the FP16 copy holds them (FP64 -> FP32 -> FP16, nearest even each time)"""
    r = np.asarray(U).view(np.float64).astype(np.float32).astype(np.float16).astype(np.float64)
    return r.view(np.complex128).reshape(np.asarray(U).shape)
