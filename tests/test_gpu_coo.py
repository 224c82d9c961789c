"""The coordinate-format operator of Sec. 2 on the GPU: the entry set built on
the device equals the oracle's coordinate-format builder bit for bit (after
sorting by (row, col, value)), and the product matches the oracle operator."""
import numpy as np
import pytest

import oracle
import paper_2111_14958_amd as wd
import wdgen
from gpu_util import dev, host, rel, say

pytestmark = pytest.mark.gpu


def _sorted(val, row, col):
    order = np.lexsort((val.imag, val.real, col, row))
    return val[order], row[order], col[order]


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (3, 5, 4, 6)])
@pytest.mark.parametrize("dagger", [False, True])
def test_coo_entries_bit_exact(dims, dagger):
    U = wdgen.gauge_field(dims, 0.6, 5)
    say("coo entries", dims, dagger)
    g = wd.Gauge(dev(U), dims)
    c = wd.Coo(g, 0.07, wd.F64, dagger)
    V = wdgen.volume(dims)
    assert c.nnz == 588 * V and c.rows == 12 * V
    val, row, col = (host(t) for t in c.export())
    rows = 12 * V                                 # entry k of row r at k * rows + r
    assert np.array_equal(row.reshape(49, rows), np.broadcast_to(np.arange(rows), (49, rows)))
    ov, orow, ocol = oracle.coo(U, dims, 0.07, dagger=dagger)
    a = _sorted(val, row.astype(np.int64), col.astype(np.int64))
    b = _sorted(ov, orow, ocol)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert np.array_equal(a[0], b[0])


@pytest.mark.parametrize("prec,tol", [(wd.F64, 1e-14), (wd.F32, 1e-6)], ids=["f64", "f32"])
def test_coo_product_matches_oracle(prec, tol):
    import torch
    dims, m0 = (8, 8, 8, 8), 0.05
    U = wdgen.gauge_field(dims, 0.5, 9)
    psi = wdgen.gaussian_source(dims, 6, 10)   # two groups of vectors: 4 and 2
    say("coo spmv", prec)
    g = wd.Gauge(dev(U), dims)
    c = wd.Coo(g, m0, prec)
    x = dev(psi).reshape(6, -1)
    if prec == wd.F32:
        x = x.to(torch.complex64)
    got = host(c.spmv(x)).reshape(psi.shape)
    want = oracle.dirac(U, psi, dims, m0)
    assert rel(got, want) <= tol
    # and it agrees with the stencil kernel
    st = host(wd.dslash(g, m0, dev(psi), wd.F64))
    assert rel(got, st) <= tol
