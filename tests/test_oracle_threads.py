"""The oracle's operator runs its site loop on several host threads (OpenMP);
each site's value must not depend on the thread count (Eq. (1) is evaluated
site by site), and the CG of Sec. 2 built on it must therefore give the same
iterates bit for bit."""
import numpy as np
import pytest

import oracle
import wdgen


@pytest.fixture
def restore_threads():
    n = oracle.set_threads(0)
    yield
    oracle.set_threads(n)


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (3, 4, 5, 6), (2, 2, 2, 2)])
@pytest.mark.parametrize("dagger", [False, True])
def test_operator_independent_of_thread_count(dims, dagger, restore_threads):
    U = wdgen.gauge_field(dims, 0.5, 41)
    psi = wdgen.gaussian_source(dims, 1, 42)[0]
    outs = []
    for n in (1, 3, 8):
        oracle.set_threads(n)
        outs.append(oracle.dirac(U, psi, dims, 0.05, dagger=dagger))
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


def test_cg_independent_of_thread_count(restore_threads):
    dims = (4, 4, 4, 4)
    U = wdgen.gauge_field(dims, 0.5, 43)
    eta = wdgen.gaussian_source(dims, 1, 44)
    res = []
    for n in (1, 4):
        oracle.set_threads(n)
        res.append(oracle.cg(U, eta, dims, 0.1, tol=1e-10))
    x1, x4 = res[0][0], res[1][0]
    assert np.array_equal(x1, x4)
