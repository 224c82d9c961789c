"""wd_dslash_noalloc, the operator entry point that allocates nothing (its packed
temporaries live in the library's static device scratch), against wd_dslash /
wd_dslash_dag on the same inputs: bitwise equal (the same packing and operator
kernels run), and against the FP64 oracle (Eq. (1)).  Calls follow one another
on one stream, the later ones smaller, so stale scratch contents of a larger
call must not leak into a smaller one."""
import numpy as np
import pytest

import oracle
import paper_2111_14958_amd as wd
from gpu_util import dev, host, rel, say, field_set

pytestmark = pytest.mark.gpu

TOL = {wd.F64: 1e-13, wd.F32: 1e-6, wd.F16N: 2e-3}


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    assert wd.device_info(0)[0].startswith("gfx950")


def _gauge(dims, seed):
    U, _ = field_set(dims, 0.5, seed, 1, seed + 1)
    return U, wd.Gauge(dev(U), dims, -1, precs=(wd.F64, wd.F32, wd.F16N))


@pytest.mark.parametrize("prec", [wd.F64, wd.F32, wd.F16N])
def test_noalloc_matches_dslash_on_shrinking_calls(prec):
    m0 = 0.05
    big, small = (8, 8, 8, 8), (4, 4, 4, 6)
    Ub, gb = _gauge(big, 3100)
    Us, gs = _gauge(small, 3200)
    try:
        _, pb = field_set(big, 0.5, 3100, 3, 3301)
        _, ps = field_set(small, 0.5, 3200, 1, 3302)
        for (U, g, psi, dims, dag) in ((Ub, gb, pb, big, False), (Us, gs, ps, small, True)):
            say("wd_dslash_noalloc", dims, "nrhs", psi.shape[0], "prec", prec, "dagger", dag)
            x = dev(psi)
            got = host(wd.dslash_noalloc(g, m0, x, prec, dagger=dag))
            ref = host(wd.dslash(g, m0, x, prec, dagger=dag))
            assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), \
                "no-alloc operator differs from wd_dslash on the same inputs"
            want = oracle.dirac(U, psi, dims, m0, -1, dagger=dag)
            assert rel(got, want) <= TOL[prec]
    finally:
        gb.close()
        gs.close()


def test_noalloc_largest_fitting_call_and_refusal():
    """12^4 in FP64: 8 fields (2 x 8 x 3.98 MB) fit the 64 MiB scratch, 9 do not."""
    dims, m0 = (12, 12, 12, 12), 0.05
    U, g = _gauge(dims, 3400)
    try:
        V = 12 ** 4
        assert 2 * 8 * V * 192 <= wd.NOALLOC_SCRATCH_BYTES < 2 * 9 * V * 192
        _, psi = field_set(dims, 0.5, 3400, 8, 3401)
        say("wd_dslash_noalloc", dims, "nrhs 8 FP64 (largest that fits)")
        x = dev(psi)
        got = host(wd.dslash_noalloc(g, m0, x, wd.F64))
        ref = host(wd.dslash(g, m0, x, wd.F64))
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
        want = oracle.dirac(U, psi[:2], dims, m0, -1)
        assert rel(got[:2], want) <= TOL[wd.F64]
        # one field more is refused before any device work, with the sizes in the detail
        import torch
        x9 = torch.zeros((9,) + tuple(x.shape[1:]), dtype=torch.complex128, device="cuda")
        with pytest.raises(wd.WDError) as e:
            wd.dslash_noalloc(g, m0, x9, wd.F64)
        assert e.value.code == wd.WD_ETOOBIG and "static scratch" in str(e.value)
        # the scratch still serves a smaller call afterwards
        say("wd_dslash_noalloc", dims, "nrhs 1 FP32 after the refusal")
        got1 = host(wd.dslash_noalloc(g, m0, x[:1], wd.F32, dagger=True))
        ref1 = host(wd.dslash(g, m0, x[:1], wd.F32, dagger=True))
        assert np.array_equal(got1.view(np.uint64), ref1.view(np.uint64))
    finally:
        g.close()


def test_noalloc_argument_errors():
    dims = (4, 4, 4, 4)
    U, g = _gauge(dims, 3500)
    try:
        l = wd.lib()
        x = dev(np.zeros((1,) + dims[::-1] + (4, 3), np.complex128))
        y = dev(np.zeros((1,) + dims[::-1] + (4, 3), np.complex128))
        assert l.wd_dslash_noalloc(g.handle, 0.1, wd.F64, 2, x.data_ptr(), y.data_ptr(), 1, None) == wd.WD_EINVAL
        assert l.wd_dslash_noalloc(g.handle, 0.1, 7, 0, x.data_ptr(), y.data_ptr(), 1, None) == wd.WD_EINVAL
        assert l.wd_dslash_noalloc(g.handle, 0.1, wd.F64, 0, x.data_ptr(), y.data_ptr(), 0, None) == wd.WD_EINVAL
        assert l.wd_dslash_noalloc(g.handle, 0.1, wd.F64, 0, None, y.data_ptr(), 1, None) == wd.WD_EINVAL
    finally:
        g.close()
