"""The CPU oracle against results fixed by mathematics (no GPU needed)."""
import math

import numpy as np
import pytest

import oracle
import pins
import wdgen


def _ok(res):
    ok, detail = res
    assert bool(ok), detail


def test_gamma_algebra():
    _ok(pins.gamma_algebra())


def test_links_unitary_det_one_and_generator_scale():
    dims = (4, 4, 4, 4)
    U = wdgen.gauge_field(dims, 0.5, 1001).reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.max(np.abs(np.conj(np.swapaxes(U, -1, -2)) @ U - eye)) <= 1e-14
    assert np.max(np.abs(np.linalg.det(U) - 1)) <= 1e-14
    # H = sum h_a lambda_a / 2 with h_a ~ N(0,1): E[tr H^2] = 8 * (1/2) = 4
    rng = np.random.default_rng(5)
    h = rng.standard_normal((200000, 8))
    H = np.einsum("na,aij->nij", h, wdgen.gell_mann()) / 2
    trH2 = np.real(np.einsum("nij,nji->n", H, H))
    assert abs(trH2.mean() - 4.0) < 5 * trH2.std() / math.sqrt(len(trH2))
    # determinism of the generator: same seed, same field
    assert np.array_equal(wdgen.gauge_field(dims, 0.5, 7), wdgen.gauge_field(dims, 0.5, 7))


@pytest.mark.parametrize("dims,m0,t_sign", [
    ((2, 2, 2, 2), 0.1, -1), ((4, 4, 4, 4), 0.1, -1), ((4, 6, 2, 8), 0.1, +1),
    ((3, 5, 4, 6), 0.02, -1), ((14, 14, 14, 14), 0.05, -1), ((16, 16, 16, 32), 0.02, -1)])
def test_free_plane_waves(dims, m0, t_sign):
    n = 1 if dims[0] >= 14 else 3
    _ok(pins.free_plane_waves(dims, m0, t_sign, n_waves=n))


def test_free_spectrum_2x4_exact():
    _ok(pins.free_spectrum_2x4(0.1))
    _ok(pins.free_spectrum_2x4(0.37))


def test_gamma5_hermiticity():
    _ok(pins.gamma5_hermiticity())
    _ok(pins.gamma5_hermiticity(dims=(2, 2, 2, 2), seed=3))


def test_adjoint_is_conjugate_transpose_dense():
    dims = (2, 2, 2, 2)
    U = wdgen.gauge_field(dims, 0.8, 99)
    D = oracle.dense(U, dims, 0.1)
    Dd = oracle.dense(U, dims, 0.1, dagger=True)
    assert np.max(np.abs(Dd - D.conj().T)) <= 1e-15
    assert D.shape == (12 * 16, 12 * 16)   # the matrix dimension is 12 V (Sec. 1)


def test_gauge_covariance():
    _ok(pins.gauge_covariance())


def test_norm_bounds():
    _ok(pins.norm_bounds())


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 4, 4)])
def test_cg_matches_dense_solve(dims):
    _ok(pins.dense_solve(dims=dims))


def test_cg_matches_dense_solve_4x4():
    _ok(pins.dense_solve(dims=(4, 4, 4, 4), m0=0.1, eps=0.3, seed=1001))


def test_cgnr_matches_dense_solve():
    _ok(pins.dense_solve(form=1))


def test_cg_matches_free_fft_solution():
    _ok(pins.free_fft_solve())


def test_cg_matches_pure_gauge_solution():
    _ok(pins.pure_gauge_solve())


def test_cgne_error_monotone():
    _ok(pins.cgne_error_monotone())


def test_cg_zero_source_and_exact_guess():
    dims = (4, 4, 4, 4)
    U = wdgen.gauge_field(dims, 0.3, 1001)
    x, it, res, st = oracle.cg(U, np.zeros((1,) + wdgen.lattice_shape(dims) + (4, 3)), dims, 0.1)
    assert it == [0] and st == [0] and not np.any(x)
    eta = wdgen.gaussian_source(dims, 1, 2001)
    x, it, res, st = oracle.cg(U, eta, dims, 0.1)
    x2, it2, res2, st2 = oracle.cg(U, eta, dims, 0.1, x0=x)
    assert it2 == [0] and st2 == [0] and np.array_equal(x, x2)


def test_cg_max_iter_reports_not_converged():
    dims = (4, 4, 4, 4)
    U = wdgen.gauge_field(dims, 0.3, 1001)
    eta = wdgen.gaussian_source(dims, 1, 2001)
    x, it, res, st = oracle.cg(U, eta, dims, 0.1, max_iter=5)
    assert st == [1] and it == [5] and res[0] > 1e-10


def test_coo_format_matches_operator():
    """The coordinate-format matrix (Sec. 2) built term by term in NumPy agrees
    with the C operator; 49 stored entries per row (duplicates on 2^4 kept)."""
    for dims in [(2, 2, 2, 2), (4, 4, 4, 4), (2, 3, 4, 5)]:
        V = wdgen.volume(dims)
        U = wdgen.gauge_field(dims, 0.6, 5)
        psi = wdgen.gaussian_source(dims, 1, 6)[0]
        for dag in (False, True):
            val, row, col = oracle.coo(U, dims, 0.07, dagger=dag)
            assert len(val) == 588 * V
            got = oracle.coo_matvec(val, row, col, psi.ravel(), 12 * V)
            want = oracle.dirac(U, psi, dims, 0.07, dagger=dag).ravel()
            assert np.linalg.norm(got - want) <= 1e-14 * np.linalg.norm(want)


def test_fp16n_encoding():
    rng = np.random.default_rng(3)
    v = (rng.standard_normal((5, 64, 4, 3)) + 1j * rng.standard_normal((5, 64, 4, 3))) * 10.0
    v32 = v.astype(np.complex64)
    codes, norms = oracle.fp16n_encode(v32)
    assert codes.dtype == np.float16 and norms.dtype == np.float32
    assert codes.shape == (5, 64, 24) and norms.shape == (5, 64)
    # the largest component of each site is coded as +-1 exactly
    assert np.all(np.max(np.abs(codes.astype(np.float32)), axis=-1) == 1.0)
    dec = oracle.fp16n_decode(codes, norms)
    err = np.abs(dec - v32).reshape(5, 64, 12)
    # half has 11 significant bits: |code - q| <= 2^-12 for |q| <= 1, times norm
    assert np.all(err.real <= norms[..., None] * 2.0 ** -11 * 1.0001)
    # all-zero site -> norm 0, codes 0
    z = np.zeros((1, 2, 4, 3), dtype=np.complex64)
    z[0, 1, 2, 1] = 0.5 + 0.25j
    c, n = oracle.fp16n_encode(z)
    assert n[0, 0] == 0 and not np.any(c[0, 0])
    assert n[0, 1] == 0.5 and c[0, 1, 14] == 1.0 and c[0, 1, 15] == 0.5
    # ties round to even: with norm 2 the scaled values are exact in FP32, and
    # 0.5 + 2^-12 sits halfway between 0.5 and 0.5 + 2^-11 (even: 0.5), 0.5 +
    # 3 2^-12 halfway between 0.5 + 2^-11 and 0.5 + 2^-10 (even: the latter)
    t = np.zeros((1, 1, 4, 3), dtype=np.complex64)
    t[0, 0, 0, 0] = 2.0                                   # the norm
    t[0, 0, 0, 1] = (1.0 + 2.0 ** -11) + 1j * (1.0 + 3 * 2.0 ** -11)
    t[0, 0, 0, 2] = -0.75 - 1j * 2.0 ** -20                # -2^-21: a half subnormal
    c, n = oracle.fp16n_encode(t)
    assert n[0, 0] == 2.0
    assert c[0, 0, 2] == 0.5 and c[0, 0, 3] == 0.5 + 2.0 ** -10
    assert c[0, 0, 4] == -0.375 and c[0, 0, 5] == -2.0 ** -21
    # a norm that is not a power of two: every code is within one half-ulp of
    # half (+1 FP32 rounding) of the exact quotient, and the site's largest
    # component is coded 1 exactly
    u = np.zeros((1, 1, 4, 3), dtype=np.complex64)
    u[0, 0, 0, 0] = 3.0
    u[0, 0, 1, 1] = 1.0 - 2.0j
    c, n = oracle.fp16n_encode(u)
    assert n[0, 0] == 3.0 and c[0, 0, 0] == 1.0
    assert abs(float(c[0, 0, 8]) - 1 / 3) <= 2.0 ** -13 and abs(float(c[0, 0, 9]) + 2 / 3) <= 2.0 ** -12
    # a subnormal norm whose reciprocal overflows FP32: codes from the quotient,
    # exact here (-1, 0.5, 0), no infinities and no NaN
    w = np.zeros((1, 1, 4, 3), dtype=np.complex64)
    w[0, 0, 0, 0] = -np.float32(2.0 ** -140) + 1j * np.float32(2.0 ** -141)
    c, n = oracle.fp16n_encode(w)
    assert n[0, 0] == np.float32(2.0 ** -140)
    assert c[0, 0, 0] == -1.0 and c[0, 0, 1] == 0.5 and np.all(c[0, 0, 2:] == 0)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 4, 4), (4, 4, 4, 4)])
def test_bicgstab_matches_dense_solve(dims):
    _ok(pins.bicgstab_dense_solve(dims=dims))


def test_bicgstab_matches_free_fft_solution():
    _ok(pins.bicgstab_free_fft_solve())


def test_bicgstab_agrees_with_cg():
    dims, m0 = (6, 6, 6, 6), 0.05
    U = wdgen.gauge_field(dims, 0.5, 1002)
    eta = wdgen.gaussian_source(dims, 2, 2002)
    xb, itb, rb, sb = oracle.bicgstab(U, eta, dims, m0)
    xc, itc, rc, sc = oracle.cg(U, eta, dims, m0)
    assert sb == [0, 0] and max(rb) <= 1e-10
    assert np.linalg.norm(xb - xc) / np.linalg.norm(xc) <= pins.kappa_bound(m0) * 2e-10


def test_bicgstab_breaks_down_on_a_point_source():
    """With r_hat = r0 = e_k, alpha = 1 / D_kk makes s orthogonal to e_k, and
    t = D s has no e_k component either ((1 - gamma)(1 + gamma) = 0 kills the
    back-and-forth hop), so <r_hat, r1> = 0: plain BiCGSTAB must stop after one
    iteration on any gauge field, with status 2 (breakdown)."""
    dims, m0 = (4, 4, 4, 4), 0.1
    U = wdgen.gauge_field(dims, 0.5, 77)
    eta = wdgen.point_sources(dims, ks=[0, 7])
    x, it, res, st = oracle.bicgstab(U, eta, dims, m0)
    assert st == [2, 2] and it == [1, 1]
    # a Gaussian source on the same links converges
    eta = wdgen.gaussian_source(dims, 1, 78)
    assert oracle.bicgstab(U, eta, dims, m0)[3] == [0]


# ------------------------------------------------------------ even-odd
def _parity_index(dims):
    """Indices of the even and odd rows of the dense operator (site-major, 12
    components per site, sites in the canonical order)."""
    par = oracle.parity(dims).ravel()
    rows = np.arange(par.size * 12)
    site_par = par[rows // 12]
    return rows[site_par == 0], rows[site_par == 1]


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 4, 4), (4, 4, 4, 4)])
@pytest.mark.parametrize("dagger", [False, True])
def test_schur_matches_dense_block_elimination(dims, dagger):
    """oracle.schur against the Schur complement D_ee - D_eo D_oo^-1 D_oe built
    from the dense operator's blocks with a generic solve (no use of the
    diagonal form of D_oo)."""
    m0 = 0.13
    U = wdgen.gauge_field(dims, 0.6, 91)
    D = oracle.dense(U, dims, m0, dagger=dagger)
    ie, io = _parity_index(dims)
    S = D[np.ix_(ie, ie)] - D[np.ix_(ie, io)] @ np.linalg.solve(D[np.ix_(io, io)], D[np.ix_(io, ie)])
    v = wdgen.gaussian_source(dims, 1, 92)[0]
    got = oracle.schur(U, v, dims, m0, dagger=dagger).ravel()
    want = S @ v.ravel()[ie]
    assert np.linalg.norm(got[ie] - want) <= 1e-13 * np.linalg.norm(want)
    assert np.all(got[io] == 0)


def test_schur_dagger_is_the_adjoint():
    dims, m0 = (4, 4, 2, 6), 0.07
    U = wdgen.gauge_field(dims, 0.5, 93)
    u, v = wdgen.gaussian_source(dims, 2, 94)
    even = (oracle.parity(dims) == 0)[..., None, None]
    u, v = np.where(even, u, 0), np.where(even, v, 0)
    lhs = np.vdot(u, oracle.schur(U, v, dims, m0))
    rhs = np.vdot(oracle.schur(U, u, dims, m0, dagger=True), v)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(u) * np.linalg.norm(v) * 10


def test_cg_eo_matches_dense_solve():
    dims, m0 = (4, 4, 4, 4), 0.1
    U = wdgen.gauge_field(dims, 0.3, 1001)
    eta = wdgen.mixed_sources(dims, 1, 1, 95)
    x, it, res, st = oracle.cg_eo(U, eta, dims, m0)
    assert st == [0, 0] and max(res) <= 1e-10
    D = oracle.dense(U, dims, m0)
    for i in range(2):
        xs = np.linalg.solve(D, eta[i].ravel())
        assert np.linalg.norm(x[i].ravel() - xs) <= pins.kappa_bound(m0) * 1e-10 * np.linalg.norm(xs)
    # the preconditioned system converges in fewer iterations than plain CGNE
    assert max(it) < min(oracle.cg(U, eta, dims, m0)[1])


def test_cg_eo_zero_source_and_free_field():
    dims, m0 = (8, 8, 8, 8), 0.05
    U = wdgen.unit_gauge(dims)
    eta = wdgen.gaussian_source(dims, 2, 96)
    eta[1] = 0
    x, it, res, st = oracle.cg_eo(U, eta, dims, m0)
    assert st == [0, 0] and it[1] == 0 and np.all(x[1] == 0)
    gam = [oracle.gamma(mu) for mu in range(4)]
    xs = pins.free_solve_fft(eta[0], dims, m0, -1, gam)
    assert np.linalg.norm(x[0] - xs) <= pins.kappa_bound(m0) * 2e-10 * np.linalg.norm(xs)


def test_third_row_of_su3_links_is_conjugated_cross_product():
    """The identity reconstruct-12 relies on: for U in SU(3), row 2 is the complex
    conjugate of row 0 x row 1; for -U (a link carrying the boundary sign -1,
    det -1) it is minus that."""
    U = wdgen.gauge_field((4, 4, 4, 4), 0.5, 531).reshape(-1, 3, 3)
    c = np.conj(np.cross(U[:, 0, :], U[:, 1, :]))
    assert np.max(np.abs(c - U[:, 2, :])) <= 1e-13
    W = -U
    cw = np.conj(np.cross(W[:, 0, :], W[:, 1, :]))
    assert np.max(np.abs(-cw - W[:, 2, :])) <= 1e-13
    # a U(3) matrix with det e^{i phi} has row 2 = e^{i phi} conj(row 0 x row 1), not the plain product
    ph = np.exp(0.3j)
    X = U[:5] * ph
    cx = np.conj(np.cross(X[:, 0, :], X[:, 1, :]))
    assert np.max(np.abs(cx - X[:, 2, :])) > 0.1
    assert np.max(np.abs(np.linalg.det(X)[:, None] * cx - X[:, 2, :])) <= 1e-13
