"""Pins for the CPU oracle: results fixed by mathematics rather than by the
oracle's own code.

Each pin returns (ok: bool, detail: str) and takes an optional `lib` (a build
of the oracle source) so that the mutation tests can run the same pins against
deliberately broken builds.

  free_plane_waves   -- closed form: with U = 1 a plane wave e^{ip.x} u is mapped
                        to e^{ip.x} D(p) u, D(p) = m0 + sum(1 - cos p) + i sum gamma sin p,
                        p_t = (2n+1) pi / Lt for the antiperiodic time boundary
  free_spectrum_2x4  -- closed form: on a 2^4 free lattice the spectrum of D is
                        {m0 + 1 + 2k +- i}, multiplicity 12 C(3,k) each
  gamma5_hermiticity -- <x, g5 D g5 y> = <D x, y>, and dirac_dag = g5 D g5 (Sec. 2)
  gauge_covariance   -- D[U^Omega](Omega psi) = Omega D[U] psi
  norm_bounds        -- |D v| <= (8 + m0)|v| and Re<v, D v> >= m0 |v|^2
  dense_solve        -- CG solution vs LAPACK solve of the dense D
  free_fft_solve     -- CG solution vs the free propagator computed with FFTs
  pure_gauge_solve   -- CG solution vs Omega D_free^{-1} Omega^dagger eta
  cgne_error_monotone-- CG on D D^dagger minimises |x_k - x*| over its Krylov
                        space, so the error never grows
"""
from __future__ import annotations

import math

import numpy as np

import oracle
import wdgen


# ----------------------------------------------------------------- closed forms
def momenta(dims, t_sign=-1):
    """Allowed momenta per axis (x, y, z, t)."""
    ps = []
    for mu, L in enumerate(dims):
        n = np.arange(L)
        if mu == 3 and t_sign == -1:
            ps.append((2 * n + 1) * np.pi / L)
        else:
            ps.append(2 * n * np.pi / L)
    return ps


def free_Dp(p, m0, gam):
    """D(p) for momenta p[..., 4] with gamma matrices gam[4] (4x4)."""
    p = np.asarray(p, dtype=np.float64)
    M = m0 + np.sum(1 - np.cos(p), axis=-1)
    out = M[..., None, None] * np.eye(4)
    for mu in range(4):
        out = out + 1j * np.sin(p[..., mu])[..., None, None] * gam[mu]
    return out


def plane_wave(dims, p, u):
    """e^{i p.x} u on the (t, z, y, x) grid; u is a (4, 3) spin-colour vector."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return ph[..., None, None] * u[None, None, None, None]


def free_solve_fft(eta, dims, m0, t_sign, gam):
    """x* = D_free^{-1} eta using FFTs; eta[t, z, y, x, 4, 3]."""
    lx, ly, lz, lt = dims
    tt = np.arange(lt)[:, None, None, None, None, None]
    tw = np.exp(1j * np.pi * tt / lt) if t_sign == -1 else np.ones_like(tt, dtype=complex)
    e = np.fft.fftn(eta / tw, axes=(0, 1, 2, 3))
    kt, kz, ky, kx = np.meshgrid(*(2 * np.pi * np.fft.fftfreq(L) for L in (lt, lz, ly, lx)),
                                 indexing="ij")
    shift = np.pi / lt if t_sign == -1 else 0.0
    p = np.stack([kx, ky, kz, kt + shift], axis=-1)
    Dp = free_Dp(p, m0, gam)
    xs = np.linalg.solve(Dp, e)          # solves over the spin index, colour as columns
    return np.fft.ifftn(xs, axes=(0, 1, 2, 3)) * tw


def kappa_bound(m0):
    """Condition-number bound of D: |D| <= 8 + m0 and sigma_min(D) >= m0."""
    return (8.0 + m0) / m0


def _gammas(lib=None):
    return [oracle.gamma(mu, lib=lib) for mu in range(4)]


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


# ----------------------------------------------------------------------- pins
def gamma_algebra(lib=None):
    G = _gammas(lib)
    for mu in range(4):
        if not np.allclose(G[mu], G[mu].conj().T, atol=0):
            return False, f"gamma_{mu} not Hermitian"
        for nu in range(4):
            ac = G[mu] @ G[nu] + G[nu] @ G[mu]
            if not np.allclose(ac, 2 * np.eye(4) * (mu == nu), atol=0):
                return False, f"Clifford relation fails for {mu},{nu}"
    g5 = G[0] @ G[1] @ G[2] @ G[3]
    if not np.allclose(g5, np.diag([1, 1, -1, -1]), atol=0):
        return False, "gamma5 != diag(1,1,-1,-1)"
    return True, "ok"


def free_plane_waves(dims, m0, t_sign=-1, n_waves=3, seed=7, lib=None, tol=1e-13):
    rng = np.random.default_rng(seed)
    G = _gammas(lib)
    U = wdgen.unit_gauge(dims)
    ps = momenta(dims, t_sign)
    worst = 0.0
    for _ in range(n_waves):
        p = np.array([ps[mu][rng.integers(len(ps[mu]))] for mu in range(4)])
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = plane_wave(dims, p, u)
        got = oracle.dirac(U, psi, dims, m0, t_sign, lib=lib)
        want = plane_wave(dims, p, free_Dp(p, m0, G) @ u)
        worst = max(worst, _rel(got, want))
        # and the normal operator D^dagger D has eigenvalue M^2 + |sin p|^2
        got2 = oracle.dirac(U, got, dims, m0, t_sign, dagger=True, lib=lib)
        M = m0 + np.sum(1 - np.cos(p))
        lam = M * M + np.sum(np.sin(p) ** 2)
        worst = max(worst, _rel(got2, lam * psi))
    return worst <= tol, f"max rel err {worst:.3e}"


def free_spectrum_2x4(m0=0.1, lib=None):
    dims = (2, 2, 2, 2)
    Dm = oracle.dense(wdgen.unit_gauge(dims), dims, m0, -1, lib=lib)
    ev = np.linalg.eigvals(Dm)
    want = []
    for k in range(4):
        for sgn in (+1, -1):
            want += [complex(m0 + 1 + 2 * k, sgn)] * (12 * math.comb(3, k))
    want = np.array(sorted(want, key=lambda z: (round(z.real, 6), round(z.imag, 6))))
    got = np.array(sorted(ev, key=lambda z: (round(z.real, 6), round(z.imag, 6))))
    err = float(np.max(np.abs(got - want)))
    return err <= 1e-12, f"max eigenvalue err {err:.3e}"


def gamma5_hermiticity(dims=(4, 4, 4, 4), m0=0.1, eps=0.7, seed=11, lib=None, tol=1e-14):
    U = wdgen.gauge_field(dims, eps, seed)
    x = wdgen.gaussian_source(dims, 1, seed + 1)[0]
    y = wdgen.gaussian_source(dims, 1, seed + 2)[0]
    g5 = np.array([1, 1, -1, -1], dtype=float)[:, None]
    Dx = oracle.dirac(U, x, dims, m0, lib=lib)
    g5Dg5y = g5 * oracle.dirac(U, g5 * y, dims, m0, lib=lib)
    lhs = np.vdot(x, g5Dg5y)
    rhs = np.vdot(Dx, y)
    e1 = abs(lhs - rhs) / (np.linalg.norm(x) * np.linalg.norm(y))
    e2 = _rel(oracle.dirac(U, y, dims, m0, dagger=True, lib=lib), g5Dg5y)
    # adjoint identity <x, D^dagger y> = <D x, y>
    e3 = abs(np.vdot(x, oracle.dirac(U, y, dims, m0, dagger=True, lib=lib)) - rhs) / (
        np.linalg.norm(x) * np.linalg.norm(y))
    worst = max(e1, e2, e3)
    return worst <= tol, f"errs {e1:.2e} {e2:.2e} {e3:.2e}"


def gauge_covariance(dims=(4, 4, 6, 8), m0=0.1, eps=0.7, seed=21, lib=None, tol=1e-14):
    U = wdgen.gauge_field(dims, eps, seed)
    Om = wdgen.site_matrices(dims, 2.0, seed + 1)
    psi = wdgen.gaussian_source(dims, 1, seed + 2)[0]
    Ug = wdgen.transform_gauge(U, Om)
    worst = 0.0
    for dag in (False, True):
        lhs = oracle.dirac(Ug, wdgen.apply_site_matrix(Om, psi), dims, m0, dagger=dag, lib=lib)
        rhs = wdgen.apply_site_matrix(Om, oracle.dirac(U, psi, dims, m0, dagger=dag, lib=lib))
        worst = max(worst, _rel(lhs, rhs))
    return worst <= tol, f"max rel err {worst:.3e}"


def norm_bounds(dims=(4, 4, 4, 4), m0=0.05, eps=1.0, seed=31, n=6, lib=None):
    U = wdgen.gauge_field(dims, eps, seed)
    vs = wdgen.gaussian_source(dims, n, seed + 1)
    for v in vs:
        Dv = oracle.dirac(U, v, dims, m0, lib=lib)
        nv = np.linalg.norm(v)
        if np.linalg.norm(Dv) > (8 + m0) * nv * (1 + 1e-12):
            return False, "|Dv| > (8+m0)|v|"
        if np.real(np.vdot(v, Dv)) < m0 * nv * nv * (1 - 1e-12):
            return False, "Re<v,Dv> < m0|v|^2"
    return True, "ok"


def dense_solve(dims=(2, 2, 4, 4), m0=0.1, eps=0.5, seed=41, tol=1e-10, lib=None,
                form=0, max_iter=5000):
    U = wdgen.gauge_field(dims, eps, seed)
    eta = wdgen.gaussian_source(dims, 1, seed + 1)[0]
    Dm = oracle.dense(U, dims, m0, lib=lib)
    xs = np.linalg.solve(Dm, eta.ravel()).reshape(eta.shape)
    x, it, res, st = oracle.cg(U, eta, dims, m0, tol=tol, form=form, max_iter=max_iter, lib=lib)
    err = _rel(x, xs)
    bound = kappa_bound(m0) * tol
    ok = st[0] == 0 and res[0] <= tol and err <= bound
    return ok, f"status {st[0]} iters {it[0]} res {res[0]:.2e} err {err:.2e} bound {bound:.2e}"


def bicgstab_dense_solve(dims=(2, 2, 4, 4), m0=0.1, eps=0.5, seed=43, tol=1e-10, lib=None,
                         max_iter=5000):
    U = wdgen.gauge_field(dims, eps, seed)
    eta = wdgen.gaussian_source(dims, 1, seed + 1)[0]
    Dm = oracle.dense(U, dims, m0, lib=lib)
    xs = np.linalg.solve(Dm, eta.ravel()).reshape(eta.shape)
    x, it, res, st = oracle.bicgstab(U, eta, dims, m0, tol=tol, max_iter=max_iter, lib=lib)
    err = _rel(x, xs)
    bound = kappa_bound(m0) * tol
    ok = st[0] == 0 and res[0] <= tol and err <= bound
    return ok, f"status {st[0]} iters {it[0]} res {res[0]:.2e} err {err:.2e} bound {bound:.2e}"


def bicgstab_free_fft_solve(dims=(8, 8, 8, 8), m0=0.05, seed=53, tol=1e-10, lib=None):
    U = wdgen.unit_gauge(dims)
    eta = wdgen.gaussian_source(dims, 1, seed)[0]
    xs = free_solve_fft(eta, dims, m0, -1, _gammas(None))
    x, it, res, st = oracle.bicgstab(U, eta, dims, m0, tol=tol, max_iter=5000, lib=lib)
    err = _rel(x, xs)
    return st[0] == 0 and err <= kappa_bound(m0) * tol, f"status {st[0]} iters {it[0]} err {err:.2e}"


def free_fft_solve(dims=(8, 8, 8, 8), m0=0.05, seed=51, tol=1e-10, lib=None, max_iter=5000):
    U = wdgen.unit_gauge(dims)
    eta = wdgen.gaussian_source(dims, 1, seed)[0]
    xs = free_solve_fft(eta, dims, m0, -1, _gammas(None))
    x, it, res, st = oracle.cg(U, eta, dims, m0, tol=tol, max_iter=max_iter, lib=lib)
    err = _rel(x, xs)
    bound = kappa_bound(m0) * tol
    return st[0] == 0 and err <= bound, f"status {st[0]} iters {it[0]} err {err:.2e}"


def pure_gauge_solve(dims=(4, 4, 4, 8), m0=0.1, seed=61, tol=1e-10, lib=None, max_iter=5000):
    Om = wdgen.site_matrices(dims, 2.0, seed)
    U = wdgen.pure_gauge(Om)
    eta = wdgen.gaussian_source(dims, 1, seed + 1)[0]
    xs = wdgen.apply_site_matrix(
        Om, free_solve_fft(wdgen.apply_site_matrix(Om, eta, dagger=True), dims, m0, -1,
                           _gammas(None)))
    x, it, res, st = oracle.cg(U, eta, dims, m0, tol=tol, max_iter=max_iter, lib=lib)
    err = _rel(x, xs)
    bound = kappa_bound(m0) * tol
    return st[0] == 0 and err <= bound, f"status {st[0]} iters {it[0]} err {err:.2e}"


def cgne_error_monotone(dims=(2, 2, 4, 4), m0=0.1, eps=0.5, seed=71, kmax=40, lib=None):
    U = wdgen.gauge_field(dims, eps, seed)
    eta = wdgen.gaussian_source(dims, 1, seed + 1)[0]
    Dm = oracle.dense(U, dims, m0, lib=lib)
    xs = np.linalg.solve(Dm, eta.ravel())
    prev = np.linalg.norm(xs)          # x_0 = 0
    for k in range(1, kmax + 1):
        x = oracle.cg(U, eta, dims, m0, tol=1e-300, max_iter=k, lib=lib)[0].ravel()
        e = np.linalg.norm(x - xs)
        if e > prev * (1 + 1e-10):
            return False, f"error grew at iteration {k}: {prev:.3e} -> {e:.3e}"
        prev = e
    return True, f"final error {prev:.3e}"
