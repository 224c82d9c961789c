"""The GPU CG keeps the search direction only as its image q = D^dagger p.

The paper's CG on D D^dagger (Sec. 2) updates p' = r' + beta p and applies
D^dagger to it; since D^dagger is linear, q' = D^dagger p' = D^dagger r' +
beta q, so the solver can form q from r and the previous q without storing p.
This test runs both recurrences side by side in FP64 with the oracle's
operator on a 4^4 lattice: the p form reproduces the oracle CG's own residual
history (so it is the paper's algorithm, not a retyped copy of the GPU's), and
the q form, carried beside it, stays equal to D^dagger p to rounding and gives
the same iterates and residuals.
"""
import numpy as np

import oracle
import wdgen


def test_direction_image_recurrence_equals_p_recurrence():
    dims, m0, iters = (4, 4, 4, 4), 0.1, 40
    U = wdgen.gauge_field(dims, 0.3, 71)
    eta = wdgen.gaussian_source(dims, 1, 72)[0]

    def D(v, dag=False):
        return oracle.dirac(U, v[None], dims, m0, -1, dagger=dag)[0]

    _, _, _, _, traces = oracle.cg(U, eta[None], dims, m0, tol=1e-14, max_iter=iters, trace=True)
    hist_oracle = traces[0]
    en = np.linalg.norm(eta)
    # p form (the paper's recurrence) and q form (the GPU's) from x0 = 0
    x_p, r_p = np.zeros_like(eta), eta.copy()
    p = r_p.copy()
    x_q, r_q = np.zeros_like(eta), eta.copy()
    q_q = D(r_q, dag=True)             # restart: q = D^dagger r
    rho_p = np.vdot(r_p, r_p).real
    rho_q = np.vdot(r_q, r_q).real
    for k in range(iters):
        q_p = D(p, dag=True)
        # the carried image equals D^dagger p up to rounding
        assert np.linalg.norm(q_q - q_p) <= 1e-12 * np.linalg.norm(q_p), k
        for x, r, q, rho in ((x_p, r_p, q_p, rho_p), (x_q, r_q, q_q, rho_q)):
            alpha = rho / np.vdot(q, q).real
            x += alpha * q
            r -= alpha * D(q)
        rho_p_new = np.vdot(r_p, r_p).real
        rho_q_new = np.vdot(r_q, r_q).real
        assert abs(np.sqrt(rho_p_new) / en - hist_oracle[k]) <= 1e-9 * hist_oracle[k], k
        assert abs(rho_q_new - rho_p_new) <= 1e-9 * rho_p_new, k
        beta_p, beta_q = rho_p_new / rho_p, rho_q_new / rho_q
        p = r_p + beta_p * p
        q_q = D(r_q, dag=True) + beta_q * q_q
        rho_p, rho_q = rho_p_new, rho_q_new
    assert np.linalg.norm(x_q - x_p) <= 1e-10 * np.linalg.norm(x_p)
    # and both are converging to the solution of D x = eta
    assert np.linalg.norm(eta - D(x_q)) / en < hist_oracle[0]
