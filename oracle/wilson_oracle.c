/*
 * TEST INFRASTRUCTURE ONLY -- the CPU oracle.
 *
 * A plain, slow, obviously correct FP64 implementation of what the solver
 * computes, used by the tests, the smoke check and the CPU baseline of the
 * benchmark to check the GPU library.  It shares no code, header, table or
 * constant with the GPU library and must never be linked into it.
 *
 * What it computes (arXiv 2111.14958):
 *  - the Wilson-Dirac operator D of Eq. (1) (Sec. 1), written out as 4x4 spin
 *    matrices (1 -+ gamma_mu) times 3x3 colour links, with no spin projection
 *    or any other rewriting;
 *  - its adjoint D^dagger, which by gamma5-hermiticity (Sec. 2) is D with the
 *    two projectors exchanged;
 *  - conjugate gradient on the normal equations D D^dagger chi = eta followed
 *    by psi = D^dagger chi (Sec. 2, the CG algorithm), carried in the solution
 *    space: x = D^dagger chi, so the update psi += alpha p of the paper becomes
 *    x += alpha D^dagger p, and the residual r = eta - D x is the residual of
 *    D psi = eta itself;
 *  - optionally CG on D^dagger D x = D^dagger eta (CGNR), the other normal form;
 *  - BiCGSTAB directly on D, one of the other Krylov methods of Sec. 1.
 *
 * Conventions (the paper is silent on them):
 *  D psi(x) = (4 + m0) psi(x)
 *             - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) s psi(x + mu)
 *                          + (1 + gamma_mu) U_mu(x - mu)^dagger s psi(x - mu) ]
 *  (Wilson parameter r = 1), s = -1 for a hop in t that wraps around the
 *  lattice when the time boundary is antiperiodic, else +1.  Gamma matrices
 *  in the DeGrand-Rossi chiral basis, gamma5 = diag(1, 1, -1, -1).
 *  Canonical layouts: U[site][mu][a][b], psi[site][spin][colour], complex128,
 *  site = x + Lx*(y + Ly*(z + Lz*t)), directions mu = 0..3 are x, y, z, t.
 *  On a lattice of extent 2 the forward and backward neighbours coincide and
 *  their contributions simply add, as in the coordinate-format product of the
 *  paper (Sec. 2), which sums duplicate entries.
 *
 * Sums are sequential in site order, FP64, no fused-multiply-add assumptions.
 * The operator's loop over sites may run on several host threads (OpenMP):
 * every site is computed by the same statements whichever thread runs it, so
 * the result does not depend on the thread count.  Dot products and norms stay
 * sequential.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* Host threads for the operator's site loop (n <= 0 leaves the setting);
 * returns the count now in force (1 without OpenMP). */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* gamma_mu[alpha][beta], DeGrand-Rossi basis */
static cplx G[4][4][4];
static int g_ready = 0;

static void init_gamma(void)
{
    if (g_ready) return;
    memset(G, 0, sizeof(G));
    /* gamma_x */
    G[0][0][3] = I;  G[0][1][2] = I;  G[0][2][1] = -I; G[0][3][0] = -I;
    /* gamma_y */
    G[1][0][3] = -1; G[1][1][2] = 1;  G[1][2][1] = 1;  G[1][3][0] = -1;
    /* gamma_z */
    G[2][0][2] = I;  G[2][1][3] = -I; G[2][2][0] = -I; G[2][3][1] = I;
    /* gamma_t */
    G[3][0][2] = 1;  G[3][1][3] = 1;  G[3][2][0] = 1;  G[3][3][1] = 1;
    g_ready = 1;
}

/* Copy of gamma_mu for the tests (row-major 4x4 complex). */
void oracle_gamma(int mu, cplx *out16)
{
    init_gamma();
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) out16[4 * a + b] = G[mu][a][b];
}

static long site_of(const int c[4], const int L[4])
{
    return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));
}

/*
 * out = D in   (dagger = 0)   or   out = D^dagger in   (dagger = 1).
 * U: [V][4][3][3], in/out: [V][4][3]; out must not alias in.
 */
void oracle_dirac(const cplx *U, const int L[4], int t_sign, double m0,
                  const cplx *in, cplx *out, int dagger)
{
    init_gamma();
    const long V = (long)L[0] * L[1] * L[2] * L[3];
    /* projector matrices P_fwd = 1 - sgn gamma, P_bwd = 1 + sgn gamma */
    const double sgn = dagger ? -1.0 : 1.0;
    cplx Pf[4][4][4], Pb[4][4][4];
    for (int mu = 0; mu < 4; ++mu)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                cplx id = (a == b) ? 1.0 : 0.0;
                Pf[mu][a][b] = id - sgn * G[mu][a][b];
                Pb[mu][a][b] = id + sgn * G[mu][a][b];
            }

#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; ++s) {
        int c[4];
        long rem = s;
        for (int d = 0; d < 4; ++d) { c[d] = (int)(rem % L[d]); rem /= L[d]; }

        cplx acc[4][3];
        memset(acc, 0, sizeof(acc));
        for (int mu = 0; mu < 4; ++mu) {
            /* forward neighbour */
            int cf[4] = {c[0], c[1], c[2], c[3]};
            cf[mu] = (c[mu] + 1) % L[mu];
            double sf = (mu == 3 && c[3] == L[3] - 1) ? (double)t_sign : 1.0;
            long nf = site_of(cf, L);
            /* backward neighbour */
            int cb[4] = {c[0], c[1], c[2], c[3]};
            cb[mu] = (c[mu] - 1 + L[mu]) % L[mu];
            double sb = (mu == 3 && c[3] == 0) ? (double)t_sign : 1.0;
            long nb = site_of(cb, L);

            const cplx *Uf = U + (s * 4 + mu) * 9;   /* U_mu(x)       */
            const cplx *Ub = U + (nb * 4 + mu) * 9;  /* U_mu(x - mu)  */
            const cplx *pf = in + nf * 12;
            const cplx *pb = in + nb * 12;

            /* colour first: v = U psi(x+mu), w = U^dagger psi(x-mu), per spin */
            cplx v[4][3], w[4][3];
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx tv = 0, tw = 0;
                    for (int b = 0; b < 3; ++b) {
                        tv += Uf[3 * a + b] * pf[3 * sp + b];
                        tw += conj(Ub[3 * b + a]) * pb[3 * sp + b];
                    }
                    v[sp][a] = sf * tv;
                    w[sp][a] = sb * tw;
                }
            /* then spin: acc += P_fwd v + P_bwd w */
            for (int al = 0; al < 4; ++al)
                for (int be = 0; be < 4; ++be) {
                    cplx f = Pf[mu][al][be], b = Pb[mu][al][be];
                    if (f == 0 && b == 0) continue;
                    for (int a = 0; a < 3; ++a) acc[al][a] += f * v[be][a] + b * w[be][a];
                }
        }
        const cplx *ps = in + s * 12;
        cplx *o = out + s * 12;
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a)
                o[3 * sp + a] = (4.0 + m0) * ps[3 * sp + a] - 0.5 * acc[sp][a];
    }
}

/* <a, b> = sum conj(a) b, sequential */
static cplx dotc(const cplx *a, const cplx *b, long n)
{
    cplx s = 0;
    for (long i = 0; i < n; ++i) s += conj(a[i]) * b[i];
    return s;
}

static double norm2(const cplx *a, long n)
{
    double s = 0;
    for (long i = 0; i < n; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

/* x = x + a*y */
static void axpy(cplx a, const cplx *y, cplx *x, long n)
{
    for (long i = 0; i < n; ++i) x[i] += a * y[i];
}

/* r = eta - D x */
static void residual(const cplx *U, const int L[4], int t_sign, double m0,
                     const cplx *eta, const cplx *x, cplx *r, cplx *tmp, long n)
{
    oracle_dirac(U, L, t_sign, m0, x, tmp, 0);
    for (long i = 0; i < n; ++i) r[i] = eta[i] - tmp[i];
}

/*
 * Conjugate gradient for D psi = eta through the normal equations.
 *  form 0 (CGNE): CG on D D^dagger chi = eta, psi = D^dagger chi, tracked in psi.
 *  form 1 (CGNR): CG on D^dagger D psi = D^dagger eta.
 * Stops when the recursively updated residual satisfies |r| <= tol |eta|, then
 * recomputes r = eta - D psi; if that true residual is still above the
 * threshold the iteration continues from it.
 * x: in = initial guess when use_x0 != 0, out = solution.
 * trace (may be NULL): |r|/|eta| after every iteration, up to max_iter entries.
 * Returns 0 on convergence, 1 if max_iter was reached, 2 on breakdown.
 */
int oracle_cg(const cplx *U, const int L[4], int t_sign, double m0,
              const cplx *eta, cplx *x, int use_x0, double tol, int max_iter,
              int form, int *iters_out, double *true_rel_res, double *trace)
{
    const long n = 12L * L[0] * L[1] * L[2] * L[3];
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *q = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    cplx *rh = malloc(sizeof(cplx) * n);
    int status = 1, it = 0;
    const double eta_norm = sqrt(norm2(eta, n));
    if (!use_x0) memset(x, 0, sizeof(cplx) * n);
    if (eta_norm == 0.0) {
        memset(x, 0, sizeof(cplx) * n);
        *iters_out = 0;
        *true_rel_res = 0.0;
        free(r); free(p); free(q); free(t); free(rh);
        return 0;
    }
    const double stop = tol * eta_norm;
    residual(U, L, t_sign, m0, eta, x, r, t, n);
    if (sqrt(norm2(r, n)) <= stop) {          /* the initial guess already solves it */
        max_iter = 0;
        status = 0;
    }

    if (form == 0) {
        /* CGNE: CG on A = D D^dagger with chi-space direction p, x = D^dagger chi */
        memcpy(p, r, sizeof(cplx) * n);
        double rho = norm2(r, n);
        while (it < max_iter) {
            oracle_dirac(U, L, t_sign, m0, p, q, 1);          /* q = D^dagger p   */
            double sigma = norm2(q, n);                         /* <p, A p>         */
            if (!(sigma > 0.0) || !isfinite(sigma)) { status = 2; break; }
            double alpha = rho / sigma;
            axpy(alpha, q, x, n);                               /* x += alpha D^+ p */
            oracle_dirac(U, L, t_sign, m0, q, t, 0);          /* t = A p          */
            axpy(-alpha, t, r, n);                              /* r -= alpha A p   */
            double rho_new = norm2(r, n);
            ++it;
            if (trace) trace[it - 1] = sqrt(rho_new) / eta_norm;
            if (sqrt(rho_new) <= stop) {
                residual(U, L, t_sign, m0, eta, x, r, t, n);
                rho_new = norm2(r, n);
                if (sqrt(rho_new) <= stop) { status = 0; break; }
            }
            double beta = rho_new / rho;
            for (long i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
            rho = rho_new;
        }
    } else {
        /* CGNR: CG on A = D^dagger D, b = D^dagger eta; r_hat = D^dagger r */
        oracle_dirac(U, L, t_sign, m0, r, rh, 1);
        memcpy(p, rh, sizeof(cplx) * n);
        double rho = norm2(rh, n);
        while (it < max_iter) {
            oracle_dirac(U, L, t_sign, m0, p, q, 0);          /* q = D p          */
            double sigma = norm2(q, n);
            if (!(sigma > 0.0) || !isfinite(sigma)) { status = 2; break; }
            double alpha = rho / sigma;
            axpy(alpha, p, x, n);
            axpy(-alpha, q, r, n);                              /* r = eta - D x    */
            double rn = norm2(r, n);
            ++it;
            if (trace) trace[it - 1] = sqrt(rn) / eta_norm;
            if (sqrt(rn) <= stop) {
                residual(U, L, t_sign, m0, eta, x, r, t, n);
                if (sqrt(norm2(r, n)) <= stop) { status = 0; break; }
            }
            oracle_dirac(U, L, t_sign, m0, r, rh, 1);          /* r_hat = D^+ r    */
            double rho_new = norm2(rh, n);
            double beta = rho_new / rho;
            for (long i = 0; i < n; ++i) p[i] = rh[i] + beta * p[i];
            rho = rho_new;
        }
    }
    residual(U, L, t_sign, m0, eta, x, r, t, n);
    *iters_out = it;
    *true_rel_res = sqrt(norm2(r, n)) / eta_norm;
    free(r); free(p); free(q); free(t); free(rh);
    return status;
}

/*
 * BiCGSTAB (van der Vorst, 1992) directly on D psi = eta -- one of the other
 * Krylov methods the paper lists (Sec. 1).  Shadow residual r_hat = r_0.
 * Stops when |r| <= tol |eta| holds for the recursive residual and then for
 * the recomputed true residual (otherwise continues from the true one).
 * Returns 0 on convergence, 1 at max_iter, 2 on breakdown (rho or <r_hat, v>
 * or <t, t> zero / not finite).
 */
int oracle_bicgstab(const cplx *U, const int L[4], int t_sign, double m0,
                    const cplx *eta, cplx *x, int use_x0, double tol, int max_iter,
                    int *iters_out, double *true_rel_res)
{
    const long n = 12L * L[0] * L[1] * L[2] * L[3];
    cplx *r = malloc(sizeof(cplx) * n), *rh = malloc(sizeof(cplx) * n);
    cplx *p = calloc(n, sizeof(cplx)), *v = calloc(n, sizeof(cplx));
    cplx *sv = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    int status = 1, it = 0;
    const double eta_norm = sqrt(norm2(eta, n));
    if (!use_x0) memset(x, 0, sizeof(cplx) * n);
    if (eta_norm == 0.0) {
        memset(x, 0, sizeof(cplx) * n);
        *iters_out = 0;
        *true_rel_res = 0.0;
        free(r); free(rh); free(p); free(v); free(sv); free(t);
        return 0;
    }
    const double stop = tol * eta_norm;
    residual(U, L, t_sign, m0, eta, x, r, t, n);
    if (sqrt(norm2(r, n)) <= stop) {
        max_iter = 0;
        status = 0;
    }
    memcpy(rh, r, sizeof(cplx) * n);
    cplx rho_old = 1.0, alpha = 1.0, omega = 1.0;
    while (it < max_iter) {
        const cplx rho = dotc(rh, r, n);
        if (rho == 0 || !isfinite(creal(rho)) || !isfinite(cimag(rho))) { status = 2; break; }
        const cplx beta = (rho / rho_old) * (alpha / omega);
        for (long i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        oracle_dirac(U, L, t_sign, m0, p, v, 0);               /* v = D p          */
        const cplx rhv = dotc(rh, v, n);
        if (rhv == 0 || !isfinite(creal(rhv))) { status = 2; break; }
        alpha = rho / rhv;
        for (long i = 0; i < n; ++i) sv[i] = r[i] - alpha * v[i];
        oracle_dirac(U, L, t_sign, m0, sv, t, 0);              /* t = D s          */
        const double tt = norm2(t, n);
        if (!(tt > 0.0) || !isfinite(tt)) { status = 2; break; }
        omega = dotc(t, sv, n) / tt;
        for (long i = 0; i < n; ++i) {
            x[i] += alpha * p[i] + omega * sv[i];
            r[i] = sv[i] - omega * t[i];
        }
        rho_old = rho;
        ++it;
        if (sqrt(norm2(r, n)) <= stop) {
            residual(U, L, t_sign, m0, eta, x, r, t, n);
            if (sqrt(norm2(r, n)) <= stop) { status = 0; break; }
        }
    }
    residual(U, L, t_sign, m0, eta, x, r, t, n);
    *iters_out = it;
    *true_rel_res = sqrt(norm2(r, n)) / eta_norm;
    free(r); free(rh); free(p); free(v); free(sv); free(t);
    return status;
}

/* <a, b> over n complex numbers, exported for tests of the reductions. */
void oracle_dotc(const cplx *a, const cplx *b, long n, cplx *out) { *out = dotc(a, b, n); }
