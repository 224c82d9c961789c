// Device side of BiCGSTAB on D itself -- one of the other Krylov methods the
// paper lists for the Dirac equation (arXiv 2111.14958, Sec. 1) -- on the same
// machinery as the CG: per-field scalars in device memory, fixed-order
// last-block reductions, the FP64 reliable update R1/R2 of cg_core.h.
//
// One iteration (van der Vorst's BiCGSTAB, shadow residual r_hat):
//   S1  p = r + beta (p - omega v)        (p = r, r_hat = r after a restart)
//   S2  v = D p,        <r_hat, v>  -> alpha = rho / <r_hat, v>
//   S3  s = r - alpha v
//   S4  t = D s,        <t, s>, <t, t>  -> omega = <t, s> / <t, t>
//   S5  x += alpha p + omega s, r = s - omega t,
//       <r_hat, r>, |r|^2  -> rho, beta = (rho / rho_old)(alpha / omega), tests
// <a, b> = sum conj(a) b.  A reliable update restarts with r_hat = r = eta - D x;
// a (near) breakdown |<r_hat, r>| <= 1e-6 |r_hat| |r| restarts with r_hat = r.
#pragma once

#include "cg_core.h"

namespace wd {

struct dc { double re, im; };
__device__ __forceinline__ dc dmul(dc a, dc b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ dc ddiv(dc a, dc b) {
    const double d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ __forceinline__ bool dfinite(dc a) { return a.re == a.re && a.im == a.im && fabs(a.re) < 1e300 && fabs(a.im) < 1e300; }
__device__ __forceinline__ dc ld(const double v[2]) { return {v[0], v[1]}; }
__device__ __forceinline__ void st(double v[2], dc a) { v[0] = a.re; v[1] = a.im; }

// ------------------------------------------------------------- S1, streaming
template <int P>
__device__ __forceinline__ void bi1_tile(const Prob &pr, int t) {
    typedef typename real_of<P>::type R;
    const int sb = t / pr.nrhs, i = t - sb * pr.nrhs;
    const int s = sb * blockDim.x + threadIdx.x;
    const Scal &c = pr.sc[i];
    if (c.state != ST_ACTIVE || !c.pending_p || s >= pr.g.V) return;
    FieldPtr fr{pr.r, pr.g.V, pr.nrhs}, fp{pr.p, pr.g.V, pr.nrhs};
    cx<R> r[12];
    Spinor<P>::load(fr, i, s, r);
    if (c.restart) {
        FieldPtr fh{pr.rh, pr.g.V, pr.nrhs};
        cx<R> rr[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) rr[k] = r[k];
        Spinor<P>::store(fh, i, s, rr);
        Spinor<P>::store(fp, i, s, r);
        return;
    }
    FieldPtr fv{pr.v, pr.g.V, pr.nrhs};
    const dc b = ld(pr.bs[i].beta), w = ld(pr.bs[i].omega);
    const R br = (R)b.re, bi = (R)b.im, wr = (R)w.re, wi = (R)w.im;
    cx<R> p[12], v[12];
    Spinor<P>::load(fp, i, s, p);
    Spinor<P>::load(fv, i, s, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        // d = p - omega v ; p = r + beta d
        const cx<R> d = {p[k].re - (wr * v[k].re - wi * v[k].im), p[k].im - (wr * v[k].im + wi * v[k].re)};
        p[k] = {r[k].re + (br * d.re - bi * d.im), r[k].im + (br * d.im + bi * d.re)};
    }
    Spinor<P>::store(fp, i, s, p);
}

// ------------------------------------------- S2 / S4, stencil plus reductions
// S2: out = v = D p, partials <r_hat, v> (2 numbers).
// S4: out = t = D s, partials <t, s> (2) and <t, t> (1).
// XY: one xy-plane per block, its input spinors staged in LDS (the x and y
// hops and the site's own spinor read them there); ORD: hop order as in the
// CG phases (5 = the memory hops z and t first); R12: links from the
// reconstruct-12 copy.
template <int P, int NR, bool S4, int ORD = 1, bool XY = false, bool R12 = false>
__device__ __forceinline__ void bi_stencil_tile(const Prob &pr, int t) {
    typedef typename real_of<P>::type R;
    typedef typename LdsSpinor<P>::word W;
    __shared__ W xy[XY ? NR * LdsWords<P>::value * 256 : 1];
    const int K = S4 ? KS4 : KS2;
    int sb, grp, s;
    stencil_tile<XY>(pr, K, t, sb, grp, s);
    const int rhs0 = grp * NR;
    const unsigned act = rhs_mask<NR>(pr, rhs0, ST_ACTIVE);
    double part[3 * NR];
#pragma unroll
    for (int j = 0; j < 3 * NR; ++j) part[j] = 0.0;
    const Geom g = pr.g;
    const int np = g.S[2];   // sites of a plane
    FieldPtr fin{S4 ? pr.sv : pr.p, g.V, pr.nrhs}, fout{S4 ? pr.tv : pr.v, g.V, pr.nrhs};
    if (XY && act) stage_plane<P, NR>(fin, rhs0, act, s, g.V, xy, np);   // act is uniform over the block
    if (act && s < g.V) {
        FieldPtr fh{pr.rh, g.V, pr.nrhs};
        const void *U = R12 ? pr.U12 : pr.U_lo;
        cx<R> acc[NR][12];
        hopping<P, false, NR, ORD, XY, false, false, R12>(g, s, U, fin, rhs0, act, acc, nullptr, xy,
                                                          s - (int)threadIdx.x, np);
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (act >> j & 1) {
                cx<R> self[12], o[12], a[12];
                if constexpr (XY) LdsSpinor<P>::get(xy, np, j, threadIdx.x, self);
                else Spinor<P>::load(fin, rhs0 + j, s, self);
                wilson_finish<R>((R)pr.diag, self, acc[j], o);
                Spinor<P>::store(fout, rhs0 + j, s, o);
                if (S4) {
#pragma unroll
                    for (int k = 0; k < 12; ++k) a[k] = self[k];   // s
                } else {
                    Spinor<P>::load(fh, rhs0 + j, s, a);            // r_hat
                }
                double re = 0, im = 0, nn = 0;
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    if (S4) {   // <t, s> = sum conj(t) s
                        re += (double)o[k].re * a[k].re + (double)o[k].im * a[k].im;
                        im += (double)o[k].re * a[k].im - (double)o[k].im * a[k].re;
                        nn += (double)norm2(o[k]);
                    } else {    // <r_hat, v> = sum conj(r_hat) v
                        re += (double)a[k].re * o[k].re + (double)a[k].im * o[k].im;
                        im += (double)a[k].re * o[k].im - (double)a[k].im * o[k].re;
                    }
                }
                part[3 * j] = re;
                part[3 * j + 1] = im;
                part[3 * j + 2] = nn;
            }
        }
    }
    if (act) {
        block_sum<3 * NR>(part);
        if (threadIdx.x == 0)
#pragma unroll
            for (int j = 0; j < NR; ++j)
                if (act >> j & 1)
                    for (int k = 0; k < 3; ++k) part_at(pr, sb, rhs0 + j, k) = part[3 * j + k];
    }
}

__device__ __forceinline__ void bi2_finish(const Prob &pr) {
    __shared__ double sums[MAX_SUMS];
    sum_all(pr, pr.nsb[KS2], 2, sums);
    for (int i = threadIdx.x; i < pr.nrhs; i += blockDim.x) {
        Scal &c = pr.sc[i];
        if (c.state == ST_ACTIVE) {
            const dc rv = {sums[2 * i], sums[2 * i + 1]};
            if (!dfinite(rv) || (rv.re == 0.0 && rv.im == 0.0)) c.state = ST_BREAKDOWN;
            else st(pr.bs[i].alpha, ddiv(ld(pr.bs[i].rho), rv));
        }
        c.pending_p = 0;
        c.restart = 0;
    }
}

__device__ __forceinline__ void bi4_finish(const Prob &pr) {
    __shared__ double sums[MAX_SUMS];
    sum_all(pr, pr.nsb[KS4], 3, sums);
    for (int i = threadIdx.x; i < pr.nrhs; i += blockDim.x) {
        Scal &c = pr.sc[i];
        if (c.state != ST_ACTIVE) continue;
        const double re = sums[3 * i], im = sums[3 * i + 1], tt = sums[3 * i + 2];
        {
            const dc w = {re / tt, im / tt};
            if (!finite_pos(tt) || !dfinite(w) || (w.re == 0.0 && w.im == 0.0)) c.state = ST_BREAKDOWN;
            else st(pr.bs[i].omega, w);
        }
    }
}

// ------------------------------------------------------------- S3, streaming
template <int P>
__device__ __forceinline__ void bi3_tile(const Prob &pr, int t) {
    typedef typename real_of<P>::type R;
    const int sb = t / pr.nrhs, i = t - sb * pr.nrhs;
    const int s = sb * blockDim.x + threadIdx.x;
    if (pr.sc[i].state != ST_ACTIVE || s >= pr.g.V) return;
    FieldPtr fr{pr.r, pr.g.V, pr.nrhs}, fv{pr.v, pr.g.V, pr.nrhs}, fs{pr.sv, pr.g.V, pr.nrhs};
    const dc a = ld(pr.bs[i].alpha);
    const R ar = (R)a.re, ai = (R)a.im;
    cx<R> r[12], v[12];
    Spinor<P>::load(fr, i, s, r);
    Spinor<P>::load(fv, i, s, v);
#pragma unroll
    for (int k = 0; k < 12; ++k)
        r[k] = {r[k].re - (ar * v[k].re - ai * v[k].im), r[k].im - (ar * v[k].im + ai * v[k].re)};
    Spinor<P>::store(fs, i, s, r);
}

// ------------------------------------------------- S5, streaming + reductions
// x_lo += alpha p + omega s ; r = s - omega t ; partials <r_hat, r>, |r|^2
template <int P>
__device__ __forceinline__ void bi5_tile(const Prob &pr, int t) {
    typedef typename real_of<P>::type R;
    constexpr int XP = XPrec<P>::value;
    typedef typename real_of<XP>::type RX;
    const int sb = t / pr.nrhs, i = t - sb * pr.nrhs;
    const int s = sb * blockDim.x + threadIdx.x;
    if (pr.sc[i].state != ST_ACTIVE) return;   // uniform over the block
    double part[3] = {0.0, 0.0, 0.0};
    if (s < pr.g.V) {
        FieldPtr fp{pr.p, pr.g.V, pr.nrhs}, fs{pr.sv, pr.g.V, pr.nrhs}, ft{pr.tv, pr.g.V, pr.nrhs};
        FieldPtr fr{pr.r, pr.g.V, pr.nrhs}, fh{pr.rh, pr.g.V, pr.nrhs}, fx{pr.x_lo, pr.g.V, pr.nrhs};
        const dc a = ld(pr.bs[i].alpha), w = ld(pr.bs[i].omega);
        cx<R> p[12], sv[12], tv[12], h[12];
        cx<RX> x[12];
        Spinor<P>::load(fp, i, s, p);
        Spinor<P>::load(fs, i, s, sv);
        Spinor<P>::load(ft, i, s, tv);
        Spinor<XP>::load(fx, i, s, x);
        const RX axr = (RX)a.re, axi = (RX)a.im, wxr = (RX)w.re, wxi = (RX)w.im;
        const R wr = (R)w.re, wi = (R)w.im;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const RX pr_ = (RX)p[k].re, pi_ = (RX)p[k].im, sr = (RX)sv[k].re, si = (RX)sv[k].im;
            x[k] = {x[k].re + (axr * pr_ - axi * pi_) + (wxr * sr - wxi * si),
                    x[k].im + (axr * pi_ + axi * pr_) + (wxr * si + wxi * sr)};
            p[k] = {sv[k].re - (wr * tv[k].re - wi * tv[k].im), sv[k].im - (wr * tv[k].im + wi * tv[k].re)};
        }
        Spinor<XP>::store(fx, i, s, x);
        Spinor<P>::store(fr, i, s, p);     // the new residual (stored values)
        Spinor<P>::load(fh, i, s, h);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            part[0] += (double)h[k].re * p[k].re + (double)h[k].im * p[k].im;
            part[1] += (double)h[k].re * p[k].im - (double)h[k].im * p[k].re;
            part[2] += (double)norm2(p[k]);
        }
    }
    block_sum<3>(part);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) part_at(pr, sb, i, k) = part[k];
}

__device__ __forceinline__ void bi5_finish(const Prob &pr) {
    __shared__ double sums[MAX_SUMS];
    sum_all(pr, pr.nsb[KS5], 3, sums);
    for (int i = threadIdx.x; i < pr.nrhs; i += blockDim.x) {
        Scal &c = pr.sc[i];
        if (c.state != ST_ACTIVE) continue;
        const double re = sums[3 * i], im = sums[3 * i + 1], r2 = sums[3 * i + 2];
        {
            BScal &b = pr.bs[i];
            const dc rho_new = {re, im};
            st(b.rho_old, ld(b.rho));
            st(b.rho, rho_new);
            st(b.beta, dmul(ddiv(rho_new, ld(b.rho_old)), ddiv(ld(b.alpha), ld(b.omega))));
            c.rho = r2;
            c.iters += 1;
            c.since_ru += 1;
            if (!(r2 < 1e300) || !dfinite(rho_new)) c.state = ST_BREAKDOWN;
            else if (r2 <= c.stop2 || c.iters >= pr.max_iter ||
                     (pr.ru_every > 0 && c.since_ru >= pr.ru_every))
                c.state = ST_FROZEN;
            else {
                // (near) breakdown, <r_hat, r> ~ 0: restart in place with
                // r_hat = p = r (the iterated residual), rho = |r|^2.  A point
                // source meets it after one iteration: with r_hat = r0 = e_k, s
                // has no component along e_k and, since (1 - gamma)(1 + gamma) = 0,
                // neither has t = D s.
                if (rho_new.re * rho_new.re + rho_new.im * rho_new.im <= 1e-12 * b.rh2 * r2) {
                    c.restart = 1;
                    b.rho[0] = r2;
                    b.rho[1] = 0.0;
                    b.rh2 = r2;
                }
                c.pending_p = 1;
            }
        }
    }
}

}  // namespace wd
