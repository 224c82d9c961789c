// Even-odd preconditioned CG (device side).
//
// Eq. (1) splits by site parity into D = [[A, D_eo], [D_oe, A]] with the
// diagonal A = 4 + m0 and the hopping blocks D_eo = -H_eo / 2, D_oe = -H_oe / 2
// (H: the hopping sum, which always joins sites of opposite parity).
// Eliminating the odd sites leaves the Schur complement on the even sites,
//     Dhat = A - D_eo A^-1 D_oe = A - c H_eo H_oe,   c = 1 / (4 A),
// with Dhat^dagger = A - c H^dagger_eo H^dagger_oe.  The CG of cg_core.h runs
// unchanged on Dhat, with every vector on the even sites only (half length):
//     b_e = eta_e - D_eo A^-1 eta_o = eta_e + H_eo eta_o / (2 A)
//     CG on Dhat Dhat^dagger, x_e = Dhat^dagger chi, until |b_e - Dhat x_e| <= tol |eta|
//     x_o = A^-1 (eta_o - D_oe x_e) = (eta_o + H_oe x_e / 2) / A
// eta - D x is then zero on the odd sites and b_e - Dhat x_e on the even ones.
// A Schur application is two half-lattice hops: the first writes the
// odd-site intermediate, the second gathers it back onto the even sites and
// applies the epilogue of the phase.
//
// Half-lattice vectors keep the packed layouts of the full ones with V/2
// sites: site n of a parity is stored at index n / 2 (Lx must be even, so the
// two sites 2k, 2k+1 have opposite parities).
#pragma once

#include "cg_core.h"

namespace wd {

// site of parity `par` stored at half index k
__device__ __forceinline__ int eo_site(const Geom &g, int k, int par) {
    int c[4];
    site_coords(g, 2 * k, c);   // x of site 2k is even
    return 2 * k + ((c[1] + c[2] + c[3] + par) & 1);
}

// tile t of an even-odd kind: site block and rhs group; k = half index or vf.
// XY: a site block is the Lx Ly / 2 sites of one parity on an xy-plane, whose
// half indices are consecutive (so are the other parity's on that plane: the
// x and y neighbours of the block's sites).
template <bool XY = false>
__device__ __forceinline__ void eo_tile(const Prob &pr, int K, int t, int &sb, int &grp, int &k) {
    sb = t / pr.ng[K];
    grp = t - sb * pr.ng[K];
    const int rows = XY ? pr.g.S[2] >> 1 : (int)blockDim.x;
    const int L = sb * rows + (int)threadIdx.x;
    k = ((int)threadIdx.x < rows && L < pr.vf) ? L : pr.vf;
}

// XY: stage the half-plane of the hop's input field (the other parity's sites
// on the block's xy-plane) in LDS; every thread of the block calls it.
template <int P, int NR, bool XY>
__device__ __forceinline__ void eo_stage(const Prob &pr, const FieldPtr &in, int rhs0, unsigned act, int k,
                                         typename LdsSpinor<P>::word *xy) {
    if constexpr (XY) stage_plane<P, NR>(in, rhs0, act, k, pr.vf, xy, pr.g.S[2] >> 1);
}

// First half hop, onto the odd sites: tmp_o = H_oe v_e (H^dagger with DAG).
// v: p for phase A (DAG), q for phase B.  QR: phase A hops r, as it forms the
// direction as q = Dhat^dagger r + beta q (see phaseA_tile).  R12 (here and in
// the second halves of phases A and B): links from the reconstruct-12 copy.
// XY (here and there): half-plane blocks, the x and y neighbours from LDS, hop
// order 5 (z and t first); one rhs per thread.
template <int P, int NR, bool DAG, bool QR = false, bool R12 = false, bool XY = false>
__device__ __forceinline__ void eo_hop1_tile(const Prob &pr, int t) {
    typedef typename real_of<P>::type R;
    typedef typename LdsSpinor<P>::word W;
    extern __shared__ uint4 eo_lds[];   // XY: the half-plane, sized at launch
    W *xy = (W *)eo_lds;
    constexpr int K = DAG ? KEA1 : KEB1;
    int sb, grp, k;
    eo_tile<XY>(pr, K, t, sb, grp, k);
    const int rhs0 = grp * NR;
    const unsigned act = rhs_mask<NR>(pr, rhs0, ST_ACTIVE);
    if (!act) return;   // uniform over the block
    FieldPtr fin{DAG ? (QR ? pr.r : pr.p) : pr.q, pr.vf, pr.nrhs}, fo{pr.tmp, pr.vf, pr.nrhs};
    eo_stage<P, NR, XY>(pr, fin, rhs0, act, k, xy);
    if (k >= pr.vf) return;
    const Geom g = pr.g;
    const int s = eo_site(g, k, 1);
    cx<R> acc[NR][12];
    hopping<P, DAG, NR, XY ? 5 : 1, XY, true, false, R12>(g, s, R12 ? pr.U12 : pr.U_lo, fin, rhs0, act, acc,
                                                          nullptr, xy, k - (int)threadIdx.x, g.S[2] >> 1);
#pragma unroll
    for (int j = 0; j < NR; ++j)
        if (act >> j & 1) Spinor<P>::store(fo, rhs0 + j, k, acc[j]);
}

// Phase A, second half: q_e = A p_e - c H^dagger_eo tmp_o, partial |q|^2.
// QR: with r in place of p, plus beta times the old q_e (not after a restart).
template <int P, int NR, bool QR = false, bool R12 = false, bool XY = false>
__device__ __forceinline__ void eo_phaseA_tile(const Prob &pr, int t) {
    typedef typename real_of<P>::type R;
    typedef typename LdsSpinor<P>::word W;
    extern __shared__ uint4 eo_lds[];   // XY: the half-plane, sized at launch
    W *xy = (W *)eo_lds;
    int sb, grp, k;
    eo_tile<XY>(pr, KA, t, sb, grp, k);
    const int rhs0 = grp * NR;
    const unsigned act = rhs_mask<NR>(pr, rhs0, ST_ACTIVE);
    double part[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) part[j] = 0.0;
    FieldPtr ft{pr.tmp, pr.vf, pr.nrhs};
    if (act) eo_stage<P, NR, XY>(pr, ft, rhs0, act, k, xy);
    if (act && k < pr.vf) {
        const Geom g = pr.g;
        const int s = eo_site(g, k, 0);
        FieldPtr fp{QR ? pr.r : pr.p, pr.vf, pr.nrhs}, fq{pr.q, pr.vf, pr.nrhs};
        cx<R> acc[NR][12];
        hopping<P, true, NR, XY ? 5 : 1, XY, true, false, R12>(g, s, R12 ? pr.U12 : pr.U_lo, ft, rhs0, act, acc,
                                                               nullptr, xy, k - (int)threadIdx.x, g.S[2] >> 1);
        const R a = (R)pr.diag, c = (R)pr.eo_c;
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (act >> j & 1) {
                cx<R> v[12], o[12];
                Spinor<P>::load(fp, rhs0 + j, k, v);
#pragma unroll
                for (int m = 0; m < 12; ++m) o[m] = {fma(-c, acc[j][m].re, a * v[m].re), fma(-c, acc[j][m].im, a * v[m].im)};
                if constexpr (QR) {
                    const Scal &sc = pr.sc[rhs0 + j];
                    if (!sc.restart) {
                        const R b = (R)sc.beta;
                        cx<R> qo[12];
                        Spinor<P>::load(fq, rhs0 + j, k, qo);
#pragma unroll
                        for (int m = 0; m < 12; ++m) o[m] = {o[m].re + b * qo[m].re, o[m].im + b * qo[m].im};
                    }
                }
                Spinor<P>::store(fq, rhs0 + j, k, o);
                double n = 0;
#pragma unroll
                for (int m = 0; m < 12; ++m) n += (double)norm2(o[m]);
                part[j] = n;
            }
        }
    }
    if (act) {
        block_sum<NR>(part);
        if (threadIdx.x == 0)
#pragma unroll
            for (int j = 0; j < NR; ++j)
                if (act >> j & 1) part_at(pr, sb, rhs0 + j, 0) = part[j];
    }
}

// Phase B, second half: t_e = A q_e - c H_eo tmp_o; r -= alpha t; x_lo += alpha q;
// partial |r|^2
template <int P, int NR, bool R12 = false, bool XY = false>
__device__ __forceinline__ void eo_phaseB_tile(const Prob &pr, int t) {
    typedef typename real_of<P>::type R;
    constexpr int XP = XPrec<P>::value;
    typedef typename real_of<XP>::type RX;
    typedef typename LdsSpinor<P>::word W;
    extern __shared__ uint4 eo_lds[];   // XY: the half-plane, sized at launch
    W *xy = (W *)eo_lds;
    int sb, grp, k;
    eo_tile<XY>(pr, KB, t, sb, grp, k);
    const int rhs0 = grp * NR;
    const unsigned act = rhs_mask<NR>(pr, rhs0, ST_ACTIVE);
    double part[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) part[j] = 0.0;
    FieldPtr ft{pr.tmp, pr.vf, pr.nrhs};
    if (act) eo_stage<P, NR, XY>(pr, ft, rhs0, act, k, xy);
    if (act && k < pr.vf) {
        const Geom g = pr.g;
        const int s = eo_site(g, k, 0);
        FieldPtr fq{pr.q, pr.vf, pr.nrhs}, fr{pr.r, pr.vf, pr.nrhs}, fx{pr.x_lo, pr.vf, pr.nrhs};
        cx<R> acc[NR][12];
        hopping<P, false, NR, XY ? 5 : 1, XY, true, false, R12>(g, s, R12 ? pr.U12 : pr.U_lo, ft, rhs0, act, acc,
                                                                nullptr, xy, k - (int)threadIdx.x, g.S[2] >> 1);
        const R a = (R)pr.diag, c = (R)pr.eo_c;
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (act >> j & 1) {
                const R al = (R)pr.sc[rhs0 + j].alpha;
                cx<R> q[12], r[12];
                Spinor<P>::load(fq, rhs0 + j, k, q);
                Spinor<P>::load(fr, rhs0 + j, k, r);
#pragma unroll
                for (int m = 0; m < 12; ++m) {
                    const cx<R> tt = {fma(-c, acc[j][m].re, a * q[m].re), fma(-c, acc[j][m].im, a * q[m].im)};
                    r[m] = {r[m].re - al * tt.re, r[m].im - al * tt.im};
                }
                Spinor<P>::store(fr, rhs0 + j, k, r);
                double n = 0;
#pragma unroll
                for (int m = 0; m < 12; ++m) n += (double)norm2(r[m]);
                part[j] = n;
                cx<RX> x[12];
                Spinor<XP>::load(fx, rhs0 + j, k, x);
                const RX ax = (RX)pr.sc[rhs0 + j].alpha;
#pragma unroll
                for (int m = 0; m < 12; ++m) x[m] = {x[m].re + ax * (RX)q[m].re, x[m].im + ax * (RX)q[m].im};
                Spinor<XP>::store(fx, rhs0 + j, k, x);
            }
        }
    }
    if (act) {
        block_sum<NR>(part);
        if (threadIdx.x == 0)
#pragma unroll
            for (int j = 0; j < NR; ++j)
                if (act >> j & 1) part_at(pr, sb, rhs0 + j, 0) = part[j];
    }
}

// Reliable update, first half (FP64, fields that are frozen): w_o = H_oe x64_e
template <int NR>
__device__ __forceinline__ void eo_ru2a_tile(const Prob &pr, int t) {
    int sb, grp, k;
    eo_tile(pr, KER2A, t, sb, grp, k);
    const int rhs0 = grp * NR;
    const unsigned act = rhs_mask<NR>(pr, rhs0, ST_FROZEN);
    if (!act || k >= pr.vf) return;
    const Geom g = pr.g;
    const int s = eo_site(g, k, 1);
    FieldPtr fx{pr.x64, pr.vf, pr.nrhs}, fw{pr.w64, pr.vf, pr.nrhs};
    cx<double> acc[NR][12];
    hopping<P64, false, NR, 1, false, true>(g, s, pr.U64, fx, rhs0, act, acc);
#pragma unroll
    for (int j = 0; j < NR; ++j)
        if (act >> j & 1) Spinor<P64>::store(fw, rhs0 + j, k, acc[j]);
}

// Reliable update, second half: r = b - (A x64 - c H_eo w_o) in FP64, stored
// in the inner precision; partial |r|^2 in FP64 (frozen fields)
template <int P, int NR>
__device__ __forceinline__ void eo_ru2b_tile(const Prob &pr, int t) {
    typedef typename real_of<P>::type R;
    int sb, grp, k;
    eo_tile(pr, KR2, t, sb, grp, k);
    const int rhs0 = grp * NR;
    const unsigned act = rhs_mask<NR>(pr, rhs0, ST_FROZEN);
    double part[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) part[j] = 0.0;
    if (act && k < pr.vf) {
        const Geom g = pr.g;
        const int s = eo_site(g, k, 0);
        FieldPtr fw{pr.w64, pr.vf, pr.nrhs}, fx{pr.x64, pr.vf, pr.nrhs}, fb{pr.eta64, pr.vf, pr.nrhs},
            fr{pr.r, pr.vf, pr.nrhs};
        cx<double> acc[NR][12];
        hopping<P64, false, NR, 1, false, true>(g, s, pr.U64, fw, rhs0, act, acc);
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (act >> j & 1) {
                cx<double> x[12], b[12];
                Spinor<P64>::load(fx, rhs0 + j, k, x);
                Spinor<P64>::load(fb, rhs0 + j, k, b);
                cx<R> rl[12];
                double n = 0;
#pragma unroll
                for (int m = 0; m < 12; ++m) {
                    const cx<double> d = {b[m].re - (pr.diag * x[m].re - pr.eo_c * acc[j][m].re),
                                          b[m].im - (pr.diag * x[m].im - pr.eo_c * acc[j][m].im)};
                    n += norm2(d);
                    rl[m] = {(R)d.re, (R)d.im};
                }
                Spinor<P>::store(fr, rhs0 + j, k, rl);
                part[j] = n;
            }
        }
    }
    if (act) {
        block_sum<NR>(part);
        if (threadIdx.x == 0)
#pragma unroll
            for (int j = 0; j < NR; ++j)
                if (act >> j & 1) part_at(pr, sb, rhs0 + j, 0) = part[j];
    }
}

// Source of the Schur system (FP64, every field): b_e = eta_e + H_eo eta_o / (2 A),
// written over eta_e.  Tile = (site block, rhs).
__device__ __forceinline__ void eo_source_tile(const Prob &pr, int t) {
    const int sb = t / pr.nrhs, i = t - sb * pr.nrhs;
    const int k = sb * (int)blockDim.x + (int)threadIdx.x;
    if (k >= pr.vf) return;
    const Geom g = pr.g;
    const int s = eo_site(g, k, 0);
    FieldPtr fo{pr.eta_o, pr.vf, pr.nrhs}, fe{pr.eta64, pr.vf, pr.nrhs};
    cx<double> acc[1][12], e[12];
    hopping<P64, false, 1, 1, false, true>(g, s, pr.U64, fo, i, 1u, acc);
    Spinor<P64>::load(fe, i, k, e);
    const double h = 0.5 / pr.diag;
#pragma unroll
    for (int m = 0; m < 12; ++m) e[m] = {fma(h, acc[0][m].re, e[m].re), fma(h, acc[0][m].im, e[m].im)};
    Spinor<P64>::store(fe, i, k, e);
}

}  // namespace wd
