// Device side of the conjugate-gradient solver (arXiv 2111.14958, Sec. 2).
//
// The paper's CG on D D^dagger chi = eta, psi = D^dagger chi, is carried in the
// solution space (x = D^dagger chi):
//     q = D^dagger p;  alpha = rho / |q|^2;  x += alpha q;  r -= alpha D q;
//     rho' = |r|^2;    beta = rho' / rho;    p = r + beta p
// so r is the residual of D x = eta itself.  The direction is kept as its
// image q alone (q' = D^dagger r + beta q equals D^dagger p'), and one
// iteration is two phases:
//     A  q = D^dagger r + beta q           + partial sums of |q|^2   -> alpha
//     B  t = D q, r -= alpha t, x += alpha q + partial sums of |r|^2   -> beta
// (phase C, p = r + beta p, with phase A reading p, remains for the z-marching
// phase-A kernel).  Every scalar lives in device memory, one record per
// right-hand side.  Phase B's blocks complete phase A's reduction themselves,
// and a one-block launch after phase B sums the per-block partials of both in
// a fixed order and updates the scalars, so nothing returns to the host inside
// an iteration and reductions are bitwise reproducible.
//
// Mixed precision: q, r, x_lo (and p) are stored in the inner precision (FP16N
// keeps x_lo in FP32).  A reliable update (R1, R2) accumulates x64 += x_lo and
// recomputes r = eta - D x64 with FP64 links and FP64 arithmetic; the solve
// ends only when that true residual satisfies |r| <= tol |eta|.
#pragma once

#include "wd_device.h"

namespace wd {

// per right-hand-side state
enum : int { ST_ACTIVE = 0, ST_FROZEN = 1, ST_DONE = 2, ST_BREAKDOWN = 3, ST_NOTCONV = 4 };
// kernel kinds: phase A, phase B, phase C, reliable update R1 (x64 += x_lo),
// reliable update R2 (r = eta - D x64), source norm N, and the five BiCGSTAB
// stages S1 (p update), S2 (v = D p), S3 (s = r - alpha v), S4 (t = D s),
// S5 (x and r updates)
// With even-odd preconditioning (eo_core.h) A, B and R2 apply the Schur
// complement in two half-lattice hops: EA1, EB1 and ER2A are the first ones.
enum : int { KA = 0, KB = 1, KC = 2, KR1 = 3, KR2 = 4, KN = 5,
             KS1 = 6, KS2 = 7, KS3 = 8, KS4 = 9, KS5 = 10,
             KEA1 = 11, KEB1 = 12, KER2A = 13, NKIND = 14 };
enum : int { METHOD_CGNE = 0, METHOD_BICGSTAB = 1 };
// doubles per (site block, rhs) partial-sum entry (complex dot products need
// up to three numbers)
constexpr int PSTRIDE = 4;

struct alignas(16) Scal {
    double rho;       // |r|^2 of the current residual
    double rho_old;   // previous rho, for beta
    double alpha, beta, sigma;
    double eta2;      // |eta|^2
    double stop2;     // (tol |eta|)^2
    double true2;     // last true residual |eta - D x64|^2
    int state;        // ST_*
    int iters;        // CG iterations done
    int since_ru;     // iterations since the last reliable update
    int n_ru;         // reliable updates done
    int pending_p;    // 1: phase C must rebuild p for this rhs
    int restart;      // 1: the next direction is p = r
    int zero_src;     // 1: eta == 0, the solution is 0
    int pad;
};

// complex scalars of BiCGSTAB, one record per right-hand side
struct alignas(16) BScal {
    double rho[2], rho_old[2], alpha[2], omega[2], beta[2];
    double rh2;       // |r_hat|^2, set when r_hat is chosen
    double pad;
};

struct alignas(16) Prob {
    Geom g;
    double diag;      // 4 + m0
    double tol2;
    int nrhs, max_iter, ru_every, method;
    int eo;           // 1: even-odd preconditioned (vectors live on the even sites)
    int vf;           // sites of a vector: V, or V/2 with even-odd
    double eo_c;      // 1 / (4 diag): Dhat = diag - eo_c H_eo H_oe
    int nsb[NKIND];   // site blocks per kernel kind
    int ng[NKIND];    // rhs groups per kernel kind
    int t0[NKIND];    // first tile of this problem in a grouped launch
    int nt[NKIND];    // tiles of this problem
    int sorder[NKIND];  // stencil kinds: strip | group-major << 16 | plane-blocked << 17
                        // | planes per block << 18 | rhs passes << 24 (see stencil_tile)
    const void *U_lo; // links in the inner precision
    const void *U12;  // reconstruct-12 copy in the inner precision, or null
    const void *U64;  // FP64 links
    void *x_lo, *r, *p, *q;   // inner-precision vectors (x_lo: FP32 for FP16N)
    void *x64, *eta64;        // FP64 packed vectors
    double *part;             // [PSTRIDE][nrhs][psb] partial sums: column (slot, field) holds the
                              // site blocks' partials one after the other
    int psb;                  // site blocks a column has room for ((V + 63) / 64)
    Scal *sc;                 // [nrhs]
    Scal *sc2;                // [nrhs] second record per field: with the fused finish, the phase-A
                              // launches of a chunk read one and write the other (iteration parity)
    void *rh, *v, *sv, *tv;   // BiCGSTAB: shadow residual r_hat, v = D p, s, t = D s
    BScal *bs;                // BiCGSTAB scalars [nrhs]
    void *eta_o;              // even-odd: odd half of the source (FP64)
    void *tmp;                // even-odd: odd-site intermediate of A and B (inner precision)
    void *w64;                // even-odd: odd-site intermediate of R2 (FP64)
};

// NT (phase tiles): the streaming accesses (fields each thread reads or writes
// once) carry the nontemporal hint.  The host sets it for FP64 solves whose
// fields exceed the 256 MB MALL: there the L2 then keeps more of the
// neighbouring input planes and phases A, B and C ran 5-9 % faster (14^4, 16
// rhs), while a single FP64 field, which the MALL holds, ran 6 % slower with
// it, and FP32/FP16 storage 13-23 % slower.

// precision x_lo is stored in
template <int P> struct XPrec { static constexpr int value = P; };
template <> struct XPrec<P16> { static constexpr int value = P32; };

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Sum v[j] over the block (at most 1024 threads) in a fixed order; result
// valid on thread 0.
template <int NR>
__device__ __forceinline__ void block_sum(double v[NR]) {
    __shared__ double red[16][NR > 0 ? NR : 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NR; ++j) v[j] = wave_sum(v[j]);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < NR; ++j) red[w][j] = v[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            double s = 0;
            for (int k = 0; k < nw; ++k) s += red[k][j];
            v[j] = s;
        }
    }
    __syncthreads();
}

// Fixed-order sums over the site blocks of partials 0..nk-1 of every column:
// one wavefront per (column, partial), lane l adding blocks l, l+64, ... in
// order, then a butterfly.  sums[i * nk + k] is valid in every thread on
// return.  The block size must be a multiple of 64.  A lane's first four
// blocks are loaded together (absent ones as 0, which leaves the sum
// unchanged), so up to 256 site blocks cost one memory round trip.
constexpr int MAX_SUMS = 64 * 3;
// The partials of slot k of field i, site block after site block (a
// wavefront reading 64 consecutive blocks reads 512 contiguous bytes).
__device__ __forceinline__ const double *part_col(const Prob &pr, int i, int k) {
    return pr.part + ((size_t)k * pr.nrhs + i) * pr.psb;
}
__device__ __forceinline__ double &part_at(const Prob &pr, int sb, int i, int k) {
    return pr.part[((size_t)k * pr.nrhs + i) * pr.psb + sb];
}

// Partials k0 .. k0 + nk - 1 of each entry are summed.
__device__ __forceinline__ void sum_all(const Prob &pr, int nsb, int nk, double *sums, int k0 = 0) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int job = w; job < pr.nrhs * nk; job += nw) {
        const int i = job / nk, k = job - i * nk;
        const double *col = part_col(pr, i, k0 + k);
        const double a0 = lane < nsb ? col[lane] : 0.0;
        const double a1 = lane + 64 < nsb ? col[lane + 64] : 0.0;
        const double a2 = lane + 128 < nsb ? col[lane + 128] : 0.0;
        const double a3 = lane + 192 < nsb ? col[lane + 192] : 0.0;
        double x = 0.0;
        x += a0;
        x += a1;
        x += a2;
        x += a3;
        for (int b = lane + 256; b < nsb; b += 64) x += col[b];
        x = wave_sum(x);
        if (lane == 0) sums[job] = x;
    }
    __syncthreads();
}

__device__ __forceinline__ bool finite_pos(double v) { return v > 0.0 && v < 1e300; }

// which problem of a grouped launch owns global tile b of kind K
__device__ __forceinline__ int find_prob(const Prob *probs, int nprob, int K, int b) {
    int j = 0;
    while (j + 1 < nprob && b >= probs[j + 1].t0[K]) ++j;
    return j;
}

// Tile t of stencil kind K: its site block, its rhs group and this thread's
// site (g.V when the thread has no site).  XY: a site block is one xy-plane
// (Lx Ly <= blockDim.x sites), as the plane-blocked variant needs.
// Passes (fp = (od >> 24) & 63 > 0): the site blocks are cut into eight
// chunks, one per XCD's tile range, and a chunk is walked in passes of fp rhs
// groups, site-block-major within a pass.  A pass holds fewer fields per
// plane, so the planes whose spinors its blocks share lie closer together in
// the XCD's L2; the links are read once per pass.
// MP (with XY): a site block is xy_kp(pr.sorder[K]) z-adjacent planes, whose
// sites are consecutive (the host picks only orders that keep them together).
__device__ __forceinline__ int xy_kp(int od) { return max(1, (od >> 18) & 7); }
template <bool XY = false, bool MP = false>
__device__ __forceinline__ void stencil_tile(const Prob &pr, int K, int t, int &sb, int &grp, int &s) {
    const int od = pr.sorder[K];
    const int fp = (od >> 24) & 63;
    if ((od >> 16) & 1) {
        grp = t / pr.nsb[K];
        sb = t - grp * pr.nsb[K];
    } else if (fp > 0 && fp < pr.ng[K]) {
        const int nsb = pr.nsb[K], ng = pr.ng[K];
        const int sc = (nsb + 7) >> 3;                  // site blocks per chunk
        const int c = t / (sc * ng), u = t - c * sc * ng;
        const int sbc = min(sc, nsb - c * sc);          // site blocks of this chunk
        const int pass = u / (sbc * fp), v = u - pass * sbc * fp;
        const int g0 = pass * fp, gp = min(fp, ng - g0);   // groups of this pass
        sb = c * sc + v / gp;
        grp = g0 + v % gp;
    } else {
        sb = t / pr.ng[K];
        grp = t - sb * pr.ng[K];
    }
    const int rows = XY ? (MP ? pr.g.S[2] * xy_kp(od) : pr.g.S[2]) : (int)blockDim.x;
    const int L = sb * rows + (int)threadIdx.x;
    s = ((int)threadIdx.x < rows && L < pr.g.V) ? order_site(pr.g, od & 0xffff, L) : pr.g.V;
}

// Plane-blocked phase kernels: LDS copy of the input field's xy-plane
template <int P> struct LdsWords { static constexpr int value = 6; };    // float4 per site
template <> struct LdsWords<P64> { static constexpr int value = 12; };   // double2 per site

// Stage the NR input spinors of this thread's site in the block's LDS plane
// (every thread of the block must call it: it ends with a barrier).
struct NoHook {
    __device__ void operator()() const {}
};
// `hook` runs after the staging and before the barrier.
template <int P, int NR, typename Hook = NoHook>
__device__ __forceinline__ void stage_plane(const FieldPtr &f, int rhs0, unsigned act, int s, int V,
                                            typename LdsSpinor<P>::word *xy, int np, Hook hook = {}) {
    typedef typename real_of<P>::type R;
    if (s < V)
#pragma unroll
        for (int j = 0; j < NR; ++j)
            if (act >> j & 1) {
                cx<R> v[12];
                Spinor<P>::load(f, rhs0 + j, s, v);
                LdsSpinor<P>::put(xy, np, j, threadIdx.x, v);
            }
    hook();
    __syncthreads();
}

// bit j set: rhs rhs0 + j is in state `want`
template <int NR>
__device__ __forceinline__ unsigned rhs_mask(const Prob &pr, const Scal *sc, int rhs0, int want) {
    unsigned m = 0;
#pragma unroll
    for (int j = 0; j < NR; ++j)
        if (rhs0 + j < pr.nrhs && sc[rhs0 + j].state == want) m |= 1u << j;
    return m;
}
template <int NR>
__device__ __forceinline__ unsigned rhs_mask(const Prob &pr, int rhs0, int want) {
    return rhs_mask<NR>(pr, pr.sc, rhs0, want);
}

// The finish of one iteration for one field (c0: its record before): phase
// A's sum sigma gives alpha (or a breakdown), phase B's sum rho the next beta,
// the counters and the state, as phaseA_finish then phaseB_finish do.  Only
// the fields the finish changes, as scalars (no record is copied through
// memory); store_fin writes them with the unchanged ones.
struct Fin {
    double sigma, alpha, rho_old, rho, beta;
    int state, iters, since_ru, pending_p;
};
__device__ __forceinline__ Fin cg_transition(const Prob &pr, const Scal &c0, double sigma, double rho) {
    Fin f{c0.sigma, c0.alpha, c0.rho_old, c0.rho, c0.beta, c0.state, c0.iters, c0.since_ru, 0};
    if (c0.state != ST_ACTIVE) return f;
    f.sigma = sigma;
    if (!finite_pos(sigma)) {
        f.state = ST_BREAKDOWN;
        return f;
    }
    f.alpha = c0.rho / sigma;
    f.iters = c0.iters + 1;
    f.since_ru = c0.since_ru + 1;
    f.rho_old = c0.rho;
    f.rho = rho;
    f.beta = rho / c0.rho;
    if (!(rho < 1e300)) f.state = ST_BREAKDOWN;   // NaN or Inf
    else if (rho <= c0.stop2 || f.iters >= pr.max_iter || (pr.ru_every > 0 && f.since_ru >= pr.ru_every))
        f.state = ST_FROZEN;                        // wants a reliable update
    else f.pending_p = 1;
    return f;
}
// the record after the finish: c0's fields with f's changes; restart cleared
// (phase A formed the direction)
__device__ __forceinline__ void store_fin(Scal &d, const Scal &c0, const Fin &f) {
    d.rho = f.rho;
    d.rho_old = f.rho_old;
    d.alpha = f.alpha;
    d.beta = f.beta;
    d.sigma = f.sigma;
    d.eta2 = c0.eta2;
    d.stop2 = c0.stop2;
    d.true2 = c0.true2;
    d.state = f.state;
    d.iters = f.iters;
    d.since_ru = f.since_ru;
    d.n_ru = c0.n_ru;
    d.pending_p = f.pending_p;
    d.restart = 0;
    d.zero_src = c0.zero_src;
    d.pad = c0.pad;
}

// ------------------------------------------------------------------ phase A
// q = D^dagger p for active rhs; partial |q|^2 (of the stored q)
// XY: plane-blocked (one xy-plane per block, x/y neighbours from LDS).
// MP (with XY): several z-adjacent planes per block (stencil_tile).  All z
// neighbours still come from memory: reading the ones inside the block from
// LDS (a branch per lane) took phases A and B from 77 to 95 VGPRs and 6 to 5
// waves per SIMD.
// R12: the links are the gauge's reconstruct-12 copy pr.U12 (two rows per link).
// QR: the direction is carried as q alone.  Since p = r + beta p_old, its image
// q = D^dagger p is D^dagger r + beta q_old: the stencil reads r and each site
// adds beta times its own old q (q = D^dagger r after a restart), so neither p
// nor a pass forming it (phase C) is needed.  Only the site's own q is read,
// so q is updated in place.
//
// Fused finish (par >= 0, with QR): the launch also completes the finish of the
// iteration before it, so an iteration is two launches.  Every block sums, for
// its own fields and in the finish's fixed order, phase A's partials of the
// previous iteration (slot 2 for par 0, slot 0 for par 1) and phase B's (slot
// 1), and applies the same transition (cg_transition) to the records it reads
// from pr.sc (par 0) or pr.sc2 (par 1); the site block 0 of each field group
// writes the results to the other array, which no block of this launch reads.
// So every block gets the same alpha, beta and state, bitwise equal to what
// k_finish would have recorded.  first = 1 (the chunk's first iteration): the
// records are final already (the reliable update or the trailing finish of the
// chunk before wrote them) and are copied unchanged.  Partials go to slot 0
// (par 0) or 2 (par 1).
template <int P, int NR, int ORD = 1, bool XY = false, bool R12 = false, bool NT = false, bool QR = false,
          bool MP = false>
__device__ __forceinline__ void phaseA_tile(const Prob &pr, int t, int par = -1, int first = 0) {
    typedef typename real_of<P>::type R;
    typedef typename LdsSpinor<P>::word W;
    __shared__ W xy[XY ? NR * LdsWords<P>::value * (MP ? 512 : 256) : 1];
    __shared__ double fsig[NR], frho[NR], fbeta[NR];
    __shared__ int fact[NR], frestart[NR];
    int sb, grp, s;
    stencil_tile<XY, MP>(pr, KA, t, sb, grp, s);
    const int rhs0 = grp * NR;
    const bool fused = QR && par >= 0;   // uniform over the launch
    const bool fin = fused && !first;
    const Scal *sin = fused && par ? pr.sc2 : pr.sc;
    Scal *sout = par ? pr.sc : pr.sc2;
    const int wslot = fused && par ? 2 : 0;
    // fields that iterate before this launch's finish (uniform over the block)
    const unsigned act0 = rhs_mask<NR>(pr, sin, rhs0, ST_ACTIVE);
    double part[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) part[j] = 0.0;
    const Geom g = pr.g;
    const int np = MP ? g.S[2] * xy_kp(pr.sorder[KA]) : g.S[2];   // sites staged in LDS
    FieldPtr fp{QR ? pr.r : pr.p, g.V, pr.nrhs}, fq{pr.q, g.V, pr.nrhs};
    // the fields of this launch's records that the finish's decision reads,
    // loaded early by the thread that decides, so the staging covers the latency
    Scal c0[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        c0[j] = Scal{};
        if (fused && threadIdx.x == 0 && rhs0 + j < pr.nrhs) {
            const Scal &m = sin[rhs0 + j];
            c0[j].state = m.state;
            c0[j].rho = m.rho;
            c0[j].stop2 = m.stop2;
            c0[j].iters = m.iters;
            c0[j].since_ru = m.since_ru;
            c0[j].beta = m.beta;
            c0[j].restart = m.restart;
        }
    }
    double as[NR][4], ar[NR][4];
    if (fin && act0) {
        col_issue<NR>(pr, rhs0, act0, as, par ? 0 : 2, pr.nsb[KA]);
        col_issue<NR>(pr, rhs0, act0, ar, 1, pr.nsb[KB]);
    }
    auto reduce = [&]() {
        if (fin && act0) {
            col_reduce<NR>(pr, rhs0, act0, as, fsig, par ? 0 : 2, pr.nsb[KA]);
            col_reduce<NR>(pr, rhs0, act0, ar, frho, 1, pr.nsb[KB]);
        }
    };
    // the plane is staged for the fields active before the finish (a field
    // that the finish freezes is staged for nothing, once per reliable update)
    if (XY && act0) stage_plane<P, NR>(fp, rhs0, act0, s, g.V, xy, np, reduce);
    else if (fin && act0) {
        reduce();
        __syncthreads();
    }
    // thread 0 applies the finish and shares the decision through LDS (one
    // barrier); site block 0 of the group stores the records at the end
    unsigned act = act0;
    if (fused) {
        if (threadIdx.x == 0)
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                const bool live = act0 >> j & 1;
                if (fin) {
                    const Fin f = cg_transition(pr, c0[j], live ? fsig[j] : 0.0, live ? frho[j] : 0.0);
                    fact[j] = live && f.state == ST_ACTIVE;
                    fbeta[j] = f.beta;
                    frestart[j] = 0;
                } else {
                    fact[j] = live;
                    fbeta[j] = c0[j].beta;
                    frestart[j] = c0[j].restart;
                }
            }
        __syncthreads();
        act = 0;
#pragma unroll
        for (int j = 0; j < NR; ++j)
            if (fact[j]) act |= 1u << j;
    }
    if (act && s < g.V) {
        const void *U = R12 ? pr.U12 : pr.U_lo;
        cx<R> acc[NR][12];
        hopping<P, true, NR, ORD, XY, false, false, R12>(g, s, U, fp, rhs0, act, acc, nullptr, xy,
                                                         s - (int)threadIdx.x, np);
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (act >> j & 1) {
                cx<R> self[12], o[12];
                if constexpr (XY) LdsSpinor<P>::get(xy, np, j, threadIdx.x, self);
                else Spinor<P>::load(fp, rhs0 + j, s, self);
                wilson_finish<R>((R)pr.diag, self, acc[j], o);
                if constexpr (QR) {
                    if (!(fused ? frestart[j] : pr.sc[rhs0 + j].restart)) {
                        const R b = (R)(fused ? fbeta[j] : pr.sc[rhs0 + j].beta);
                        cx<R> qo[12];
                        Spinor<P>::template load<NT>(fq, rhs0 + j, s, qo);
#pragma unroll
                        for (int k = 0; k < 12; ++k) o[k] = {o[k].re + b * qo[k].re, o[k].im + b * qo[k].im};
                    }
                }
                Spinor<P>::template store<NT>(fq, rhs0 + j, s, o);
                double n = 0;
#pragma unroll
                for (int k = 0; k < 12; ++k) n += (double)norm2(o[k]);
                part[j] = n;
            }
        }
    }
    if (act) {
        block_sum<NR>(part);
        if (threadIdx.x == 0)
#pragma unroll
            for (int j = 0; j < NR; ++j)
                if (act >> j & 1) part_at(pr, sb, rhs0 + j, wslot) = part[j];
    }
    // the group's records after the finish (or copied unchanged in the chunk's
    // first iteration), from the complete records read again
    if (fused && sb == 0 && threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < NR; ++j)
            if (rhs0 + j < pr.nrhs) {
                const Scal full = sin[rhs0 + j];
                if (fin) {
                    const bool live = act0 >> j & 1;
                    store_fin(sout[rhs0 + j], full, cg_transition(pr, full, live ? fsig[j] : 0.0, live ? frho[j] : 0.0));
                } else {
                    sout[rhs0 + j] = full;
                }
            }
}

// The finish functions run in one block; thread i updates the scalars of
// right-hand side i.
// Each reads its thread's scalar record before the partial sums, so the two
// loads overlap (nrhs <= 64 < blockDim.x: one field per thread).
__device__ __forceinline__ void phaseA_finish(const Prob &pr) {
    __shared__ double sums[MAX_SUMS];
    const int i = threadIdx.x;
    Scal c0;
    if (i < pr.nrhs) c0 = pr.sc[i];
    if (!__syncthreads_or(i < pr.nrhs && c0.state == ST_ACTIVE)) {   // nothing to sum
        if (i < pr.nrhs) pr.sc[i].pending_p = pr.sc[i].restart = 0;
        return;
    }
    sum_all(pr, pr.nsb[KA], 1, sums);
    if (i < pr.nrhs) {
        Scal &c = pr.sc[i];
        if (c0.state == ST_ACTIVE) {
            const double sigma = sums[i];
            c.sigma = sigma;
            if (!finite_pos(sigma)) c.state = ST_BREAKDOWN;
            else c.alpha = c0.rho / sigma;
        }
        c.pending_p = 0;
        c.restart = 0;
    }
}

// ------------------------------------------------------------------ phase B
// Phase A's reduction inside the phase-B blocks (FA): each block sums phase
// A's partials of its own fields, so alpha = rho / sigma is known without a
// finish launch between the phases.  Wave w takes fields j = w, w + nw, ...
// of the tile and adds exactly as sum_all does (same lanes, same order, same
// butterfly), so every block gets the sigma the finish after phase B records.
// fa_issue loads a lane's first four partials (before the plane staging, whose
// latency then covers them); fa_reduce completes the sums into sig[j] (LDS,
// read after the block's next barrier).
template <int NR>
__device__ __forceinline__ void col_issue(const Prob &pr, int rhs0, unsigned act, double (&a)[NR][4], int slot,
                                          int nsb) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        a[j][0] = a[j][1] = a[j][2] = a[j][3] = 0.0;
        if (j % nw == w && (act >> j & 1)) {
            const double *col = part_col(pr, rhs0 + j, slot);
            if (lane < nsb) a[j][0] = col[lane];
            if (lane + 64 < nsb) a[j][1] = col[lane + 64];
            if (lane + 128 < nsb) a[j][2] = col[lane + 128];
            if (lane + 192 < nsb) a[j][3] = col[lane + 192];
        }
    }
}

template <int NR>
__device__ __forceinline__ void col_reduce(const Prob &pr, int rhs0, unsigned act, const double (&a)[NR][4],
                                           double *out, int slot, int nsb) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (j % nw == w && (act >> j & 1)) {
            const double *col = part_col(pr, rhs0 + j, slot);
            double x = 0.0;
            x += a[j][0];
            x += a[j][1];
            x += a[j][2];
            x += a[j][3];
            for (int b = lane + 256; b < nsb; b += 64) x += col[b];
            x = wave_sum(x);
            if (lane == 0) out[j] = x;
        }
    }
}

template <int NR>
__device__ __forceinline__ void fa_issue(const Prob &pr, int rhs0, unsigned act, double (&a)[NR][4], int slot = 0) {
    col_issue<NR>(pr, rhs0, act, a, slot, pr.nsb[KA]);
}
template <int NR>
__device__ __forceinline__ void fa_reduce(const Prob &pr, int rhs0, unsigned act, const double (&a)[NR][4],
                                          double *sig, int slot = 0) {
    col_reduce<NR>(pr, rhs0, act, a, sig, slot, pr.nsb[KA]);
}

// t = D q; r -= alpha t; x_lo += alpha q(s); partial |r|^2 (of the stored r)
// FA: phase A's reduction is completed here (alpha from sigma of fa_reduce;
// a field whose sigma is not finite and positive is skipped, as the finish
// marks it broken down) and the |r|^2 partials go to slot 1, beside phase A's
// in slot 0, for phaseAB_finish.
// par >= 0 (with FA; the fused finish, see phaseA_tile): the records are those
// the phase-A launch of iteration parity par wrote (pr.sc2 for par 0, pr.sc for
// 1) and phase A's partials are in slot 0 (par 0) or 2 (par 1).
template <int P, int NR, int ORD = 1, bool XY = false, bool R12 = false, bool NT = false, bool FA = false,
          bool MP = false>
__device__ __forceinline__ void phaseB_tile(const Prob &pr, int t, int par = -1) {
    typedef typename real_of<P>::type R;
    constexpr int XP = XPrec<P>::value;
    typedef typename real_of<XP>::type RX;
    typedef typename LdsSpinor<P>::word W;
    __shared__ W xy[XY ? NR * LdsWords<P>::value * (MP ? 512 : 256) : 1];
    __shared__ double sig[NR];
    int sb, grp, s;
    stencil_tile<XY, MP>(pr, KB, t, sb, grp, s);
    const int rhs0 = grp * NR;
    const Scal *sc = par < 0 ? pr.sc : (par ? pr.sc : pr.sc2);
    const int aslot = par > 0 ? 2 : 0;
    unsigned act = rhs_mask<NR>(pr, sc, rhs0, ST_ACTIVE);
    double part[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) part[j] = 0.0;
    const Geom g = pr.g;
    const int np = MP ? g.S[2] * xy_kp(pr.sorder[KB]) : g.S[2];   // sites staged in LDS
    FieldPtr fq{pr.q, g.V, pr.nrhs}, fr{pr.r, g.V, pr.nrhs}, fx{pr.x_lo, g.V, pr.nrhs};
    if constexpr (FA) {
        if (act) {   // uniform over the block
            double a[NR][4];
            fa_issue<NR>(pr, rhs0, act, a, aslot);
            if constexpr (XY) {
                stage_plane<P, NR>(fq, rhs0, act, s, g.V, xy, np,
                                   [&]() { fa_reduce<NR>(pr, rhs0, act, a, sig, aslot); });
            } else {
                fa_reduce<NR>(pr, rhs0, act, a, sig, aslot);
                __syncthreads();
            }
#pragma unroll
            for (int j = 0; j < NR; ++j)
                if ((act >> j & 1) && !finite_pos(sig[j])) act &= ~(1u << j);
        }
    } else if (XY && act) {
        stage_plane<P, NR>(fq, rhs0, act, s, g.V, xy, np);
    }
    if (act && s < g.V) {
        const void *U = R12 ? pr.U12 : pr.U_lo;
        cx<R> acc[NR][12];
        hopping<P, false, NR, ORD, XY, false, false, R12>(g, s, U, fq, rhs0, act, acc, nullptr, xy,
                                                          s - (int)threadIdx.x, np);
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (act >> j & 1) {
                const double al = FA ? sc[rhs0 + j].rho / sig[j] : sc[rhs0 + j].alpha;
                const R a = (R)al;
                cx<R> q[12], o[12], r[12];
                if constexpr (XY) LdsSpinor<P>::get(xy, np, j, threadIdx.x, q);
                else Spinor<P>::load(fq, rhs0 + j, s, q);
                wilson_finish<R>((R)pr.diag, q, acc[j], o);
                Spinor<P>::template load<NT>(fr, rhs0 + j, s, r);
#pragma unroll
                for (int k = 0; k < 12; ++k) r[k] = {r[k].re - a * o[k].re, r[k].im - a * o[k].im};
                Spinor<P>::template store<NT>(fr, rhs0 + j, s, r);
                double n = 0;
#pragma unroll
                for (int k = 0; k < 12; ++k) n += (double)norm2(r[k]);
                part[j] = n;
                cx<RX> x[12];
                Spinor<XP>::template load<NT>(fx, rhs0 + j, s, x);
                const RX ax = (RX)al;
#pragma unroll
                for (int k = 0; k < 12; ++k) x[k] = {x[k].re + ax * (RX)q[k].re, x[k].im + ax * (RX)q[k].im};
                Spinor<XP>::template store<NT>(fx, rhs0 + j, s, x);
            }
        }
    }
    if (act) {
        block_sum<NR>(part);
        if (threadIdx.x == 0)
#pragma unroll
            for (int j = 0; j < NR; ++j)
                if (act >> j & 1) part_at(pr, sb, rhs0 + j, FA ? 1 : 0) = part[j];
    }
}

// the scalar updates after phase B of an active field (c0: its record before)
__device__ __forceinline__ void phaseB_update(const Prob &pr, Scal &c, const Scal &c0, double rho) {
    const int iters = c0.iters + 1, since_ru = c0.since_ru + 1;
    c.rho_old = c0.rho;
    c.rho = rho;
    c.beta = rho / c0.rho;
    c.iters = iters;
    c.since_ru = since_ru;
    if (!(rho < 1e300)) c.state = ST_BREAKDOWN;   // NaN or Inf
    else if (rho <= c0.stop2 || iters >= pr.max_iter || (pr.ru_every > 0 && since_ru >= pr.ru_every))
        c.state = ST_FROZEN;                       // wants a reliable update
    else c.pending_p = 1;
}

__device__ __forceinline__ void phaseB_finish(const Prob &pr) {
    __shared__ double sums[MAX_SUMS];
    const int i = threadIdx.x;
    Scal c0;
    if (i < pr.nrhs) c0 = pr.sc[i];
    if (!__syncthreads_or(i < pr.nrhs && c0.state == ST_ACTIVE)) return;   // nothing to sum
    sum_all(pr, pr.nsb[KB], 1, sums);
    if (i < pr.nrhs && c0.state == ST_ACTIVE) phaseB_update(pr, pr.sc[i], c0, sums[i]);
}

// Phase A's (slot 0) and phase B's (slot 1) sums of every field in one memory
// round trip: wave w takes fields i = w, w + nw, ... and loads the first four
// blocks of both columns before adding either, each in sum_all's order (so
// the values are the ones sum_all returns, and fa_reduce's sigma).
__device__ __forceinline__ void sum_ab(const Prob &pr, double *sa, double *sb, int aslot = 0) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int na = pr.nsb[KA], nb = pr.nsb[KB];
    for (int i = w; i < pr.nrhs; i += nw) {
        const double *ca = part_col(pr, i, aslot), *cb = part_col(pr, i, 1);
        double a[4], b[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a[k] = lane + 64 * k < na ? ca[lane + 64 * k] : 0.0;
            b[k] = lane + 64 * k < nb ? cb[lane + 64 * k] : 0.0;
        }
        double x = 0.0, y = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x += a[k];
            y += b[k];
        }
        for (int j = lane + 256; j < na; j += 64) x += ca[j];
        for (int j = lane + 256; j < nb; j += 64) y += cb[j];
        x = wave_sum(x);
        y = wave_sum(y);
        if (lane == 0) {
            sa[i] = x;
            sb[i] = y;
        }
    }
    __syncthreads();
}

// After an FA phase B: phase A's finish (sigma, alpha, breakdown) from its
// slot (0 or 2), then phase B's from slot 1, with the results phaseA_finish
// followed by phaseB_finish give.  The records are read from sin and written
// to sout (the same array in the three-launch iteration; with the fused
// finish, the chunk's last records into pr.sc).
__device__ __forceinline__ void phaseAB_finish(const Prob &pr, const Scal *sin, Scal *sout, int aslot) {
    __shared__ double sa[MAX_SUMS], sbb[MAX_SUMS];
    const int i = threadIdx.x;
    Scal c0;
    if (i < pr.nrhs) c0 = sin[i];
    if (!__syncthreads_or(i < pr.nrhs && c0.state == ST_ACTIVE)) {   // nothing to sum
        if (i < pr.nrhs) store_fin(sout[i], c0, cg_transition(pr, c0, 0.0, 0.0));
        return;
    }
    sum_ab(pr, sa, sbb, aslot);
    if (i < pr.nrhs) store_fin(sout[i], c0, cg_transition(pr, c0, sa[i], sbb[i]));
}
__device__ __forceinline__ void phaseAB_finish(const Prob &pr) { phaseAB_finish(pr, pr.sc, pr.sc, 0); }

// ---------------------------------------------- z-marching phases A and B
// A tile is a column of xy-planes: one t, one rhs, the planes z0 <= z < z1 of
// z-chunk c (the chunk count is pr.sorder[K]).  The block walks the column
// with two LDS plane buffers `lds` (dynamic, 2 x np sites): at each step it
// stages plane z+1, then forms phase A's or B's epilogue for plane z with the
// x, y and forward-z neighbours from LDS, the backward-z hop carried in
// registers from the previous step (hopping() with ZM) and only the t
// neighbours from memory.  A site of the column is thus read from memory once
// (plus one plane before the chunk), against five times (own plane and four
// neighbour planes) for plane blocks.  Tiles are ordered rhs fastest, then t,
// then the chunk, so the blocks sharing links or t neighbours run together on
// one XCD.  Partial sums are per column: part[c Lt + t][rhs].
// Needs Lx Ly <= blockDim.x and one rhs per tile; FP32 and FP16 storage.
template <int P, int ORD, bool B>
__device__ __forceinline__ void zm_tile(const Prob &pr, int t, typename LdsSpinor<P>::word *lds) {
    typedef typename real_of<P>::type R;
    constexpr int XP = XPrec<P>::value;
    typedef typename real_of<XP>::type RX;
    constexpr int K = B ? KB : KA;
    const Geom g = pr.g;
    const int np = g.S[2], Lz = g.L[2], Lt = g.L[3];
    const int nzc = pr.sorder[K] & 0xffff;
    const int rhs = t % pr.nrhs, col = t / pr.nrhs;
    const int c = col / Lt, tt = col - c * Lt;
    const int z0 = (c * Lz) / nzc, z1 = ((c + 1) * Lz) / nzc;
    const unsigned act = rhs_mask<1>(pr, rhs, ST_ACTIVE);
    if (!act) return;   // the same for every thread of the block
    const int i = threadIdx.x;
    const bool on = i < np;
    typename LdsSpinor<P>::word *buf[2] = {lds, lds + LdsWords<P>::value * np};
    FieldPtr fin{B ? pr.q : pr.p, g.V, pr.nrhs};
    FieldPtr fr{pr.r, g.V, pr.nrhs}, fx{pr.x_lo, g.V, pr.nrhs}, fq{pr.q, g.V, pr.nrhs};
    const void *U = pr.U_lo;
    constexpr int SB = B ? +1 : -1;   // backward-hop sign of D (B) or D^dagger (A)
    cx<R> carry[1][12];
    if (on) {   // backward z hop of plane z0 from plane z0 - 1; stage plane z0
        const int sp = i + np * ((z0 == 0 ? Lz - 1 : z0 - 1) + Lz * tt);
        cx<R> u[9], v[12], h[6], w[6];
        Link<P>::load(U, g, 2, sp, false, u);
        Spinor<P>::load(fin, rhs, sp, v);
        project<2, SB>(v, h);
        link_adj_mul(u, h, w);
#pragma unroll
        for (int k = 0; k < 12; ++k) carry[0][k] = {R(0), R(0)};
        accumulate<2, SB>(w, carry[0]);
        Spinor<P>::load(fin, rhs, i + np * (z0 + Lz * tt), v);
        LdsSpinor<P>::put(buf[0], np, 0, i, v);
    }
    double part = 0.0;
    for (int z = z0; z < z1; ++z) {
        const int cur = (z - z0) & 1;
        const int s = i + np * (z + Lz * tt);
        if (on) {   // stage plane z + 1 (the forward z neighbours)
            cx<R> v[12];
            Spinor<P>::load(fin, rhs, i + np * ((z + 1 == Lz ? 0 : z + 1) + Lz * tt), v);
            LdsSpinor<P>::put(buf[cur ^ 1], np, 0, i, v);
        }
        __syncthreads();
        if (on) {
            cx<R> acc[1][12], self[12], o[12];
            hopping<P, !B, 1, ORD, true, false, true>(g, s, U, fin, rhs, act, acc, nullptr, buf[cur], s - i, np,
                                                      buf[cur ^ 1], carry);
            LdsSpinor<P>::get(buf[cur], np, 0, i, self);
            wilson_finish<R>((R)pr.diag, self, acc[0], o);
            double n = 0;
            if constexpr (B) {   // r -= alpha D q; x_lo += alpha q
                const R a = (R)pr.sc[rhs].alpha;
                cx<R> r[12];
                Spinor<P>::template load<false>(fr, rhs, s, r);
#pragma unroll
                for (int k = 0; k < 12; ++k) r[k] = {r[k].re - a * o[k].re, r[k].im - a * o[k].im};
                Spinor<P>::template store<false>(fr, rhs, s, r);
#pragma unroll
                for (int k = 0; k < 12; ++k) n += (double)norm2(r[k]);
                cx<RX> x[12];
                Spinor<XP>::template load<false>(fx, rhs, s, x);
                const RX ax = (RX)pr.sc[rhs].alpha;
#pragma unroll
                for (int k = 0; k < 12; ++k)
                    x[k] = {x[k].re + ax * (RX)self[k].re, x[k].im + ax * (RX)self[k].im};
                Spinor<XP>::template store<false>(fx, rhs, s, x);
            } else {             // q = D^dagger p
                Spinor<P>::template store<false>(fq, rhs, s, o);
#pragma unroll
                for (int k = 0; k < 12; ++k) n += (double)norm2(o[k]);
            }
            part += n;
        }
        __syncthreads();   // buf[cur] is overwritten by the next step
    }
    double pv[1] = {part};
    block_sum<1>(pv);
    if (threadIdx.x == 0) part_at(pr, col, rhs, 0) = pv[0];
}

// ------------------------------------------------------------------ phase C
// p = r + beta p (or p = r after a restart), streaming, tile = (site block, rhs)
template <int P, bool NT = false>
__device__ __forceinline__ void phaseC_tile(const Prob &pr, int t) {
    typedef typename real_of<P>::type R;
    const int sb = t / pr.nrhs, i = t - sb * pr.nrhs;
    const int s = sb * blockDim.x + threadIdx.x;
    const Scal &c = pr.sc[i];
    if (c.state != ST_ACTIVE || !c.pending_p || s >= pr.vf) return;
    FieldPtr fr{pr.r, pr.vf, pr.nrhs}, fp{pr.p, pr.vf, pr.nrhs};
    cx<R> r[12], p[12];
    Spinor<P>::template load<NT>(fr, i, s, r);
    if (!c.restart) {
        const R b = (R)c.beta;
        Spinor<P>::template load<NT>(fp, i, s, p);
#pragma unroll
        for (int k = 0; k < 12; ++k) r[k] = {r[k].re + b * p[k].re, r[k].im + b * p[k].im};
    }
    Spinor<P>::template store<NT>(fp, i, s, r);
}

// ------------------------------------------------------- reliable update R1
// x64 += x_lo; x_lo = 0   (rhs that are frozen)
template <int P>
__device__ __forceinline__ void ru1_tile(const Prob &pr, int t) {
    constexpr int XP = XPrec<P>::value;
    typedef typename real_of<XP>::type RX;
    const int sb = t / pr.nrhs, i = t - sb * pr.nrhs;
    const int s = sb * blockDim.x + threadIdx.x;
    if (pr.sc[i].state != ST_FROZEN || s >= pr.vf) return;
    FieldPtr fx{pr.x_lo, pr.vf, pr.nrhs}, f64{pr.x64, pr.vf, pr.nrhs};
    cx<RX> xl[12];
    cx<double> x[12];
    Spinor<XP>::load(fx, i, s, xl);
    Spinor<P64>::load(f64, i, s, x);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        x[k] = {x[k].re + (double)xl[k].re, x[k].im + (double)xl[k].im};
        xl[k] = {RX(0), RX(0)};
    }
    Spinor<P64>::store(f64, i, s, x);
    Spinor<XP>::store(fx, i, s, xl);
}

// ------------------------------------------------------- reliable update R2
// r = eta - D x64 in FP64 with FP64 links; r_lo = r rounded to the inner
// precision; partial |r|^2 in FP64 (frozen rhs).  XY: one xy-plane per block,
// x64 of the plane staged in LDS (x and y neighbours and the site itself).
// ZX: x64 is zero (the first residual of a solve without an initial guess):
// D x64 is exactly zero, so r = eta without the stencil, bitwise the same.
template <int P, int NR, bool XY = false, bool ZX = false>
__device__ __forceinline__ void ru2_tile(const Prob &pr, int t) {
    typedef typename real_of<P>::type R;
    typedef typename LdsSpinor<P64>::word W;
    __shared__ W xy[XY ? NR * LdsWords<P64>::value * 256 : 1];
    int sb, grp, s;
    stencil_tile<XY>(pr, KR2, t, sb, grp, s);
    const int rhs0 = grp * NR;
    const unsigned act = rhs_mask<NR>(pr, rhs0, ST_FROZEN);
    double part[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) part[j] = 0.0;
    const Geom g = pr.g;
    const int np = g.S[2];
    FieldPtr fx{pr.x64, g.V, pr.nrhs}, fe{pr.eta64, g.V, pr.nrhs}, fr{pr.r, g.V, pr.nrhs};
    if (!ZX && XY && act) stage_plane<P64, NR>(fx, rhs0, act, s, g.V, xy, np);
    if (act && s < g.V) {
        const void *U = pr.U64;
        cx<double> acc[NR][12];
        if constexpr (!ZX)
            hopping<P64, false, NR, XY ? 3 : 1, XY>(g, s, U, fx, rhs0, act, acc, nullptr, xy, s - (int)threadIdx.x,
                                                    np);
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (act >> j & 1) {
                cx<double> x[12], e[12], o[12];
                if constexpr (ZX) {
#pragma unroll
                    for (int k = 0; k < 12; ++k) o[k] = {0.0, 0.0};
                } else {
                    if constexpr (XY) LdsSpinor<P64>::get(xy, np, j, threadIdx.x, x);
                    else Spinor<P64>::load(fx, rhs0 + j, s, x);
                    wilson_finish<double>(pr.diag, x, acc[j], o);
                }
                Spinor<P64>::load(fe, rhs0 + j, s, e);
                cx<R> rl[12];
                double n = 0;
#pragma unroll
                for (int k = 0; k < 12; ++k) {
                    const cx<double> d = e[k] - o[k];
                    n += norm2(d);
                    rl[k] = {(R)d.re, (R)d.im};
                }
                Spinor<P>::store(fr, rhs0 + j, s, rl);
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

__device__ __forceinline__ void ru2_finish(const Prob &pr) {
    __shared__ double sums[MAX_SUMS];
    sum_all(pr, pr.nsb[KR2], 1, sums);
    for (int i = threadIdx.x; i < pr.nrhs; i += blockDim.x) {
        Scal &c = pr.sc[i];
        if (c.state != ST_FROZEN) {
            // CG: the chunk's last phase C has consumed the flag.  BiCGSTAB: a
            // field still iterating keeps it for the next p update.
            if (pr.method == METHOD_CGNE) c.pending_p = 0;
            continue;
        }
        const double r2 = sums[i];
        {
            c.true2 = r2;
            c.n_ru += 1;
            c.since_ru = 0;
            c.pending_p = 0;
            if (r2 <= c.stop2) c.state = ST_DONE;
            else if (!(r2 < 1e300)) c.state = ST_BREAKDOWN;
            else if (c.iters >= pr.max_iter) c.state = ST_NOTCONV;
            else {
                // Continue from the true residual.  beta stays the value of the
                // last iteration (iterated |r|^2 over its predecessor); forming it
                // from the true |r|^2 instead stalls when the stored residual has
                // drifted far from the true one (FP16 storage).
                c.rho = r2;
                c.state = ST_ACTIVE;
                c.pending_p = 1;
                if (pr.method == METHOD_BICGSTAB) {
                    // restart from the true residual: r_hat = r, p = r, rho = |r|^2
                    c.restart = 1;
                    pr.bs[i].rho[0] = r2;
                    pr.bs[i].rho[1] = 0.0;
                    pr.bs[i].rh2 = r2;
                }
            }
        }
    }
}

// -------------------------------------------------------- source norm |eta|^2
__device__ __forceinline__ void norm_tile(const Prob &pr, int t) {
    const int sb = t / pr.nrhs, i = t - sb * pr.nrhs;
    const int s = sb * blockDim.x + threadIdx.x;
    double part[1] = {0.0};
    if (s < pr.vf) {
        FieldPtr fe{pr.eta64, pr.vf, pr.nrhs};
        cx<double> e[12];
        Spinor<P64>::load(fe, i, s, e);
#pragma unroll
        for (int k = 0; k < 12; ++k) part[0] += norm2(e[k]);
        if (pr.eo) {   // |eta|^2 of the whole field: the odd half too
            FieldPtr fo{pr.eta_o, pr.vf, pr.nrhs};
            Spinor<P64>::load(fo, i, s, e);
#pragma unroll
            for (int k = 0; k < 12; ++k) part[0] += norm2(e[k]);
        }
    }
    block_sum<1>(part);
    if (threadIdx.x == 0) part_at(pr, sb, i, 0) = part[0];
}

__device__ __forceinline__ void norm_finish(const Prob &pr) {
    __shared__ double sums[MAX_SUMS];
    sum_all(pr, pr.nsb[KN], 1, sums);
    for (int i = threadIdx.x; i < pr.nrhs; i += blockDim.x) {
        const double e2 = sums[i];
        {
            Scal &c = pr.sc[i];
            c.eta2 = e2;
            c.stop2 = pr.tol2 * e2;
            if (e2 == 0.0) { c.state = ST_DONE; c.zero_src = 1; c.true2 = 0.0; }
            else if (!(e2 < 1e300)) c.state = ST_BREAKDOWN;
        }
    }
}

}  // namespace wd
