// The Wilson-Dirac operator D and its adjoint (Eq. (1), Sec. 1; D^dagger by
// gamma5-hermiticity, Sec. 2) as a matrix-free stencil on packed fields.
//
// One thread computes one lattice site for NR right-hand sides, so each link
// is loaded once per NR fields.  A block covers `block` consecutive sites (of
// the processing order, order_site) of one group of NR right-hand sides.
// Tiles are ordered site-block-major (group-minor) or group-major, and
// optionally remapped so each XCD works through one contiguous range of them.
// `order` = strip width | group-major << 16.
#include <algorithm>
#include <mutex>

#include "wd_device.h"
#include "wd_host.h"

namespace wd {

// R12: U is the gauge's reconstruct-12 FP32 copy (two rows per link)
template <int P, bool DAG, int NR, int ORD, bool R12 = false>
__global__ __launch_bounds__(256) void k_dslash(Geom g, double diag, const void *__restrict__ U,
                                                FieldPtr in, FieldPtr out, int ngroups, int remap, int rloop,
                                                int order) {
    typedef typename real_of<P>::type R;
    // tile = (site block, group of rloop consecutive rhs groups); the block
    // handles its rhs groups one after the other, so fewer distinct fields are
    // in flight per XCD at a time
    const int nouter = (ngroups + rloop - 1) / rloop;
    const int b = remap ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    int sb, go;
    if (order >> 16) {
        const int nsb = (int)gridDim.x / nouter;
        go = b / nsb;
        sb = b - go * nsb;
    } else {
        sb = b / nouter;
        go = b - sb * nouter;
    }
    const int L = sb * blockDim.x + threadIdx.x;
    if (L >= g.V) return;
    const int s = order_site(g, order & 0xffff, L);
    for (int gi = 0; gi < rloop; ++gi) {
        const int grp = go * rloop + gi;
        if (grp >= ngroups) break;
        const int rhs0 = grp * NR;
        const int nact = min(NR, in.nrhs - rhs0);
        const unsigned act = (1u << nact) - 1u;
        cx<R> acc[NR][12];
        if constexpr (ORD == 4) {
            cx<R> self[NR][12];
#pragma unroll
            for (int j = 0; j < NR; ++j)
                if (act >> j & 1) Spinor<P>::load(in, rhs0 + j, s, self[j]);
            hopping<P, DAG, NR, ORD, false, false, false, R12>(g, s, U, in, rhs0, act, acc, self);
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                if (act >> j & 1) {
                    cx<R> o[12];
                    wilson_finish<R>((R)diag, self[j], acc[j], o);
                    Spinor<P>::store(out, rhs0 + j, s, o);
                }
            }
        } else {
            hopping<P, DAG, NR, ORD, false, false, false, R12>(g, s, U, in, rhs0, act, acc);
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                if (act >> j & 1) {
                    cx<R> self[12], o[12];
                    Spinor<P>::load(in, rhs0 + j, s, self);
                    wilson_finish<R>((R)diag, self, acc[j], o);
                    Spinor<P>::store(out, rhs0 + j, s, o);
                }
            }
        }
    }
}

// Plane-blocked variant: a block is one xy-plane (np = Lx Ly <= 256 sites) of
// one group of NR right-hand sides.  The block first copies its plane's
// spinors to LDS; the x and y neighbours then come from LDS, so only the own
// spinor and the z and t neighbours are read from memory.  The own spinor is
// read back from LDS for the diagonal term.
// MP: a block is k z-adjacent planes of one rhs (blockDim.x = k Lx Ly <= 512
// consecutive sites; the processing order keeps such planes together).  A
// 14 x 14 plane fills 196 of a 256-thread block's lanes, two planes 392 of
// 448; and a z neighbour inside the block comes from LDS.
template <int P, bool DAG, int NR, int ORD, bool R12 = false, bool MP = false>
__global__ __launch_bounds__(MP ? 512 : 256) void k_dslash_xy(Geom g, double diag, const void *__restrict__ U,
                                                   FieldPtr in, FieldPtr out, int ngroups, int remap, int order) {
    typedef typename real_of<P>::type R;
    typedef typename LdsSpinor<P>::word W;
    extern __shared__ uint4 lds_raw[];
    W *xy = (W *)lds_raw;
    const int np = (int)blockDim.x;
    const int b = remap ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int npl = (int)gridDim.x / ngroups;
    int pl, grp;
    if (order >> 16) {
        grp = b / npl;
        pl = b - grp * npl;
    } else {
        pl = b / ngroups;
        grp = b - pl * ngroups;
    }
    const int s = order_site(g, order & 0xffff, pl * np + (int)threadIdx.x);
    const int rhs0 = grp * NR;
    const int nact = min(NR, in.nrhs - rhs0);
    const unsigned act = (1u << nact) - 1u;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (act >> j & 1) {
            cx<R> self[12];
            Spinor<P>::load(in, rhs0 + j, s, self);
            LdsSpinor<P>::put(xy, np, j, threadIdx.x, self);
        }
    }
    __syncthreads();
    cx<R> acc[NR][12];
    hopping<P, DAG, NR, ORD, true, false, false, R12, MP>(g, s, U, in, rhs0, act, acc, nullptr, xy,
                                                          s - (int)threadIdx.x, np);
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        if (act >> j & 1) {
            cx<R> self[12], o[12];
            LdsSpinor<P>::get(xy, np, j, threadIdx.x, self);
            wilson_finish<R>((R)diag, self, acc[j], o);
            Spinor<P>::store(out, rhs0 + j, s, o);
        }
    }
}

// z-marching variant: a block walks a column of xy-planes along z (one rhs,
// one t, the planes of z-chunk c), so every spinor is read from memory about
// once by its own block instead of once per neighbouring plane.  Per plane:
// the next plane's own spinors are loaded first (they are the z neighbours on
// that side), one barrier, x and y neighbours from LDS (two plane buffers),
// t neighbours from memory, the z hop from the other side carried in registers
// (march_hopping).  Even chunks walk upward, odd chunks downward (nchunk is
// even), so the two blocks meeting at a chunk boundary load the planes there
// at the same time, both at the start or both at the end of their walks.
// Tile order 0: chunk-major, then rhs, then t (an XCD's contiguous range of
// tiles holds whole t-rings of a few rhs of one chunk); 1: rhs-major, then t,
// then chunk (whole t-rings and both chunks of fewer rhs).  With those on one
// XCD and walking in step, the t neighbours and the boundary planes a block
// reads were loaded by another block of that XCD moments before.
// blockDim.x = Lx Ly.
template <int P, bool DAG, bool DOWN, bool R12, int ORD>
__device__ __forceinline__ void zm_walk(const Geom &g, double diag, const void *U, const FieldPtr &in,
                                        const FieldPtr &out, int rhs, int tt, int z0, int z1,
                                        typename LdsSpinor<P>::word *buf0, typename LdsSpinor<P>::word *buf1) {
    typedef typename real_of<P>::type R;
    const int np = g.S[2], Lz = g.L[2];
    const int i = threadIdx.x;
    const int tb = np * Lz * tt + i;   // this thread's site on plane 0 of the t-slice
    const int zf = DOWN ? z1 - 1 : z0;
    cx<R> self[12], carry[12];
    {   // the z hop into the first plane from the plane on the far side
        const int zb = DOWN ? (zf + 1 == Lz ? 0 : zf + 1) : (zf == 0 ? Lz - 1 : zf - 1);
        const int sb = tb + np * zb;
        cx<R> u[9], v[12], h[6], w[6];
        Link<P>::template load<R12>(U, g, 2, DOWN ? tb + np * zf : sb, false, u);
        Spinor<P>::load(in, rhs, sb, v);
#pragma unroll
        for (int k = 0; k < 12; ++k) carry[k] = {R(0), R(0)};
        constexpr int SF = DAG ? +1 : -1;
        if constexpr (DOWN) {
            project<2, SF>(v, h);
            link_mul(u, h, w);
            accumulate<2, SF>(w, carry);
        } else {
            project<2, -SF>(v, h);
            link_adj_mul(u, h, w);
            accumulate<2, -SF>(w, carry);
        }
        Spinor<P>::load(in, rhs, tb + np * zf, self);
        LdsSpinor<P>::put(buf0, np, 0, i, self);
    }
    const int nz = z1 - z0;
    for (int k = 0; k < nz; ++k) {
        const int z = DOWN ? zf - k : zf + k;
        const int zn = DOWN ? (z == 0 ? Lz - 1 : z - 1) : (z + 1 == Lz ? 0 : z + 1);
        const int s = tb + np * z, sn = tb + np * zn;
        typename LdsSpinor<P>::word *cur = (k & 1) ? buf1 : buf0;
        cx<R> nxt[12], acc[12], o[12];
        Spinor<P>::load(in, rhs, sn, nxt);
        __syncthreads();   // plane z is complete in its buffer
        march_hopping<P, DAG, DOWN, R12, ORD>(g, s, sn, U, in, rhs, cur, s - i, np, nxt, carry, acc);
        LdsSpinor<P>::get(cur, np, 0, i, self);
        wilson_finish<R>((R)diag, self, acc, o);
        Spinor<P>::store(out, rhs, s, o);
        // the other buffer was last read before this step's barrier
        if (k + 1 < nz) LdsSpinor<P>::put((k & 1) ? buf0 : buf1, np, 0, i, nxt);
    }
}

template <int P, bool DAG, bool R12 = false, int ORD = 3>
__global__ __launch_bounds__(256) void k_dslash_zm(Geom g, double diag, const void *__restrict__ U, FieldPtr in,
                                                   FieldPtr out, int nchunk, int remap, int order) {
    typedef typename LdsSpinor<P>::word W;
    extern __shared__ uint4 lds_raw[];
    const int np = g.S[2], Lz = g.L[2], Lt = g.L[3];
    W *buf0 = (W *)lds_raw, *buf1 = buf0 + (LdsSpinor<P>::BYTES / 16) * np;
    const int b = remap ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    int rhs, tt, c;
    if (order == 0) {
        tt = b % Lt;
        const int q = b / Lt;
        rhs = q % in.nrhs;
        c = q / in.nrhs;
    } else {
        c = b % nchunk;
        const int q = b / nchunk;
        tt = q % Lt;
        rhs = q / Lt;
    }
    const int z0 = (c * Lz) / nchunk, z1 = ((c + 1) * Lz) / nchunk;
    if (c & 1) zm_walk<P, DAG, true, R12, ORD>(g, diag, U, in, out, rhs, tt, z0, z1, buf0, buf1);
    else zm_walk<P, DAG, false, R12, ORD>(g, diag, U, in, out, rhs, tt, z0, z1, buf0, buf1);
}

// LDS bytes of the plane-blocked variant
static size_t xy_lds_bytes(int prec, int nr, int np) {
    return (size_t)nr * (prec == WD_F64 ? 192 : 96) * np;
}

int xy_planes(const Shape &sh, const Geom &g, int prec, int nr) {
    const int k = sh.planes;
    const int strip = (sh.strip > 0 && sh.strip < g.L[2]) ? sh.strip : 0;
    // k z-adjacent planes are consecutive sites in every processing order
    // whose strips hold whole groups of k planes
    if (k < 2 || prec == WD_F64 || nr != 1 || k * g.S[2] > 512 || g.L[2] % k || strip % k) return 1;
    return k;
}

template <int P, bool DAG, bool R12 = false>
static void launch_xy(int nr, int ord, dim3 grid, int np, size_t lds, hipStream_t st, const Geom &g, double diag,
                      const void *U, FieldPtr in, FieldPtr out, int ngroups, int remap, int od, bool mp) {
    const dim3 block(np);
    if (mp) {   // several planes per block: one rhs per thread, hop order 3 or 5, not FP64
        if constexpr (P != P64) {
            if (ord == 5) hipLaunchKernelGGL((k_dslash_xy<P, DAG, 1, 5, R12, true>), grid, block, lds, st, g, diag, U, in, out, ngroups, remap, od);
            else hipLaunchKernelGGL((k_dslash_xy<P, DAG, 1, 3, R12, true>), grid, block, lds, st, g, diag, U, in, out, ngroups, remap, od);
        }
    } else if (nr == 1) {
        if (ord == 5) hipLaunchKernelGGL((k_dslash_xy<P, DAG, 1, 5, R12>), grid, block, lds, st, g, diag, U, in, out, ngroups, remap, od);
        else if (ord == 3) hipLaunchKernelGGL((k_dslash_xy<P, DAG, 1, 3, R12>), grid, block, lds, st, g, diag, U, in, out, ngroups, remap, od);
        else hipLaunchKernelGGL((k_dslash_xy<P, DAG, 1, 1, R12>), grid, block, lds, st, g, diag, U, in, out, ngroups, remap, od);
    } else {   // hop order 5 exists for one rhs per thread: 3 here
        if (ord == 3 || ord == 5) hipLaunchKernelGGL((k_dslash_xy<P, DAG, 2, 3, R12>), grid, block, lds, st, g, diag, U, in, out, ngroups, remap, od);
        else hipLaunchKernelGGL((k_dslash_xy<P, DAG, 2, 1, R12>), grid, block, lds, st, g, diag, U, in, out, ngroups, remap, od);
    }
}

template <int P, bool DAG, int ORD, bool R12 = false>
static void launch_nr_o(int nr, dim3 grid, dim3 block, hipStream_t st, const Geom &g, double diag,
                        const void *U, FieldPtr in, FieldPtr out, int ngroups, int remap, int rl, int od) {
    if constexpr (ORD == 4) {
        // the own spinors of several rhs do not fit in registers: only NR = 1
        if (nr == 1)
            hipLaunchKernelGGL((k_dslash<P, DAG, 1, 4, R12>), grid, block, 0, st, g, diag, U, in, out, ngroups, remap, rl, od);
        else
            launch_nr_o<P, DAG, 3, R12>(nr, grid, block, st, g, diag, U, in, out, ngroups, remap, rl, od);
    } else {
        switch (nr) {
        case 1: hipLaunchKernelGGL((k_dslash<P, DAG, 1, ORD, R12>), grid, block, 0, st, g, diag, U, in, out, ngroups, remap, rl, od); break;
        case 2: hipLaunchKernelGGL((k_dslash<P, DAG, 2, ORD, R12>), grid, block, 0, st, g, diag, U, in, out, ngroups, remap, rl, od); break;
        default: hipLaunchKernelGGL((k_dslash<P, DAG, 4, ORD, R12>), grid, block, 0, st, g, diag, U, in, out, ngroups, remap, rl, od); break;
        }
    }
}

template <int P, bool DAG, bool R12 = false>
static void launch_nr(int nr, int ordered, int rl, dim3 grid, dim3 block, hipStream_t st, const Geom &g, double diag,
                      const void *U, FieldPtr in, FieldPtr out, int ngroups, int remap, int od) {
    if (ordered == 1) launch_nr_o<P, DAG, 1, R12>(nr, grid, block, st, g, diag, U, in, out, ngroups, remap, rl, od);
    else if (ordered == 2) launch_nr_o<P, DAG, 2, R12>(nr, grid, block, st, g, diag, U, in, out, ngroups, remap, rl, od);
    else if (ordered == 3 || ordered == 5)   // site blocks read every neighbour from memory: 5 is 3
        launch_nr_o<P, DAG, 3, R12>(nr, grid, block, st, g, diag, U, in, out, ngroups, remap, rl, od);
    else if (ordered == 4) launch_nr_o<P, DAG, 4, R12>(nr, grid, block, st, g, diag, U, in, out, ngroups, remap, rl, od);
    else launch_nr_o<P, DAG, 0, R12>(nr, grid, block, st, g, diag, U, in, out, ngroups, remap, rl, od);
}

Geom make_geom(const wd_gauge *gg) { return geom_of(gg->dims, gg->tsign); }

int launch_dslash(const wd_gauge *gg, double m0, int prec, bool dag, const void *in, void *out,
                  int nrhs, const Shape &sh, hipStream_t st) {
    const Geom g = make_geom(gg);
    const int nr = (sh.nr == 1 || sh.nr == 2 || sh.nr == 4) ? sh.nr : 1;
    const int blk = (sh.block == 64 || sh.block == 128 || sh.block == 256) ? sh.block : 256;
    const int ngroups = (nrhs + nr - 1) / nr;
    const int rl = sh.rloop >= 1 ? std::min(sh.rloop, ngroups) : 1;
    const int nsb = (g.V + blk - 1) / blk;
    const int strip = (sh.strip > 0 && sh.strip < g.L[2]) ? sh.strip : 0;
    const int od = strip | (sh.gmajor ? 1 << 16 : 0);
    const int np = g.L[0] * g.L[1];
    // FP32 with a reconstruct-12 copy: every shape reads the two-row links
    const bool r12 = prec == WD_F32 && gg->U12[WD_F32] != nullptr;
    if (sh.xylds == 2 && np <= 256 && prec != WD_F64 && g.L[2] >= 2) {
        // z-marching columns: nchunk (even, at most Lz) chunks per column
        int nch = sh.strip >= 2 ? sh.strip & ~1 : 2;
        if (nch > g.L[2]) nch = g.L[2] & ~1;
        const size_t lds = 2 * (size_t)(prec == WD_F64 ? 192 : 96) * np;
        FieldPtr fi{(void *)in, g.V, nrhs}, fo{out, g.V, nrhs};
        const void *U = r12 ? gg->U12[WD_F32] : gg->U[prec];
        const dim3 grid(nch * g.L[3] * nrhs), block(np);
        const int ord = sh.gmajor;
        const double diag = 4.0 + m0;
        switch (prec * 2 + (dag ? 1 : 0)) {
        case 2:
            if (r12) hipLaunchKernelGGL((k_dslash_zm<P32, false, true>), grid, block, lds, st, g, diag, U, fi, fo, nch, sh.remap, ord);
            else hipLaunchKernelGGL((k_dslash_zm<P32, false>), grid, block, lds, st, g, diag, U, fi, fo, nch, sh.remap, ord);
            break;
        case 3:
            if (r12) hipLaunchKernelGGL((k_dslash_zm<P32, true, true>), grid, block, lds, st, g, diag, U, fi, fo, nch, sh.remap, ord);
            else hipLaunchKernelGGL((k_dslash_zm<P32, true>), grid, block, lds, st, g, diag, U, fi, fo, nch, sh.remap, ord);
            break;
        case 4: hipLaunchKernelGGL((k_dslash_zm<P16, false>), grid, block, lds, st, g, diag, U, fi, fo, nch, sh.remap, ord); break;
        case 5: hipLaunchKernelGGL((k_dslash_zm<P16, true>), grid, block, lds, st, g, diag, U, fi, fo, nch, sh.remap, ord); break;
        default: return fail(WD_EINVAL, "unknown precision %d", prec);
        }
        WD_HIP(hipGetLastError());
        return WD_OK;
    }
    if (sh.xylds && np <= 256) {   // else the site-blocked kernel below
        const int nrx = prec == WD_F64 ? 1 : std::min(nr, 2);
        const int ngx = (nrhs + nrx - 1) / nrx;
        const int kp = xy_planes(sh, g, prec, nrx);
        const int npb = kp * np;   // sites per block
        size_t lds = xy_lds_bytes(prec, nrx, npb);
        // fewer resident blocks keep an XCD's in-flight data within its L2: the
        // LDS request is padded so at most occ blocks fit the 160 KB of a CU
        if (sh.occ > 0 && (size_t)(163840 / sh.occ) > lds) lds = std::min<size_t>(163840 / sh.occ, 65536);
        FieldPtr fi{(void *)in, g.V, nrhs}, fo{out, g.V, nrhs};
        const void *U = r12 ? gg->U12[WD_F32] : gg->U[prec];
        const dim3 grid((g.V / npb) * ngx);
        int ord = sh.ordered == 3 || sh.ordered == 5 ? sh.ordered : 1;
        if (kp > 1 && ord == 1) ord = 3;
        switch (prec * 2 + (dag ? 1 : 0)) {
        case 0: launch_xy<P64, false>(nrx, ord, grid, npb, lds, st, g, 4.0 + m0, U, fi, fo, ngx, sh.remap, od, kp > 1); break;
        case 1: launch_xy<P64, true>(nrx, ord, grid, npb, lds, st, g, 4.0 + m0, U, fi, fo, ngx, sh.remap, od, kp > 1); break;
        case 2:
            if (r12) launch_xy<P32, false, true>(nrx, ord, grid, npb, lds, st, g, 4.0 + m0, U, fi, fo, ngx, sh.remap, od, kp > 1);
            else launch_xy<P32, false>(nrx, ord, grid, npb, lds, st, g, 4.0 + m0, U, fi, fo, ngx, sh.remap, od, kp > 1);
            break;
        case 3:
            if (r12) launch_xy<P32, true, true>(nrx, ord, grid, npb, lds, st, g, 4.0 + m0, U, fi, fo, ngx, sh.remap, od, kp > 1);
            else launch_xy<P32, true>(nrx, ord, grid, npb, lds, st, g, 4.0 + m0, U, fi, fo, ngx, sh.remap, od, kp > 1);
            break;
        case 4: launch_xy<P16, false>(nrx, ord, grid, npb, lds, st, g, 4.0 + m0, U, fi, fo, ngx, sh.remap, od, kp > 1); break;
        case 5: launch_xy<P16, true>(nrx, ord, grid, npb, lds, st, g, 4.0 + m0, U, fi, fo, ngx, sh.remap, od, kp > 1); break;
        default: return fail(WD_EINVAL, "unknown precision %d", prec);
        }
        WD_HIP(hipGetLastError());
        return WD_OK;
    }
    const dim3 grid(nsb * ((ngroups + rl - 1) / rl)), block(blk);
    FieldPtr fi{(void *)in, g.V, nrhs}, fo{out, g.V, nrhs};
    const void *U = r12 ? gg->U12[WD_F32] : gg->U[prec];
    const double diag = 4.0 + m0;
    switch (prec * 2 + (dag ? 1 : 0)) {
    case 0: launch_nr<P64, false>(nr, sh.ordered, rl, grid, block, st, g, diag, U, fi, fo, ngroups, sh.remap, od); break;
    case 1: launch_nr<P64, true>(nr, sh.ordered, rl, grid, block, st, g, diag, U, fi, fo, ngroups, sh.remap, od); break;
    case 2:
        if (r12) launch_nr<P32, false, true>(nr, sh.ordered, rl, grid, block, st, g, diag, U, fi, fo, ngroups, sh.remap, od);
        else launch_nr<P32, false>(nr, sh.ordered, rl, grid, block, st, g, diag, U, fi, fo, ngroups, sh.remap, od);
        break;
    case 3:
        if (r12) launch_nr<P32, true, true>(nr, sh.ordered, rl, grid, block, st, g, diag, U, fi, fo, ngroups, sh.remap, od);
        else launch_nr<P32, true>(nr, sh.ordered, rl, grid, block, st, g, diag, U, fi, fo, ngroups, sh.remap, od);
        break;
    case 4: launch_nr<P16, false>(nr, sh.ordered, rl, grid, block, st, g, diag, U, fi, fo, ngroups, sh.remap, od); break;
    case 5: launch_nr<P16, true>(nr, sh.ordered, rl, grid, block, st, g, diag, U, fi, fo, ngroups, sh.remap, od); break;
    default: return fail(WD_EINVAL, "unknown precision %d", prec);
    }
    WD_HIP(hipGetLastError());
    return WD_OK;
}

// Device memory of wd_dslash_noalloc: the packed input and output of one call.
// Host code never passes the name itself to a kernel (on the host it is a
// stand-in, not a device address); it uses the address hipGetSymbolAddress
// returns for the current device, taken once per device.
static __device__ __align__(256) unsigned char scratch[WD_NOALLOC_SCRATCH_BYTES];

static int scratch_ptr(unsigned char **out) {
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static unsigned char *ptr[MAX_DEVICES];
    int dev = 0;
    WD_HIP(hipGetDevice(&dev));
    WD_CHECK(dev >= 0 && dev < MAX_DEVICES, WD_ENODEV, "device ordinal %d beyond %d", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(WD_EHIP, "hipGetSymbolAddress of the static scratch on device %d: %s", dev,
                        hipGetErrorString(e));
        ptr[dev] = (unsigned char *)p;
    }
    *out = ptr[dev];
    return WD_OK;
}

// scratch_a/scratch_b: where the canonical path keeps the packed in/out; null =
// allocate them on the stream
static int dslash_entry(const wd_gauge *g, double m0, int32_t prec, const void *in, void *out,
                        int32_t nrhs, uint32_t flags, void *stream, bool dag, bool noalloc = false) {
    clear_error();
    WD_CHECK(g && in && out, WD_EINVAL, "null argument");
    WD_CHECK(prec >= 0 && prec <= 2, WD_EINVAL, "unknown precision %d", prec);
    WD_CHECK(nrhs >= 1 && nrhs <= MAX_RHS, WD_EINVAL, "nrhs %d out of range 1..%d", nrhs, MAX_RHS);
    WD_CHECK((flags & ~WD_PACKED) == 0, WD_EINVAL, "unknown flags 0x%x", flags);
    WD_CHECK(g->U[prec] != nullptr, WD_EINVAL, "gauge handle holds no links in precision %d", prec);
    WD_CHECK(in != out, WD_EINVAL, "in and out must not overlap");
    WD_CHECK(m0 == m0, WD_EINVAL, "m0 is NaN");
    int rc = require_gfx950();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    ShapeKey key{{g->dims[0], g->dims[1], g->dims[2], g->dims[3]}, prec, nrhs, dag ? 1 : 0};
    const Shape sh = shape_lookup(key);
    if (flags & WD_PACKED) return launch_dslash(g, m0, prec, dag, in, out, nrhs, sh, st);

    // canonical complex128 in/out: pack, apply, unpack through temporaries
    const size_t nb = spinor_bytes(prec, g->V, nrhs);
    if (noalloc) {
        // the two packed buffers, each at a 256-byte boundary, in the static scratch
        const size_t nba = (nb + 255) & ~(size_t)255;
        WD_CHECK(2 * nba <= (size_t)WD_NOALLOC_SCRATCH_BYTES, WD_ETOOBIG,
                 "%d fields of %lld sites in precision %d need %zu bytes of scratch, the static scratch holds %zu",
                 nrhs, (long long)g->V, prec, 2 * nba, (size_t)WD_NOALLOC_SCRATCH_BYTES);
        unsigned char *sp = nullptr;
        rc = scratch_ptr(&sp);
        if (rc) return rc;
        rc = launch_pack_spinor(prec, in, sp, (int)g->V, nrhs, st);
        if (!rc) rc = launch_dslash(g, m0, prec, dag, sp, sp + nba, nrhs, sh, st);
        if (!rc) rc = launch_unpack_spinor(prec, sp + nba, out, (int)g->V, nrhs, st);
        return rc;
    }
    void *a = nullptr, *b = nullptr;
    WD_HIP(hipMallocAsync(&a, nb, st));
    hipError_t e = hipMallocAsync(&b, nb, st);
    if (e != hipSuccess) {
        hipFreeAsync(a, st);
        return fail(WD_ENOMEM, "hipMallocAsync: %s", hipGetErrorString(e));
    }
    rc = launch_pack_spinor(prec, in, a, (int)g->V, nrhs, st);
    if (!rc) rc = launch_dslash(g, m0, prec, dag, a, b, nrhs, sh, st);
    if (!rc) rc = launch_unpack_spinor(prec, b, out, (int)g->V, nrhs, st);
    hipFreeAsync(a, st);
    hipFreeAsync(b, st);
    return rc;
}

}  // namespace wd

extern "C" {
int wd_dslash(const wd_gauge *g, double m0, int32_t prec, const void *in_dev, void *out_dev,
              int32_t nrhs, uint32_t flags, void *stream) {
    return wd::dslash_entry(g, m0, prec, in_dev, out_dev, nrhs, flags, stream, false);
}
int wd_dslash_dag(const wd_gauge *g, double m0, int32_t prec, const void *in_dev, void *out_dev,
                  int32_t nrhs, uint32_t flags, void *stream) {
    return wd::dslash_entry(g, m0, prec, in_dev, out_dev, nrhs, flags, stream, true);
}
int wd_dslash_noalloc(const wd_gauge *g, double m0, int32_t prec, int32_t dagger, const void *in_dev,
                      void *out_dev, int32_t nrhs, void *stream) {
    if (dagger != 0 && dagger != 1) {
        wd::clear_error();
        return wd::fail(WD_EINVAL, "dagger must be 0 or 1, not %d", dagger);
    }
    return wd::dslash_entry(g, m0, prec, in_dev, out_dev, nrhs, 0u, stream, dagger == 1, true);
}
}
