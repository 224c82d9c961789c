// Device-side building blocks of libwd: complex arithmetic, lattice geometry,
// packed field accessors in three storage precisions, and the spin-projected
// Wilson hopping term of Eq. (1) (arXiv 2111.14958, Sec. 1).
//
// Storage precisions:
//   P64  FP64 links and spinors, FP64 arithmetic
//   P32  FP32 links and spinors, FP32 arithmetic
//   P16  FP16 links, FP16 spinors with one FP32 norm per site, FP32 arithmetic
//
// Packed layouts (structure of arrays, sites fastest, so that the 64 lanes of a
// wavefront read 64 consecutive sites with one wide load per component chunk):
//   spinor P64  double2 [rhs][12][V]
//          P32  float4  [rhs][6][V]      (two complex components per float4)
//          P16  half8   [rhs][3][V]      (four complex components per 16 bytes)
//               + float [rhs][V] norms after the codes of all rhs
//   links  P64  double2 [mu][9][V]       (U_mu(x)[a][b] at index 3a+b)
//          P32  float2  [mu][9][V]       (reconstruct-12: [mu][6][V], rows 0 and 1)
//          P16  half2   [mu][9][V]       (reconstruct-12: [mu][6][V])
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wd {

enum : int { P64 = 0, P32 = 1, P16 = 2 };

typedef _Float16 h16;
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef _Float16 half8v __attribute__((ext_vector_type(8)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

// Field pointers handed to kernels through device-side records are generic
// pointers; accessing them through the global address space lets the compiler
// emit global (not flat) loads and stores.
template <typename T> using gptr = __attribute__((address_space(1))) T *;
template <typename T> __device__ __forceinline__ gptr<T> as_global(void *p) { return (gptr<T>)p; }
template <typename T> __device__ __forceinline__ gptr<const T> as_global(const void *p) { return (gptr<const T>)p; }

// Element of a plane.  base + plane must be the same in every lane of the
// wavefront (a field pointer plus plane number times plane bytes); it is moved
// to scalar registers, so each access is one load or store with a scalar base
// and a 32-bit vector byte offset and needs no 64-bit address arithmetic.
typedef __attribute__((address_space(1))) char gchar;
__device__ __forceinline__ gchar *wave_uniform(gchar *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (gchar *)(((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ gptr<const T> at(const void *base, size_t plane, uint32_t off) {
    return (gptr<const T>)(wave_uniform((gchar *)base + plane) + off);
}
template <typename T>
__device__ __forceinline__ gptr<T> at(void *base, size_t plane, uint32_t off) {
    return (gptr<T>)(wave_uniform((gchar *)base + plane) + off);
}

// Loads and stores of data a kernel touches once.  NT sets the nontemporal
// hint, which makes the L2 evict these lines first, so that stencil inputs
// which neighbouring blocks read again stay resident.
template <bool NT, typename T> __device__ __forceinline__ T ld(gptr<const T> p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename T> __device__ __forceinline__ void st(gptr<T> p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <int P> struct real_of { typedef float type; };
template <> struct real_of<P64> { typedef double type; };

template <typename R> struct cx { R re, im; };

template <typename R> __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> __device__ __forceinline__ cx<R> times_i(cx<R> a) { return {-a.im, a.re}; }
template <typename R> __device__ __forceinline__ cx<R> times_mi(cx<R> a) { return {a.im, -a.re}; }
// a * b
template <typename R> __device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename R> __device__ __forceinline__ cx<R> cjmul(cx<R> a, cx<R> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R> __device__ __forceinline__ R norm2(cx<R> a) { return a.re * a.re + a.im * a.im; }

// ------------------------------------------------------------------ geometry
// Division by a lattice extent without the integer divide sequence (about 20
// vector instructions): division by an invariant integer through
// multiplication (Granlund and Montgomery, 1994).  For a divisor
// 1 <= d < 2^31 let l = ceil(log2 d) and M = floor(2^(32+l) / d) + 1.  Then
// e = M d - 2^(32+l) lies in (0, d], d <= 2^l, so n M / 2^(32+l) exceeds n / d
// by less than 1/d and floor(n M / 2^(32+l)) = floor(n / d) for n < 2^32.
// M = 2^32 + m with m = floor(2^32 (2^l - d) / d) + 1 < 2^32, hence
// floor(n M / 2^32) = mulhi(n, m) + n, which stays below 2^32 for n < 2^31
// (mulhi(n, m) < n): n / d = (mulhi(n, m) + n) >> l for 0 <= n < 2^31.
struct FastDiv {
    uint32_t m, l;
};
__host__ __device__ inline FastDiv fastdiv_make(uint32_t d) {
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    return FastDiv{(uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1), l};
}
__host__ __device__ __forceinline__ int fastdiv(int n, FastDiv f) {
    const uint32_t u = (uint32_t)n;
    return (int)(((uint32_t)(((uint64_t)u * f.m) >> 32) + u) >> f.l);
}

struct Geom {
    int L[4];     // Lx, Ly, Lz, Lt
    int S[4];     // strides 1, Lx, Lx*Ly, Lx*Ly*Lz
    int V;        // sites
    int tsign;    // time boundary sign, carried by the t-links of the last slice
    FastDiv dL[3];   // division by Lx, Ly, Lz
    FastDiv dP;      // division by the sites of an xy-plane, Lx Ly
};
// the geometry of a dims[0] x dims[1] x dims[2] x dims[3] lattice
__host__ __device__ inline Geom geom_of(const int dims[4], int tsign) {
    Geom g;
    for (int d = 0; d < 4; ++d) g.L[d] = dims[d];
    g.S[0] = 1;
    g.S[1] = g.L[0];
    g.S[2] = g.L[0] * g.L[1];
    g.S[3] = g.L[0] * g.L[1] * g.L[2];
    g.V = g.S[3] * g.L[3];
    g.tsign = tsign;
    for (int d = 0; d < 3; ++d) g.dL[d] = fastdiv_make((uint32_t)g.L[d]);
    g.dP = fastdiv_make((uint32_t)g.S[2]);
    return g;
}

// coordinates of site 0 <= s < V
__device__ __forceinline__ void site_coords(const Geom &g, int s, int c[4]) {
    const int q0 = fastdiv(s, g.dL[0]), q1 = fastdiv(q0, g.dL[1]), q2 = fastdiv(q1, g.dL[2]);
    c[0] = s - q0 * g.L[0];
    c[1] = q0 - q1 * g.L[1];
    c[2] = q1 - q2 * g.L[2];
    c[3] = q2;
}

// ------------------------------------------------------------- spinor views
// Base pointer of a packed field holding nrhs right-hand sides on V sites.
struct FieldPtr {
    void *p;
    int V;
    int nrhs;
};

template <int P> struct Spinor;

template <> struct Spinor<P64> {
    typedef double R;
    static constexpr int BYTES_PER_SITE = 192;
    template <bool NT = false>
    __device__ static __forceinline__ void load(const FieldPtr &f, int r, int s, cx<R> o[12]) {
        const size_t pb = (size_t)f.V * 16;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const d2v v = ld<NT>(at<d2v>((const void *)f.p, (size_t)(r * 12 + k) * pb, (uint32_t)s * 16u));
            o[k] = {v.x, v.y};
        }
    }
    template <bool NT = false>
    __device__ static __forceinline__ void store(const FieldPtr &f, int r, int s, const cx<R> o[12]) {
        const size_t pb = (size_t)f.V * 16;
#pragma unroll
        for (int k = 0; k < 12; ++k)
            st<NT>(at<d2v>(f.p, (size_t)(r * 12 + k) * pb, (uint32_t)s * 16u), d2v{o[k].re, o[k].im});
    }
};

template <> struct Spinor<P32> {
    typedef float R;
    static constexpr int BYTES_PER_SITE = 96;
    template <bool NT = false>
    __device__ static __forceinline__ void load(const FieldPtr &f, int r, int s, cx<R> o[12]) {
        const size_t pb = (size_t)f.V * 16;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const f4v v = ld<NT>(at<f4v>((const void *)f.p, (size_t)(r * 6 + j) * pb, (uint32_t)s * 16u));
            o[2 * j] = {v.x, v.y};
            o[2 * j + 1] = {v.z, v.w};
        }
    }
    template <bool NT = false>
    __device__ static __forceinline__ void store(const FieldPtr &f, int r, int s, const cx<R> o[12]) {
        const size_t pb = (size_t)f.V * 16;
#pragma unroll
        for (int j = 0; j < 6; ++j)
            st<NT>(at<f4v>(f.p, (size_t)(r * 6 + j) * pb, (uint32_t)s * 16u),
                   f4v{o[2 * j].re, o[2 * j].im, o[2 * j + 1].re, o[2 * j + 1].im});
    }
};

template <> struct Spinor<P16> {
    typedef float R;
    static constexpr int BYTES_PER_SITE = 52;
    // byte offset of the norm plane of rhs r
    __device__ static __forceinline__ size_t norm_plane(const FieldPtr &f, int r) {
        return (size_t)f.nrhs * 3 * f.V * 16 + (size_t)r * f.V * 4;
    }
    template <bool NT = false>
    __device__ static __forceinline__ void load(const FieldPtr &f, int r, int s, cx<R> o[12]) {
        const size_t pb = (size_t)f.V * 16;
        const float n = ld<NT>(at<float>((const void *)f.p, norm_plane(f, r), (uint32_t)s * 4u));
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const half8v v = ld<NT>(at<half8v>((const void *)f.p, (size_t)(r * 3 + j) * pb, (uint32_t)s * 16u));
#pragma unroll
            for (int k = 0; k < 4; ++k) o[4 * j + k] = {n * (float)v[2 * k], n * (float)v[2 * k + 1]};
        }
    }
    // Quantise: norm = max |re|,|im| over the site, inv = 1 / norm (FP32, one
    // division per site); the scaled value q = v inv is the FP32 product, or
    // the FP32 quotient v / norm where 1 / norm overflows (norm < 2^-128);
    // code = half(q), rounded to nearest even.  Returns the stored values in o.
    template <bool NT = false>
    __device__ static __forceinline__ void store(const FieldPtr &f, int r, int s, cx<R> o[12]) {
        float n = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) n = fmaxf(n, fmaxf(fabsf(o[k].re), fabsf(o[k].im)));
        const float inv = n > 0.f ? 1.f / n : 0.f;
        float q[24];
        if (inv < INFINITY) {   // also n == 0 (inv 0: the codes are 0)
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                q[2 * k] = n > 0.f ? o[k].re * inv : 0.f;
                q[2 * k + 1] = n > 0.f ? o[k].im * inv : 0.f;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                q[2 * k] = o[k].re / n;
                q[2 * k + 1] = o[k].im / n;
            }
        }
        const size_t pb = (size_t)f.V * 16;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            half8v v;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                // the FP32 value is final before the conversion (no fused
                // multiply-and-round-to-half)
                asm volatile("" : "+v"(q[8 * j + k]));
                v[k] = (h16)q[8 * j + k];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) o[4 * j + k] = {n * (float)v[2 * k], n * (float)v[2 * k + 1]};
            st<NT>(at<half8v>(f.p, (size_t)(r * 3 + j) * pb, (uint32_t)s * 16u), v);
        }
        st<NT>(at<float>(f.p, norm_plane(f, r), (uint32_t)s * 4u), n);
    }
};

// --------------------------------------------------------------- link views
// Link<P>::load<R12>(U, g, mu, s, last_t, u): the link U_mu at site s.  last_t:
// s is on the last time slice and mu = t, so the stored link carries the
// boundary sign.  With reconstruct-12 (R12: a gauge's extra FP32/FP16 copies
// in the [mu][6][V] layout) only rows 0 and 1 are stored.  The third row of an SU(3) matrix is the complex conjugate of the
// cross product of the first two.  A link stored times the boundary sign -1
// has determinant -1, so its third row is that product times -1.
template <int P> struct Link;

template <typename R>
__device__ __forceinline__ void third_row(cx<R> u[9], R sg) {
    const cx<R> c0 = cmul(u[1], u[5]) - cmul(u[2], u[4]);
    const cx<R> c1 = cmul(u[2], u[3]) - cmul(u[0], u[5]);
    const cx<R> c2 = cmul(u[0], u[4]) - cmul(u[1], u[3]);
    u[6] = {sg * c0.re, -sg * c0.im};
    u[7] = {sg * c1.re, -sg * c1.im};
    u[8] = {sg * c2.re, -sg * c2.im};
}

template <> struct Link<P64> {
    typedef double R;
    static constexpr int BYTES_PER_LINK = 144;
    template <bool R12 = false>   // the FP64 copy is always complete
    __device__ static __forceinline__ void load(const void *U, const Geom &g, int mu, int s, bool, cx<R> u[9]) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const d2v v = *at<d2v>(U, (size_t)(mu * 9 + k) * g.V * 16, (uint32_t)s * 16u);
            u[k] = {v.x, v.y};
        }
    }
};
template <> struct Link<P32> {
    typedef float R;
    static constexpr int BYTES_PER_LINK = 72;
    template <bool R12 = false>
    __device__ static __forceinline__ void load(const void *U, const Geom &g, int mu, int s, bool last_t,
                                                cx<R> u[9]) {
        constexpr int nk = R12 ? 6 : 9;   // stored entries per link
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const f2v v = *at<f2v>(U, (size_t)(mu * nk + k) * g.V * 8, (uint32_t)s * 8u);
            u[k] = {v.x, v.y};
        }
        if constexpr (R12) {
            third_row<R>(u, last_t ? (R)g.tsign : R(1));
        } else {
#pragma unroll
            for (int k = 6; k < 9; ++k) {
                const f2v v = *at<f2v>(U, (size_t)(mu * 9 + k) * g.V * 8, (uint32_t)s * 8u);
                u[k] = {v.x, v.y};
            }
        }
    }
};
template <> struct Link<P16> {
    typedef float R;
    static constexpr int BYTES_PER_LINK = 36;
    template <bool R12 = false>
    __device__ static __forceinline__ void load(const void *U, const Geom &g, int mu, int s, bool last_t,
                                                cx<R> u[9]) {
        constexpr int nk = R12 ? 6 : 9;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const half2v v = *at<half2v>(U, (size_t)(mu * nk + k) * g.V * 4, (uint32_t)s * 4u);
            u[k] = {(float)v.x, (float)v.y};
        }
        if constexpr (R12) {
            third_row<R>(u, last_t ? (R)g.tsign : R(1));
        } else {
#pragma unroll
            for (int k = 6; k < 9; ++k) {
                const half2v v = *at<half2v>(U, (size_t)(mu * 9 + k) * g.V * 4, (uint32_t)s * 4u);
                u[k] = {(float)v.x, (float)v.y};
            }
        }
    }
};

// ------------------------------------------------- spin projection, Eq. (1)
// In the DeGrand-Rossi basis gamma_mu = [[0, B_mu], [B_mu^dagger, 0]] with
// B_x = i sigma_1, B_y = -i sigma_2, B_z = i sigma_3, B_t = 1.  For a spinor
// psi = (u; d) (spins 0,1 | 2,3):
//   (1 + S gamma_mu) psi = (h ; S B_mu^dagger h),   h = u + S B_mu d,   S = +-1.
// The colour link commutes with the spin structure, so a hop multiplies only
// the two-spin half spinor h by the link and rebuilds the lower spins after.

// h = u + S * B_mu d  (h: 2 spins x 3 colours)
template <int MU, int S, typename R>
__device__ __forceinline__ void project(const cx<R> p[12], cx<R> h[6]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cx<R> d0 = p[6 + c], d1 = p[9 + c];
        cx<R> b0, b1;
        if constexpr (MU == 0) { b0 = times_i(d1); b1 = times_i(d0); }
        else if constexpr (MU == 1) { b0 = -d1; b1 = d0; }
        else if constexpr (MU == 2) { b0 = times_i(d0); b1 = times_mi(d1); }
        else { b0 = d0; b1 = d1; }
        if constexpr (S > 0) { h[c] = p[c] + b0; h[3 + c] = p[3 + c] + b1; }
        else { h[c] = p[c] - b0; h[3 + c] = p[3 + c] - b1; }
    }
}

// acc_upper += w, acc_lower += S * B_mu^dagger w
template <int MU, int S, typename R>
__device__ __forceinline__ void accumulate(const cx<R> w[6], cx<R> acc[12]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cx<R> w0 = w[c], w1 = w[3 + c];
        acc[c] = acc[c] + w0;
        acc[3 + c] = acc[3 + c] + w1;
        cx<R> l0, l1;
        if constexpr (MU == 0) { l0 = times_mi(w1); l1 = times_mi(w0); }
        else if constexpr (MU == 1) { l0 = w1; l1 = -w0; }
        else if constexpr (MU == 2) { l0 = times_mi(w0); l1 = times_i(w1); }
        else { l0 = w0; l1 = w1; }
        if constexpr (S > 0) { acc[6 + c] = acc[6 + c] + l0; acc[9 + c] = acc[9 + c] + l1; }
        else { acc[6 + c] = acc[6 + c] - l0; acc[9 + c] = acc[9 + c] - l1; }
    }
}

// w = U h   (per spin component).  Each output component is one multiply and
// five fused multiply-adds.
template <typename R>
__device__ __forceinline__ void link_mul(const cx<R> u[9], const cx<R> h[6], cx<R> w[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const cx<R> u0 = u[3 * a], u1 = u[3 * a + 1], u2 = u[3 * a + 2];
            const cx<R> h0 = h[3 * sp], h1 = h[3 * sp + 1], h2 = h[3 * sp + 2];
            R re = u0.re * h0.re;
            re = fma(-u0.im, h0.im, re);
            re = fma(u1.re, h1.re, re);
            re = fma(-u1.im, h1.im, re);
            re = fma(u2.re, h2.re, re);
            re = fma(-u2.im, h2.im, re);
            R im = u0.re * h0.im;
            im = fma(u0.im, h0.re, im);
            im = fma(u1.re, h1.im, im);
            im = fma(u1.im, h1.re, im);
            im = fma(u2.re, h2.im, im);
            im = fma(u2.im, h2.re, im);
            w[3 * sp + a] = {re, im};
        }
}

// w = U^dagger h
template <typename R>
__device__ __forceinline__ void link_adj_mul(const cx<R> u[9], const cx<R> h[6], cx<R> w[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const cx<R> u0 = u[a], u1 = u[3 + a], u2 = u[6 + a];
            const cx<R> h0 = h[3 * sp], h1 = h[3 * sp + 1], h2 = h[3 * sp + 2];
            R re = u0.re * h0.re;
            re = fma(u0.im, h0.im, re);
            re = fma(u1.re, h1.re, re);
            re = fma(u1.im, h1.im, re);
            re = fma(u2.re, h2.re, re);
            re = fma(u2.im, h2.im, re);
            R im = u0.re * h0.im;
            im = fma(-u0.im, h0.re, im);
            im = fma(u1.re, h1.im, im);
            im = fma(-u1.im, h1.re, im);
            im = fma(u2.re, h2.im, im);
            im = fma(-u2.im, h2.re, im);
            w[3 * sp + a] = {re, im};
        }
}

template <int MU> struct IntC { static constexpr int value = MU; };

// A block's copy of one xy-plane of spinors in LDS, [NR][components][np]
// with np = sites of the plane (the block size): FP64 as 12 double2 per site,
// FP32 and FP16N (decoded) as 6 float4 per site.  Consecutive sites are
// consecutive 16-byte words, so a wavefront's accesses are conflict free.
template <int P> struct LdsSpinor {
    static constexpr int BYTES = 96;
    __device__ static __forceinline__ void put(f4v *b, int np, int j, int i, const cx<float> v[12]) {
#pragma unroll
        for (int k = 0; k < 6; ++k) b[(j * 6 + k) * np + i] = f4v{v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im};
    }
    __device__ static __forceinline__ void get(const f4v *b, int np, int j, int i, cx<float> v[12]) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const f4v w = b[(j * 6 + k) * np + i];
            v[2 * k] = {w.x, w.y};
            v[2 * k + 1] = {w.z, w.w};
        }
    }
    typedef f4v word;
};
template <> struct LdsSpinor<P64> {
    static constexpr int BYTES = 192;
    __device__ static __forceinline__ void put(d2v *b, int np, int j, int i, const cx<double> v[12]) {
#pragma unroll
        for (int k = 0; k < 12; ++k) b[(j * 12 + k) * np + i] = d2v{v[k].re, v[k].im};
    }
    __device__ static __forceinline__ void get(const d2v *b, int np, int j, int i, cx<double> v[12]) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const d2v w = b[(j * 12 + k) * np + i];
            v[k] = {w.x, w.y};
        }
    }
    typedef d2v word;
};

// Hopping sum of Eq. (1) at site s for NR right-hand sides of field `in`
// starting at rhs0 (only those whose bit is set in `act` are touched):
//   acc = sum_mu [ (1 + SF gamma_mu) U_mu(s) psi(s+mu) + (1 + SB gamma_mu) U_mu(s-mu)^dag psi(s-mu) ]
// with SF = -1, SB = +1 for D and SF = +1, SB = -1 for D^dagger.  The boundary
// sign of the hops in t that wrap around is carried by the packed t-links of
// the last time slice (both such hops use those links).  Each link is loaded
// once and applied to all NR right-hand sides.
//
// XYLDS: the neighbours in x and y are read from the block's LDS copy of its
// xy-plane (`xy`, plane starting at site `plane0`, np sites) instead of memory.
// HALF: `in` holds only the sites of the other parity, site n at index n / 2
// (even-odd preconditioning; needs an even Lx); with XYLDS, plane0 and np
// count half indices (the block's half-plane).
// R12: U is a reconstruct-12 copy (two rows per link, FP32/FP16).
// ZIN (with XYLDS; a block of several z-adjacent xy-planes, whose sites are
// consecutive, all staged in `xy`): a z neighbour that lies in the block's
// planes is read from LDS, the others from memory.
// ZM (with XYLDS; for a block that walks a column of xy-planes in z): `zn` is
// the LDS copy of the next plane, which supplies the forward z neighbour.  The
// backward z hop is not formed here: acc starts from `carry`, which holds it
// on entry, and on return `carry` holds the backward z hop of site s + z,
// (1 + SB gamma_z) U_z(s)^dag psi(s), made from the link the forward z hop loads.
template <int P, bool DAG, int NR, int ORDERED = 1, bool XYLDS = false, bool HALF = false, bool ZM = false,
          bool R12 = false, bool ZIN = false>
__device__ __forceinline__ void hopping(const Geom &g, int s, const void *U, const FieldPtr &in,
                                        int rhs0, unsigned act, cx<typename real_of<P>::type> acc[NR][12],
                                        const cx<typename real_of<P>::type> (*first)[12] = nullptr,
                                        const typename LdsSpinor<P>::word *xy = nullptr, int plane0 = 0,
                                        int np = 0, const typename LdsSpinor<P>::word *zn = nullptr,
                                        cx<typename real_of<P>::type> (*carry)[12] = nullptr) {
    static_assert(!ZM || XYLDS, "z-marching reads the x and y neighbours from LDS");
    static_assert(!ZIN || (XYLDS && !ZM && !HALF), "z neighbours from LDS: multi-plane blocks only");
    typedef typename real_of<P>::type R;
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    int c[4];
    site_coords(g, s, c);
#pragma unroll
    for (int j = 0; j < NR; ++j)
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[j][k] = ZM ? carry[j][k] : cx<R>{R(0), R(0)};

    // ORDERED (1): one hop at a time.  Each hop's load addresses pass through empty asm
    // statements that also consume every accumulator of the previous hop, so
    // the compiler cannot
    // hoist the loads of all eight hops ahead of the arithmetic (it treats the
    // field loads as unclobbered and would otherwise do so, exhausting the
    // register file: FP64 needs 36 registers per link and 48 per neighbour
    // spinor, and the kernel spills to scratch).  Latency is hidden by
    // occupancy instead.  Unordered, the compiler schedules freely (kept for
    // the operator kernel, where the autotuner may prefer it).
    // make the index values depend on every accumulator (no instructions)
    auto after_acc = [&](int &a, int &b) {
#pragma unroll
        for (int j = 0; j < NR; ++j)
#pragma unroll
            for (int k = 0; k < 12; ++k)
                asm volatile("" : "+v"(a), "+v"(b) : "v"(acc[j][k].re), "v"(acc[j][k].im));
    };
    // neighbour and link-site index of every hop h = 2 mu + (backward ? 1 : 0)
    int nbi[8], lsi[8];
    // ORDERED 4: as 3, and the caller's values `first` (the site's own spinor,
    // loaded before the call) are in registers before any hop is issued, so
    // the own-site load and the x/y neighbour loads touch their common cache
    // lines close together in time
    auto after_first = [&](int &a) {
        if (first)
#pragma unroll
            for (int j = 0; j < NR; ++j)
                asm volatile("" : "+v"(a) : "v"(first[j][0].re), "v"(first[j][11].im));
    };
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        nbi[2 * mu] = c[mu] == g.L[mu] - 1 ? s - (g.L[mu] - 1) * g.S[mu] : s + g.S[mu];
        nbi[2 * mu + 1] = c[mu] == 0 ? s + (g.L[mu] - 1) * g.S[mu] : s - g.S[mu];
        lsi[2 * mu] = s;
        lsi[2 * mu + 1] = nbi[2 * mu + 1];
    }
    auto hop = [&](auto hc) {
        constexpr int H = decltype(hc)::value;
        constexpr int MU = H / 2;
        constexpr bool FWD = (H % 2) == 0;
        constexpr int S = FWD ? SF : SB;
        // ORDERED 1: this hop's loads wait for every earlier hop's arithmetic.
        // ORDERED 2: a direction's two hops are issued together.
        // ORDERED 3: software pipeline, the loads of hop H+1 are released as soon
        //            as hop H-1's arithmetic is done (two hops in flight).
        if constexpr (ORDERED == 1) after_acc(nbi[H], lsi[H]);
        if constexpr (ORDERED == 2 && FWD) after_acc(nbi[H], lsi[H]);
        if constexpr (ORDERED == 2 && FWD) after_acc(nbi[H + 1], lsi[H + 1]);
        if constexpr ((ORDERED == 3 || ORDERED == 4) && H + 1 < 8) after_acc(nbi[H + 1], lsi[H + 1]);
        // ORDERED 5: as 3 in the sequence z+ z- t+ t- x+ x- y+ y- (the hops that
        // read memory first, close in time to the neighbouring blocks' loads of
        // their own planes; the LDS hops last)
        if constexpr (ORDERED == 5 && H != 3) after_acc(nbi[H == 7 ? 0 : H + 1], lsi[H == 7 ? 0 : H + 1]);
        if constexpr (ORDERED == 4 && H == 0) after_first(nbi[0]);
        if constexpr (ZM && MU == 2 && !FWD) return;   // carried in from the previous plane
        const int nb = nbi[H];
        cx<R> u[9];
        // the t-link of the last slice: the forward hop from t = Lt-1, the backward hop from t = 0
        Link<P>::template load<R12>(U, g, MU, lsi[H], MU == 3 && c[3] == (FWD ? g.L[3] - 1 : 0), u);
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            if (act >> j & 1) {
                cx<R> p[12], h[6], w[6];
                if constexpr (XYLDS && MU < 2) LdsSpinor<P>::get(xy, np, j, (HALF ? nb >> 1 : nb) - plane0, p);
                else if constexpr (ZM && MU == 2) LdsSpinor<P>::get(zn, np, j, s - plane0, p);
                else if constexpr (ZIN && MU == 2) {
                    const int li = nb - plane0;   // in the block's planes: only one wave can diverge
                    if ((unsigned)li < (unsigned)np) LdsSpinor<P>::get(xy, np, j, li, p);
                    else Spinor<P>::load(in, rhs0 + j, nb, p);
                } else Spinor<P>::load(in, rhs0 + j, HALF ? nb >> 1 : nb, p);
                project<MU, S>(p, h);
                if constexpr (FWD) link_mul(u, h, w);
                else link_adj_mul(u, h, w);
                accumulate<MU, S>(w, acc[j]);
                if constexpr (ZM && MU == 2) {   // backward z hop of s + z from this link and psi(s)
                    LdsSpinor<P>::get(xy, np, j, s - plane0, p);
                    project<2, SB>(p, h);
                    link_adj_mul(u, h, w);
#pragma unroll
                    for (int k = 0; k < 12; ++k) carry[j][k] = {R(0), R(0)};
                    accumulate<2, SB>(w, carry[j]);
                }
            }
        }
    };
    if constexpr (ORDERED == 5) {
        hop(IntC<4>{});
        hop(IntC<5>{});
        hop(IntC<6>{});
        hop(IntC<7>{});
        hop(IntC<0>{});
        hop(IntC<1>{});
        hop(IntC<2>{});
        hop(IntC<3>{});
    } else {
        hop(IntC<0>{});
        hop(IntC<1>{});
        hop(IntC<2>{});
        hop(IntC<3>{});
        hop(IntC<4>{});
        hop(IntC<5>{});
        hop(IntC<6>{});
        hop(IntC<7>{});
    }
}

// Hopping sum of Eq. (1) at site s for a block that walks a column of
// xy-planes along z (one rhs, one t).  The block's LDS holds plane z (`xy`,
// first site plane0, np sites: the x and y neighbours); the thread holds its
// own spinor (read back from `xy`) and `nxt`, its site's spinor on the next plane of the walk
// (z + 1 upward, z - 1 downward), which is its z neighbour on that side; the
// z hop from the other side arrives in `carry`, formed on the previous plane.
// sn is the site of nxt.  The t neighbours come from memory.
//   upward:   acc = carry + ... + (1 + SF g_z) U_z(s) nxt,
//             carry <- (1 + SB g_z) U_z(s)^dag self   (the backward hop of sn)
//   downward: acc = carry + ... + (1 + SB g_z) U_z(sn)^dag nxt,
//             carry <- (1 + SF g_z) U_z(sn) self      (the forward hop of sn)
// Both use the one link between the two planes.  Loads are issued hop by hop,
// one (ORD 1) or two (ORD 3) hops in flight, as in hopping().
template <int P, bool DAG, bool DOWN, bool R12 = false, int ORD = 3>
__device__ __forceinline__ void march_hopping(const Geom &g, int s, int sn, const void *U, const FieldPtr &in,
                                              int rhs, const typename LdsSpinor<P>::word *xy, int plane0, int np,
                                              const cx<typename real_of<P>::type> nxt[12],
                                              cx<typename real_of<P>::type> carry[12],
                                              cx<typename real_of<P>::type> acc[12]) {
    typedef typename real_of<P>::type R;
    constexpr int SF = DAG ? +1 : -1;
    constexpr int SB = -SF;
    int c[4];
    site_coords(g, s, c);
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = carry[k];
    // neighbour and link site of the x, y and t hops: h = 0..5 is x+, x-, y+, y-, t+, t-
    int nbi[6], lsi[6];
#pragma unroll
    for (int h = 0; h < 3; ++h) {
        const int mu = h == 2 ? 3 : h;
        nbi[2 * h] = c[mu] == g.L[mu] - 1 ? s - (g.L[mu] - 1) * g.S[mu] : s + g.S[mu];
        nbi[2 * h + 1] = c[mu] == 0 ? s + (g.L[mu] - 1) * g.S[mu] : s - g.S[mu];
        lsi[2 * h] = s;
        lsi[2 * h + 1] = nbi[2 * h + 1];
    }
    int zl = DOWN ? sn : s;   // site of the z link
    auto after_acc = [&](int &a, int &b) {
#pragma unroll
        for (int k = 0; k < 12; ++k) asm volatile("" : "+v"(a), "+v"(b) : "v"(acc[k].re), "v"(acc[k].im));
    };
    auto hop = [&](auto hc) {
        constexpr int H = decltype(hc)::value;
        constexpr int MU = H < 4 ? H / 2 : 3;
        constexpr bool FWD = (H % 2) == 0;
        constexpr int S = FWD ? SF : SB;
        if constexpr (ORD == 1) after_acc(nbi[H], lsi[H]);
        else if constexpr (H + 1 < 6) after_acc(nbi[H + 1], lsi[H + 1]);
        else after_acc(zl, zl);
        cx<R> u[9], p[12], h[6], w[6];
        Link<P>::template load<R12>(U, g, MU, lsi[H], MU == 3 && c[3] == (FWD ? g.L[3] - 1 : 0), u);
        if constexpr (MU < 2) LdsSpinor<P>::get(xy, np, 0, nbi[H] - plane0, p);
        else Spinor<P>::load(in, rhs, nbi[H], p);
        project<MU, S>(p, h);
        if constexpr (FWD) link_mul(u, h, w);
        else link_adj_mul(u, h, w);
        accumulate<MU, S>(w, acc);
    };
    hop(IntC<0>{});
    hop(IntC<1>{});
    hop(IntC<2>{});
    hop(IntC<3>{});
    hop(IntC<4>{});
    hop(IntC<5>{});
    {   // the z hop towards the next plane, and the carry for it (own spinor from LDS)
        if constexpr (ORD == 1) after_acc(zl, zl);
        cx<R> u[9], h[6], w[6], self[12];
        Link<P>::template load<R12>(U, g, 2, zl, false, u);
        LdsSpinor<P>::get(xy, np, 0, s - plane0, self);
        if constexpr (DOWN) {
            project<2, SB>(nxt, h);
            link_adj_mul(u, h, w);
            accumulate<2, SB>(w, acc);
            project<2, SF>(self, h);
            link_mul(u, h, w);
#pragma unroll
            for (int k = 0; k < 12; ++k) carry[k] = {R(0), R(0)};
            accumulate<2, SF>(w, carry);
        } else {
            project<2, SF>(nxt, h);
            link_mul(u, h, w);
            accumulate<2, SF>(w, acc);
            project<2, SB>(self, h);
            link_adj_mul(u, h, w);
#pragma unroll
            for (int k = 0; k < 12; ++k) carry[k] = {R(0), R(0)};
            accumulate<2, SB>(w, carry);
        }
    }
}

// Apply D (or D^dagger): o = diag * psi(s) - 1/2 acc, with diag = 4 + m0.
template <typename R>
__device__ __forceinline__ void wilson_finish(R diag, const cx<R> self[12], const cx<R> acc[12], cx<R> o[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k)
        o[k] = {fma(R(-0.5), acc[k].re, diag * self[k].re), fma(R(-0.5), acc[k].im, diag * self[k].im)};
}

// Blocks are handed to the 8 XCDs round robin (block b runs on XCD b % 8).
// Remap so that each XCD works on one contiguous range of tiles: lattice
// neighbours then share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int xcd = b & 7, idx = b >> 3;
    const int per = n >> 3, rem = n & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// Site at position L of a kernel's processing order.  strip == 0: lexicographic
// order (x fastest).  strip = W > 0: the (z, t) planes are walked in strips of
// W consecutive z-planes, t-major within a strip, so a site's t neighbours are
// W planes away in the order (instead of Lz planes) and the data a block
// shares with the blocks processed around it stays in the XCD's L2.  Every
// xy-plane stays contiguous, so a wavefront's accesses remain coalesced.
__host__ __device__ __forceinline__ int order_site(const Geom &g, int strip, int L) {
    if (strip <= 0) return L;
    const int P = g.S[2];                           // sites per xy-plane
    const int q = fastdiv(L, g.dP), off = L - q * P; // plane number in the order, offset
    const int per = strip * g.L[3];       // planes of a full strip
    const int zb = q / per, qq = q - zb * per;
    const int w = g.L[2] - zb * strip < strip ? g.L[2] - zb * strip : strip;   // last strip may be narrower
    const int t = qq / w, zi = qq - t * w;
    return off + P * (zb * strip + zi + g.L[2] * t);
}

}  // namespace wd
