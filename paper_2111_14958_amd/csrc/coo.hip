// The Wilson-Dirac operator stored explicitly in coordinate format, as the
// paper does (arXiv 2111.14958, Sec. 2): three arrays Val, Row, Col hold every
// non-zero entry with its row and column index, and the product is
// out[Row[k]] += Val[k] * in[Col[k]].
//
// The entries are generated on the device from the packed FP64 links, row by
// row: row r = 12 n + 3 alpha + a (site n, spin alpha, colour a) holds 49
// entries -- the diagonal (4 + m0), then for mu = x, y, z, t the forward hop
// (spin beta with (1 -+ gamma_mu)_{alpha beta} != 0, colours b) and the
// backward hop.  Entry k of row r is stored at index k * rows + r (entry 0 of
// every row, then entry 1, ...): the product gives each row to one thread,
// which sums its 49 terms in entry order without atomics, and the threads of
// a wavefront read consecutive values and column indices (a row-after-row
// order would put a wavefront's loads 49 entries apart).  Row is kept as the
// format defines it (and for export).
// On lattices of extent 2 the forward and backward columns coincide; both
// entries are kept and summed, like duplicate coordinate entries.
#include "wd_device.h"
#include "wd_host.h"

namespace wd {

constexpr int COO_PER_ROW = 49;

// DeGrand-Rossi gamma matrices as (column, value) of the single non-zero of
// each row: gamma_mu[alpha][gcol[mu][alpha]] = gval[mu][alpha].
__constant__ int g_gcol[4][4] = {{3, 2, 1, 0}, {3, 2, 1, 0}, {2, 3, 0, 1}, {2, 3, 0, 1}};
// value as (re, im)
__constant__ double g_gval[4][4][2] = {
    {{0, 1}, {0, 1}, {0, -1}, {0, -1}},     // gamma_x = [[0, i sigma1], [-i sigma1, 0]]
    {{-1, 0}, {1, 0}, {1, 0}, {-1, 0}},     // gamma_y = [[0, -i sigma2], [i sigma2, 0]]
    {{0, 1}, {0, -1}, {0, -1}, {0, 1}},     // gamma_z = [[0, i sigma3], [-i sigma3, 0]]
    {{1, 0}, {1, 0}, {1, 0}, {1, 0}}};      // gamma_t = [[0, 1], [1, 0]]

template <typename T> struct CVal;
template <> struct CVal<double> { typedef double2 type; };
template <> struct CVal<float> { typedef float2 type; };

// One thread per row: write its 49 entries.
template <typename T>
__global__ void k_coo_build(Geom g, double diag, const double2 *__restrict__ U64, int dagger,
                            typename CVal<T>::type *__restrict__ val, int *__restrict__ row,
                            int *__restrict__ col) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= 12 * g.V) return;
    const int s = r / 12, al = (r % 12) / 3, a = r % 3;
    int c[4];
    site_coords(g, s, c);
    const size_t rows = (size_t)12 * g.V;
    int k = 0;
    auto put = [&](int cc, double re, double im) {
        const size_t e = (size_t)k * rows + r;
        val[e] = {(T)re, (T)im};
        row[e] = r;
        col[e] = cc;
        ++k;
    };
    put(r, diag, 0.0);
    const double sg = dagger ? -1.0 : 1.0;
    for (int mu = 0; mu < 4; ++mu) {
        const bool fwrap = c[mu] == g.L[mu] - 1, bwrap = c[mu] == 0;
        const int fw = fwrap ? s - (g.L[mu] - 1) * g.S[mu] : s + g.S[mu];
        const int bw = bwrap ? s + (g.L[mu] - 1) * g.S[mu] : s - g.S[mu];
        // projector row alpha: identity at beta = alpha, -+ sg gamma at beta = gcol
        const int gb = g_gcol[mu][al];
        const double gre = g_gval[mu][al][0], gim = g_gval[mu][al][1];
        for (int dir = 0; dir < 2; ++dir) {
            // forward: -1/2 (1 - sg gamma) U_mu(x) s_f ; backward: -1/2 (1 + sg gamma) U_mu(x-mu)^dag s_b
            const double ps = dir == 0 ? -sg : sg;
            const double sfac = -0.5;   // the boundary sign is in the packed t-links
            const int nb = dir == 0 ? fw : bw;
            const int ls = dir == 0 ? s : bw;
            for (int pass = 0; pass < 2; ++pass) {
                const int be = pass == 0 ? al : gb;
                const double pre = pass == 0 ? 1.0 : ps * gre, pim = pass == 0 ? 0.0 : ps * gim;
                for (int b = 0; b < 3; ++b) {
                    // link element: U_ab (forward) or conj(U_ba) (backward)
                    double2 u = dir == 0 ? U64[((size_t)mu * 9 + 3 * a + b) * g.V + ls]
                                         : U64[((size_t)mu * 9 + 3 * b + a) * g.V + ls];
                    if (dir == 1) u.y = -u.y;
                    const double re = sfac * (pre * u.x - pim * u.y);
                    const double im = sfac * (pre * u.y + pim * u.x);
                    put(12 * nb + 3 * be + b, re, im);
                }
            }
        }
    }
}

// out[row] = sum over the row's entries of Val * in[Col], nrhs vectors, up to
// four at a time (each entry read once per group of four vectors).  Every sum
// runs over the row's entries in entry order.
template <typename T>
__global__ void k_coo_spmv(const typename CVal<T>::type *__restrict__ val, const int *__restrict__ col,
                           const typename CVal<T>::type *__restrict__ in, typename CVal<T>::type *__restrict__ out,
                           int nrows, int nrhs) {
    typedef typename CVal<T>::type C;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    for (int v0 = 0; v0 < nrhs; v0 += 4) {
        const int nv = min(4, nrhs - v0);
        T sre[4] = {0, 0, 0, 0}, sim[4] = {0, 0, 0, 0};
        for (int k = 0; k < COO_PER_ROW; ++k) {
            const size_t e = (size_t)k * nrows + r;
            const C a = val[e];
            const int c = col[e];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (j < nv) {
                    const C b = in[(size_t)(v0 + j) * nrows + c];
                    sre[j] += a.x * b.x - a.y * b.y;
                    sim[j] += a.x * b.y + a.y * b.x;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < nv) out[(size_t)(v0 + j) * nrows + r] = {sre[j], sim[j]};
    }
}

}  // namespace wd

struct wd_coo {
    int prec;          // WD_F64 or WD_F32
    int64_t rows, nnz;
    void *val;
    int *row, *col;
    int device;
};

using namespace wd;

extern "C" {

int wd_coo_create(const wd_gauge *g, double m0, int32_t prec, int32_t dagger, void *stream, wd_coo **out) {
    clear_error();
    WD_CHECK(g && out, WD_EINVAL, "null argument");
    WD_CHECK(prec == WD_F64 || prec == WD_F32, WD_EINVAL, "coordinate format supports FP64 and FP32");
    WD_CHECK(m0 == m0, WD_EINVAL, "m0 is NaN");
    const int64_t rows = 12 * g->V, nnz = rows * COO_PER_ROW;
    WD_CHECK(nnz < ((int64_t)1 << 31) * 4, WD_EINVAL, "lattice too large for the coordinate format");
    int rc = require_gfx950();
    if (rc) return rc;
    wd_coo *h = new wd_coo();
    h->prec = prec;
    h->rows = rows;
    h->nnz = nnz;
    (void)hipGetDevice(&h->device);
    const size_t vb = (size_t)nnz * (prec == WD_F64 ? 16 : 8);
    h->val = nullptr;
    h->row = h->col = nullptr;
    if (hipMalloc(&h->val, vb) != hipSuccess || hipMalloc((void **)&h->row, nnz * 4) != hipSuccess ||
        hipMalloc((void **)&h->col, nnz * 4) != hipSuccess) {
        if (h->val) (void)hipFree(h->val);
        if (h->row) (void)hipFree(h->row);
        delete h;
        return fail(WD_ENOMEM, "coordinate-format arrays (%zu bytes) do not fit", vb + (size_t)nnz * 8);
    }
    const Geom geo = make_geom(g);
    hipStream_t st = (hipStream_t)stream;
    const int blocks = (int)((rows + 255) / 256);
    if (prec == WD_F64)
        hipLaunchKernelGGL(k_coo_build<double>, dim3(blocks), dim3(256), 0, st, geo, 4.0 + m0,
                           (const double2 *)g->U[WD_F64], dagger, (double2 *)h->val, h->row, h->col);
    else
        hipLaunchKernelGGL(k_coo_build<float>, dim3(blocks), dim3(256), 0, st, geo, 4.0 + m0,
                           (const double2 *)g->U[WD_F64], dagger, (float2 *)h->val, h->row, h->col);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(h->val);
        (void)hipFree(h->row);
        (void)hipFree(h->col);
        delete h;
        return fail(WD_EHIP, "building the coordinate format: %s", hipGetErrorString(e));
    }
    *out = h;
    return WD_OK;
}

int wd_coo_destroy(wd_coo *h) {
    clear_error();
    if (!h) return WD_OK;
    (void)hipFree(h->val);
    (void)hipFree(h->row);
    (void)hipFree(h->col);
    delete h;
    return WD_OK;
}

int wd_coo_info(const wd_coo *h, int64_t *nnz, int64_t *rows, size_t *bytes) {
    clear_error();
    WD_CHECK(h, WD_EINVAL, "null handle");
    if (nnz) *nnz = h->nnz;
    if (rows) *rows = h->rows;
    if (bytes) *bytes = (size_t)h->nnz * ((h->prec == WD_F64 ? 16 : 8) + 8);
    return WD_OK;
}

int wd_coo_export(const wd_coo *h, void *val_dev, void *row_dev, void *col_dev, void *stream) {
    clear_error();
    WD_CHECK(h && val_dev && row_dev && col_dev, WD_EINVAL, "null argument");
    hipStream_t st = (hipStream_t)stream;
    WD_HIP(hipMemcpyAsync(val_dev, h->val, (size_t)h->nnz * (h->prec == WD_F64 ? 16 : 8), hipMemcpyDeviceToDevice, st));
    WD_HIP(hipMemcpyAsync(row_dev, h->row, (size_t)h->nnz * 4, hipMemcpyDeviceToDevice, st));
    WD_HIP(hipMemcpyAsync(col_dev, h->col, (size_t)h->nnz * 4, hipMemcpyDeviceToDevice, st));
    return WD_OK;
}

int wd_coo_spmv(const wd_coo *h, const void *in_dev, void *out_dev, int32_t nrhs, void *stream) {
    clear_error();
    WD_CHECK(h && in_dev && out_dev, WD_EINVAL, "null argument");
    WD_CHECK(in_dev != out_dev, WD_EINVAL, "in and out must not overlap");
    WD_CHECK(nrhs >= 1 && nrhs <= MAX_RHS, WD_EINVAL, "nrhs %d out of range", nrhs);
    hipStream_t st = (hipStream_t)stream;
    const int nrows = (int)h->rows;
    const int blocks = (nrows + 255) / 256;
    if (h->prec == WD_F64)
        hipLaunchKernelGGL(k_coo_spmv<double>, dim3(blocks), dim3(256), 0, st, (const double2 *)h->val, h->col,
                           (const double2 *)in_dev, (double2 *)out_dev, nrows, nrhs);
    else
        hipLaunchKernelGGL(k_coo_spmv<float>, dim3(blocks), dim3(256), 0, st, (const float2 *)h->val, h->col,
                           (const float2 *)in_dev, (float2 *)out_dev, nrows, nrhs);
    WD_HIP(hipGetLastError());
    return WD_OK;
}

}  // extern "C"
