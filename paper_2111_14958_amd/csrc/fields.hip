// Library plumbing and field conversion: errors, device checks, the gauge
// handle (packing the canonical complex128 links into the structure-of-arrays
// layouts of each precision) and spinor pack / unpack.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "wd_device.h"
#include "wd_host.h"

namespace wd {

static thread_local char g_detail[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_detail, sizeof(g_detail), fmt, ap);
    va_end(ap);
    return code;
}
void clear_error() { g_detail[0] = 0; }

int require_gfx950(int *num_cu) {
    static std::mutex mu;
    static std::map<int, int> cu_of;   // device -> CU count (0 = not gfx950)
    int dev = 0;
    WD_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = cu_of.find(dev);
    if (it == cu_of.end()) {
        hipDeviceProp_t prop;
        WD_HIP(hipGetDeviceProperties(&prop, dev));
        int ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        it = cu_of.emplace(dev, ok ? prop.multiProcessorCount : 0).first;
    }
    if (it->second == 0) return fail(WD_ENODEV, "device %d is not a gfx950", dev);
    if (num_cu) *num_cu = it->second;
    return WD_OK;
}

size_t spinor_bytes(int prec, int64_t V, int nrhs) {
    switch (prec) {
    case WD_F64: return (size_t)nrhs * V * 192;
    case WD_F32: return (size_t)nrhs * V * 96;
    case WD_F16N: return (size_t)nrhs * V * 52;
    }
    return 0;
}

size_t link_bytes(int prec, int64_t V, bool r12) {
    switch (prec) {
    case WD_F64: return (size_t)V * 4 * 144;
    case WD_F32: return (size_t)V * 4 * (r12 ? 48 : 72);
    case WD_F16N: return (size_t)V * 4 * (r12 ? 24 : 36);
    }
    return 0;
}

// ------------------------------------------------------------------ kernels
// canonical U[site][mu][a][b] (complex128) -> packed [mu][9][V] in precision P
// t-links of the last time slice (sites >= last0) are stored times -1 when
// flip is set: the antiperiodic boundary sign of both hops across it.
// R12: rows 0 and 1 only ([mu][6][V]); a link whose row 2 is not
// sign * conj(row 0 x row 1) to 1e-6 (sign -1 for a flipped link) sets *bad.
template <int P, bool R12>
__global__ void k_pack_links(const double2 *__restrict__ in, void *__restrict__ out, int V, int last0, int flip,
                             int *bad) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= V) return;
    constexpr int NK = R12 ? 6 : 9;
    for (int mu = 0; mu < 4; ++mu) {
        const double2 *src = in + ((size_t)s * 4 + mu) * 9;
        const bool neg = flip && mu == 3 && s >= last0;
        if constexpr (R12) {   // check the input matrix (before the sign): det 1 and unitary rows
            cx<double> u[9];
            for (int k = 0; k < 9; ++k) u[k] = {src[k].x, src[k].y};
            const cx<double> r2[3] = {u[6], u[7], u[8]};
            third_row<double>(u, 1.0);
            double dev = 0.0;
            for (int k = 0; k < 3; ++k) dev = fmax(dev, fabs(r2[k].re - u[6 + k].re) + fabs(r2[k].im - u[6 + k].im));
            if (!(dev <= 1e-6)) *bad = 1;   // a plain store from the lanes that found one
        }
        for (int k = 0; k < NK; ++k) {
            double2 v = src[k];
            if (neg) v = make_double2(-v.x, -v.y);
            const size_t o = ((size_t)mu * NK + k) * V + s;
            if constexpr (P == P64) {
                ((double2 *)out)[o] = v;
            } else if constexpr (P == P32) {
                ((float2 *)out)[o] = make_float2((float)v.x, (float)v.y);
            } else {
                half2v h;
                h.x = (h16)(float)v.x;   // FP64 -> FP32 -> FP16, each round to nearest even
                h.y = (h16)(float)v.y;
                ((half2v *)out)[o] = h;
            }
        }
    }
}

// canonical psi[rhs][site][12] (complex128) -> packed precision P
template <int P>
__global__ void k_pack_spinor(const double2 *__restrict__ in, void *__restrict__ out, int V, int nrhs) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= V || r >= nrhs) return;
    typedef typename real_of<P>::type R;
    const double2 *src = in + ((size_t)r * V + s) * 12;
    cx<R> v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const double2 d = src[k];
        v[k] = {(R)d.x, (R)d.y};
    }
    FieldPtr f{out, V, nrhs};
    Spinor<P>::store(f, r, s, v);
}

template <int P>
__global__ void k_unpack_spinor(const void *__restrict__ in, double2 *__restrict__ out, int V, int nrhs) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (s >= V || r >= nrhs) return;
    typedef typename real_of<P>::type R;
    cx<R> v[12];
    FieldPtr f{(void *)in, V, nrhs};
    Spinor<P>::load(f, r, s, v);
    double2 *dst = out + ((size_t)r * V + s) * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) dst[k] = make_double2((double)v[k].re, (double)v[k].im);
}

int launch_pack_links(int prec, const void *in, void *out, const int dims[4], int tsign, hipStream_t st, bool r12,
                      int *bad) {
    const int V = dims[0] * dims[1] * dims[2] * dims[3];
    const int last0 = V - dims[0] * dims[1] * dims[2];
    const int flip = tsign < 0 ? 1 : 0;
    const int blocks = (V + 255) / 256;
    WD_CHECK(!r12 || (prec != WD_F64 && bad), WD_EINVAL, "reconstruct-12 packs FP32/FP16 copies with a flag");
    const double2 *src = (const double2 *)in;
    switch (prec * 2 + (r12 ? 1 : 0)) {
    case WD_F64 * 2: hipLaunchKernelGGL((k_pack_links<P64, false>), dim3(blocks), dim3(256), 0, st, src, out, V, last0, flip, bad); break;
    case WD_F32 * 2: hipLaunchKernelGGL((k_pack_links<P32, false>), dim3(blocks), dim3(256), 0, st, src, out, V, last0, flip, bad); break;
    case WD_F32 * 2 + 1: hipLaunchKernelGGL((k_pack_links<P32, true>), dim3(blocks), dim3(256), 0, st, src, out, V, last0, flip, bad); break;
    case WD_F16N * 2: hipLaunchKernelGGL((k_pack_links<P16, false>), dim3(blocks), dim3(256), 0, st, src, out, V, last0, flip, bad); break;
    case WD_F16N * 2 + 1: hipLaunchKernelGGL((k_pack_links<P16, true>), dim3(blocks), dim3(256), 0, st, src, out, V, last0, flip, bad); break;
    default: return fail(WD_EINVAL, "unknown precision %d", prec);
    }
    WD_HIP(hipGetLastError());
    return WD_OK;
}

int launch_pack_spinor(int prec, const void *in, void *out, int V, int nrhs, hipStream_t st) {
    dim3 grid((V + 255) / 256, nrhs);
    switch (prec) {
    case WD_F64: hipLaunchKernelGGL(k_pack_spinor<P64>, grid, dim3(256), 0, st, (const double2 *)in, out, V, nrhs); break;
    case WD_F32: hipLaunchKernelGGL(k_pack_spinor<P32>, grid, dim3(256), 0, st, (const double2 *)in, out, V, nrhs); break;
    case WD_F16N: hipLaunchKernelGGL(k_pack_spinor<P16>, grid, dim3(256), 0, st, (const double2 *)in, out, V, nrhs); break;
    default: return fail(WD_EINVAL, "unknown precision %d", prec);
    }
    WD_HIP(hipGetLastError());
    return WD_OK;
}

int launch_unpack_spinor(int prec, const void *in, void *out, int V, int nrhs, hipStream_t st) {
    dim3 grid((V + 255) / 256, nrhs);
    switch (prec) {
    case WD_F64: hipLaunchKernelGGL(k_unpack_spinor<P64>, grid, dim3(256), 0, st, in, (double2 *)out, V, nrhs); break;
    case WD_F32: hipLaunchKernelGGL(k_unpack_spinor<P32>, grid, dim3(256), 0, st, in, (double2 *)out, V, nrhs); break;
    case WD_F16N: hipLaunchKernelGGL(k_unpack_spinor<P16>, grid, dim3(256), 0, st, in, (double2 *)out, V, nrhs); break;
    default: return fail(WD_EINVAL, "unknown precision %d", prec);
    }
    WD_HIP(hipGetLastError());
    return WD_OK;
}

}  // namespace wd

using namespace wd;

// ------------------------------------------------------------------- C ABI
extern "C" {

int wd_version(void) { return 10000; }

const char *wd_strerror(int code) {
    switch (code) {
    case WD_OK: return "success";
    case WD_EINVAL: return "invalid argument";
    case WD_ENODEV: return "no gfx950 device";
    case WD_EHIP: return "HIP runtime error";
    case WD_ENOMEM: return "out of memory / workspace too small";
    case WD_ENOTCONV: return "not converged within max_iter";
    case WD_EBREAKDOWN: return "CG breakdown (NaN/Inf or non-positive curvature)";
    case WD_ETOOBIG: return "request larger than the server arena or the static scratch";
    case WD_ENOTFOUND: return "unknown ticket";
    }
    return "unknown error";
}

const char *wd_last_error_detail(void) { return g_detail; }

int wd_device_info(int device, char *arch, size_t arch_len, int32_t *num_cu) {
    clear_error();
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return fail(WD_ENODEV, "no HIP device");
    WD_CHECK(device >= 0 && device < n, WD_EINVAL, "device %d out of range (%d devices)", device, n);
    hipDeviceProp_t prop;
    WD_HIP(hipGetDeviceProperties(&prop, device));
    if (arch && arch_len) {
        strncpy(arch, prop.gcnArchName, arch_len - 1);
        arch[arch_len - 1] = 0;
    }
    if (num_cu) *num_cu = prop.multiProcessorCount;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(WD_ENODEV, "device %d is %s, not gfx950", device, prop.gcnArchName);
    return WD_OK;
}

int wd_gauge_create(const int32_t dims[4], int32_t t_sign, const void *U_dev, uint32_t prec_mask,
                    void *stream, wd_gauge **out) {
    clear_error();
    WD_CHECK(dims && U_dev && out, WD_EINVAL, "null argument");
    WD_CHECK(t_sign == 1 || t_sign == -1, WD_EINVAL, "t_sign must be +1 or -1, got %d", t_sign);
    WD_CHECK((prec_mask & ~(7u | WD_GAUGE_RECON12)) == 0, WD_EINVAL, "bad precision mask 0x%x", prec_mask);
    int64_t V = 1;
    for (int d = 0; d < 4; ++d) {
        WD_CHECK(dims[d] >= 1 && dims[d] <= 4096, WD_EINVAL, "bad lattice extent dims[%d] = %d", d, dims[d]);
        V *= dims[d];
    }
    WD_CHECK(V <= MAX_SITES, WD_EINVAL, "lattice of %lld sites exceeds the limit", (long long)V);
    int rc = require_gfx950();
    if (rc) return rc;
    *out = nullptr;
    wd_gauge *g = new wd_gauge();
    for (int d = 0; d < 4; ++d) g->dims[d] = dims[d];
    g->tsign = t_sign;
    g->V = V;
    g->mask = prec_mask | WD_GAUGE_F64;
    const bool r12 = (g->mask & WD_GAUGE_RECON12) != 0;
    hipGetDevice(&g->device);
    hipStream_t st = (hipStream_t)stream;
    int *bad = nullptr;   // reconstruct-12: set by the packing kernels for a non-SU(3) link
    auto release = [&]() {
        for (int p = 0; p < 3; ++p) {
            if (g->U[p]) hipFree(g->U[p]);
            if (g->U12[p]) hipFree(g->U12[p]);
        }
        if (bad) hipFree(bad);
        delete g;
    };
    for (int p = 0; p < 3; ++p) g->U[p] = g->U12[p] = nullptr;
    if (r12) {
        hipError_t e = hipMalloc(&bad, sizeof(int));
        if (e != hipSuccess) {
            bad = nullptr;
            release();
            return fail(WD_ENOMEM, "hipMalloc of the link check flag: %s", hipGetErrorString(e));
        }
        hipMemsetAsync(bad, 0, sizeof(int), st);
    }
    // the complete copies, then (reconstruct-12) the two-row FP32 copy beside them
    for (int c = 0; c < 4; ++c) {
        const int p = c < 3 ? c : WD_F32;
        const bool pr12 = c == 3;
        if (!(g->mask & (1u << p)) || (pr12 && !r12)) continue;
        void **dst = pr12 ? &g->U12[p] : &g->U[p];
        hipError_t e = hipMalloc(dst, link_bytes(p, V, pr12));
        if (e != hipSuccess) {
            *dst = nullptr;
            release();
            return fail(WD_ENOMEM, "hipMalloc of %zu link bytes: %s", link_bytes(p, V, pr12), hipGetErrorString(e));
        }
        launch_pack_links(p, U_dev, *dst, g->dims, g->tsign, st, pr12, bad);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    int nonsu3 = 0;
    if (e == hipSuccess && bad) e = hipMemcpy(&nonsu3, bad, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        release();
        return fail(WD_EHIP, "packing links: %s", hipGetErrorString(e));
    }
    if (nonsu3) {
        release();
        return fail(WD_EINVAL, "reconstruct-12 needs SU(3) links: a link's third row differs from the "
                               "conjugated cross product of its first two by more than 1e-6");
    }
    if (bad) hipFree(bad);
    *out = g;
    return WD_OK;
}

int wd_gauge_destroy(wd_gauge *g) {
    clear_error();
    if (!g) return WD_OK;
    int cur = 0;
    hipGetDevice(&cur);
    if (cur != g->device) hipSetDevice(g->device);
    for (int p = 0; p < 3; ++p) {
        if (g->U[p]) hipFree(g->U[p]);
        if (g->U12[p]) hipFree(g->U12[p]);
    }
    if (cur != g->device) hipSetDevice(cur);
    delete g;
    return WD_OK;
}

int wd_gauge_info(const wd_gauge *g, int32_t dims[4], int32_t *t_sign, int64_t *sites, uint32_t *mask) {
    clear_error();
    WD_CHECK(g, WD_EINVAL, "null gauge");
    if (dims) for (int d = 0; d < 4; ++d) dims[d] = g->dims[d];
    if (t_sign) *t_sign = g->tsign;
    if (sites) *sites = g->V;
    if (mask) *mask = g->mask;
    return WD_OK;
}

size_t wd_spinor_bytes(const wd_gauge *g, int32_t prec, int32_t nrhs) {
    if (!g || nrhs < 0 || prec < 0 || prec > 2) return 0;
    return spinor_bytes(prec, g->V, nrhs);
}

int wd_pack_spinor(const wd_gauge *g, int32_t prec, const void *in_dev, void *out_dev, int32_t nrhs, void *stream) {
    clear_error();
    WD_CHECK(g && in_dev && out_dev, WD_EINVAL, "null argument");
    WD_CHECK(prec >= 0 && prec <= 2, WD_EINVAL, "unknown precision %d", prec);
    WD_CHECK(nrhs >= 1 && nrhs <= MAX_RHS, WD_EINVAL, "nrhs %d out of range", nrhs);
    if (nrhs == 0) return WD_OK;
    return launch_pack_spinor(prec, in_dev, out_dev, (int)g->V, nrhs, (hipStream_t)stream);
}

int wd_unpack_spinor(const wd_gauge *g, int32_t prec, const void *in_dev, void *out_dev, int32_t nrhs, void *stream) {
    clear_error();
    WD_CHECK(g && in_dev && out_dev, WD_EINVAL, "null argument");
    WD_CHECK(prec >= 0 && prec <= 2, WD_EINVAL, "unknown precision %d", prec);
    WD_CHECK(nrhs >= 1 && nrhs <= MAX_RHS, WD_EINVAL, "nrhs %d out of range", nrhs);
    return launch_unpack_spinor(prec, in_dev, out_dev, (int)g->V, nrhs, (hipStream_t)stream);
}

}  // extern "C"
