// Streaming bandwidth probe: read, copy and write kernels with wide (16-byte)
// coalesced accesses and four independent accesses per thread in flight.  They
// measure the memory ceiling that the operator's bandwidth is compared with
// (the naive roofline of Sec. 3.1 needs the machine's attainable bandwidth).
#include "wd_host.h"

namespace wd {

// KIND 0: read src (every word is combined into a value that is written only
// in a case that does not occur for finite data, so no load can be dropped);
// KIND 1: copy src -> dst; KIND 2: write a constant to dst.
template <int KIND>
__global__ __launch_bounds__(256) void k_stream(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    const uint4 pat = make_uint4(0x3f800000u, 0u, 0x3f800000u, 0u);
    for (; i + 3 * stride < n; i += 4 * stride) {
        if constexpr (KIND == 2) {
            dst[i] = pat;
            dst[i + stride] = pat;
            dst[i + 2 * stride] = pat;
            dst[i + 3 * stride] = pat;
        } else {
            const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
            if constexpr (KIND == 1) {
                dst[i] = a;
                dst[i + stride] = b;
                dst[i + 2 * stride] = c;
                dst[i + 3 * stride] = d;
            } else {
                acc.x ^= a.x ^ b.x ^ c.x ^ d.x;
                acc.y ^= a.y ^ b.y ^ c.y ^ d.y;
                acc.z ^= a.z ^ b.z ^ c.z ^ d.z;
                acc.w ^= a.w ^ b.w ^ c.w ^ d.w;
            }
        }
    }
    for (; i < n; i += stride) {
        if constexpr (KIND == 2) {
            dst[i] = pat;
        } else {
            const uint4 a = src[i];
            if constexpr (KIND == 1) dst[i] = a;
            else {
                acc.x ^= a.x;
                acc.y ^= a.y;
                acc.z ^= a.z;
                acc.w ^= a.w;
            }
        }
    }
    if constexpr (KIND == 0)
        if ((acc.x & acc.y & acc.z & acc.w) == 0xffffffffu) dst[0] = acc;   // all-ones words only
}

}  // namespace wd

extern "C" int wd_stream(int32_t kind, const void *src_dev, void *dst_dev, size_t bytes, void *stream) {
    using namespace wd;
    clear_error();
    WD_CHECK(kind >= WD_STREAM_READ && kind <= WD_STREAM_WRITE, WD_EINVAL, "unknown stream kind %d", kind);
    WD_CHECK(dst_dev && (src_dev || kind == WD_STREAM_WRITE), WD_EINVAL, "null argument");
    WD_CHECK(bytes % 16 == 0 && ((uintptr_t)dst_dev & 15) == 0 && ((uintptr_t)src_dev & 15) == 0, WD_EINVAL,
             "bytes and pointers must be multiples of 16");
    int rc = require_gfx950();
    if (rc) return rc;
    const size_t n = bytes / 16;
    if (n == 0) return WD_OK;
    // 8192 blocks of 256 threads fill the 256 compute units several times over
    const size_t want = (n + 4 * 256 - 1) / (4 * 256);
    const dim3 grid((unsigned)(want < 8192 ? want : 8192)), block(256);
    hipStream_t st = (hipStream_t)stream;
    const uint4 *s = (const uint4 *)src_dev;
    uint4 *d = (uint4 *)dst_dev;
    switch (kind) {
    case WD_STREAM_READ: hipLaunchKernelGGL(k_stream<0>, grid, block, 0, st, s, d, n); break;
    case WD_STREAM_COPY: hipLaunchKernelGGL(k_stream<1>, grid, block, 0, st, s, d, n); break;
    default: hipLaunchKernelGGL(k_stream<2>, grid, block, 0, st, s, d, n); break;
    }
    WD_HIP(hipGetLastError());
    return WD_OK;
}
