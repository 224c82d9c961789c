// Host-side internals of libwd: error reporting, the gauge handle, launch
// shapes and the launch helpers shared by the translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "wd.h"
#include "wd_device.h"

namespace wd {

// Record a failure for wd_last_error_detail (thread-local) and return `code`.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define WD_HIP(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return ::wd::fail(WD_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                              __FILE__, __LINE__);                                         \
    } while (0)

#define WD_CHECK(cond, code, ...)                   \
    do {                                            \
        if (!(cond)) return ::wd::fail(code, __VA_ARGS__); \
    } while (0)

// Largest supported lattice (keeps every per-field offset in 32 bits).
constexpr int64_t MAX_SITES = int64_t(1) << 26;
constexpr int MAX_RHS = 64;

// Verify that the current device is a gfx950; caches the answer per device.
int require_gfx950(int *num_cu = nullptr);

size_t spinor_bytes(int prec, int64_t V, int nrhs);
size_t link_bytes(int prec, int64_t V, bool r12 = false);   // all four directions; r12: two rows (FP32/FP16)

// Launch shape of one operator kernel.
struct Shape {
    int block = 256;         // threads per block (64, 128 or 256)
    int nr = 1;              // right-hand sides per thread (1, 2 or 4)
    int remap = 1;           // XCD-contiguous tile order
    int ordered = 1;         // hops issued one at a time (see hopping())
    int rloop = 1;           // rhs groups a block handles one after the other
    int strip = 0;           // processing order: z-strips of this width (0: lexicographic)
    int gmajor = 0;          // tiles ordered rhs-group-major (1) or site-block-major (0)
    int xylds = 0;           // plane-blocked: one xy-plane per block, x/y neighbours from LDS
    int occ = 0;             // plane-blocked operator: at most occ blocks per CU (0: no limit)
    int fpass = 0;           // CG phases: each eighth of the site blocks is walked in passes of
                             // fpass rhs groups (0: all groups of a site block together)
    int planes = 1;          // plane-blocked, one rhs per thread, FP32/FP16 storage: k z-adjacent
                             // xy-planes per block (k Lx Ly <= 512 sites)
};

// Key of the launch-shape table: lattice, precision, rhs count, dagger, and
// the kernel family (operator kernel, or one of the CG phase kernels, whose
// fused epilogues move more data per site and prefer other shapes).
enum : int { FAM_DSLASH = 0, FAM_CG_A = 1, FAM_CG_B = 2, FAM_CG_R = 3 };
struct ShapeKey {
    int L[4];
    int prec, nrhs, dag;
    int fam = FAM_DSLASH;
    bool operator<(const ShapeKey &o) const;
};
Shape shape_lookup(const ShapeKey &k);      // tuned entry or the default
void shape_store(const ShapeKey &k, const Shape &s);
// shape_store, and append the entry to the cache file WD_TUNE_CACHE names (if any)
void shape_store_persist(const ShapeKey &k, const Shape &s, double us);
Shape default_shape(int prec, int nrhs, int fam = FAM_DSLASH);
int encode_order(const Shape &s);           // wd_tune_result.site_order of a shape

}  // namespace wd

struct wd_gauge {
    int dims[4];
    int tsign;
    int64_t V;
    uint32_t mask;
    int device;
    void *U[3];     // packed links per precision (device), nullptr when absent
    void *U12[3];   // reconstruct-12 copies (FP32, FP16; WD_GAUGE_RECON12), nullptr when absent
};

namespace wd {
Geom make_geom(const wd_gauge *g);
// planes per plane-blocked block that shape sh gets on lattice g (1 where k
// planes do not fit: FP64 storage, several rhs per thread, k Lx Ly > 512, Lz or
// the strip width not a multiple of k)
int xy_planes(const Shape &sh, const Geom &g, int prec, int nr);
// Launchers implemented in the .hip units (all asynchronous on `stream`).
// canonical complex128 links -> packed precision prec; the t-links of the last
// time slice carry the boundary sign (tsign) from here on
// r12 (FP32/FP16): keep rows 0 and 1 only, and set *bad (device int) to 1 where
// row 2 is not the conjugated cross product of rows 0 and 1 to 1e-6
int launch_pack_links(int prec, const void *U_c128, void *out, const int dims[4], int tsign, hipStream_t st,
                      bool r12 = false, int *bad = nullptr);
int launch_pack_spinor(int prec, const void *in_c128, void *out, int V, int nrhs, hipStream_t st);
int launch_unpack_spinor(int prec, const void *in, void *out_c128, int V, int nrhs, hipStream_t st);
int launch_dslash(const wd_gauge *g, double m0, int prec, bool dag, const void *in, void *out,
                  int nrhs, const Shape &sh, hipStream_t st);
}  // namespace wd
