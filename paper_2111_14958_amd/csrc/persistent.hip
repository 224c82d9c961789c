// Persistent CG chunk kernel: K iterations of phases A and B (the CG of
// arXiv 2111.14958, Sec. 2, carried in the solution space, with the search
// direction kept as q = D^dagger p) in one launch.
//
// The grid is sized so that every block is resident at once (occupancy x CU
// count, or one 1024-thread block on each of max_cus compute units).  Blocks
// sweep the tiles of a phase (XCD by XCD in contiguous ranges when the grid is
// whole XCD rounds), then meet at a grid barrier.  The last block to arrive performs the phase's
// fixed-order reduction (alpha or beta and the convergence tests) and releases
// the others, so a CG iteration costs two grid-wide synchronisations and no
// kernel launches.  Every wait is bounded: a block that waits longer than the
// limit sets an abort flag, every other waiter sees it and exits, and the host
// reports the failure; no wave can spin forever.
#include "cg_host.h"

namespace wd {

struct Barrier {
    unsigned *count;   // arrivals, monotonic within a launch
    unsigned *gen;     // released barrier generations
    int *abort;        // set when a wait exceeded its limit
    unsigned long long limit;   // wall-clock ticks a block may wait
};

// Arrive at barrier number e; true (in every thread) for the last block.
__device__ __forceinline__ bool bar_arrive(const Barrier &b, unsigned nblk, unsigned e) {
    __shared__ int last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned old = atomicAdd(b.count, 1u);
        last = (old + 1 == nblk * (e + 1));
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

__device__ __forceinline__ void bar_release(const Barrier &b, unsigned e) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_store(b.gen, e + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Wait for barrier e to be released; returns nonzero if the launch aborted.
// The generation is polled with relaxed loads and acquired once, by the fence
// after the loop: an acquiring load at device scope invalidates the XCD's L2
// on every poll, under the blocks of that XCD that are still computing.
__device__ __forceinline__ int bar_wait(const Barrier &b, unsigned e) {
    __shared__ int aborted;
    if (threadIdx.x == 0) {
        const unsigned long long t0 = wall_clock64();
        int ab = 0;
        while (__hip_atomic_load(b.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < e + 1) {
            if (__hip_atomic_load(b.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ab = 1; break; }
            if (wall_clock64() - t0 > b.limit) {
                __hip_atomic_store(b.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ab = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __threadfence();
        aborted = ab;
    }
    __syncthreads();
    return aborted;
}

// Tiles of one phase for this block.  With a grid of whole XCD rounds the XCD
// of block b (b mod 8) owns the contiguous range [x nt / 8, (x+1) nt / 8) and
// its blocks stride through it; any other grid strides through all tiles.
#define FOR_MY_TILES(nt, t)                                                       \
    const bool xr_ = (gridDim.x & 7) == 0;                                        \
    const int x_ = xr_ ? (int)(blockIdx.x & 7) : 0;                               \
    const int i_ = xr_ ? (int)(blockIdx.x >> 3) : (int)blockIdx.x;                \
    const int per_ = xr_ ? (int)(gridDim.x >> 3) : (int)gridDim.x;                \
    const int lo_ = xr_ ? (int)(((long long)(nt) * x_) / 8) : 0;                  \
    const int hi_ = xr_ ? (int)(((long long)(nt) * (x_ + 1)) / 8) : (nt);         \
    for (int t = lo_ + i_; t < hi_; t += per_)

// BLK is the block size the kernel is compiled for: 256, or 1024 for the
// launch with one block per compute unit (FP32 and FP16 storage).  R12: links
// from the reconstruct-12 copy (FP32).  The phase tiles take one hop at a time
// (pipelining two hops, hop order 3, timed the same at 14^4 x 16).
template <int P, int NR, int BLK = 256, bool R12 = false>
__global__ __launch_bounds__(BLK) void k_persistent(const Prob *__restrict__ probs, int K, Barrier b) {
    const Prob &pr = probs[0];
    const unsigned nblk = gridDim.x;
    unsigned e = 0;
    for (int it = 0; it < K; ++it) {
        {   // phase A: the direction q = D^dagger r + beta q (no p, no phase C)
            FOR_MY_TILES(pr.nt[KA], t) phaseA_tile<P, NR, 1, false, R12, false, true>(pr, t);
        }
        if (bar_arrive(b, nblk, e)) {
            phaseA_finish(pr);
            bar_release(b, e);
        } else if (bar_wait(b, e)) {
            return;
        }
        ++e;
        {   // phase B
            FOR_MY_TILES(pr.nt[KB], t) phaseB_tile<P, NR, 1, false, R12>(pr, t);
        }
        if (bar_arrive(b, nblk, e)) {
            phaseB_finish(pr);
            bar_release(b, e);
        } else if (bar_wait(b, e)) {
            return;
        }
        ++e;
    }
}

// zero the barrier words (a kernel: no memset node in the chunk graph)
__global__ void k_bar_reset(unsigned *p) {
    if (threadIdx.x == 0) {
        p[BAR_GEN / 4] = 0u;
        p[BAR_ABORT / 4] = 0u;
        p[BAR_COUNT / 4] = 0u;
    }
}

static void make_barrier(Barrier &b, void *bar, int khz) {
    char *c = (char *)bar;
    b.count = (unsigned *)(c + BAR_COUNT);
    b.gen = (unsigned *)(c + BAR_GEN);
    b.abort = (int *)(c + BAR_ABORT);
    b.limit = (unsigned long long)khz * 1000ull * 2ull;   // two seconds
}

template <int P, int NR>
static int launch_persistent(int blk, hipStream_t st, const Prob *d, int K, void *bar, int max_tiles) {
    int dev = 0, ncu = 0, per_cu = 0, khz = 0;
    WD_HIP(hipGetDevice(&dev));
    WD_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    WD_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    WD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<P, NR>, blk, 0));
    WD_CHECK(per_cu >= 1, WD_EHIP, "persistent kernel does not fit a compute unit");
    int nblk = per_cu * ncu;
    if (nblk > max_tiles) nblk = max_tiles;
    nblk &= ~7;   // whole XCD rounds
    if (nblk < 8) nblk = 8;
    Barrier b;
    make_barrier(b, bar, khz);
    hipLaunchKernelGGL(k_bar_reset, dim3(1), dim3(64), 0, st, (unsigned *)bar);
    hipLaunchKernelGGL((k_persistent<P, NR>), dim3(nblk), dim3(blk), 0, st, d, K, b);
    WD_HIP(hipGetLastError());
    return WD_OK;
}

// min(max_cus, compute units) blocks of 1024 threads (FP32 and FP16 storage;
// the FP64 kernel would spill registers at this block size).  A compute unit has room
// for one such block only (checked), so every block runs on a compute unit of
// its own: the launch uses exactly that many compute units.  All blocks are
// resident at once, which the grid barriers need.
template <int P, bool R12>
static int launch_persistent_cus(hipStream_t st, const Prob *d, int K, void *bar, int max_cus) {
    int dev = 0, ncu = 0, per_cu = 0, khz = 0;
    WD_HIP(hipGetDevice(&dev));
    WD_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    WD_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    WD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<P, 1, 1024, R12>, 1024, 0));
    WD_CHECK(per_cu == 1, WD_EHIP, "the compute-unit-limited kernel fits %d times on a compute unit", per_cu);
    const int nblk = max_cus < ncu ? max_cus : ncu;
    Barrier b;
    make_barrier(b, bar, khz);
    hipLaunchKernelGGL(k_bar_reset, dim3(1), dim3(64), 0, st, (unsigned *)bar);
    hipLaunchKernelGGL((k_persistent<P, 1, 1024, R12>), dim3(nblk), dim3(1024), 0, st, d, K, b);
    WD_HIP(hipGetLastError());
    return WD_OK;
}

int record_persistent_chunk(int inner, const LaunchSet &ls, hipStream_t st, const Prob *d, int nprob,
                            int K, void *bar, int max_cus) {
    WD_CHECK(nprob == 1, WD_EINVAL, "the persistent kernel serves one problem");
    const KindShape &ka = ls.k[KA], &kb = ls.k[KB];
    WD_CHECK(ka.block == kb.block && ka.nr == kb.nr, WD_EINVAL,
             "persistent kernel needs one block shape for phases A and B");
    if (max_cus > 0) {
        WD_CHECK(ka.block == 1024 && ka.nr == 1 && (!ka.r12 || inner == P32), WD_EINVAL,
                 "kernel with a block per compute unit: 1024 threads, 1 rhs");
        switch (inner) {
        case P32:
            return ka.r12 ? launch_persistent_cus<P32, true>(st, d, K, bar, max_cus)
                          : launch_persistent_cus<P32, false>(st, d, K, bar, max_cus);
        case P16: return launch_persistent_cus<P16, false>(st, d, K, bar, max_cus);
        }
        return fail(WD_EINVAL, "no compute-unit-limited kernel for precision %d", inner);
    }
    const int max_tiles = std::max(ka.grid, kb.grid);
    const int blk = ka.block;
    switch (inner * 4 + ka.nr) {
    case P64 * 4 + 1: return launch_persistent<P64, 1>(blk, st, d, K, bar, max_tiles);
    case P64 * 4 + 2: return launch_persistent<P64, 2>(blk, st, d, K, bar, max_tiles);
    case P32 * 4 + 1: return launch_persistent<P32, 1>(blk, st, d, K, bar, max_tiles);
    case P32 * 4 + 2: return launch_persistent<P32, 2>(blk, st, d, K, bar, max_tiles);
    case P32 * 4 + 4: return launch_persistent<P32, 4>(blk, st, d, K, bar, max_tiles);
    case P16 * 4 + 1: return launch_persistent<P16, 1>(blk, st, d, K, bar, max_tiles);
    case P16 * 4 + 2: return launch_persistent<P16, 2>(blk, st, d, K, bar, max_tiles);
    case P16 * 4 + 4: return launch_persistent<P16, 4>(blk, st, d, K, bar, max_tiles);
    }
    return fail(WD_EINVAL, "no persistent kernel for precision %d with %d rhs per thread", inner, ka.nr);
}

}  // namespace wd
