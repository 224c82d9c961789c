// Host-side pieces of the CG solver shared by the batch solver and the server.
#pragma once

#include <vector>

#include "cg_core.h"
#include "wd_host.h"

namespace wd {

struct KindShape {
    int block = 256, nr = 1, remap = 0, grid = 0;
    int ordered = 1;   // hop order of phases A and B: 1, 3 (pipelined) or 5 (pipelined, memory hops first)
    int order = 0;     // stencil kinds: processing order, strip | group-major << 16 | plane-blocked << 17
                       // | planes per block << 18
    int xy = 0;        // phases A and B: 1 plane-blocked variant (x/y neighbours from LDS),
                       // 2 z-marching columns of planes (zm_tile)
    int lds = 0;       // dynamic LDS bytes per block (z-marching)
    int r12 = 0;       // phases A and B: links from the reconstruct-12 copy
    int nt = 0;        // phases A, B and C: nontemporal streaming accesses (FP64)
    int planes = 1;    // phases A and B, plane-blocked: z-adjacent xy-planes per block
};
struct LaunchSet {
    KindShape k[NKIND];
    int eo = 0;   // even-odd preconditioned solve: A, B, R2 are Schur kernels
    int qrec = 0; // phase A forms the direction q = D^dagger r + beta q (Dhat for even-odd): no p, no phase C
    int fused = 0; // phase A completes the previous iteration's finish (launch_iterations): two launches
                   // per iteration and one trailing finish per chunk
    int pcus = 0;  // persistent kernel: one 1024-thread block on each of min(pcus, CUs) compute units
                   // (0: phase B's blocks, as many as are resident at once)
};

// The persistent kernel's grid-barrier words, each on a 256-byte line of its
// own (the line every waiting block polls is not the one the arrivals update):
// the released generation, the abort flag and the arrival counter.
constexpr size_t BAR_GEN = 0, BAR_ABORT = 256, BAR_COUNT = 512;
constexpr size_t BAR_BYTES = 768;

// Byte offsets of the pieces of a solve workspace.
struct WsLayout {
    size_t prob, scal, scal2, bar, summary, part, eta64, x64, xlo, r, p, q;
    size_t bscal, rh, sv, tv;   // BiCGSTAB only (0 otherwise)
    size_t eta_o, tmp, w64;     // even-odd only (0 otherwise)
    size_t total;
};

WsLayout ws_layout(int64_t V, int nrhs, int inner, int method, int eo = 0);
void plan_shapes(const wd_gauge *g, int nrhs, int inner, LaunchSet &ls, Prob &pr);
void plan_persistent(LaunchSet &ls, Prob &pr, int64_t V, int nrhs, int inner, int max_cus = 0);
void fill_prob(Prob &pr, const wd_gauge *g, double m0, int nrhs, const wd_cg_params &p, char *ws,
               const WsLayout &L);
void init_scalars(std::vector<Scal> &sc, int nrhs);
// One kernel kind of a CG iteration (and the finish after it).  par >= 0, first:
// phase A or B of a fused-finish iteration (see launch_iterations).
void launch_kind(int kind, int inner, const LaunchSet &ls, hipStream_t st, const Prob *d, int nprob, int par = -1,
                 int first = 0);
// the first true residual of a solve; x_zero: x64 is zero (no stencil needed)
void launch_first_residual(int inner, const LaunchSet &ls, hipStream_t st, const Prob *d, int nprob, bool x_zero);
// K CG iterations: with ls.fused, phases A and B per iteration (A finishing the
// iteration before it) and one trailing finish; else A, B (with its finish)
// and C, with the even-odd hops where ls.eo.
void launch_iterations(int inner, const LaunchSet &ls, hipStream_t st, const Prob *d, int nprob, int K);
// WD_CG_UNFUSED set (and not "0"): solves and the server use the three-launch iteration
bool unfused_requested();
void launch_summary(hipStream_t st, const Prob *d, int nprob, int *out, const int *abort_flag);
void launch_zero(void *p, size_t bytes, hipStream_t st);
int check_params(const wd_cg_params *p);
// Even-odd preconditioning (one problem record at d, vf = V/2 sites per half):
// split a canonical complex128 field into its FP64 even and odd halves; form
// the Schur system's source b_e over eta_e; rebuild the odd half of x and write
// the canonical complex128 solution.
void launch_eo_split(const Prob *d, int64_t vf, int nrhs, const void *src, void *even, void *odd, hipStream_t st);
void launch_eo_source(const Prob *d, int64_t vf, int nrhs, hipStream_t st);
void launch_eo_merge(const Prob *d, int64_t vf, int nrhs, void *sol, hipStream_t st);
int cg_status_of(int state);
// Record one persistent chunk kernel (K iterations of phases A and B with grid
// barriers) on `st`; `bar` is BAR_BYTES of device scratch for the barrier.
// max_cus > 0: one 1024-thread block on each of min(max_cus, CUs) compute
// units (ls.pcus after plan_persistent).
int record_persistent_chunk(int inner, const LaunchSet &ls, hipStream_t st, const Prob *d, int nprob,
                            int K, void *bar, int max_cus = 0);

}  // namespace wd
