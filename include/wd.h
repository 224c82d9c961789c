/*
 * wd.h -- C ABI of libwd, a Wilson-Dirac conjugate-gradient library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library solves the lattice-QCD linear system D psi = eta of Eq. (1) of
 * arXiv 2111.14958 (Sec. 1): D is the Wilson-Dirac operator acting on fields
 * with 3 colours and 4 spins per lattice site (12 complex numbers per site).
 * It solves by conjugate gradient on the normal equations, as in Sec. 2: CG on
 * D D^dagger chi = eta, then psi = D^dagger chi, the multiplication by
 * D^dagger being folded into the iteration (psi is updated directly).
 *
 * Operator convention (Wilson parameter r = 1, bare mass m0):
 *   D psi(x) = (4 + m0) psi(x)
 *              - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) s psi(x + mu)
 *                           + (1 + gamma_mu) U_mu(x - mu)^dagger s psi(x - mu) ]
 * with s = t_sign for a hop in t that wraps around the lattice, else 1.
 * Gamma matrices in the DeGrand-Rossi chiral basis, gamma5 = diag(1,1,-1,-1).
 * D^dagger = gamma5 D gamma5 (gamma5-hermiticity, Sec. 2) exchanges the two
 * projectors.
 *
 * Canonical (user) layouts, C order, complex128 = (double re, double im):
 *   gauge   U[t][z][y][x][mu][a][b]     mu = 0..3 is x, y, z, t; U_mu(x) is the
 *                                       link x -> x + mu, (U psi)_a = sum_b U_ab psi_b
 *   spinor  psi[rhs][t][z][y][x][spin][colour]
 * dims are (Lx, Ly, Lz, Lt); site = x + Lx*(y + Ly*(z + Lz*t)).
 *
 * Packed (internal, structure-of-arrays) spinor layouts, used when a call
 * passes WD_PACKED; V = number of sites, component k = 3*spin + colour:
 *   WD_F64   double2 [rhs][12][V]          element (k, site) = component k
 *   WD_F32   float4  [rhs][6][V]           chunk j = components 2j, 2j+1 as (re,im,re,im)
 *   WD_F16N  16-byte [rhs][3][V] codes, then float [rhs][V] norms, in one buffer:
 *            chunk j = 8 halves = components 4j..4j+3 as (re,im) pairs; value =
 *            norm * code; norm = max |real or imaginary part| over the site's 24
 *            numbers (FP32), code = half(v * inv) with inv = 1 / norm rounded to
 *            FP32 (the FP32 product, then round-to-nearest-even to half; the
 *            FP32 quotient v / norm where 1 / norm overflows, norm < 2^-128);
 *            an all-zero site has norm 0.
 *
 * Memory ownership: every pointer argument named *_dev is device memory owned by
 * the caller (for example a PyTorch tensor); the library never frees it.  A
 * wd_gauge owns the packed link copies it allocates until wd_gauge_destroy.
 * A server owns nothing but what it carves out of the caller's arena.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null stream).
 * wd_dslash* and the pack functions are asynchronous on that stream.
 * wd_cg_solve* enqueue their work on that stream and return once the solution
 * and the reports are final (they synchronise the stream).
 *
 * Errors: functions return WD_OK (0) or a negative code; wd_strerror gives the
 * text, wd_last_error_detail the detail of the most recent failure on the
 * calling thread.  No function aborts the process.
 */
#ifndef WD_H
#define WD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    WD_OK = 0,
    WD_EINVAL = -1,      /* bad dimensions, null pointer, nrhs, tolerance, flags    */
    WD_ENODEV = -2,      /* no gfx950 device visible                                */
    WD_EHIP = -3,        /* HIP runtime error (detail string has the runtime text)  */
    WD_ENOMEM = -4,      /* workspace too small or device allocation failed         */
    WD_ENOTCONV = -5,    /* max_iter reached before the true residual met tol       */
    WD_EBREAKDOWN = -6,  /* NaN/Inf or <q,q> <= 0 inside CG                         */
    WD_ETOOBIG = -7,     /* request larger than the server arena or static scratch  */
    WD_ENOTFOUND = -8    /* unknown server ticket                                   */
};

typedef enum { WD_F64 = 0, WD_F32 = 1, WD_F16N = 2 } wd_prec;

/* flags of wd_dslash / wd_dslash_dag */
#define WD_PACKED 1u     /* in/out are in the packed layout of `prec` (see above) */

/* ------------------------------------------------------------------ library */
int         wd_version(void);                 /* 10000*major + 100*minor + patch  */
const char *wd_strerror(int code);
const char *wd_last_error_detail(void);       /* thread-local, "" when none        */
/* name of device `device` (gcnArchName) and its compute-unit count; WD_ENODEV
 * when the device is not gfx950 */
int wd_device_info(int device, char *arch, size_t arch_len, int32_t *num_cu);

/* ------------------------------------------------------------------ gauge field */
typedef struct wd_gauge wd_gauge;

#define WD_GAUGE_F64  (1u << WD_F64)
#define WD_GAUGE_F32  (1u << WD_F32)
#define WD_GAUGE_F16  (1u << WD_F16N)
/* Reconstruct-12: beside the FP32 copy, keep one with rows 0 and 1 of each link
 * only (12 reals instead of 18); the FP32 operator (wd_dslash, wd_dslash_dag),
 * the kernels of phases A and B of CG with FP32 inner iterations (plane or site
 * blocks, the even-odd half-lattice hops and the persistent kernel's phases;
 * not the z-marching kernels, not the server) and BiCGSTAB's plane-blocked stencils read it and
 * rebuild row 2 as the complex conjugate of the
 * cross product of rows 0 and 1, which holds for SU(3) matrices (unitary, det 1).
 * That cuts a third of their link bytes.  (With FP16 storage the rebuilt row
 * cost more than the bytes saved, so those kernels keep the complete copy.)  The paper's Conclusions ask for
 * operator representations better suited to the Dirac operator; this is a
 * standard one.  wd_gauge_create returns WD_EINVAL (and keeps nothing) when a
 * link's row 2 differs from that product by more than 1e-6 in any component. */
#define WD_GAUGE_RECON12 (1u << 8)

/* Pack the canonical complex128 links U_dev (dims, see above) into device-resident
 * copies in the precisions of prec_mask, optionally | WD_GAUGE_RECON12 (the FP64
 * copy is always made: the solver uses it for true residuals).  t_sign is -1 (antiperiodic time boundary) or +1.
 * Lower-precision copies are rounded to nearest even (FP16 via FP32).
 * Synchronises `stream` before returning; U_dev may be freed afterwards. */
int wd_gauge_create(const int32_t dims[4], int32_t t_sign, const void *U_dev,
                    uint32_t prec_mask, void *stream, wd_gauge **out);
int wd_gauge_destroy(wd_gauge *g);
/* dims[4], t_sign, sites and the precision mask of a gauge handle */
int wd_gauge_info(const wd_gauge *g, int32_t dims[4], int32_t *t_sign, int64_t *sites,
                  uint32_t *prec_mask);

/* --------------------------------------------------------- spinor conversion */
/* bytes of a packed spinor buffer holding nrhs fields of the gauge's lattice */
size_t wd_spinor_bytes(const wd_gauge *g, int32_t prec, int32_t nrhs);
/* canonical complex128 [nrhs][V][12] -> packed `prec` layout (RNE rounding) */
int wd_pack_spinor(const wd_gauge *g, int32_t prec, const void *in_dev, void *out_dev,
                   int32_t nrhs, void *stream);
/* packed `prec` layout -> canonical complex128 */
int wd_unpack_spinor(const wd_gauge *g, int32_t prec, const void *in_dev, void *out_dev,
                     int32_t nrhs, void *stream);

/* ----------------------------------------------------------------- operator */
/* out = D in (wd_dslash) or out = D^dagger in (wd_dslash_dag) for nrhs fields,
 * Eq. (1) with the convention above; arithmetic in the precision `prec`
 * (WD_F16N: half storage with per-site norms, FP32 arithmetic).  With
 * WD_PACKED the buffers are in the packed layout of `prec`; otherwise they are
 * canonical complex128 and the call packs / unpacks through stream-ordered
 * temporary buffers.  The gauge handle must hold the links in `prec`.
 * in and out must not overlap.  Asynchronous on `stream`. */
int wd_dslash(const wd_gauge *g, double m0, int32_t prec, const void *in_dev, void *out_dev,
              int32_t nrhs, uint32_t flags, void *stream);
int wd_dslash_dag(const wd_gauge *g, double m0, int32_t prec, const void *in_dev,
                  void *out_dev, int32_t nrhs, uint32_t flags, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): wd_dslash (dagger = 0)
 * or wd_dslash_dag (dagger = 1) on canonical complex128 in/out, with the packed
 * temporaries kept in a static device array of WD_NOALLOC_SCRATCH_BYTES that
 * the library holds on every device it runs on until the process ends, instead
 * of buffers allocated per call.  The call allocates nothing.  Both packed
 * fields (each rounded up to 256 bytes) must fit the array: 2 * nrhs * V *
 * (192 | 96 | 52) bytes for FP64 | FP32 | FP16N, else WD_ETOOBIG.  Every call on
 * one device shares that device's array, so calls that overlap on one device
 * (other streams, other threads) race; calls ordered on one stream do not.
 * dagger other than 0/1 is WD_EINVAL.  Asynchronous on `stream`. */
#define WD_NOALLOC_SCRATCH_BYTES (64u << 20)
int wd_dslash_noalloc(const wd_gauge *g, double m0, int32_t prec, int32_t dagger,
                      const void *in_dev, void *out_dev, int32_t nrhs, void *stream);

/* ------------------------------------------- coordinate-format operator */
/* The operator stored explicitly as in Sec. 2 of the paper: arrays Val, Row,
 * Col of the non-zero entries of D (or D^dagger), 49 per row (the diagonal,
 * then per direction x, y, z, t the 6 forward and 6 backward entries) of the
 * rows r = 12 site + 3 spin + colour; entry k of row r sits at index
 * k * rows + r (entry 0 of every row first); duplicate entries of extent-2
 * lattices are kept.  Built on the device from the gauge handle's
 * FP64 links; prec is WD_F64 (complex128 values) or WD_F32 (complex64).
 * Row and Col are int32.  The handle owns the arrays (nnz*(16 or 8) + nnz*8
 * bytes). */
typedef struct wd_coo wd_coo;
int wd_coo_create(const wd_gauge *g, double m0, int32_t prec, int32_t dagger, void *stream,
                  wd_coo **out);
int wd_coo_destroy(wd_coo *h);
int wd_coo_info(const wd_coo *h, int64_t *nnz, int64_t *rows, size_t *bytes);
/* copy Val, Row, Col into caller buffers (device) */
int wd_coo_export(const wd_coo *h, void *val_dev, void *row_dev, void *col_dev, void *stream);
/* out[Row[k]] += Val[k] * in[Col[k]] for nrhs vectors of 12 V complex numbers
 * (canonical layout, complex128 for WD_F64, complex64 for WD_F32); out is
 * overwritten.  Asynchronous on `stream`. */
int wd_coo_spmv(const wd_coo *h, const void *in_dev, void *out_dev, int32_t nrhs, void *stream);

/* -------------------------------------------------------------- CG solvers */
typedef struct {
    double  tol;            /* target |eta - D x| / |eta| (true residual, FP64), > 0   */
    int32_t max_iter;       /* CG iterations per right-hand side                        */
    int32_t reliable_every; /* inner iterations between reliable updates; 0 = only when
                               the iterated residual reaches tol                         */
    int32_t inner;          /* wd_prec of the inner iteration                           */
    int32_t use_x0;         /* 1: sol_dev holds the initial guess on entry              */
    int32_t persistent;     /* 0: one kernel per CG phase, 1: one persistent kernel per
                               chunk with grid barriers, -1: library default             */
    int32_t chunk;          /* CG iterations per graph replay (the host checks for
                               convergence between replays).  0 = library default:
                               reliable_every (or 50), and for CG a replay cut
                               short, in multiples of 8, once the fields' decrease of
                               |r|^2 says they need fewer; the results do not depend
                               on the replay lengths                                  */
    int32_t method;         /* WD_METHOD_CGNE (default) or WD_METHOD_BICGSTAB           */
    int32_t precondition;   /* WD_PRECOND_NONE (default) or WD_PRECOND_EO               */
    int32_t max_cus;        /* 0: all compute units.  n > 0: the CG iterations run on n
                               compute units (see below); needs persistent = 1         */
} wd_cg_params;

/* Compute-unit-limited CG (max_cus = n > 0), for speedup-versus-compute-units
 * studies (Sec. 3.1, Fig. 2).  The persistent kernel is launched with
 * min(n, compute units) blocks of 1024 threads whose register demand leaves room
 * for one block per compute unit, so each block holds a compute unit of its own
 * and the CG iterations use exactly that many.  The set-up, the reliable
 * updates and the final FP64 residual still run on the whole device.  Results
 * are identical (bitwise) for every n.  Returns WD_EHIP if the kernel would fit
 * twice on a compute unit.  FP32 or FP16N inner iterations only.  Not for the
 * server.  With persistent = 1 and max_cus = 0, FP32 and FP16N solves whose
 * phase shapes take one rhs per thread (the defaults) use this launch on every
 * compute unit, and the same bits as max_cus = n; FP64 (and shapes with several
 * rhs per thread) run phase B's block size instead, as many blocks as are
 * resident at once. */

/* Krylov method of wd_cg_solve / wd_cg_solve_batch.
 * WD_METHOD_CGNE: CG on the normal equations D D^dagger chi = eta, x = D^dagger chi
 *   (Sec. 2, the paper's solver), two operator applications per iteration.
 * WD_METHOD_BICGSTAB: BiCGSTAB on D x = eta (one of the Krylov methods Sec. 1
 *   names for the Dirac equation), two applications of D per iteration; a
 *   reliable update restarts it from the FP64 true residual (shadow residual
 *   r_hat = r).  Runs without the persistent kernel and without profiling. */
#define WD_METHOD_CGNE     0
#define WD_METHOD_BICGSTAB 1

/* Preconditioning of wd_cg_solve / wd_cg_solve_batch.
 * WD_PRECOND_EO: even-odd.  The odd sites are eliminated (D's diagonal 4 + m0
 *   is site-local and its hopping term joins opposite parities), CG runs on the
 *   normal equations of the Schur complement Dhat = A - D_eo A^-1 D_oe on the
 *   even sites, and the odd half of x follows from the even half.  The test
 *   |b_e - Dhat x_e| <= tol |eta| is the full system's true residual.  CG
 *   (WD_METHOD_CGNE) only, not with the persistent kernel; Lx must be even.
 *   The paper asks for operator forms better suited to the Dirac operator
 *   (Conclusions) without describing one; this is the textbook elimination. */
#define WD_PRECOND_NONE 0
#define WD_PRECOND_EO   1

typedef struct {
    int32_t status;           /* WD_OK, WD_ENOTCONV or WD_EBREAKDOWN                    */
    int32_t iters;            /* CG iterations performed                                */
    int32_t reliable_updates; /* true-residual recomputations, the final one included   */
    int32_t reserved;
    double  true_rel_res;     /* |eta - D x| / |eta|, recomputed in FP64 at the end    */
    double  iter_rel_res;     /* last recursively updated residual / |eta|             */
    double  seconds;          /* wall time of the whole call                           */
} wd_cg_report;

/* tol 1e-10, max_iter 20000, reliable_every 50, inner WD_F32, use_x0 0,
 * persistent -1, chunk 0, method WD_METHOD_CGNE, precondition WD_PRECOND_NONE */
void   wd_cg_default_params(wd_cg_params *p);
/* device workspace a solve of nrhs fields on g's lattice needs, in bytes */
size_t wd_cg_workspace_bytes(const wd_gauge *g, int32_t nrhs, const wd_cg_params *p);

/* Solve D x = eta for one field (src/sol canonical complex128 [V][12]).
 * ws_dev: caller-owned device workspace of at least wd_cg_workspace_bytes.
 * The inner iteration runs in p->inner precision; the solution is accumulated
 * in FP64 and every reliable update recomputes eta - D x with the FP64 links.
 * Returns WD_OK when the FP64 true residual is <= tol, else the first failing
 * per-field status.  Synchronises `stream`. */
int wd_cg_solve(const wd_gauge *g, double m0, const void *src_dev, void *sol_dev,
                const wd_cg_params *p, void *ws_dev, size_t ws_bytes, wd_cg_report *rep,
                void *stream);
/* The same for nrhs fields that share the links (src/sol [nrhs][V][12]); one
 * report per field.  All fields advance in the same kernels, each with its own
 * CG scalars; converged fields stop doing work. */
int wd_cg_solve_batch(const wd_gauge *g, double m0, const void *src_dev, void *sol_dev,
                      int32_t nrhs, const wd_cg_params *p, void *ws_dev, size_t ws_bytes,
                      wd_cg_report *reps, void *stream);

/* --------------------------------------------------------------- autotuner */
typedef struct {
    int32_t block;        /* threads per block                                   */
    int32_t rhs_per_thread;
    int32_t xcd_remap;    /* 1: tiles mapped to XCDs in contiguous ranges        */
    int32_t hop_order;    /* 1: hops one at a time, 2: a direction's two hops together,
                             3: two hops in flight, 4: 3 with the own spinor loaded
                             first, 5: 3 with the hops that read memory (z, t) before
                             the ones that read LDS (x, y; plane blocks, one rhs per
                             thread), 0: compiler order                           */
    int32_t rhs_loop;     /* rhs groups one block handles one after the other    */
    int32_t site_order;   /* strip | xy_planes << 12 | group_major << 16
                             | xy_lds << 17 | occ << 18 | z_march << 24
                             | rhs_pass << 25.
                             strip = W in 1..4095: sites are processed in strips
                             of W z-planes, t-major inside a strip (0:
                             lexicographic); xy_planes = k in 2..4 (with xy_lds
                             = 1, one rhs per thread; the operator with hop
                             order 3 or 5, CG phases A and B with hop order
                             5): a block is k
                             z-adjacent xy-planes (k Lx Ly <= 512 sites), a z
                             neighbour inside it read from LDS too; a lattice,
                             precision or strip where k planes do not fit (FP64,
                             Lz or W not a multiple of k) uses one (0 or 1:
                             one plane);
                             group_major = 1: tiles are ordered rhs-group-major
                             instead of site-block-major; xy_lds = 1: one xy-plane
                             per block with the x/y neighbours in LDS; occ > 0: at
                             most occ plane blocks per compute unit (operator);
                             z_march = 1 (with xy_lds = 1; CG phases A and B in
                             FP32/FP16N storage): a block walks a column of
                             xy-planes along z with two planes in LDS, and strip
                             is then the number of z-chunks (0: automatic);
                             rhs_pass = n in 1..63 (CG phases A and B, not with
                             group_major or z_march): the site blocks are cut
                             into eight chunks, one per XCD's tile range, each
                             walked in passes of n rhs groups (0: all at once);
                             results are bitwise the same for every order    */
    double  us;           /* median time of one application, microseconds        */
    double  gbps;         /* algorithmic bytes / time                             */
} wd_tune_result;

/* Time every candidate launch shape of the operator for (g, prec, nrhs, dagger)
 * on scratch data, reject candidates whose output differs from the reference
 * shape's by more than rounding (shapes that sum the hops in another order round
 * differently: per component FP64 1e-12, FP32 2e-5 of the largest component,
 * FP16N two half ulps of the site norm), and store the fastest in the in-process table (and in the cache file
 * named by WD_TUNE_CACHE, if set).  Later calls with the same key use it.
 * Synchronises `stream`. */
int wd_tune_dslash(const wd_gauge *g, int32_t prec, int32_t nrhs, int32_t dagger,
                   wd_tune_result *best, void *stream);
/* the launch shape currently used for the key (tuned or default) */
int wd_tune_lookup(const wd_gauge *g, int32_t prec, int32_t nrhs, int32_t dagger,
                   wd_tune_result *cfg);

/* Autotune the CG phase kernels as Sec. 3.1 tunes the workgroup size of the
 * whole CG (Fig. 1): one launch shape for phases A and B (families
 * WD_FAMILY_CG_A and WD_FAMILY_CG_B) of g's lattice, inner precision `inner`
 * and nrhs fields.  Every candidate (plane or site blocks, 1 or 2 rhs per
 * thread, hop order 1, 3 or 5 (5: plane blocks, one rhs per thread), z-strips of
 * 0/2/4/7 planes, with hop order 5 one or two planes per block where two fit)
 * runs `iters` (1..1000)
 * CG iterations from the nrhs canonical fields src_dev (as wd_cg_solve_batch
 * takes them) with the mass m0; the median of three runs is kept; a candidate
 * whose iterate differs from the first candidate's by more than 1e-3 relative
 * is rejected.  The fastest shape is stored for later solves and returned in
 * best (best->us: its median time of the whole run, microseconds).  Allocates
 * and frees its own device scratch; synchronises `stream`.  On an error the
 * previous shapes are restored. */
int wd_tune_cg(const wd_gauge *g, double m0, int32_t inner, const void *src_dev, int32_t nrhs,
               int32_t iters, wd_tune_result *best, void *stream);

/* kernel families of the shape table */
#define WD_FAMILY_DSLASH 0   /* wd_dslash / wd_dslash_dag                       */
#define WD_FAMILY_CG_A   1   /* CG phase A: q = D^dagger r + beta q, |q|^2     */
#define WD_FAMILY_CG_B   2   /* CG phase B: D q, r and x updates, |r|^2; also
                                 BiCGSTAB's two stencil stages (its plane-blocked
                                 bit; they take hop order 5, one rhs per thread) */
#define WD_FAMILY_CG_R   3   /* reliable update r = eta - D x (FP64)           */
/* Set the launch shape of one kernel family for (g's lattice, prec, nrhs,
 * dagger) by hand -- e.g. to sweep the block size of the whole CG as the paper
 * does for its workgroup size (Sec. 3.1, Fig. 1).  block in {64,128,256},
 * rhs_per_thread in {1,2,4}, hop_order 0..5 (CG phases: 1, 3 or 5), rhs_loop >= 1,
 * site_order as in wd_tune_result; z_march = 1 for the operator kernel (FP32 and
 * FP16N storage): a block walks a column of xy-planes along z, strip is then the
 * (even) number of z-chunks, alternate chunks walk downward, and group_major
 * selects the tile order (0: chunk, rhs, t; 1: rhs, t, chunk). */
int wd_shape_set(const wd_gauge *g, int32_t prec, int32_t nrhs, int32_t dagger, int32_t family,
                 const wd_tune_result *shape);
/* The launch shape a kernel family uses for the key (set, tuned or default);
 * us and gbps are 0. */
int wd_shape_get(const wd_gauge *g, int32_t prec, int32_t nrhs, int32_t dagger, int32_t family,
                 wd_tune_result *shape);


/* --------------------------------------------------------------- profiling */
/* Per-kernel statistics of CG solves.  While profiling is on, wd_cg_solve*
 * launch the kernels of each chunk one by one (instead of replaying the chunk
 * graph) and launch every phase-A/B/C tile kernel with HIP start/stop events
 * on the solve's stream, recorded at the kernel's own begin and end (the
 * one-block reduction launch after B is not included).  Launched one by
 * one, the kernels run somewhat slower than inside the graph.  bytes_total sums the algorithmic bytes of those launches (links
 * once, every spinor of every active right-hand side once per read or write).
 * Meant for measurement runs; CG (WD_METHOD_CGNE) without the persistent
 * kernel only. */
typedef struct {
    char    name[32];       /* "cg_phaseA" (q = D^dagger r + beta q), "cg_phaseB" (D q +
                               updates), "cg_phaseC" (p = r + beta p: only in solves
                               whose phase A reads p, i.e. z-marching phase A; 0
                               launches otherwise)                                    */
    int64_t launches;
    double  total_ms;       /* summed event time                                    */
    double  bytes_total;    /* summed algorithmic bytes                             */
} wd_kernel_stat;

int wd_profile_enable(int32_t on);                       /* process-wide switch   */
int wd_profile_reset(void);
/* copy up to max_n entries into out, *n = number of entries available */
int wd_profile_read(wd_kernel_stat *out, int32_t max_n, int32_t *n);

/* Chunk graphs of the CG solvers: *built = graphs captured since the library
 * was loaded, *cached = graphs held now (at most 32, least recently used ones
 * are dropped).  A solve replays the graph of its key (workspace address,
 * lattice, rhs count, inner precision, chunk length, method and every field
 * of every kernel's launch shape) and captures a new one when none matches. */
int wd_cg_graph_stats(int64_t *built, int32_t *cached);

/* --------------------------------------------------------- bandwidth probe */
/* The memory ceiling the operator's bandwidth is measured against (the naive
 * roofline P = min(peak flops, bandwidth x intensity) of Sec. 3.1 needs the
 * attainable bandwidth): one streaming kernel with 16-byte coalesced accesses.
 *   WD_STREAM_READ   reads `bytes` of src_dev (dst_dev: 16 bytes the kernel may
 *                    write, so that no load can be dropped)
 *   WD_STREAM_COPY   copies `bytes` from src_dev to dst_dev (no overlap)
 *   WD_STREAM_WRITE  writes `bytes` of a constant pattern to dst_dev (src_dev unused)
 * bytes and both pointers must be multiples of 16 (WD_EINVAL otherwise).
 * Asynchronous on `stream`. */
#define WD_STREAM_READ  0
#define WD_STREAM_COPY  1
#define WD_STREAM_WRITE 2
int wd_stream(int32_t kind, const void *src_dev, void *dst_dev, size_t bytes, void *stream);

/* ----------------------------------------------------------------- serving */
typedef struct wd_server wd_server;

typedef struct {
    void   *arena_dev;     /* caller-owned device memory the server carves from       */
    size_t  arena_bytes;
    int32_t max_slots;     /* requests resident on the device at once (<= 64)         */
    int32_t chunk;         /* CG iterations per scheduling step (0 = default 25)     */
    int32_t device;        /* HIP device ordinal                                      */
    int32_t reserved;
} wd_serve_config;

typedef struct {
    int32_t     dims[4];
    int32_t     t_sign;
    int32_t     nrhs;
    double      m0;
    const void *gauge_dev;  /* canonical complex128 links; read during admission     */
    const void *src_dev;    /* canonical complex128 [nrhs][V][12]; read at admission */
    void       *sol_dev;    /* canonical complex128 [nrhs][V][12]; written at retire */
    wd_cg_params params;    /* inner WD_F32 or WD_F64; WD_METHOD_CGNE; precondition
                               WD_PRECOND_NONE or WD_PRECOND_EO (even Lx)              */
} wd_request;

typedef struct {
    uint64_t submitted, admitted, completed;
    uint64_t steps;             /* scheduling steps run                           */
    uint64_t arena_high_water;  /* largest number of arena bytes in use           */
    int32_t  active, pending;
    uint64_t arena_capacity;    /* arena bytes left for requests once the server's
                                   own tables are carved out: the largest footprint
                                   wd_serve_submit accepts                        */
} wd_serve_stats;

/* Device bytes a request occupies in the arena while it is resident. */
size_t wd_serve_footprint(const wd_request *req);
/* Start the scheduler thread.  The arena is used as a first-fit heap. */
int wd_serve_create(const wd_serve_config *cfg, wd_server **out);
/* Queue a request; returns at once.  WD_ETOOBIG if its footprint exceeds the
 * arena capacity (wd_serve_stats.arena_capacity), so it could never be admitted;
 * every accepted request is admitted once enough of the arena is free.
 * The caller keeps gauge_dev/src_dev/sol_dev alive until the ticket is done. */
int wd_serve_submit(wd_server *s, const wd_request *req, uint64_t *ticket);
/* *done = 1 and reps[nrhs] filled once the request is finished, else *done = 0.
 * Thread-safe, non-blocking.  The per-field seconds are submit -> done. */
int wd_serve_poll(wd_server *s, uint64_t ticket, wd_cg_report *reps, int32_t *done);
int wd_serve_stats_get(wd_server *s, wd_serve_stats *st);
/* Finish the requests already admitted, drop the pending ones, stop the thread. */
int wd_serve_destroy(wd_server *s);

#ifdef __cplusplus
}
#endif
#endif /* WD_H */
