// Continuous-batching solve server: many CG solves of the Wilson-Dirac
// operator (arXiv 2111.14958, Eq. (1) and the CG of Sec. 2) resident on one
// GPU at once.
//
// A scheduler thread owns a caller-given device arena, managed as a first-fit
// heap.  At every step boundary it admits pending requests in arrival order
// while their footprint (packed links, CG vectors, scalars) fits the free arena
// and a slot is free; a request that has waited too long blocks later ones
// from jumping ahead of it.  A step is `chunk` CG iterations for every resident
// request at once: each kernel of the iteration is one grouped launch over the
// tiles of all requests (each record carries its own lattice, links, vectors
// and scalars), so work of different requests shares the device.  After the
// step the scheduler reads every request's per-field state, retires finished
// requests (solution unpacked to the caller's buffer, reports filed, arena
// freed) and admits new ones.  The per-field arithmetic does not depend on
// which other requests share a launch, so a request's result is the same
// alone and in a mix.
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "cg_host.h"

namespace wd {

static size_t al256s(size_t x) { return (x + 255) & ~size_t(255); }

struct Arena {
    size_t size = 0, used = 0, high = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    void init(size_t n) {
        size = n;
        free_.clear();
        free_[0] = n;
        used = high = 0;
    }
    bool alloc(size_t n, size_t *off) {
        n = al256s(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t o = it->first, rem = it->second - n;
            free_.erase(it);
            if (rem) free_[o + n] = rem;
            *off = o;
            used += n;
            if (used > high) high = used;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = al256s(n);
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct SlotLayout {
    size_t links64, links_lo, ws, total;
    WsLayout L;
};

static SlotLayout slot_layout(int64_t V, int nrhs, int inner, int eo) {
    SlotLayout s;
    size_t o = 0;
    s.links64 = o;
    o += al256s(link_bytes(WD_F64, V));
    if (inner != WD_F64) {
        s.links_lo = o;
        o += al256s(link_bytes(inner, V));
    } else {
        s.links_lo = s.links64;
    }
    s.ws = o;
    s.L = ws_layout(V, nrhs, inner, METHOD_CGNE, eo);
    o += s.L.total;
    s.total = o;
    return s;
}

struct Pending {
    uint64_t ticket;
    wd_request req;
    std::chrono::steady_clock::time_point t_submit;
    int waited = 0;
};

struct Slot {
    uint64_t ticket;
    wd_request req;
    int64_t V;
    size_t off;
    SlotLayout sl;
    Prob prob;      // record with t0 = 0 (standalone launches)
    std::vector<Scal> sc;
    std::chrono::steady_clock::time_point t_submit;
};

// Fixed server-wide launch shapes: results must not depend on the mix.
static void server_shapes(int inner, int &blk, int &nr_ab) {
    blk = 256;
    nr_ab = inner == WD_F64 ? 1 : 2;
}

// Phases A and B of an FP32 or FP64 request without even-odd preconditioning
// whose xy-planes hold 128..256 sites run on plane blocks (one plane per
// 256-thread block, x and y neighbours from LDS, hop order 5, one rhs per
// thread); every other kernel, and every other request, on site blocks.  The
// choice depends on the request alone, so its results do not depend on the mix.
static bool server_xy(int inner, int eo, const int dims[4]) {
    const int np = dims[0] * dims[1];
    return !eo && inner != WD_F16N && np >= 128 && np <= 256;
}
static bool prob_xy(const Prob &pr) { return (pr.sorder[KA] >> 17) & 1; }

// tiles of every kernel kind for one request (vectors of vf sites)
static void prob_tiles(Prob &pr, int inner, int64_t vf, int nrhs, bool xy) {
    int blk, nr;
    server_shapes(inner, blk, nr);
    for (int k = 0; k < NKIND; ++k) {
        const bool plane = xy && (k == KA || k == KB);
        const int knr = plane ? 1 : (k == KA || k == KB || k == KEA1 || k == KEB1) ? nr : 1;
        pr.nsb[k] = plane ? (int)(vf / pr.g.S[2]) : (int)((vf + blk - 1) / blk);
        pr.ng[k] = (k == KC || k == KR1 || k == KN) ? nrhs : (nrhs + knr - 1) / knr;
        pr.nt[k] = pr.nsb[k] * pr.ng[k];
        pr.t0[k] = 0;
        pr.sorder[k] = plane ? 1 << 17 : 0;   // plane-blocked tiles, lexicographic planes
    }
}

// launch shapes of the server's kernels, with the grid of every kind
static LaunchSet server_launch(int inner, int eo, int xy, const int grid[NKIND]) {
    int blk, nr;
    server_shapes(inner, blk, nr);
    LaunchSet ls;
    ls.eo = eo;
    ls.qrec = 1;   // k_phaseA and the even-odd phase A carry the direction as q
    ls.fused = !eo && !unfused_requested();   // site blocks, phase A's reduction in phase B: phase A
                                              // finishes the iteration before it
    for (int k = 0; k < NKIND; ++k) {
        const bool stencil = k == KA || k == KB || k == KR2 || k == KEA1 || k == KEB1 || k == KER2A;
        ls.k[k].block = blk;
        ls.k[k].nr = (k == KA || k == KB || k == KEA1 || k == KEB1) ? nr : 1;
        ls.k[k].remap = stencil ? 1 : 0;
        ls.k[k].grid = grid[k];
        if (xy && (k == KA || k == KB)) {
            ls.k[k].xy = 1;
            ls.k[k].nr = 1;
            ls.k[k].ordered = 5;
            ls.k[k].order = 1 << 17;
        }
    }
    return ls;
}

static LaunchSet single_launch(const Prob &pr, int inner) { return server_launch(inner, pr.eo, prob_xy(pr), pr.nt); }

}  // namespace wd

struct wd_server {
    wd_serve_config cfg;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<wd::Pending> pending;
    std::map<uint64_t, std::vector<wd_cg_report>> done;
    std::vector<wd::Slot> active;   // scheduler thread only
    wd::Arena arena;                // guarded by mu
    uint64_t next_ticket = 1;
    bool stop = false;
    int error = 0;
    std::thread th;
    hipStream_t st = nullptr;
    wd_serve_stats stats{};
    // per (inner precision, even-odd, plane-blocked phases) group: max_slots Prob records
    static constexpr int NGROUP = 12;
    size_t table_off[NGROUP] = {};
    size_t table_bytes = 0;             // arena bytes the tables occupy
    std::vector<wd::Prob> table[NGROUP];   // host staging of the tables (alive until the step syncs)
    int chunk = 25;
};

namespace wd {

static char *arena_ptr(wd_server *s, size_t off) { return (char *)s->cfg.arena_dev + off; }

// Pack links and source, reset the CG state and run the first true residual.
static int init_slot(wd_server *s, Slot &sl) {
    const wd_request &rq = sl.req;
    const int inner = rq.params.inner;
    const int64_t V = sl.V;
    char *base = arena_ptr(s, sl.off);
    hipStream_t st = s->st;
    int rc = launch_pack_links(WD_F64, rq.gauge_dev, base + sl.sl.links64, rq.dims, rq.t_sign, st);
    if (!rc && inner != WD_F64)
        rc = launch_pack_links(inner, rq.gauge_dev, base + sl.sl.links_lo, rq.dims, rq.t_sign, st);
    if (rc) return rc;
    wd_gauge g;   // a view of the arena copies, for the record
    memset(&g, 0, sizeof(g));
    for (int d = 0; d < 4; ++d) g.dims[d] = rq.dims[d];
    g.tsign = rq.t_sign;
    g.V = V;
    g.U[WD_F64] = base + sl.sl.links64;
    g.U[inner] = base + sl.sl.links_lo;
    char *w = base + sl.sl.ws;
    const WsLayout &L = sl.sl.L;
    memset(&sl.prob, 0, sizeof(sl.prob));
    fill_prob(sl.prob, &g, rq.m0, rq.nrhs, rq.params, w, L);
    const int eo = sl.prob.eo;
    const int64_t vf = sl.prob.vf;
    prob_tiles(sl.prob, inner, vf, rq.nrhs, server_xy(inner, eo, rq.dims));
    init_scalars(sl.sc, rq.nrhs);
    WD_HIP(hipMemcpyAsync(w + L.prob, &sl.prob, sizeof(Prob), hipMemcpyHostToDevice, st));
    WD_HIP(hipMemcpyAsync(w + L.scal, sl.sc.data(), sizeof(Scal) * rq.nrhs, hipMemcpyHostToDevice, st));
    WD_HIP(hipMemsetAsync(w + L.bar, 0, BAR_BYTES, st));
    const Prob *dp = (const Prob *)(w + L.prob);
    if (eo) {
        launch_eo_split(dp, vf, rq.nrhs, rq.src_dev, w + L.eta64, w + L.eta_o, st);
        if (rq.params.use_x0) launch_eo_split(dp, vf, rq.nrhs, rq.sol_dev, w + L.x64, w + L.w64, st);
        else launch_zero(w + L.x64, spinor_bytes(WD_F64, vf, rq.nrhs), st);
    } else {
        rc = launch_pack_spinor(WD_F64, rq.src_dev, w + L.eta64, (int)V, rq.nrhs, st);
        if (rc) return rc;
        if (rq.params.use_x0) rc = launch_pack_spinor(WD_F64, rq.sol_dev, w + L.x64, (int)V, rq.nrhs, st);
        else launch_zero(w + L.x64, spinor_bytes(WD_F64, V, rq.nrhs), st);
        if (rc) return rc;
    }
    launch_zero(w + L.xlo, spinor_bytes(inner == WD_F16N ? WD_F32 : inner, vf, rq.nrhs), st);
    const LaunchSet ls = single_launch(sl.prob, inner);
    launch_kind(KN, inner, ls, st, dp, 1);
    if (eo) {
        launch_eo_source(dp, vf, rq.nrhs, st);
        launch_kind(KER2A, inner, ls, st, dp, 1);
    }
    launch_first_residual(inner, ls, st, dp, 1, !rq.params.use_x0);
    launch_kind(KC, inner, ls, st, dp, 1);
    WD_HIP(hipGetLastError());
    return WD_OK;
}

// One step: `chunk` iterations plus a reliable update for every resident
// request of one group (inner precision, even-odd or not, plane-blocked phases
// or not: gkey = (inner 2 + eo) 2 + xy), as grouped launches.
static int group_key(const Slot &sl) { return (sl.req.params.inner * 2 + sl.prob.eo) * 2 + (prob_xy(sl.prob) ? 1 : 0); }
static int step_group(wd_server *s, int gkey, const std::vector<Slot *> &grp) {
    if (grp.empty()) return WD_OK;
    const int inner = gkey >> 2, eo = (gkey >> 1) & 1, xy = gkey & 1;
    std::vector<Prob> &table = s->table[gkey];
    table.clear();
    int tot[NKIND] = {};
    for (Slot *sl : grp) {
        Prob p = sl->prob;
        for (int k = 0; k < NKIND; ++k) {
            p.t0[k] = tot[k];
            tot[k] += p.nt[k];
        }
        table.push_back(p);
    }
    const LaunchSet ls = server_launch(inner, eo, xy, tot);
    Prob *dt = (Prob *)arena_ptr(s, s->table_off[gkey]);
    const int n = (int)table.size();
    WD_HIP(hipMemcpyAsync(dt, table.data(), sizeof(Prob) * n, hipMemcpyHostToDevice, s->st));
    launch_iterations(inner, ls, s->st, dt, n, s->chunk);
    launch_kind(KR1, inner, ls, s->st, dt, n);
    if (eo) launch_kind(KER2A, inner, ls, s->st, dt, n);
    launch_kind(KR2, inner, ls, s->st, dt, n);
    launch_kind(KC, inner, ls, s->st, dt, n);
    WD_HIP(hipGetLastError());
    return WD_OK;
}

static bool slot_finished(const Slot &sl) {
    for (const Scal &c : sl.sc)
        if (c.state == ST_ACTIVE || c.state == ST_FROZEN) return false;
    return true;
}

static void fill_reports(const Slot &sl, std::vector<wd_cg_report> &reps, double secs, int force_status) {
    reps.assign(sl.req.nrhs, wd_cg_report());
    for (int i = 0; i < sl.req.nrhs; ++i) {
        const Scal &c = sl.sc[i];
        wd_cg_report &r = reps[i];
        memset(&r, 0, sizeof(r));
        r.status = force_status ? force_status : cg_status_of(c.state);
        r.iters = c.iters;
        r.reliable_updates = c.n_ru;
        r.true_rel_res = c.eta2 > 0 ? sqrt(c.true2 / c.eta2) : 0.0;
        r.iter_rel_res = c.eta2 > 0 ? sqrt(c.rho / c.eta2) : 0.0;
        r.seconds = secs;
    }
}

static double since(std::chrono::steady_clock::time_point t) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t).count();
}

// Fail every resident and pending request (after a runtime error).
static void fail_all(wd_server *s, int code) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->error = code;
    for (Slot &sl : s->active) {
        std::vector<wd_cg_report> reps;
        fill_reports(sl, reps, since(sl.t_submit), code);
        s->done[sl.ticket] = reps;
        s->arena.release(sl.off, sl.sl.total);
    }
    s->active.clear();
    for (Pending &p : s->pending) {
        std::vector<wd_cg_report> reps(p.req.nrhs);
        memset(reps.data(), 0, sizeof(wd_cg_report) * p.req.nrhs);
        for (auto &r : reps) r.status = code;
        s->done[p.ticket] = reps;
    }
    s->pending.clear();
    s->stats.active = 0;
    s->stats.pending = 0;
    s->stats.completed = s->done.size();
}

static void scheduler(wd_server *s) {
    (void)hipSetDevice(s->cfg.device);
    const int max_wait_steps = 8;
    for (;;) {
        std::vector<Slot> admitted;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] { return s->stop || !s->pending.empty() || !s->active.empty(); });
            if (s->stop && s->active.empty()) break;
            if (s->stop) s->pending.clear();
            // admission in arrival order, by footprint and free slots
            bool blocked = false;
            for (auto it = s->pending.begin(); it != s->pending.end() && !blocked;) {
                const int nslots = (int)(s->active.size() + admitted.size());
                const SlotLayout lay = slot_layout((int64_t)it->req.dims[0] * it->req.dims[1] *
                                                       it->req.dims[2] * it->req.dims[3],
                                                   it->req.nrhs, it->req.params.inner,
                                                   it->req.params.precondition == WD_PRECOND_EO);
                size_t off = 0;
                if (nslots < s->cfg.max_slots && s->arena.alloc(lay.total, &off)) {
                    Slot sl;
                    sl.ticket = it->ticket;
                    sl.req = it->req;
                    sl.V = (int64_t)it->req.dims[0] * it->req.dims[1] * it->req.dims[2] * it->req.dims[3];
                    sl.off = off;
                    sl.sl = lay;
                    sl.t_submit = it->t_submit;
                    admitted.push_back(sl);
                    it = s->pending.erase(it);
                    s->stats.admitted++;
                } else if (s->active.empty() && admitted.empty() && nslots < s->cfg.max_slots) {
                    // the arena is empty and still too small (submit's capacity
                    // check rules this out): fail the request rather than wait
                    // for space that can never appear
                    std::vector<wd_cg_report> reps(it->req.nrhs);
                    memset(reps.data(), 0, sizeof(wd_cg_report) * it->req.nrhs);
                    for (auto &r : reps) r.status = WD_ETOOBIG;
                    s->done[it->ticket] = reps;
                    s->stats.completed++;
                    it = s->pending.erase(it);
                } else {
                    // keep the order fair: a request that has waited long enough
                    // stops later requests from overtaking it
                    if (++it->waited > max_wait_steps) blocked = true;
                    ++it;
                }
            }
            s->stats.arena_high_water = s->arena.high;
        }
        int rc = WD_OK;
        for (Slot &sl : admitted) {
            if (!rc) rc = init_slot(s, sl);
            s->active.push_back(sl);
        }
        if (rc) { fail_all(s, rc); continue; }
        // one step over every resident request
        std::vector<Slot *> grp[wd_server::NGROUP];
        for (Slot &sl : s->active) grp[group_key(sl)].push_back(&sl);
        for (int p = 0; p < wd_server::NGROUP && !rc; ++p) rc = step_group(s, p, grp[p]);
        if (!rc && hipStreamSynchronize(s->st) != hipSuccess) rc = WD_EHIP;
        for (Slot &sl : s->active) {
            if (rc) break;
            if (hipMemcpyAsync(sl.sc.data(), arena_ptr(s, sl.off) + sl.sl.ws + sl.sl.L.scal,
                               sizeof(Scal) * sl.req.nrhs, hipMemcpyDeviceToHost, s->st) != hipSuccess)
                rc = WD_EHIP;
        }
        if (!rc && hipStreamSynchronize(s->st) != hipSuccess) rc = WD_EHIP;
        if (rc) { fail_all(s, rc); continue; }
        // retire finished requests
        std::vector<Slot> keep, fin;
        for (Slot &sl : s->active) (slot_finished(sl) ? fin : keep).push_back(sl);
        for (Slot &sl : fin) {
            char *w = arena_ptr(s, sl.off) + sl.sl.ws;
            if (sl.prob.eo) {
                launch_eo_merge((const Prob *)(w + sl.sl.L.prob), sl.prob.vf, sl.req.nrhs, sl.req.sol_dev, s->st);
                if (hipGetLastError() != hipSuccess) rc = WD_EHIP;
            } else {
                rc = launch_unpack_spinor(WD_F64, w + sl.sl.L.x64, sl.req.sol_dev, (int)sl.V, sl.req.nrhs, s->st);
            }
            for (int i = 0; i < sl.req.nrhs && !rc; ++i)
                if (sl.sc[i].zero_src &&
                    hipMemsetAsync((char *)sl.req.sol_dev + (size_t)i * sl.V * 192, 0, (size_t)sl.V * 192,
                                   s->st) != hipSuccess)
                    rc = WD_EHIP;
            if (rc) break;
        }
        if (!rc && !fin.empty() && hipStreamSynchronize(s->st) != hipSuccess) rc = WD_EHIP;
        if (rc) { fail_all(s, rc); continue; }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (Slot &sl : fin) {
                std::vector<wd_cg_report> reps;
                fill_reports(sl, reps, since(sl.t_submit), 0);
                s->done[sl.ticket] = reps;
                s->arena.release(sl.off, sl.sl.total);
                s->stats.completed++;
            }
            s->active = keep;
            s->stats.steps++;
            s->stats.active = (int32_t)s->active.size();
            s->stats.pending = (int32_t)s->pending.size();
        }
    }
}

static int check_request(const wd_request *r) {
    WD_CHECK(r, WD_EINVAL, "null request");
    WD_CHECK(r->gauge_dev && r->src_dev && r->sol_dev, WD_EINVAL, "null field pointer");
    WD_CHECK(r->src_dev != r->sol_dev, WD_EINVAL, "src and sol must not overlap");
    WD_CHECK(r->t_sign == 1 || r->t_sign == -1, WD_EINVAL, "t_sign must be +1 or -1");
    WD_CHECK(r->nrhs >= 1 && r->nrhs <= MAX_RHS, WD_EINVAL, "nrhs %d out of range", r->nrhs);
    WD_CHECK(r->m0 > -4.0 && r->m0 < 1e6, WD_EINVAL, "m0 %g out of range", r->m0);
    int64_t V = 1;
    for (int d = 0; d < 4; ++d) {
        WD_CHECK(r->dims[d] >= 1 && r->dims[d] <= 4096, WD_EINVAL, "bad extent %d", r->dims[d]);
        V *= r->dims[d];
    }
    WD_CHECK(V <= MAX_SITES, WD_EINVAL, "lattice too large");
    int rc = check_params(&r->params);
    if (rc) return rc;
    WD_CHECK(r->params.inner == WD_F32 || r->params.inner == WD_F64, WD_EINVAL,
             "the server runs FP32 or FP64 inner iterations");
    WD_CHECK(r->params.method == METHOD_CGNE, WD_EINVAL, "the server runs CG on the normal equations only");
    WD_CHECK(r->params.max_cus == 0, WD_EINVAL, "the server runs on the whole device (max_cus 0)");
    WD_CHECK(r->params.precondition == WD_PRECOND_NONE || r->dims[0] % 2 == 0, WD_EINVAL,
             "even-odd preconditioning needs an even Lx");
    return WD_OK;
}

}  // namespace wd

using namespace wd;

extern "C" {

size_t wd_serve_footprint(const wd_request *req) {
    if (check_request(req) != WD_OK) return 0;
    const int64_t V = (int64_t)req->dims[0] * req->dims[1] * req->dims[2] * req->dims[3];
    return al256s(slot_layout(V, req->nrhs, req->params.inner, req->params.precondition == WD_PRECOND_EO).total);
}

int wd_serve_create(const wd_serve_config *cfg, wd_server **out) {
    clear_error();
    WD_CHECK(cfg && out, WD_EINVAL, "null argument");
    WD_CHECK(cfg->arena_dev && cfg->arena_bytes > 0, WD_EINVAL, "empty arena");
    WD_CHECK(cfg->max_slots >= 1 && cfg->max_slots <= 64, WD_EINVAL, "max_slots %d out of 1..64", cfg->max_slots);
    WD_CHECK(cfg->chunk >= 0 && cfg->chunk <= 1000, WD_EINVAL, "chunk %d out of range", cfg->chunk);
    WD_CHECK(((uintptr_t)cfg->arena_dev & 255) == 0, WD_EINVAL, "arena must be 256-byte aligned");
    int prev_dev = 0;
    WD_HIP(hipGetDevice(&prev_dev));
    WD_HIP(hipSetDevice(cfg->device));
    int rc = require_gfx950();
    (void)hipSetDevice(prev_dev);
    if (rc) return rc;
    wd_server *s = new wd_server();
    s->cfg = *cfg;
    s->chunk = cfg->chunk > 0 ? cfg->chunk : 25;
    s->arena.init(cfg->arena_bytes);
    const size_t tb = al256s(sizeof(Prob) * cfg->max_slots);
    for (int p = 0; p < wd_server::NGROUP; ++p) {
        if (!s->arena.alloc(tb, &s->table_off[p])) {
            delete s;
            return fail(WD_ETOOBIG, "arena too small for the request tables");
        }
    }
    s->table_bytes = s->arena.used;
    s->arena.high = s->arena.used;
    (void)hipSetDevice(cfg->device);
    const hipError_t e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking);
    (void)hipSetDevice(prev_dev);
    if (e != hipSuccess) {
        delete s;
        return fail(WD_EHIP, "stream creation failed");
    }
    s->th = std::thread(scheduler, s);
    *out = s;
    return WD_OK;
}

int wd_serve_submit(wd_server *s, const wd_request *req, uint64_t *ticket) {
    clear_error();
    WD_CHECK(s && ticket, WD_EINVAL, "null argument");
    int rc = check_request(req);
    if (rc) return rc;
    const size_t need = wd_serve_footprint(req);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->error) return fail(s->error, "server stopped after a runtime error");
    WD_CHECK(!s->stop, WD_EINVAL, "server is shutting down");
    // what is left of the arena once the request tables are carved out: a
    // request of at most this footprint fits as soon as nothing else is resident
    const size_t capacity = s->arena.size - s->table_bytes;
    if (need > capacity)
        return fail(WD_ETOOBIG, "request needs %zu bytes, the arena offers %zu", need, capacity);
    Pending p;
    p.ticket = s->next_ticket++;
    p.req = *req;
    p.t_submit = std::chrono::steady_clock::now();
    s->pending.push_back(p);
    s->stats.submitted++;
    s->stats.pending = (int32_t)s->pending.size();
    *ticket = p.ticket;
    s->cv.notify_all();
    return WD_OK;
}

int wd_serve_poll(wd_server *s, uint64_t ticket, wd_cg_report *reps, int32_t *done) {
    clear_error();
    WD_CHECK(s && done, WD_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->done.find(ticket);
    if (it == s->done.end()) {
        bool known = ticket > 0 && ticket < s->next_ticket;
        *done = 0;
        return known ? WD_OK : fail(WD_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    }
    if (reps) memcpy(reps, it->second.data(), sizeof(wd_cg_report) * it->second.size());
    *done = 1;
    return WD_OK;
}

int wd_serve_stats_get(wd_server *s, wd_serve_stats *st) {
    clear_error();
    WD_CHECK(s && st, WD_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *st = s->stats;
    st->arena_high_water = s->arena.high;
    st->arena_capacity = s->arena.size - s->table_bytes;
    st->pending = (int32_t)s->pending.size();
    return WD_OK;
}

int wd_serve_destroy(wd_server *s) {
    clear_error();
    if (!s) return WD_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    if (s->st) (void)hipStreamDestroy(s->st);
    delete s;
    return WD_OK;
}

}  // extern "C"
