"""Experiments beyond the benchmark line, on MI355X.

    python -m paper_2111_14958_amd.experiments fig1    # whole-CG time vs block size
    python -m paper_2111_14958_amd.experiments fig2    # whole-CG speedup vs compute units
    python -m paper_2111_14958_amd.experiments serve   # open-loop serving latency
    python -m paper_2111_14958_amd.experiments serve eo   # the same, even-odd preconditioned
    python -m paper_2111_14958_amd.experiments solve [f32|f64|f16n]   # one profiled 14^4 x 16 solve
    python -m paper_2111_14958_amd.experiments dslash f32|f64|f16n hot|cold [reps]
                                                       # the 14^4 x 16 operator alone

Fig. 1 of the paper times the whole CG at 14^4 while varying the SYCL
workgroup size with the number of compute units fixed; here the block size of
every CG kernel is swept (64, 128, 256 threads) through wd_shape_set, using the
single-field FP64 CG of the paper's algorithm (plain CG on D D^dagger,
true-residual check at 1e-10) on seeded synthetic fields (links exp(i 0.5 H),
Gaussian source, m0 = 0.05).  Prints one JSON line per point.

Fig. 2 of the paper plots the speedup of the whole CG at 14^4 against the
number of compute units, relative to one compute unit.  Here the persistent CG
kernel is confined to n compute units (wd_cg_params.max_cus: n blocks of 1024
threads, one per compute unit) and the speedup is T(1) / T(n), for one
Gaussian source and for the 16-source batch (12 point + 4 Gaussian), FP32
inner iterations with FP64 reliable updates every 50.
"""
from __future__ import annotations

import json
import sys
import time


def _setup(dims=(14, 14, 14, 14), m0=0.05, nrhs=1):
    import torch

    import paper_2111_14958_amd as wd
    import wdgen
    U = wdgen.gauge_field(dims, 0.5, 1002)
    src = wdgen.gaussian_source(dims, 1, 2002) if nrhs == 1 else wdgen.mixed_sources(dims, 12, nrhs - 12, 2002)
    g = wd.Gauge(torch.from_numpy(U).cuda(), dims)
    dsrc = torch.from_numpy(src).cuda()
    return wd, torch, g, dsrc, m0


def _time_solve(wd, torch, g, dsrc, m0, params, reps=3):
    sol = torch.zeros_like(dsrc)
    ws = torch.empty(wd.cg_workspace_bytes(g, dsrc.shape[0], params), dtype=torch.uint8, device="cuda")
    wd.cg_solve_batch(g, m0, dsrc, sol=sol, params=params, ws=ws)   # warm (graph capture)
    torch.cuda.synchronize()
    best, rep = 1e30, None
    for _ in range(reps):
        t0 = time.perf_counter()
        _, reps_, rc = wd.cg_solve_batch(g, m0, dsrc, sol=sol, params=params, ws=ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if dt < best:
            best, rep = dt, reps_[0]
    return best, rep


def fig1(blocks=(64, 128, 256)):
    wd, torch, g, dsrc, m0 = _setup()
    p = wd.cg_default_params(inner=wd.F64, reliable_every=0)
    for blk in blocks:
        for fam, dag in ((wd.FAMILY_CG_A, True), (wd.FAMILY_CG_B, False), (wd.FAMILY_CG_R, False)):
            wd.shape_set(g, wd.F64, 1, dag, fam, blk, rhs_per_thread=1)
        t, rep = _time_solve(wd, torch, g, dsrc, m0, p)
        print(json.dumps({"figure": 1, "lattice": "14^4", "block": blk, "seconds": t,
                          "iters": rep["iters"], "true_rel_res": rep["true_rel_res"],
                          "gflops": 2 * 1368.0 * 14 ** 4 * rep["iters"] / t / 1e9}), flush=True)


def fig2(cus=(1, 2, 4, 8, 16, 32, 64, 128, 256), batches=(1, 16)):
    for nrhs in batches:
        wd, torch, g, dsrc, m0 = _setup(nrhs=nrhs)
        t1 = None
        for n in cus:
            p = wd.cg_default_params(inner=wd.F32, reliable_every=50, persistent=1, max_cus=n)
            t, rep = _time_solve(wd, torch, g, dsrc, m0, p, reps=2 if n < 8 else 3)
            t1 = t if t1 is None else t1
            print(json.dumps({"figure": 2, "lattice": "14^4", "rhs": nrhs, "compute_units": n, "seconds": t,
                              "speedup": t1 / t, "iters": rep["iters"], "true_rel_res": rep["true_rel_res"]}),
                  flush=True)
        p = wd.cg_default_params(inner=wd.F32, reliable_every=50)
        t, rep = _time_solve(wd, torch, g, dsrc, m0, p)
        print(json.dumps({"figure": 2, "lattice": "14^4", "rhs": nrhs, "compute_units": "all, default kernels",
                          "seconds": t, "speedup": t1 / t, "iters": rep["iters"]}), flush=True)
        del g


def serve(n_requests=600, rates=(0.25, 0.5, 1.0, 1.5, 2.0), pool=2, arena_gib=24, max_slots=16, seed=10_000,
          eo=False):
    """Continuous-batching solve server under Poisson arrivals.

    Request i (seeded by seed + i): lattice drawn uniformly from 4^4, 8^4, 12^4, 14^4, 16^3 x 32,
    1..12 Gaussian right-hand sides, m0 uniform in [0.02, 0.2], FP32 inner CG
    with FP64 reliable updates, tol 1e-10.  Gauge fields (links exp(i 0.5 H))
    come from a pre-generated pool of `pool` fields per volume; sources are
    drawn on the device.  Everything is generated before the clock starts.
    First a closed-loop run (all requests at t = 0) measures the capacity in
    requests/s; then open-loop runs submit at `rates` x capacity with
    exponential inter-arrival times.  Latency = submit -> result, measured by
    the server.  eo: every request even-odd preconditioned.  Prints one JSON
    line per run.
    """
    import numpy as np
    import torch

    import paper_2111_14958_amd as wd
    import wdgen
    rng = np.random.default_rng(seed)
    volumes = wdgen.SERVING_VOLUMES
    gauges = {}
    for vi, dims in enumerate(volumes):
        gauges[vi] = [torch.from_numpy(wdgen.gauge_field(dims, 0.5, seed + 100 * vi + k)).cuda()
                      for k in range(pool)]
    print(json.dumps({"serve": "pool ready"}), flush=True)
    reqs = []
    gen = torch.Generator(device="cuda")
    for i in range(n_requests):
        vi = int(rng.integers(0, len(volumes)))
        dims = volumes[vi]
        nrhs = int(rng.integers(1, 13))
        m0 = float(rng.uniform(0.02, 0.2))
        V = dims[0] * dims[1] * dims[2] * dims[3]
        gen.manual_seed(seed + 50_000 + i)
        src = torch.randn((nrhs, dims[3], dims[2], dims[1], dims[0], 4, 3), dtype=torch.complex128,
                          device="cuda", generator=gen)
        reqs.append(dict(dims=dims, nrhs=nrhs, m0=m0, V=V, U=gauges[vi][i % pool], src=src))
    arena = torch.empty(int(arena_gib) << 30, dtype=torch.uint8, device="cuda")
    params = wd.cg_default_params(inner=wd.F32, reliable_every=50,
                                  precondition=wd.PRECOND_EO if eo else wd.PRECOND_NONE)

    def run(arrivals):
        srv = wd.Server(arena, max_slots=max_slots)
        sols = [torch.zeros_like(r["src"]) for r in reqs]
        torch.cuda.synchronize()
        tickets, reps = [None] * len(reqs), [None] * len(reqs)
        t0 = time.perf_counter()
        nxt = 0
        while any(r is None for r in reps):
            now = time.perf_counter() - t0
            while nxt < len(reqs) and arrivals[nxt] <= now:
                r = reqs[nxt]
                req = wd.Server.request(r["dims"], r["nrhs"], r["m0"], r["U"], r["src"], sols[nxt], params)
                tickets[nxt] = srv.submit(req)
                nxt += 1
            for i in range(nxt):
                if reps[i] is None:
                    reps[i] = srv.poll(tickets[i])
            time.sleep(0.0005)
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        lat = np.array([rep[0]["seconds"] for rep in reps])
        ok = all(x["status"] == 0 and x["true_rel_res"] <= 1e-10 for rep in reps for x in rep)
        nrhs_tot = sum(r["nrhs"] for r in reqs)
        return dict(requests=len(reqs), wall_s=wall, requests_per_s=len(reqs) / wall,
                    rhs_solves_per_s=nrhs_tot / wall, p50_latency_s=float(np.percentile(lat, 50)),
                    p99_latency_s=float(np.percentile(lat, 99)), all_converged=ok,
                    arena_high_water_gib=st["arena_high_water"] / 2**30, steps=st["steps"])

    closed = run(np.zeros(len(reqs)))
    print(json.dumps({"serve": "closed-loop", "even_odd": eo, **closed}), flush=True)
    cap = closed["requests_per_s"]
    for f in rates:
        arr = np.cumsum(rng.exponential(1.0 / (f * cap), size=len(reqs)))
        res = run(arr - arr[0])
        print(json.dumps({"serve": "poisson", "even_odd": eo, "rate_x_capacity": f, "offered_per_s": f * cap,
                          **res}), flush=True)


def solve(inner_name="f32"):
    """One solve of the 14^4 x 16 benchmark workload (reconstruct-12 links, as the
    benchmark; inner precision f32 (mixed, the benchmark's), f64 or f16n) with
    the library's profiling mode on (every chunk kernel launched on its own,
    bracketed by events), then one 256 MiB streaming copy of known size: the
    program that hardware-counter runs profile (the copy calibrates the byte
    counters).  Prints the per-kernel statistics as JSON."""
    import torch

    import paper_2111_14958_amd as wd
    import wdgen
    cfg = wdgen.CONFIGS["lat14x4_16rhs"]
    dims = cfg["dims"]
    U = wdgen.gauge_field(dims, cfg["eps"], cfg["gauge_seed"])
    src = wdgen.mixed_sources(dims, cfg["n_point"], cfg["n_gauss"], cfg["src_seed"])
    g = wd.Gauge(torch.from_numpy(U).cuda(), dims, recon12=True)   # as the benchmark
    dsrc = torch.from_numpy(src).cuda()
    inner = {"f64": wd.F64, "f32": wd.F32, "f16n": wd.F16N}[inner_name]
    p = wd.cg_default_params(tol=cfg["tol"], inner=inner, reliable_every=0 if inner == wd.F64 else 50)
    sol = torch.zeros_like(dsrc)
    ws = torch.empty(wd.cg_workspace_bytes(g, dsrc.shape[0], p), dtype=torch.uint8, device="cuda")
    wd.profile_reset()
    wd.profile_enable(True)
    _, reps, rc = wd.cg_solve_batch(g, cfg["m0"], dsrc, sol=sol, params=p, ws=ws)
    torch.cuda.synchronize()
    wd.profile_enable(False)
    prof = wd.profile_read()
    a = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    wd.stream(wd.STREAM_COPY, a, b, a.numel())
    torch.cuda.synchronize()
    print(json.dumps({"solve": "14^4 x 16, inner " + inner_name, "rc": rc, "iters": max(r["iters"] for r in reps),
                      "kernels": prof, "copy_bytes_each_way": a.numel()}), flush=True)


def dslash(prec_name="f32", mode="hot", reps=20):
    """The stand-alone operator on the 14^4 x 16 benchmark fields (reconstruct-12
    gauge, as the benchmark; default launch shapes): `reps` applications back to
    back (mode hot: fields and links stay in the 256 MB MALL) or each after a
    1 GiB buffer is written (mode cold), then one 256 MiB streaming copy of
    known size that calibrates the byte counters: the program that the
    operator's hardware-counter runs profile.  Prints the timing as JSON."""
    import torch

    import paper_2111_14958_amd as wd
    import wdgen
    prec = {"f64": wd.F64, "f32": wd.F32, "f16n": wd.F16N}[prec_name]
    reps = int(reps)
    cfg = wdgen.CONFIGS["lat14x4_16rhs"]
    dims, nrhs = cfg["dims"], cfg["n_point"] + cfg["n_gauss"]
    U = wdgen.gauge_field(dims, cfg["eps"], cfg["gauge_seed"])
    src = wdgen.mixed_sources(dims, cfg["n_point"], cfg["n_gauss"], cfg["src_seed"])
    g = wd.Gauge(torch.from_numpy(U).cuda(), dims, recon12=True)
    pin = wd.pack_spinor(g, torch.from_numpy(src).cuda(), prec)
    pout = wd.empty_packed(g, prec, nrhs)
    flush = torch.empty(1 << 30, dtype=torch.uint8, device="cuda") if mode == "cold" else None
    times = []
    for _ in range(reps):
        if flush is not None:
            flush.fill_(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        wd.dslash(g, cfg["m0"], pin, prec, packed=True, nrhs=nrhs, out=pout)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) * 1e3)
    a = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    wd.stream(wd.STREAM_COPY, a, b, a.numel())
    torch.cuda.synchronize()
    print(json.dumps({"dslash": "14^4 x 16", "prec": prec_name, "mode": mode, "reps": reps,
                      "shape": wd.shape_get(g, prec, nrhs, False, wd.FAMILY_DSLASH),
                      "median_us": sorted(times)[len(times) // 2], "copy_bytes_each_way": a.numel()}),
          flush=True)


if __name__ == "__main__":
    if sys.argv[1] == "serve" and sys.argv[2:] == ["eo"]:
        serve(eo=True)
    elif sys.argv[1] == "dslash":
        dslash(*sys.argv[2:])
    elif sys.argv[1] == "solve":
        solve(*sys.argv[2:])
    else:
        {"fig1": fig1, "fig2": fig2, "serve": serve, "solve": solve}[sys.argv[1]]()
