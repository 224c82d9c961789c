#!/usr/bin/env python3
"""Benchmark: multi-right-hand-side mixed-precision CG for the Wilson-Dirac
operator on one MI355X (arXiv 2111.14958, the CG of Sec. 2 on Eq. (1)).

Workload (one step = one full batched solve, every step of the hot path):
  14^4 lattice, antiperiodic time boundary, m0 = 0.05, links exp(i 0.5 H),
  16 right-hand sides (12 spin-colour point sources at the origin, 4 complex
  Gaussian sources), FP32 inner CG with FP64 reliable updates every 50
  iterations, stop at true relative residual 1e-10 (FP64).  Inputs (links,
  sources) are resident in HBM before the timed region; the links are packed
  once (gauge setup), sources are packed inside every solve.

Prints ONE JSON line: value = right-hand-side solves per second.  Beside it:
the plain FP64 CG on the same GPU (the "mixed vs FP64" ratio), the roofline of
the dominant kernel measured with HIP events (the library's profiling mode),
the stand-alone operator bandwidth and HBM traffic, the streaming-kernel ceilings,
the persistent kernel at the same shape and the CPU oracle.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dslash GB/s (% HBM peak); CG solves/s at res 1e-10, mixed vs FP64"
HBM_PEAK_GBPS = 8000.0
# hardware-counter summary of the dominant kernel (FETCH_SIZE / WRITE_SIZE runs)
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_phaseB_f32_14x4_16rhs_pmc.md")
# sources that define the phase-B kernel; the counter figures hold only for them
KERNEL_SOURCES = ("wd_device.h", "cg_core.h", "cg.hip")
# the stand-alone operator's counter summary and the sources of its kernels
PMC_DSLASH = os.path.join(ROOT, "profiles", "k_dslash_xy_14x4_16rhs_pmc.md")
DSLASH_SOURCES = ("wd_device.h", "dslash.hip")


def kernel_sources_sha256(sources=KERNEL_SOURCES):
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2111_14958_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pmc_traffic(path=PMC_SUMMARY, sources=KERNEL_SOURCES, key="traffic_bytes_per_launch"):
    """HBM-side bytes per launch from a committed counter summary, or None when
    it is missing or was taken on other kernel sources."""
    try:
        text = open(path).read()
    except OSError:
        return None, "no counter summary"
    sha = re.search(r"kernel_sources_sha256: ([0-9a-f]+)", text)
    val = re.search(re.escape(key) + r": ([0-9.eE+]+)", text)
    if not sha or not val:
        return None, "counter summary unreadable"
    if sha.group(1) != kernel_sources_sha256(sources):
        return None, "kernel changed since the counters were taken"
    return float(val.group(1)), "FETCH_SIZE x2 + WRITE_SIZE (copy-calibrated), per launch"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-big", action="store_true", help="skip the 16^3x32 FP16N context run")
    ap.add_argument("--cpu-iters", type=int, default=150,
                    help="oracle CG iterations timed for the CPU baseline sample")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(independent solves would shard by request)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2111_14958_amd as wd
    import wdgen

    if not os.path.exists(wd.LIB_PATH):
        from paper_2111_14958_amd import build
        build.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    arch, ncu = wd.device_info(0)

    cfg = wdgen.CONFIGS["lat14x4_16rhs"]
    dims, m0, tol = cfg["dims"], cfg["m0"], cfg["tol"]
    nrhs = cfg["n_point"] + cfg["n_gauss"]
    V = wdgen.volume(dims)
    log("generating inputs", dims, nrhs)
    U = wdgen.gauge_field(dims, cfg["eps"], cfg["gauge_seed"])
    src = wdgen.mixed_sources(dims, cfg["n_point"], cfg["n_gauss"], cfg["src_seed"])
    dU = torch.from_numpy(U).to(dev)
    dsrc = torch.from_numpy(src).to(dev)
    # links: the complete copies plus a two-row (reconstruct-12) FP32 copy, which
    # the FP32 operator and the stencils of every FP32-inner solver read
    g = wd.Gauge(dU, dims, -1, recon12=True)
    sol = torch.zeros_like(dsrc)

    p_mixed = wd.cg_default_params(tol=tol, inner=wd.F32, reliable_every=50)
    p_fp64 = wd.cg_default_params(tol=tol, inner=wd.F64, reliable_every=0)
    p_bicg = wd.cg_default_params(tol=tol, inner=wd.F32, reliable_every=50, method=wd.METHOD_BICGSTAB)
    p_bicg64 = wd.cg_default_params(tol=tol, inner=wd.F64, reliable_every=0, method=wd.METHOD_BICGSTAB)
    p_eo = wd.cg_default_params(tol=tol, inner=wd.F32, reliable_every=50, precondition=wd.PRECOND_EO)
    p_eo64 = wd.cg_default_params(tol=tol, inner=wd.F64, reliable_every=0, precondition=wd.PRECOND_EO)
    ws = torch.empty(max(wd.cg_workspace_bytes(g, nrhs, p)
                         for p in (p_mixed, p_fp64, p_bicg, p_bicg64, p_eo, p_eo64)),
                     dtype=torch.uint8, device=dev)

    def solve(params):
        x, reps, rc = wd.cg_solve_batch(g, m0, dsrc, sol=sol, params=params, ws=ws)
        return reps, rc

    # ------------------------------------------------------------- timed: mixed
    log("warmup", args.warmup)
    for _ in range(args.warmup):
        solve(p_mixed)
    torch.cuda.synchronize()
    log("timed", args.steps, "steps")
    t0 = time.perf_counter()
    all_reps = []
    for _ in range(args.steps):
        reps, rc = solve(p_mixed)
        all_reps.append((reps, rc))
    torch.cuda.synchronize()
    t_mixed = time.perf_counter() - t0
    ok = all(rc == wd.WD_OK and all(r["status"] == 0 and r["true_rel_res"] <= tol for r in reps)
             for reps, rc in all_reps)
    reps_mixed = all_reps[-1][0]
    x_mixed = sol.clone()
    value = nrhs * args.steps / t_mixed
    log(f"mixed: {value:.2f} solves/s, iters {[r['iters'] for r in reps_mixed]}")

    # ------------------------------------------------------------- FP64 beside
    solve(p_fp64)  # warm the graph
    torch.cuda.synchronize()
    n64 = max(1, min(args.steps, 2))
    t0 = time.perf_counter()
    for _ in range(n64):
        reps64, rc64 = solve(p_fp64)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    fp64_value = nrhs * n64 / t64
    x64 = sol.clone()
    diff = (x_mixed - x64).reshape(nrhs, -1)
    err_vs_fp64 = (diff.norm(dim=1) / x64.reshape(nrhs, -1).norm(dim=1)).max().item()
    log(f"fp64: {fp64_value:.2f} solves/s, iters {[r['iters'] for r in reps64]}")

    # ------------------------------------------- FP16-storage inner (context)
    p16 = wd.cg_default_params(tol=tol, inner=wd.F16N, reliable_every=50)
    solve(p16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps16, rc16 = solve(p16)
    torch.cuda.synchronize()
    f16_value = nrhs / (time.perf_counter() - t0)
    err16 = ((sol - x64).reshape(nrhs, -1).norm(dim=1) / x64.reshape(nrhs, -1).norm(dim=1)).max().item()

    # ------------- BiCGSTAB on D (Sec. 1 alternative) and even-odd CG, context
    bicg, eocg = {}, {}
    for name, pb, dst in (("f32", p_bicg, bicg), ("f64", p_bicg64, bicg), ("f32", p_eo, eocg),
                          ("f64", p_eo64, eocg)):
        solve(pb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        repsb, rcb = solve(pb)
        torch.cuda.synchronize()
        dst[name] = {"solves_per_s": nrhs / (time.perf_counter() - t0), "converged": rcb == wd.WD_OK,
                      "iters": [r["iters"] for r in repsb],
                      "err_vs_fp64_cg_solution": ((sol - x64).reshape(nrhs, -1).norm(dim=1) /
                                                  x64.reshape(nrhs, -1).norm(dim=1)).max().item()}

    # ------------------------------------ roofline of the dominant CG kernel
    wd.profile_reset()
    wd.profile_enable(True)
    solve(p_mixed)
    torch.cuda.synchronize()
    wd.profile_enable(False)
    prof = wd.profile_read()
    dom_name = max(prof, key=lambda k: prof[k]["total_ms"])
    dom = prof[dom_name]
    dom_gbps = dom["bytes_total"] / (dom["total_ms"] * 1e-3) / 1e9
    fam = {"cg_phaseA": wd.FAMILY_CG_A, "cg_phaseB": wd.FAMILY_CG_B}.get(dom_name)
    if fam is not None:
        sh = wd.shape_get(g, wd.F32, nrhs, fam == wd.FAMILY_CG_A, fam)
        xy = sh["xy_lds"] and dims[0] * dims[1] <= 256
        nr = min(sh["rhs_per_thread"], 2) if xy else sh["rhs_per_thread"]
        mp = bool(xy) and nr == 1 and sh["hop_order"] == 5 and sh.get("xy_planes", 1) > 1
        kernel_symbol = "wd::k_%s<1, %d, %d, %s, true, false, %s>" % (
            dom_name[3:], nr, sh["hop_order"] if sh["hop_order"] in (3, 5) else 1, "true" if xy else "false",
            "true" if mp else "false")
    else:
        kernel_symbol = dom_name
    traffic, traffic_note = pmc_traffic() if dom_name == "cg_phaseB" else (None, "not measured")
    per_launch = {k: {"launches": v["launches"],
                      "avg_us": 1e3 * v["total_ms"] / max(v["launches"], 1),
                      "GBps": v["bytes_total"] / max(v["total_ms"], 1e-12) / 1e6}
                  for k, v in prof.items() if v["launches"] > 0}

    # -------- the same solve with the complete 18-real links (context)
    gfull = wd.Gauge(dU, dims, -1)
    xf, rfs, rcf = wd.cg_solve_batch(gfull, m0, dsrc, sol=sol, params=p_mixed, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xf, rfs, rcf = wd.cg_solve_batch(gfull, m0, dsrc, sol=sol, params=p_mixed, ws=ws)
    torch.cuda.synchronize()
    full_value = nrhs / (time.perf_counter() - t0)
    wd.profile_reset()
    wd.profile_enable(True)
    wd.cg_solve_batch(gfull, m0, dsrc, sol=sol, params=p_mixed, ws=ws)
    torch.cuda.synchronize()
    wd.profile_enable(False)
    proff = wd.profile_read()
    complete_links = {"solves_per_s": full_value, "converged": rcf == wd.WD_OK,
                      "max_true_rel_res": max(r["true_rel_res"] for r in rfs),
                      "err_vs_fp64_cg_solution": ((sol - x64).reshape(nrhs, -1).norm(dim=1) /
                                                  x64.reshape(nrhs, -1).norm(dim=1)).max().item(),
                      "kernels_avg_us": {k: 1e3 * v["total_ms"] / max(v["launches"], 1) for k, v in proff.items()
                                         if v["launches"] > 0}}
    del gfull
    log(f"complete links: {full_value:.2f} solves/s")

    # ---- the same batch in one persistent launch per chunk (grid barriers)
    p_pers = wd.cg_default_params(tol=tol, inner=wd.F32, reliable_every=50, persistent=1)
    solve(p_pers)   # graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    repsp, rcp = solve(p_pers)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    it_p = max(r["iters"] for r in repsp)
    per_it_graph = sum(1e3 * prof[k]["total_ms"] / max(prof[k]["launches"], 1)
                       for k in ("cg_phaseA", "cg_phaseB") if k in prof)
    persistent = {"solves_per_s": nrhs / tp, "converged": rcp == wd.WD_OK, "iters_max": it_p,
                  "us_per_iteration": 1e6 * tp / it_p,
                  "graph_path_phase_A_plus_B_us": per_it_graph,
                  # one 1024-thread block per compute unit, site blocks, the
                  # reconstruct-12 links as the graph path; against the graph
                  # path's plane-blocked phases, per grid barrier (two per
                  # iteration): an upper bound of the barrier's cost
                  "overhead_us_per_barrier": (1e6 * tp / it_p - per_it_graph) / 2,
                  "max_true_rel_res": max(r["true_rel_res"] for r in repsp)}
    log(f"persistent: {nrhs / tp:.2f} solves/s")

    # ------------------------------------------ stand-alone operator, 16 rhs
    dslash = {}
    for prec, name in ((wd.F32, "f32"), (wd.F64, "f64"), (wd.F16N, "f16n")):
        pin = wd.pack_spinor(g, dsrc, prec)
        pout = wd.empty_packed(g, prec, nrhs)
        for _ in range(3):
            wd.dslash(g, m0, pin, prec, packed=True, nrhs=nrhs, out=pout)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps_n = 50
        e0.record()
        for _ in range(reps_n):
            wd.dslash(g, m0, pin, prec, packed=True, nrhs=nrhs, out=pout)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps_n
        # the gauge holds the reconstruct-12 copy: the FP32 operator reads two rows per link
        link = {wd.F64: 576, wd.F32: 192, wd.F16N: 144}[prec]
        spin = {wd.F64: 192, wd.F32: 96, wd.F16N: 52}[prec]
        alg = V * (link + 2 * nrhs * spin)
        # cold: a 1 GiB buffer is written between applications, so the fields and
        # links come from HBM instead of the 256 MB MALL; each application is
        # bracketed by its own events
        flush = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        cold = []
        for _ in range(20):
            flush.fill_(1)
            c0 = torch.cuda.Event(enable_timing=True)
            c1 = torch.cuda.Event(enable_timing=True)
            c0.record()
            wd.dslash(g, m0, pin, prec, packed=True, nrhs=nrhs, out=pout)
            c1.record()
            torch.cuda.synchronize()
            cold.append(c0.elapsed_time(c1) * 1e3)
        cold_us = sorted(cold)[len(cold) // 2]
        del flush
        dslash[name] = {"us": us, "GBps": alg / (us * 1e-6) / 1e9, "link_bytes_per_site": link,
                        "alg_bytes_per_launch": alg,
                        "GFLOPs": 1368.0 * V * nrhs / (us * 1e-6) / 1e9,
                        "frac_hbm": alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBPS,
                        "cold_us_median": cold_us, "cold_GBps": alg / (cold_us * 1e-6) / 1e9,
                        "cold_frac_hbm": alg / (cold_us * 1e-6) / 1e9 / HBM_PEAK_GBPS}
        for mode in ("hot", "cold"):
            tb, note = pmc_traffic(PMC_DSLASH, DSLASH_SOURCES, f"traffic_{name}_{mode}")
            dslash[name][f"traffic_{mode}_bytes_per_launch"] = tb
            dslash[name][f"traffic_{mode}_over_algorithmic"] = tb / alg if tb else None
        dslash[name]["traffic_note"] = note
        del pin, pout

    # ------------------------- the paper's coordinate-format operator (Sec. 2)
    coo = {}
    x1 = dsrc[cfg["n_point"]:cfg["n_point"] + 1].reshape(1, -1).contiguous()
    for prec, name in ((wd.F64, "f64"), (wd.F32, "f32")):
        c = wd.Coo(g, m0, prec)
        xin = x1 if prec == wd.F64 else x1.to(torch.complex64)
        yout = torch.empty_like(xin)
        for _ in range(3):
            c.spmv(xin, out=yout)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            c.spmv(xin, out=yout)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / 20
        vb = 16 if prec == wd.F64 else 8
        alg = c.nnz * (vb + 4) + 2 * c.rows * vb     # Val, Col, in, out
        coo[name] = {"us": us, "GBps": alg / (us * 1e-6) / 1e9,
                     "GFLOPs_useful": 1368.0 * V / (us * 1e-6) / 1e9,
                     "GFLOPs_executed": 8.0 * c.nnz / (us * 1e-6) / 1e9,
                     "bytes_per_site": alg / V, "nnz": c.nnz}
        c.close()

    # ------------------------------------ memory ceiling: the streaming kernels
    # wd_stream read / copy / write with 16-byte coalesced accesses; 128 MiB stays
    # in the 256 MB MALL when repeated (the operator's 125 MB working set does
    # too), 4 GiB streams from HBM
    stream = {}
    buf_a = torch.empty(4 << 30, dtype=torch.uint8, device=dev)
    buf_b = torch.empty(4 << 30, dtype=torch.uint8, device=dev)
    for label, nbytes, n_rep in (("128MiB_repeated", 128 << 20, 20), ("4GiB", 4 << 30, 5)):
        row = {}
        for kind, kname, fac in ((wd.STREAM_READ, "read", 1), (wd.STREAM_COPY, "copy", 2),
                                 (wd.STREAM_WRITE, "write", 1)):
            for _ in range(2):
                wd.stream(kind, buf_a, buf_b, nbytes)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(n_rep):
                wd.stream(kind, buf_a, buf_b, nbytes)
            e1.record()
            torch.cuda.synchronize()
            row[kname + "_GBps"] = fac * nbytes * n_rep / (e0.elapsed_time(e1) * 1e-3) / 1e9
        stream[label] = row
    del buf_a, buf_b
    copy_gbps = stream["4GiB"]["copy_GBps"]

    # ------ 8^4, 12^4, 14^4 single field: operator alone and CG, FP64 and FP32 (context)
    single = {}
    for key in ("lat8x4_1rhs", "lat12x4_1rhs", "lat14x4_1rhs"):
        sfcfg = wdgen.CONFIGS[key]
        d2 = sfcfg["dims"]
        V2 = wdgen.volume(d2)
        U2 = torch.from_numpy(wdgen.gauge_field(d2, sfcfg["eps"], sfcfg["gauge_seed"])).to(dev)
        s2 = torch.from_numpy(wdgen.gaussian_source(d2, 1, sfcfg["src_seed"])).to(dev)
        g2 = wd.Gauge(U2, d2, -1, recon12=True)
        row = {}
        for prec, name in ((wd.F64, "f64"), (wd.F32, "f32")):
            pin = wd.pack_spinor(g2, s2, prec)
            pout = wd.empty_packed(g2, prec, 1)
            for _ in range(3):
                wd.dslash(g2, sfcfg["m0"], pin, prec, packed=True, nrhs=1, out=pout)
            torch.cuda.synchronize()
            # 100 applications captured in one graph and replayed: the time per
            # application is the kernel's (plus the graph's gap between kernels),
            # not the host's call rate
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                for _ in range(100):
                    wd.dslash(g2, sfcfg["m0"], pin, prec, packed=True, nrhs=1, out=pout)
            graph.replay()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                graph.replay()
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / 500
            del graph
            alg = V2 * ({wd.F64: 576, wd.F32: 192}[prec] + 2 * {wd.F64: 192, wd.F32: 96}[prec])
            pc = wd.cg_default_params(tol=sfcfg["tol"], inner=prec, reliable_every=0 if prec == wd.F64 else 50)
            sol2 = torch.zeros_like(s2)
            ws2 = torch.empty(wd.cg_workspace_bytes(g2, 1, pc), dtype=torch.uint8, device=dev)
            wd.cg_solve_batch(g2, sfcfg["m0"], s2, sol=sol2, params=pc, ws=ws2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                _, rep2, rc2 = wd.cg_solve_batch(g2, sfcfg["m0"], s2, sol=sol2, params=pc, ws=ws2)
            torch.cuda.synchronize()
            row[name] = {"dslash_us": us, "dslash_GBps": alg / (us * 1e-6) / 1e9,
                         "cg_solves_per_s": 3 / (time.perf_counter() - t0), "cg_iters": rep2[0]["iters"],
                         "true_rel_res": rep2[0]["true_rel_res"], "converged": rc2 == wd.WD_OK}
            del pin, pout
        single["x".join(str(d) for d in d2)] = row
        del g2
    log("single-field context", json.dumps(single))

    # ------------------- 16^3 x 32, m0 0.02, 12 point sources: FP16N vs FP64 (context)
    big = None
    if not args.no_big:
        bigcfg = wdgen.CONFIGS["lat16x3x32_12rhs"]
        log("big 16^3x32 inputs")
        Ub = torch.from_numpy(wdgen.gauge_field(bigcfg["dims"], bigcfg["eps"], bigcfg["gauge_seed"])).to(dev)
        gb = wd.Gauge(Ub, bigcfg["dims"], -1, recon12=True)
        srcb = torch.from_numpy(wdgen.point_sources(bigcfg["dims"])).to(dev)
        solb = torch.zeros_like(srcb)
        big = {"workload": "16^3x32, m0 0.02, eps 0.5, 12 point sources, tol 1e-10"}
        xsb = {}
        for name, pc in (("f16n", wd.cg_default_params(tol=tol, inner=wd.F16N, reliable_every=50)),
                         ("f32", wd.cg_default_params(tol=tol, inner=wd.F32, reliable_every=50)),
                         ("f64", wd.cg_default_params(tol=tol, inner=wd.F64, reliable_every=0))):
            wsb = torch.empty(wd.cg_workspace_bytes(gb, 12, pc), dtype=torch.uint8, device=dev)
            wd.cg_solve_batch(gb, bigcfg["m0"], srcb, sol=solb, params=pc, ws=wsb)   # graph capture
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, repsb, rcb = wd.cg_solve_batch(gb, bigcfg["m0"], srcb, sol=solb, params=pc, ws=wsb)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            xsb[name] = solb.clone()
            big[name] = {"solves_per_s": 12 / dt, "converged": rcb == wd.WD_OK,
                        "max_true_rel_res": max(r["true_rel_res"] for r in repsb),
                        "iters_max": max(r["iters"] for r in repsb)}
            del wsb
        for name in ("f16n", "f32"):
            db = (xsb[name] - xsb["f64"]).reshape(12, -1).norm(dim=1) / xsb["f64"].reshape(12, -1).norm(dim=1)
            big[name]["err_vs_fp64_solution"] = db.max().item()
        big["f16n_vs_f64_speedup"] = big["f16n"]["solves_per_s"] / big["f64"]["solves_per_s"]
        del Ub, gb, srcb, solb, xsb

    # ----------------------------------------------------- CPU oracle baseline
    cpu = None
    if not args.no_cpu:
        import oracle
        i_g = cfg["n_point"]   # first Gaussian source
        iters_needed = reps64[i_g]["iters"]
        n_it = min(args.cpu_iters, iters_needed)
        threads_all = oracle.set_threads(0)   # OMP_NUM_THREADS, else every host core
        runs = {}
        for nt in sorted({1, threads_all}):
            oracle.set_threads(nt)
            log(f"cpu oracle: {n_it} CG iterations on one 14^4 field, {nt} thread(s)")
            t0 = time.perf_counter()
            oracle.cg(U, src[i_g:i_g + 1], dims, m0, tol=1e-300, max_iter=n_it)
            t_cpu = time.perf_counter() - t0
            runs[nt] = {"solves_per_s": 1.0 / (t_cpu / n_it * iters_needed), "seconds": t_cpu}
        oracle.set_threads(threads_all)
        model = "unknown"
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        cpu = {"value": runs[threads_all]["solves_per_s"], "unit": "solves/s", "cores": threads_all,
               "kind": "oracle",
               "sample": f"FP64 C oracle CG on 1 Gaussian field of this 14^4 workload: {n_it} iterations "
                         f"timed ({runs[threads_all]['seconds']:.1f} s on {threads_all} threads; the "
                         f"operator's site loop is OpenMP-parallel, dot products sequential), scaled to "
                         f"the {iters_needed} iterations the FP64 solve needs",
               "seconds": runs[threads_all]["seconds"],
               "one_thread_solves_per_s": runs[1]["solves_per_s"], "one_thread_seconds": runs[1]["seconds"],
               "cpu_model": model, "host_cpus_visible": os.cpu_count()}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_mixed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "wilson-dirac cg 14^4 x 16 rhs (12 point + 4 gaussian), m0 0.05, "
                               "eps 0.5, tol 1e-10, fp32 inner + fp64 reliable updates every 50, "
                               "reconstruct-12 fp32 links in the inner operator",
                   "lattice": list(dims), "nrhs": nrhs, "global_batch": nrhs,
                   "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "kernel": kernel_symbol, "achieved": dom_gbps,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": dom_gbps / HBM_PEAK_GBPS,
                     "traffic": traffic},
        "cpu_baseline": cpu,
        "details": {
            "device": f"{arch} ({ncu} CUs)",
            "all_solves_converged": ok,
            "max_true_rel_res": max(r["true_rel_res"] for r in reps_mixed),
            "iters_mixed": [r["iters"] for r in reps_mixed],
            "reliable_updates": [r["reliable_updates"] for r in reps_mixed],
            "fp64_solves_per_s": fp64_value,
            "mixed_vs_fp64": value / fp64_value,
            "iters_fp64": [r["iters"] for r in reps64],
            "mixed_err_vs_fp64_solution": err_vs_fp64,
            "f16n_solves_per_s": f16_value,
            "f16n_all_converged": rc16 == wd.WD_OK,
            "f16n_err_vs_fp64_solution": err16,
            "cg_kernels": per_launch,
            "dominant_kernel_alg_bytes_per_launch": dom["bytes_total"] / max(dom["launches"], 1),
            "traffic_note": traffic_note,
            "bicgstab_16rhs": bicg,
            "even_odd_cg_16rhs": eocg,
            "complete_links_cg_16rhs": complete_links,
            "dslash_16rhs": dslash,
            "coo_spmv_1rhs": coo,
            "copy_GBps": copy_gbps,
            "stream": stream,
            "persistent_cg_16rhs": persistent,
            "single_field": single,
            "lat16x3x32_12rhs": big,
        },
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
