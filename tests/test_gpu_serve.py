"""Serving: continuous batching of solves of different lattices on one GPU.

Checks that every result is accepted by the oracle (true residual <= 1e-10),
that each result is bit-for-bit the same alone and in a mix (the per-field
arithmetic of a grouped launch does not depend on the other requests), that
admission never exceeds the arena, and the error paths."""
import time

import numpy as np
import pytest

import oracle
import paper_2111_14958_amd as wd
import wdgen
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _requests():
    rng = np.random.default_rng(10_000)
    vols = [(4, 4, 4, 4), (6, 6, 6, 6), (4, 4, 6, 8), (8, 8, 8, 8), (6, 4, 4, 6)]
    out = []
    for i in range(7):
        dims = vols[i % len(vols)]
        nrhs = int(rng.integers(1, 4))
        m0 = float(rng.uniform(0.05, 0.2))
        U = wdgen.gauge_field(dims, 0.5, 10_000 + i)
        src = wdgen.gaussian_source(dims, nrhs, 60_000 + i)
        inner = wd.F64 if i % 3 == 2 else wd.F32
        eo = i % 2   # every other request even-odd preconditioned
        out.append(dict(dims=dims, nrhs=nrhs, m0=m0, U=U, src=src, inner=inner, eo=eo))
    return out


def _big_requests():
    """The serving workload's largest volumes beside small ones: 14^4 and
    16^3 x 32 with 12 right-hand sides at m0 0.02 (the hardest conditioning the
    stream draws), one of them even-odd preconditioned, and three smaller
    requests, the 12^4 one in FP64.  The 14^4 and 12^4 requests run their
    phases on plane blocks, the others on site blocks."""
    out = []
    specs = [((14, 14, 14, 14), 12, 0.02, 0), ((16, 16, 16, 32), 12, 0.02, 1),
             ((4, 4, 4, 4), 3, 0.2, 0), ((8, 8, 8, 8), 5, 0.07, 1), ((12, 12, 12, 12), 2, 0.11, 0)]
    for i, (dims, nrhs, m0, eo) in enumerate(specs):
        U = wdgen.gauge_field(dims, 0.5, 11_000 + i)
        src = wdgen.gaussian_source(dims, nrhs, 61_000 + i)
        inner = wd.F64 if i == 4 else wd.F32
        out.append(dict(dims=dims, nrhs=nrhs, m0=m0, U=U, src=src, inner=inner, eo=eo))
    return out


def _run(reqs, arena_bytes, max_slots=8, chunk=10):
    import torch
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    srv = wd.Server(arena, max_slots=max_slots, chunk=chunk)
    tickets, keep = [], []
    for r in reqs:
        dU, dsrc = dev(r["U"]), dev(r["src"])
        sol = torch.zeros_like(dsrc)
        p = wd.cg_default_params(inner=r["inner"], reliable_every=0 if r["inner"] == wd.F64 else 50,
                                 precondition=wd.PRECOND_EO if r["eo"] else wd.PRECOND_NONE)
        req = wd.Server.request(r["dims"], r["nrhs"], r["m0"], dU, dsrc, sol, p)
        tickets.append(srv.submit(req, keep=(dU, dsrc, sol)))
        keep.append(sol)
    reps = [None] * len(reqs)
    t0 = time.time()
    while any(r is None for r in reps):
        for i, t in enumerate(tickets):
            if reps[i] is None:
                reps[i] = srv.poll(t)
        assert time.time() - t0 < 100, "server did not finish"
        time.sleep(0.002)
    st = srv.stats()
    srv.close()
    return [host(s) for s in keep], reps, st


def test_serve_mix_matches_oracle_and_alone():
    reqs = _requests()
    say("serve mix", len(reqs))
    xs, reps, st = _run(reqs, 256 << 20)
    assert st["completed"] == len(reqs) and st["submitted"] == len(reqs)
    for r, x, rep in zip(reqs, xs, reps):
        assert all(e["status"] == 0 for e in rep), rep
        res = oracle.true_residual(r["U"], r["src"], x, r["dims"], r["m0"])
        assert np.all(res <= TOL * 1.0000001), res
    # each request alone gives the identical bits
    for i in (0, 3, 5):
        say("serve alone", i)
        xa, repa, _ = _run([reqs[i]], 64 << 20)
        assert np.array_equal(xa[0], xs[i])
        assert [e["iters"] for e in repa[0]] == [e["iters"] for e in reps[i]]


def test_serve_mix_at_the_largest_volumes():
    """Grouped launches with many tiles per request (14^4 and 16^3 x 32 at 12
    right-hand sides) give oracle-accepted results that are bitwise the same
    alone and in the mix."""
    reqs = _big_requests()
    say("serve big mix", [r["dims"] for r in reqs])
    xs, reps, st = _run(reqs, 3 << 30, chunk=25)
    assert st["completed"] == len(reqs)
    for r, x, rep in zip(reqs, xs, reps):
        assert all(e["status"] == 0 for e in rep), (r["dims"], rep)
        res = oracle.true_residual(r["U"], r["src"], x, r["dims"], r["m0"])
        assert np.all(res <= TOL * 1.0000001), (r["dims"], res)
        for e, o in zip(rep, res):
            assert abs(e["true_rel_res"] - o) <= 1e-3 * TOL + 1e-6 * o
    for i in (0, 1, 4):
        say("serve big alone", reqs[i]["dims"])
        xa, repa, _ = _run([reqs[i]], 2 << 30, chunk=25)
        assert np.array_equal(xa[0], xs[i]), reqs[i]["dims"]
        assert [e["iters"] for e in repa[0]] == [e["iters"] for e in reps[i]]


def test_serve_largest_accepted_request_completes():
    """A request whose footprint equals the arena's capacity is accepted and
    completes; one slightly larger is refused at submission (it could never be
    admitted)."""
    import torch
    small = dict(dims=(4, 4, 4, 4), nrhs=1, m0=0.1)
    large = dict(dims=(4, 4, 4, 4), nrhs=2, m0=0.1)
    U = wdgen.gauge_field(small["dims"], 0.3, 12_001)
    dU = dev(U)
    p = wd.cg_default_params(inner=wd.F32)
    fps = []
    for r in (small, large):
        req = wd.Request()
        req.dims[:] = list(r["dims"])
        req.t_sign, req.nrhs, req.m0 = -1, r["nrhs"], r["m0"]
        req.gauge_dev = req.src_dev = 1
        req.sol_dev = 2
        req.params = p
        fps.append(wd.Server.footprint(req))
    # the bytes the server keeps for itself, from a probe server's capacity
    probe_arena = torch.empty(1 << 22, dtype=torch.uint8, device="cuda")
    probe = wd.Server(probe_arena, max_slots=4)
    own = probe_arena.numel() - probe.stats()["arena_capacity"]
    probe.close()
    assert own > 0
    for arena_bytes, accept in ((own + fps[0], (True, False)), (own + fps[1] - 256, (True, False)),
                                (own + fps[1], (True, True))):
        say("serve capacity", arena_bytes, accept)
        arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
        srv = wd.Server(arena, max_slots=4)
        assert srv.stats()["arena_capacity"] == arena_bytes - own
        for r, ok in zip((small, large), accept):
            src = wdgen.gaussian_source(r["dims"], r["nrhs"], 62_000 + r["nrhs"])
            dsrc = dev(src)
            sol = torch.zeros_like(dsrc)
            req = wd.Server.request(r["dims"], r["nrhs"], r["m0"], dU, dsrc, sol, p)
            if not ok:
                with pytest.raises(wd.WDError) as e:
                    srv.submit(req)
                assert e.value.code == wd.WD_ETOOBIG
                continue
            t = srv.submit(req, keep=(dsrc, sol))
            t0 = time.time()
            rep = None
            while rep is None:
                rep = srv.poll(t)
                assert time.time() - t0 < 60, "an accepted request was never completed"
                time.sleep(0.002)
            assert all(e["status"] == 0 for e in rep), rep
            res = oracle.true_residual(U, src, host(sol), r["dims"], r["m0"])
            assert np.all(res <= TOL * 1.0000001)
        srv.close()


def test_serve_admission_respects_arena():
    reqs = _requests()[:5]
    fps = []
    for r in reqs:
        p = wd.cg_default_params(inner=r["inner"], precondition=wd.PRECOND_EO if r["eo"] else wd.PRECOND_NONE)
        req = wd.Request()
        req.dims[:] = list(r["dims"])
        req.t_sign, req.nrhs, req.m0 = -1, r["nrhs"], r["m0"]
        req.gauge_dev = req.src_dev = 1
        req.sol_dev = 2
        req.params = p
        fps.append(wd.Server.footprint(req))
    assert all(f > 0 for f in fps)
    table = 6 * 8 * 1024   # request tables (6 groups x max_slots records), see wd_serve_create
    arena = table + max(fps) + min(fps) + 4096      # room for about two requests at once
    say("serve small arena", arena)
    xs, reps, st = _run(reqs, arena, max_slots=8)
    assert st["arena_high_water"] <= arena
    assert st["completed"] == len(reqs)
    for r, x, rep in zip(reqs, xs, reps):
        assert all(e["status"] == 0 for e in rep)
        assert np.all(oracle.true_residual(r["U"], r["src"], x, r["dims"], r["m0"]) <= TOL * 1.0000001)


def test_serve_errors():
    import torch
    arena = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    srv = wd.Server(arena, max_slots=2)
    dims = (16, 16, 16, 16)
    U = torch.zeros((16, 16, 16, 16, 4, 3, 3), dtype=torch.complex128, device="cuda")
    src = torch.zeros((1, 16, 16, 16, 16, 4, 3), dtype=torch.complex128, device="cuda")
    sol = torch.zeros_like(src)
    req = wd.Server.request(dims, 1, 0.1, U, src, sol)
    say("serve errors")
    with pytest.raises(wd.WDError) as e:
        srv.submit(req)
    assert e.value.code == wd.WD_ETOOBIG
    with pytest.raises(wd.WDError) as e:
        srv.poll(wd.Ticket(12345, 1))
    assert e.value.code == wd.WD_ENOTFOUND
    bad = wd.Server.request(dims, 1, 0.1, U, src, sol, wd.cg_default_params(inner=wd.F16N))
    with pytest.raises(wd.WDError) as e:
        srv.submit(bad)
    assert e.value.code == wd.WD_EINVAL
    srv.close()
