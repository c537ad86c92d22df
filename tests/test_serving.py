"""Serving loop (many systems resident in one arena) through the C-ABI."""
import ctypes as C

import numpy as np
import pytest

from paper_2005_08348_amd import systems as S


def _lib():
    from paper_2005_08348_amd import membx
    return membx


def test_submit_validation_host_only():
    """Submission only prepares host data: a request that can never fit the
    arena is refused with E_NOMEM, a malformed request with E_INVAL; no device
    call is made before a job is admitted."""
    M = _lib()
    L = M.lib()
    srv = C.c_void_p()
    fake = C.c_void_p(1 << 40)          # never dereferenced: nothing is admitted here
    assert L.membx_server_create(fake, 1 << 20, C.byref(srv)) == 0
    s = S.make("c0")
    b = M._DescBuilder(s, M.MIXED, *M._tuning({}))
    jid = C.c_int64()
    ok = M.Request(0, 1, 10, 0, 0, 0, 0)
    assert L.membx_server_submit(srv, C.byref(b.desc), C.byref(ok), C.byref(jid)) == 2  # E_NOMEM
    bad = M.Request(0, 0, 10, 0, 0, 0, 0)
    assert L.membx_server_submit(srv, C.byref(b.desc), C.byref(bad), C.byref(jid)) == 1
    bad2 = M.Request(0, 1, 0, 0, 0, 0, 0)
    assert L.membx_server_submit(srv, C.byref(b.desc), C.byref(bad2), C.byref(jid)) == 1
    assert L.membx_server_destroy(srv) == 0
    # a large enough arena takes the job (queued, not admitted)
    srv2 = C.c_void_p()
    assert L.membx_server_create(fake, 64 << 20, C.byref(srv2)) == 0
    assert L.membx_server_submit(srv2, C.byref(b.desc), C.byref(ok), C.byref(jid)) == 0
    assert jid.value == 1
    assert L.membx_server_destroy(srv2) == 0


@pytest.mark.gpu
def test_jobs_alone_equal_jobs_in_a_mix():
    """Each job's final state and counters are bit-identical whether it runs
    alone (System API) or resident with others under a budget that forces
    queueing."""
    M = _lib()
    jobs = [S.serving_job(j, n, 200508348100 + j) for j, n in enumerate((1500, 3000, 2200, 4000))]
    req = dict(minimize_iters=100, md_cycles=2, md_steps=20, mdas_cycles=2, mdas_pairs=4,
               mdas_k=5, mdas_m=1)
    alone, pair_int = [], []
    for s in jobs:
        g = M.System(s, precision="mixed")
        g.minimize(req["minimize_iters"], 1e-4, 0.01)
        pi = 0
        for _ in range(req["md_cycles"]):
            g.md_step(req["md_steps"])
            pi += g.energies()["n_pairs_in_cutoff"] * req["md_steps"]
        for _ in range(req["mdas_cycles"]):
            g.mdas_cycle(req["mdas_pairs"], req["mdas_k"], req["mdas_m"], results=False)
            pi += g.energies()["n_pairs_in_cutoff"] * req["mdas_k"] * req["mdas_m"]
        e = g.energies()
        alone.append((e["potential"], e["step"], e["n_pairs_in_cutoff"]))
        pair_int.append(pi)
        g.close()
    sizes = [M.arena_bytes(s, precision="mixed") for s in jobs]
    budget = int(max(sizes) * 1.6) + 4096        # at most two of these fit at once
    srv = M.Server(budget)
    # every other job counts its pair interactions per cycle (an extra
    # energy pass that must leave the trajectory untouched)
    ids = [srv.submit(s, count_pairs=(q % 2 == 0), **req) for q, s in enumerate(jobs)]
    done, max_wait = {}, 0
    for _ in range(200000):
        res, nres, nwait = srv.poll()
        max_wait = max(max_wait, nwait)
        for r in res:
            done[r["job_id"]] = r
        if len(done) == len(jobs):
            break
    assert len(done) == len(jobs)
    assert max_wait >= 1, "the budget should have forced queueing"
    for q, (jid, s, (pot, steps, pairs)) in enumerate(zip(ids, jobs, alone)):
        r = done[jid]
        assert r["pair_interactions"] == (pair_int[q] if q % 2 == 0 else -1)
        assert r["status"] == 0
        assert r["n_cycles"] == req["md_cycles"] + req["mdas_cycles"]
        assert r["potential"] == pot
        assert r["md_steps"] == steps
        assert r["pairs_in_cutoff"] == pairs
        assert r["cycle_ms_p50"] > 0
    assert len(srv.cycle_times()) == len(jobs) * 4
    cp = srv.cycle_pairs()
    assert len(cp) == len(jobs) * 4
    assert cp[cp >= 0].sum() == sum(pair_int[q] for q in range(0, len(jobs), 2))
    srv.close()
