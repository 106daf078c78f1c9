"""Batched solves and the serving loop through the C ABI (bl_batch_solve, bl_server_*):
every problem's eigenvalues match the dense oracle, and a problem's results do not depend
on the other problems it shares launches with (alone == in batch == in a served mix; the
slots of an engine share kernels but not arithmetic, so the agreement is to the last bit)."""
import math
import time

import numpy as np
import pytest

import synth
from oracle import fem
from oracle.dense import dense_eigs

pytestmark = pytest.mark.gpu


def _problems():
    """Two shapes (16x16 and 32x32, p = 6 and p = 9), different eps, nev and paths; two
    of the 16x16 problems share p with different nev."""
    out = []
    specs = [
        (16, 4, 2, synth.eps_disc(16, 16, 1.0, 1.0, 8.9, 0.3), [(0.9, -0.4), (1.1, -0.3)], 11),
        (16, 5, 1, synth.eps_disc(16, 16, 1.0, 1.0, 4.0, 0.25), [(0.0, 0.0), (0.3, 0.0)], 12),
        (32, 6, 3, synth.eps_disc_lattice(32, 32, 1.0, 1.0, 12.0, 0.3), [(math.pi, 0.5)], 13),
        (16, 4, 2, np.ones(256), [(math.pi, math.pi), (2.8, 3.0), (2.6, 2.9)], 14),
        (32, 6, 3, synth.eps_random_field(32, 32, 1.0, 1.0, 5), [(0.4, 1.9), (0.6, 1.8)], 15),
    ]
    for n, nev, nthrow, eps, ks, seed in specs:
        out.append(dict(n=n, m=n, a=1.0, b=1.0, eps=eps, nev=nev, nthrow=nthrow,
                        ks=np.array(ks, dtype=float),
                        start=synth.start_block(2 * n * n, nev + nthrow, seed)))
    return out


OPTS = dict(tol=1e-9, max_iter=300, coarsest_min=4)
_DENSE = {}


def _dense(pr, t):
    key = (pr["eps"].tobytes(), pr["n"], tuple(pr["ks"][t]), pr["nev"])
    if key not in _DENSE:
        d = fem.Discretization(pr["n"], pr["m"], 1.0, 1.0, pr["eps"], *pr["ks"][t])
        _DENSE[key] = dense_eigs(d, pr["nev"])[0]
    return _DENSE[key]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_dense_and_alone(precision):
    from paper_2304_00337_amd import batch_solve
    probs = _problems()
    together = batch_solve(probs, precision=precision, **OPTS)
    tol = 1e-9 if precision == "fp64" else 1e-6
    for pr, r in zip(probs, together):
        assert r["status"] == 0, r
        for t in range(len(pr["ks"])):
            ref = _dense(pr, t)
            assert np.max(np.abs(r["evals"][t] - ref) / ref) < tol, (t, r["evals"][t], ref)
    # alone: each problem in a batch of its own, one slot per engine
    for pr, r in zip(probs, together):
        a = batch_solve([pr], precision=precision, **OPTS)[0]
        assert np.array_equal(a["evals"], r["evals"])
        assert np.array_equal(a["iterations"], r["iterations"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_with_soft_locking_matches_dense(precision):
    """Soft locking, and one preconditioned throw-away vector, in engines of several slots (the three 16x16 problems share one, with
    different nev): the slots share one column count, so a slot may keep converged pairs
    unlocked; every problem still matches the dense oracle.  (Alone and in a batch may differ
    in the last bits here: the shared column count couples the slots' bases.)"""
    from paper_2304_00337_amd import batch_solve
    probs = _problems()
    res = batch_solve(probs, precision=precision, lock_rel=1.0, throw_precond=1, **OPTS)
    tol = 1e-9 if precision == "fp64" else 1e-6
    for pr, r in zip(probs, res):
        assert r["status"] == 0, r
        for t in range(len(pr["ks"])):
            ref = _dense(pr, t)
            assert np.max(np.abs(r["evals"][t] - ref) / ref) < tol, (t, r["evals"][t], ref)


def test_batch_nested_start_for_problems_without_a_start_block():
    """With nested_start, batched problems without a start block start from the nested
    iteration on their own slot while the others iterate: every problem matches the dense
    eigenvalues, the problems that have start blocks give what they give without the option,
    and a nested problem gives in the batch what it gives alone."""
    from paper_2304_00337_amd import batch_solve
    probs = _problems()
    for i in (0, 2, 4):
        probs[i] = dict(probs[i], start=None)
    mixed = batch_solve(probs, nested_start=1, **OPTS)
    for pr, r in zip(probs, mixed):
        assert r["status"] == 0, r
        for t in range(len(pr["ks"])):
            ref = _dense(pr, t)
            assert np.max(np.abs(r["evals"][t] - ref) / ref) < 1e-9
    plain = batch_solve([pr for pr in probs if pr["start"] is not None], **OPTS)
    for r, q in zip([r for pr, r in zip(probs, mixed) if pr["start"] is not None], plain):
        assert np.array_equal(r["evals"], q["evals"]) and np.array_equal(r["iterations"], q["iterations"])
    alone = batch_solve([probs[2]], nested_start=1, **OPTS)[0]
    assert np.array_equal(alone["evals"], mixed[2]["evals"])
    assert np.array_equal(alone["iterations"], mixed[2]["iterations"])


def test_batch_equals_single_handle_and_slot_limits():
    """A batched problem equals the same path on a one-problem handle (bl_solve_path), and
    engines with fewer slots than problems (slots re-used as problems finish) give the same
    results."""
    from paper_2304_00337_amd import Solver, batch_solve
    probs = _problems()
    full = batch_solve(probs, **OPTS)
    tight = batch_solve(probs, max_slots=1, **OPTS)
    for r, q in zip(full, tight):
        assert np.array_equal(r["evals"], q["evals"])
    pr = probs[2]
    s = Solver(pr["n"], pr["m"], 1.0, 1.0, pr["eps"], nev=pr["nev"], nthrow=pr["nthrow"], **OPTS)
    one = s.solve_path(pr["ks"], start=pr["start"])
    assert np.array_equal(one["evals"], full[2]["evals"])
    assert np.array_equal(one["iterations"], full[2]["iterations"])


def test_batch_reports_invalid_problems_without_stopping_others():
    from paper_2304_00337_amd import batch_solve
    probs = _problems()[:2]
    bad = dict(probs[0])
    bad["ks"] = np.array([[float("nan"), 0.0]])
    res = batch_solve([probs[0], bad, probs[1]], **OPTS)
    assert res[0]["status"] == 0 and res[2]["status"] == 0
    assert res[1]["status"] == -1


def _serve(srv, reqs, rate_hz, seed):
    """Submit at Poisson arrival times; poll until all are done."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=len(reqs))
    tickets, results = [], {}
    for g, rq in zip(gaps, reqs):
        time.sleep(g)
        tickets.append(srv.submit(**rq))
        for t in tickets:
            if t not in results:
                r = srv.poll(t)
                if r is not None:
                    results[t] = r
    deadline = time.time() + 120
    while len(results) < len(tickets):
        assert time.time() < deadline, "server did not finish"
        for t in tickets:
            if t not in results:
                r = srv.poll(t)
                if r is not None:
                    results[t] = r
        time.sleep(0.002)
    return [results[t] for t in tickets]


def test_server_alone_equals_in_mix():
    from paper_2304_00337_amd import Server
    probs = _problems()
    reqs = [dict(n=p["n"], m=p["m"], a=1.0, b=1.0, eps=p["eps"], nev=p["nev"], nthrow=p["nthrow"],
                 ks=p["ks"], start=p["start"]) for p in probs]
    mix = reqs * 2     # every request twice, the copies arriving while the first ones run
    with Server(max_slots=4, precision="mixed", **OPTS) as srv:
        got = _serve(srv, mix, rate_hz=200.0, seed=0)
        st = srv.stats()
        assert st["pending"] == 0 and st["queued"] == 0
    for r in got:
        assert r["status"] == 0
        assert r["latency_s"] >= r["run_s"] >= 0 and r["queue_s"] >= 0
    for i in range(len(reqs)):
        assert np.array_equal(got[i]["evals"], got[i + len(reqs)]["evals"])
    with Server(precision="mixed", **OPTS) as srv:
        alone = _serve(srv, [reqs[2]], rate_hz=1000.0, seed=1)[0]
    assert np.array_equal(alone["evals"], got[2]["evals"])
    assert np.array_equal(alone["iterations"], got[2]["iterations"])


def test_server_small_budget_swaps_engines():
    """A budget that holds one engine at a time: requests of two shapes still all finish,
    the engines being released and created as the queue demands."""
    from paper_2304_00337_amd import Server, Solver
    probs = _problems()
    reqs = [dict(n=p["n"], m=p["m"], a=1.0, b=1.0, eps=p["eps"], nev=p["nev"], nthrow=p["nthrow"],
                 ks=p["ks"], start=p["start"]) for p in probs]
    big = max(Solver.footprint_bytes(p["n"], p["m"], 1.0, 1.0, nev=p["nev"] + p["nthrow"], nthrow=0,
                                     coarsest_min=4) for p in probs)
    with Server(hbm_budget=int(big * 1.05), max_slots=1, **OPTS) as srv:
        got = _serve(srv, reqs, rate_hz=1000.0, seed=2)
    ref = __import__("paper_2304_00337_amd").batch_solve(probs, **OPTS)
    for g, r in zip(got, ref):
        assert g["status"] == 0
        assert np.array_equal(g["evals"], r["evals"])


def test_server_errors():
    from paper_2304_00337_amd import Server
    from paper_2304_00337_amd.native import BlochError
    p = _problems()[0]
    with Server(**OPTS) as srv:
        with pytest.raises(BlochError):
            srv.submit(n=p["n"], m=p["m"], a=1.0, b=1.0, eps=p["eps"], nev=p["nev"], nthrow=p["nthrow"],
                       ks=np.array([[float("inf"), 0.0]]), start=p["start"])
        from paper_2304_00337_amd.native import check
        with pytest.raises(BlochError):
            check(srv.lib.bl_server_poll(srv.h, 12345, None, None, None, None), "bl_server_poll")


def test_batch_context_reuses_engines():
    """A batch context keeps its engines: a second run of the same problems allocates no new
    engine and gives identical results; per-point times are reported and the smoother timing
    counts launches of the finest-level smoother (run per level here: with fused coarse
    cycles these small grids have no separate finest-level launch), whose results equal the
    fused engines' bit for bit."""
    from paper_2304_00337_amd import Batch, batch_solve
    probs = _problems()
    with Batch(max_slots=4, coarse_fuse=0, **OPTS) as b:
        b.set_timing(True)
        r1 = b.run(probs)
        t1 = b.timing()
        r2 = b.run(probs)
    ref = batch_solve(probs, **OPTS)
    for x, y, z in zip(r1, r2, ref):
        assert x["status"] == 0
        assert np.array_equal(x["evals"], y["evals"]) and np.array_equal(x["evals"], z["evals"])
        assert np.all(x["point_ms"] > 0)
    assert t1["launches"] > 0 and t1["total_ms"] > 0 and t1["columns"] >= t1["launches"]
    assert t1["alg_bytes"] > 0


def test_server_large_request_is_not_starved():
    """A budget that holds the large request only when nothing else is on the device, and a
    stream of small requests arriving with and after it: admission lets at most a few later
    requests pass the large one, then drains the small engine, releases it and admits the
    large request, which therefore finishes before most of the small requests submitted
    after it, with the same result as alone."""
    from paper_2304_00337_amd import Server, Solver
    eps_small = synth.eps_disc(32, 32, 1.0, 1.0, 8.9, 0.3)
    eps_big = synth.eps_disc_lattice(128, 128, 1.0, 1.0, 12.0, 0.3)
    small = [dict(n=32, m=32, a=1.0, b=1.0, eps=eps_small, nev=4, nthrow=2,
                  ks=np.array([(0.9, -0.4), (1.0, -0.35), (1.1, -0.3)]),
                  start=synth.start_block(2 * 32 * 32, 6, 40 + i)) for i in range(14)]
    big = dict(n=128, m=128, a=1.0, b=1.0, eps=eps_big, nev=4, nthrow=2, ks=np.array([(0.7, 0.2), (0.8, 0.25)]),
               start=synth.start_block(2 * 128 * 128, 6, 99))
    fb = Solver.footprint_bytes(128, 128, 1.0, 1.0, nev=6, nthrow=0, coarsest_min=4)
    fs = Solver.footprint_bytes(32, 32, 1.0, 1.0, nev=6, nthrow=0, coarsest_min=4)
    reqs = small[:2] + [big] + small[2:]
    with Server(hbm_budget=int(fb + 0.5 * fs), max_slots=2, precision="mixed", **OPTS) as srv:
        t_sub = []
        tickets = []
        for rq in reqs:
            t_sub.append(time.perf_counter())
            tickets.append(srv.submit(**rq))
        done, t_done = {}, {}
        deadline = time.time() + 120
        while len(done) < len(tickets):
            assert time.time() < deadline, "server did not finish"
            for t in tickets:
                if t not in done:
                    r = srv.poll(t)
                    if r is not None:
                        done[t] = r
                        t_done[t] = time.perf_counter()
            time.sleep(0.001)
    res = [done[t] for t in tickets]
    assert all(r["status"] == 0 for r in res)
    big_done = t_done[tickets[2]]
    later_small_after = sum(1 for t in tickets[3:] if t_done[t] > big_done)
    assert later_small_after >= 6, later_small_after
    with Server(precision="mixed", **OPTS) as srv:
        alone = _serve(srv, [big], rate_hz=1000.0, seed=3)[0]
    assert np.array_equal(alone["evals"], res[2]["evals"])


def test_reduced_mixed_batch_against_oracle():
    """A reduced batch of the 64-problem kind in one batch context: n in {64, 96, 128} and
    nev in {4, 8, 16}, mixed precision, every problem converged and its eigenvalues within
    1e-6 of the oracle's ARPACK values (tests/golden/arpack_c4small.json); the plain FP64
    batch within 1e-9."""
    import json
    import os
    from paper_2304_00337_amd import batch_solve
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "arpack_c4small.json")) as f:
        gold = json.load(f)["points"]
    probs = synth.config_c4_small()
    items = [dict(n=p.n, m=p.m, a=p.a, b=p.b, eps=p.eps, nev=p.nev, nthrow=p.nthrow, ks=np.asarray(p.ks),
                  start=p.start()) for p in probs]
    for precision, tol in (("mixed", 1e-6), ("fp64", 1e-9)):
        res = batch_solve(items, precision=precision, tol=1e-8, max_iter=300)
        for p, r, g in zip(probs, res, gold):
            assert r["status"] == 0, (precision, p.n, p.nev)
            ref = np.array(g["evals"])
            err = np.max(np.abs(r["evals"][0] - ref) / ref)
            assert err <= tol, (precision, p.n, p.nev, err)


def test_server_alone_equals_in_mix_large_request():
    """A 512 x 512 request served among smaller ones gives the same result, to the last
    bit, as when it is served alone."""
    from paper_2304_00337_amd import Server
    probs = _problems()
    reqs = [dict(n=p["n"], m=p["m"], a=1.0, b=1.0, eps=p["eps"], nev=p["nev"], nthrow=p["nthrow"],
                 ks=p["ks"], start=p["start"]) for p in probs]
    big = dict(n=512, m=512, a=1.0, b=1.0, eps=synth.eps_random_field(512, 512, 1.0, 1.0, 21), nev=8, nthrow=4,
               ks=np.array([(0.6, 0.3), (0.7, 0.35), (0.8, 0.4)]), start=synth.start_block(2 * 512 * 512, 12, 77))
    mix = reqs[:2] + [big] + reqs[2:]
    with Server(max_slots=4, precision="mixed", **OPTS) as srv:
        got = _serve(srv, mix, rate_hz=200.0, seed=5)
    assert all(r["status"] == 0 for r in got)
    with Server(precision="mixed", **OPTS) as srv:
        alone = _serve(srv, [big], rate_hz=1000.0, seed=6)[0]
    assert np.array_equal(alone["evals"], got[2]["evals"])
    assert np.array_equal(alone["iterations"], got[2]["iterations"])
