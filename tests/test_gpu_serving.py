"""Batched and served solves on the GPU: every LP's result is the same alone,
in a batch and in the serving mix (continuous batching)."""
import time

import numpy as np
import pytest

import lpgen

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2508_08062_amd")

OPTS = dict(precision=0, memory=8, kkt_every=16, tol=1e-4, max_iter=4000, ruiz_iters=10, dhat_mode=0, epoch=32)


def _lps(count, seed0):
    rng = np.random.default_rng(seed0)
    out = []
    for i in range(count):
        m = int(rng.integers(300, 3000))
        out.append(lpgen.mip_like_lp(seed0 * 100 + i, m=m, n=2 * m, nnz=int(rng.integers(3, 8)) * 2 * m))
    return out


def _solo(lp, **extra):
    s = P.Solver(lp, **{**OPTS, **extra})
    s.solve()
    r = s.result()
    s.close()
    return r


@pytest.mark.parametrize("extra", [{}, {"variant": 3, "restart_period": 50}, {"pw_period": 64, "sg_div": 3.0}],
                         ids=["aa", "restarted", "primal-weight"])
def test_served_results_equal_solo_results(extra):
    lps = _lps(10, 7)
    solo = [_solo(lp, **extra) for lp in lps]
    srv = P.Server(hbm_budget_bytes=1 << 30, max_slots=4, **{**OPTS, **extra})
    tickets = []
    for i, lp in enumerate(lps):  # staggered arrivals: some join while others run
        tickets.append(srv.submit(lp))
        time.sleep(0.002 * (i % 3))
    results = {}
    t0 = time.time()
    while len(results) < len(tickets):
        assert time.time() - t0 < 90, srv.stats()
        for t in tickets:
            if t not in results:
                r = srv.poll(t)
                if r is not None:
                    results[t] = r
        time.sleep(0.001)
    st = srv.stats()
    srv.close()
    assert st["submitted"] == st["admitted"] == st["finished"] == len(lps)
    for t, ref in zip(tickets, solo):
        r = results[t]
        assert r["status"] == ref["status"] and r["iters"] == ref["iters"]
        assert np.array_equal(r["x"], ref["x"]) and np.array_equal(r["y"], ref["y"])
        assert r["t_done"] >= r["t_admit"] >= 0.0


def test_server_budget_queues_and_rejects():
    lps = _lps(3, 8)
    est = 40 * 1024 * 1024
    srv = P.Server(hbm_budget_bytes=est, max_slots=8, **OPTS)
    big = lpgen.mip_like_lp(99, m=200000, n=400000, nnz=2000000)
    tb = srv.submit(big)  # larger than the whole budget: rejected, not a crash
    ts = [srv.submit(lp) for lp in lps]
    done = {}
    t0 = time.time()
    while len(done) < len(ts):
        assert time.time() - t0 < 60
        for t in ts:
            if t not in done:
                r = srv.poll(t, want_solution=False)
                if r is not None:
                    done[t] = r
    with pytest.raises(P.AAPDHGError) as e:
        srv.poll(tb)
    assert e.value.status == P.E_NOMEM
    srv.close()


def test_batch_of_uneven_lps_equals_solo():
    lps = _lps(12, 9)
    solo = [_solo(lp) for lp in lps]
    members = [P.Solver(lp, **OPTS) for lp in lps]
    b = P.Batch(members)
    b.solve()
    for g, ref in zip(members, solo):
        r = g.result()
        assert r["status"] == ref["status"] and r["iters"] == ref["iters"]
        assert np.array_equal(r["x"], ref["x"])
    b.close()


def test_batch_of_mixed_methods_equals_solo():
    """Every member of one batch runs its own method and options (each LP has
    its own descriptor): vanilla PDHG, AA-PDHG, FAA-PDHG under both angle
    filter readings, restarted PDHG and AA-PDHG with the primal-weight
    update share the launches, and each result equals the LP's solo run bit
    for bit."""
    lps = _lps(6, 11)
    methods = [dict(variant=0), dict(variant=1), dict(variant=2, cs=0.5), dict(variant=2, cs=0.5, angle_mode=1),
               dict(variant=3, restart_period=40), dict(variant=1, pw_period=64, sg_div=2.0)]
    solo = [_solo(lp, **mth) for lp, mth in zip(lps, methods)]
    members = [P.Solver(lp, **{**OPTS, **mth}) for lp, mth in zip(lps, methods)]
    b = P.Batch(members)
    b.solve()
    for r, ref, mth in zip(b.results(), solo, methods):  # aapdhg_batch_result
        assert (r["status"], r["iters"], r["aa_steps"]) == (ref["status"], ref["iters"], ref["aa_steps"]), mth
        assert np.array_equal(r["x"], ref["x"]) and np.array_equal(r["y"], ref["y"]), mth
    with pytest.raises(P.AAPDHGError, match="out of range"):
        b.result(len(members))
    b.close()


def _infeasible_lp():
    # x0 + x1 = 1 and x0 + x1 = 3 with 0 <= x <= 10: no feasible point
    return lpgen.LPData(m=2, n=2, rowptr=np.array([0, 2, 4], dtype=np.int64),
                        colidx=np.array([0, 1, 0, 1], dtype=np.int32), val=np.ones(4), c=np.ones(2),
                        q=np.array([1.0, 3.0]), l=np.zeros(2), u=np.full(2, 10.0),
                        rowtype=np.zeros(2, dtype=np.uint8))


def test_a_request_that_cannot_converge_does_not_disturb_the_others():
    """An infeasible request shares the server's epochs with ordinary ones: it
    ends at its pass limit while the others finish exactly as alone."""
    lps = _lps(4, 13)
    solo = [_solo(lp) for lp in lps]
    srv = P.Server(hbm_budget_bytes=1 << 30, max_slots=8, **OPTS)
    bad = srv.submit(_infeasible_lp())
    tickets = [srv.submit(lp) for lp in lps]
    results = {}
    t0 = time.time()
    while len(results) < len(tickets) + 1:
        assert time.time() - t0 < 90, srv.stats()
        for t in [bad] + tickets:
            if t not in results:
                r = srv.poll(t)
                if r is not None:
                    results[t] = r
        time.sleep(0.001)
    srv.close()
    rb = results[bad]
    assert rb["status"] == "iter_limit" and rb["iters"] == OPTS["max_iter"] + 1
    assert np.all(np.isfinite(rb["x"])) and np.all(np.isfinite(rb["y"]))
    for t, ref in zip(tickets, solo):
        r = results[t]
        assert r["status"] == ref["status"] and r["iters"] == ref["iters"]
        assert np.array_equal(r["x"], ref["x"]) and np.array_equal(r["y"], ref["y"])
