"""Asynchronous entry points on the GPU.

* aapdhg_solve enqueues the solve and returns at once: a 20k x 50k LP held
  for 30,000 loop passes (about 0.6 s of device time) is still running when
  the call returns; aapdhg_wait returns once it has finished, and the result
  equals that of the same solve waited for at once, bit for bit.
* A second call on the handle (here aapdhg_result) waits for the solve
  itself.
* The server with caller-given compute and copy streams (torch streams):
  requests submitted together, some while others run, give their solo
  results bit for bit.
"""
import time

import numpy as np
import pytest

import lpgen

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2508_08062_amd")


def test_solve_returns_before_the_work_completes():
    lp = lpgen.mip_like_lp(1)
    kw = dict(precision=0, memory=10, kkt_every=64, ruiz_iters=10, dhat_mode=0, tol=0.0, max_iter=30000)
    g = P.Solver(lp, **kw)
    t0 = time.perf_counter()
    g.solve(wait=False)
    t_ret = time.perf_counter() - t0
    g.wait()
    t_done = time.perf_counter() - t0
    r = g.result()
    assert r["status"] == "iter_limit" and r["iters"] == 30001
    assert t_done > 0.2 and t_ret < 0.25 * t_done, (t_ret, t_done)
    # the next call on the handle waits by itself
    g2 = P.Solver(lp, **kw)
    g2.solve(wait=False)
    r2 = g2.result()
    assert r2["iters"] == 30001
    assert np.array_equal(r["x"], r2["x"]) and np.array_equal(r["y"], r2["y"])
    g.close()
    g2.close()


def test_server_with_caller_streams_equals_solo():
    import torch
    compute, copy = torch.cuda.Stream(), torch.cuda.Stream()
    lps = [lpgen.mip_like_lp(40 + i, m=m, n=int(2.5 * m), nnz=int(12.5 * m))
           for i, m in enumerate((2000, 9000, 4000, 15000, 1000))]
    opts = dict(variant=1, precision=0, memory=10, kkt_every=64, ruiz_iters=10, dhat_mode=0, tol=1e-4,
                max_iter=100000, epoch=64)
    srv = P.Server(hbm_budget_bytes=4 << 30, max_slots=8, compute_stream=compute, copy_stream=copy, **opts)
    tickets = [srv.submit(lp) for lp in lps[:3]]
    time.sleep(0.05)  # the rest arrive while the first ones run
    tickets += [srv.submit(lp) for lp in lps[3:]]
    served = {}
    deadline = time.monotonic() + 120.0
    while len(served) < len(tickets):
        assert time.monotonic() < deadline, "served requests did not finish"
        for t in tickets:
            if t not in served:
                r = srv.poll(t)
                if r is not None:
                    served[t] = r
        time.sleep(0.005)
    st = srv.stats()
    srv.close()
    assert st["finished"] == len(lps) and st["resident"] == 0
    for lp, t in zip(lps, tickets):
        g = P.Solver(lp, **opts)
        g.solve()
        ref = g.result()
        r = served[t]
        assert r["status"] == ref["status"] == "converged"
        assert r["iters"] == ref["iters"] and r["kkt"] == ref["kkt"]
        assert np.array_equal(r["x"], ref["x"]) and np.array_equal(r["y"], ref["y"])
        g.close()
