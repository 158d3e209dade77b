"""Launch-side options of the batched path on the GPU: the passes captured in
a HIP graph and replayed (option graph), and the autotuned work tables
(option autotune).  Neither changes the method; the graph does not change the
kernels or their order, so results are equal bit for bit with and without
it, and a tuned LP keeps its tables alone and in a batch, so its iterates are
the same in both."""
import os

import numpy as np
import pytest

import lpgen

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2508_08062_amd")

OPTS = dict(variant=1, precision=0, memory=8, kkt_every=16, ruiz_iters=10, dhat_mode=0, tol=1e-4,
            max_iter=4000, epoch=64)


def _lps():
    return [lpgen.mip_like_lp(60 + i, m=m, n=2 * m, nnz=6 * m) for i, m in enumerate((1200, 5000, 2500, 9000))]


def _states(solvers):
    return [(g.get_state()["k"], g.get_state()["u"]) for g in solvers]


def test_graph_replay_equals_direct_launches():
    lps = _lps()
    out = []
    for graph in (0, 1):
        members = [P.Solver(lp, loop_kernel=1, graph=graph, **OPTS) for lp in lps]
        b = P.Batch(members)
        b.solve()
        out.append(_states(members))
        b.close()
        for g in members:
            g.close()
    for (ka, ua), (kb, ub) in zip(*out):
        assert ka == kb and np.array_equal(ua, ub)
    # one LP in three launches per pass, solved on its own
    res = []
    for graph in (0, 1):
        g = P.Solver(lps[1], loop_kernel=1, graph=graph, **OPTS)
        g.solve()
        res.append(g.result())
        g.close()
    assert res[0]["iters"] == res[1]["iters"] and np.array_equal(res[0]["x"], res[1]["x"])


def test_autotuned_lps_equal_alone_and_in_a_graph_batch(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("AAPDHG_TUNE_CACHE", str(cache))
    lps = _lps()
    solo = []
    for lp in lps:
        # three launches per pass alone and in the graph batch (the tuner keeps the loop
        # kernel the options ask for and tunes the tables)
        g = P.Solver(lp, autotune=1, loop_kernel=1, **OPTS)
        g.solve()
        solo.append((g.result(), g.get_state()["u"]))
        g.close()
    lines = cache.read_text().splitlines()
    assert 1 <= len(lines) <= len(lps)  # LPs of one shape class share an entry
    for ln in lines:
        key, w, cpb, lk, ms = ln.split()
        assert key.count(":") == 12 and int(w) in (2, 4, 8) and int(cpb) in (0, 2) and int(lk) == 1
    # members created again take the cached choices (no new entries) and, in a
    # batch replayed from a graph, give their solo results bit for bit
    members = [P.Solver(lp, autotune=1, graph=1, loop_kernel=1, **OPTS) for lp in lps]
    assert cache.read_text().splitlines() == lines
    b = P.Batch(members)
    b.solve()
    for (r, u), g in zip(solo, members):
        r2 = g.result()
        assert r2["iters"] == r["iters"] and r2["kkt"] == r["kkt"]
        assert np.array_equal(g.get_state()["u"], u)
    b.close()
    for g in members:
        g.close()
