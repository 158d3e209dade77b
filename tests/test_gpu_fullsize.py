"""GPU checks at the benchmark's full sizes and launch configurations.

After a benchmark-sized launch (the 20k x 50k LP: one persistent launch of
500 loop passes; the 1M x 2M LP: 250 passes of the three-launch kernels; the
256-LP batch: 200 passes of its launch set, sampled members), the device
state must agree with the oracle evaluated on the same seeded, equilibrated,
float32-rounded LP (requests of the serving mix are checked at their
solution instead, after going through the server):

  * the last PDHG point: u_prev + g_prev equals the oracle's T(u_prev)
    (eq. pdhg) element by element, to relative 1e-5 of the vector's norm
    (the float32 storage of x_hat, x_bar and y_hat; the products are exact
    in float64);
  * the history: every Gram entry is the float64 dot product of the stored
    difference columns and ||g|| the norm of the stored residual (float64
    sums of the same float32 values in another order: relative 1e-9); every
    right-hand side is the dot product with the stored residual up to the
    rounding of the float32 difference columns it was updated with (the
    library adds each new Gram row to the right-hand sides, which is exact
    for exact differences: each update adds at most 2^-24 ||dG_a|| ||dG_s||,
    allowed for 4 M updates of the largest live column);
  * the counters add up (i + j = k - 1), the iterate lies in X x Y, and the
    KKT residuals reported at the returned point equal the oracle's there.
"""
import time

import numpy as np
import pytest

import lpgen
import oracle

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2508_08062_amd")


def _scaled_oracle_problem(lp, ruiz_iters):
    Po = oracle.Problem.from_lpdata(lp)
    if ruiz_iters:
        Po, _, _ = oracle.ruiz(Po, ruiz_iters)
    return Po.rounded_fp32()


def _check_state(lp, Po, g, tau, sigma, st, M, fp32=True):
    n = lp.n
    up, gp = st["u_prev"], st["g_prev"]
    # the last PDHG point
    xh, yh = oracle.pdhg_map(Po, up[:n], up[n:], tau, sigma)
    ref = np.r_[xh, yh]
    got = up + gp
    err = np.abs(got - ref)
    scale = np.linalg.norm(ref)
    assert np.linalg.norm(got - ref) / scale < 1e-5
    assert err.max() / np.abs(ref).max() < 1e-5
    # the history and its Gram matrix
    live = st["live"]
    assert len(live) <= M
    G, rhs = st["G"], st["rhs"]
    for a in live:
        for b in live:
            want = float(np.dot(st["dG"][a], st["dG"][b]))
            tol = 1e-9 * np.sqrt(G[a, a] * G[b, b]) + 1e-300
            assert abs(G[a, b] - want) <= tol, (a, b, G[a, b], want)
        want = float(np.dot(st["dG"][a], gp))
        big = max(np.sqrt(G[b, b]) for b in live)
        upd = 4 * M * 2.0 ** -24 * np.sqrt(G[a, a]) * big if fp32 else 0.0
        assert abs(rhs[a] - want) <= 1e-9 * np.sqrt(G[a, a] * float(gp @ gp)) + upd + 1e-300, (a, rhs[a], want)
    assert st["gnorm"] == pytest.approx(float(np.linalg.norm(gp)), rel=1e-9)
    # counters and projections
    assert st["i"] + st["j"] == st["k"] - 1
    x, y = st["u"][:n], st["u"][n:]
    # (the bounds of both sides are float32 roundings of the same scaled values)
    slack = 1e-6 * (1.0 + np.abs(np.where(np.isfinite(Po.l), Po.l, 0.0)) + np.abs(np.where(np.isfinite(Po.u), Po.u, 0.0)))
    assert np.all(x >= Po.l - slack) and np.all(x <= Po.u + slack)
    assert np.all(y[Po.rowtype == oracle.ROW_GE] >= 0.0)
    # KKT at the returned point, measured on the problem as solved
    r = g.result()
    ko = oracle.kkt(Po, x, y)
    for key, gkey in (("r_p", "r_pri"), ("r_d", "r_dual"), ("r_g", "r_gap")):
        assert r[gkey] == pytest.approx(ko[key], rel=1e-6, abs=1e-9), key


def test_mip20k_after_one_persistent_launch_of_500_passes():
    lp = lpgen.mip_like_lp(1)
    opts = dict(variant=1, precision=0, memory=10, kkt_every=64, ruiz_iters=10, dhat_mode=0)
    Po = _scaled_oracle_problem(lp, 10)
    tau = sigma = 0.9 / oracle.power_norm(Po)
    g = P.Solver(lp, tol=0.0, max_iter=10 ** 9, tau=tau, sigma=sigma, **opts)
    g.iterate(1)  # the init step
    t = g.iterate_timed(500)  # the benchmark's launch: one persistent launch of 500 passes
    assert t["kernel"] == "persistent" and t["passes"] == 500
    st = g.get_state()
    assert st["k"] == 501 and st["status"] == 4
    _check_state(lp, Po, g, tau, sigma, st, 10)
    g.close()


def test_powerlaw1m_after_250_three_launch_passes():
    lp = lpgen.powerlaw_lp(2)
    opts = dict(variant=2, precision=0, memory=10, kkt_every=64, ruiz_iters=10, dhat_mode=0)
    Po = _scaled_oracle_problem(lp, 10)
    tau = sigma = 0.9 / oracle.power_norm(Po)
    g = P.Solver(lp, tol=0.0, max_iter=10 ** 9, tau=tau, sigma=sigma, **opts)
    g.iterate(1)
    t = g.iterate_timed(250)
    assert t["kernel"] == "three"
    st = g.get_state()
    assert st["k"] == 251 and st["status"] == 4
    _check_state(lp, Po, g, tau, sigma, st, 10)
    g.close()


@pytest.mark.timeout(300)
def test_batch256_after_200_passes_of_the_whole_batch():
    """The batch workload at full size (256 LPs, 44.6M entries) advanced by
    the launches of one launch set; the state of sampled members (the
    first, a middle one, the last and the largest) is checked as above
    against the oracle on that member's own scaled LP, with the member's
    own step sizes."""
    lps = lpgen.batch_lps(256, 3)
    opts = dict(variant=1, precision=0, memory=8, kkt_every=64, ruiz_iters=10, dhat_mode=0)
    members = [P.Solver(lp, tol=0.0, max_iter=10 ** 9, **opts) for lp in lps]
    b = P.Batch(members)
    b.iterate(200)  # a member that has not started takes its init step first: k = 201
    big = int(np.argmax([lp.nnz for lp in lps]))
    for i in sorted({0, 128, 255, big}):
        g = members[i]
        st = g.get_state()
        assert st["k"] == 201 and st["status"] == 4, i
        d = g.dims()
        Po = _scaled_oracle_problem(lps[i], 10)
        _check_state(lps[i], Po, g, d["tau"], d["sigma"], st, 8)
    b.close()
    for g in members:
        g.close()


@pytest.mark.timeout(300)
def test_serving_mix_requests_through_the_server():
    """Requests of the serving workload's pool (Poisson stream seed 4: the
    largest, 96,675 columns and 483,375 entries, and two typical ones) go
    through the server with the workload's options, submitted together; each
    result equals the LP's solo solve bit for bit, and the KKT residuals the
    server reports equal the oracle's at the returned point on the LP's
    scaled, float32-rounded problem."""
    reqs = lpgen.serving_requests(rate=4.0, duration=10.0, seed=4)[:16]
    pick = [5, 0, 6]
    lps = [lpgen.mip_like_lp(reqs[i][4], m=reqs[i][1], n=reqs[i][2], nnz=reqs[i][3]) for i in pick]
    opts = dict(variant=1, precision=0, memory=10, kkt_every=64, ruiz_iters=10, dhat_mode=0, tol=1e-4,
                max_iter=200000, epoch=64)
    srv = P.Server(hbm_budget_bytes=8 << 30, max_slots=64, **opts)
    tickets = [srv.submit(lp) for lp in lps]
    served = {}
    deadline = time.monotonic() + 240.0
    while len(served) < len(tickets):
        assert time.monotonic() < deadline, "served requests did not finish"
        for t in tickets:
            if t not in served:
                r = srv.poll(t)
                if r is not None:
                    served[t] = r
        time.sleep(0.01)
    srv.close()
    for lp, t in zip(lps, tickets):
        r = served[t]
        g = P.Solver(lp, **opts)
        g.solve()
        ref = g.result()
        assert r["status"] == ref["status"] == "converged"
        assert r["iters"] == ref["iters"] and r["kkt"] == ref["kkt"]
        assert np.array_equal(r["x"], ref["x"]) and np.array_equal(r["y"], ref["y"])
        d_row, d_col = g.scaling()
        Po = _scaled_oracle_problem(lp, 10)
        ko = oracle.kkt(Po, r["x"] / d_col, r["y"] / d_row)
        for key, gkey in (("r_p", "r_pri"), ("r_d", "r_dual"), ("r_g", "r_gap")):
            assert ref[gkey] == pytest.approx(ko[key], rel=1e-5, abs=1e-9), key
        assert ko["kkt"] <= 1.01e-4
        g.close()
