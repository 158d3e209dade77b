"""GPU parity at the benchmark's sizes, in the benchmark's configurations.

* The 20k x 50k LP (AA-PDHG, m_A = 10, 10 Ruiz sweeps, float32, KKT test
  every 64 passes, the persistent loop kernel): 50 free-running loop passes
  compared with the oracle entry by entry after every pass, and the same 50
  passes run as one launch give the same bits as 50 launches of one pass.
* The 1M x 2M LP (FAA-PDHG, m_A = 10, float32, three launches per pass): one
  pass at a time from the GPU's own state loaded into the oracle (teacher
  forcing), every step accelerated (large D) so that the filters of Alg 3-5
  run on each pass; the kept memory, gamma and u^{k+1} are compared.
* Solves to relative KKT 1e-4 and 1e-6 of the smallest LP of the 256-LP
  batch: in float64 the objective equals the oracle's to 1e-6; in float32
  the returned point passes the oracle's KKT test and its objective is
  compared with the planted optimum of the generator.  The 20k x 50k LP
  solved to 1e-4 in both precisions: the oracle's KKT at the returned point
  and the planted optimum.

Tolerances: err32 / err64 of tests/_util.py for iterates; one pass from the
same state (teacher forcing) is compared entry by entry to 1e-5 of each
entry's size or of 1e-3 of the vector's largest entry.
"""
import numpy as np
import pytest

import lpgen
import oracle
from _util import entrywise_err, err32

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2508_08062_amd")



def _scaled(lp, ruiz_iters=10, fp32=True):
    """The LP as the library solves it: Ruiz-scaled, and rounded to float32
    for the float32 path (the float64 path keeps the scaled values)."""
    Po = oracle.Problem.from_lpdata(lp)
    if ruiz_iters:
        Po, _, _ = oracle.ruiz(Po, ruiz_iters)
    return Po.rounded_fp32() if fp32 else Po


@pytest.mark.timeout(300)
def test_mip20k_50_free_running_passes_in_the_persistent_kernel():
    lp = lpgen.mip_like_lp(1)
    opts = dict(variant=1, memory=10, kkt_every=64, dhat_mode=0)
    Po = _scaled(lp)
    tau = sigma = 0.9 / oracle.power_norm(Po)
    g = P.Solver(lp, precision=0, ruiz_iters=10, tol=0.0, max_iter=10 ** 9, tau=tau, sigma=sigma, **opts)
    o = oracle.Solver(Po, oracle.Options(tol=0.0, max_iter=10 ** 9, tau=tau, sigma=sigma, **opts))
    o.start()
    t = g.iterate_timed(1)  # the init step, then one loop pass
    assert t["kernel"] == "persistent"
    o.step()
    errs = []
    for k in range(50):
        if k:
            o.step()
            g.iterate(1)
        st = g.get_state()
        ref = np.r_[o.state.x, o.state.y]
        errs.append(err32(st["u"], ref))
        assert (st["i"], st["j"]) == (o.state.i, o.state.j), k
        assert errs[-1] < 1e-5, (k, errs[-1])
    u50 = st["u"].copy()
    g.close()
    # the same 50 passes as one launch of the persistent kernel: the same bits
    g2 = P.Solver(lp, precision=0, ruiz_iters=10, tol=0.0, max_iter=10 ** 9, tau=tau, sigma=sigma, **opts)
    g2.iterate(1)
    t = g2.iterate_timed(50)
    assert t["kernel"] == "persistent" and t["passes"] == 50
    assert np.array_equal(g2.get_state()["u"], u50)
    g2.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("cs,kappa_bar", [(0.2, 1e8), (0.6, 1e4)])
def test_powerlaw1m_faa_teacher_forced_passes(cs, kappa_bar):
    """Every pass an FAA step (D = 1e6): after 14 passes from the start
    (memory full), three passes each from the GPU's state loaded into the
    oracle.  Per pass: the branch and counters; the kept memory (the same
    number of columns, and the GPU's live columns are the oracle's filtered
    ones: the columns carried over are the ones loaded, and the new
    difference column agrees to the float32 rounding of the two residuals
    it is formed from); gamma (the GPU solves the normal equations of the
    kept columns by Cholesky, the oracle factors them by QR) to 1e-4 of the
    largest coefficient; and the next iterate entry by entry."""
    lp = lpgen.powerlaw_lp(2)
    Po = _scaled(lp)
    n = lp.n
    tau = sigma = 0.9 / oracle.power_norm(Po, iters=60)
    opts = dict(variant=2, memory=10, kkt_every=64, dhat_mode=0, cs=cs, kappa_bar=kappa_bar, D=1e6)
    g = P.Solver(lp, precision=0, ruiz_iters=10, tol=0.0, max_iter=10 ** 9, tau=tau, sigma=sigma, **opts)
    g.iterate(1)
    g.iterate(14)
    o = oracle.Solver(Po, oracle.Options(tol=0.0, max_iter=10 ** 9, tau=tau, sigma=sigma, **opts))
    kept = []
    for _ in range(3):
        st = g.get_state()
        S = oracle.State(k=st["k"], x=st["u"][:n].copy(), y=st["u"][n:].copy(), u_prev=st["u_prev"].copy(),
                         g_prev=st["g_prev"].copy(), dU=[st["W"][t] - o.Dhat * st["dG"][t] for t in st["live"]],
                         dG=[st["dG"][t].copy() for t in st["live"]], i=st["i"], j=st["j"], n0=st["n0"])
        o.state = S
        before = len(S.dG) + 1  # the new pair joins the memory (oldest dropped when full)
        o.step()
        g.iterate(1)
        st2 = g.get_state()
        assert o.last_branch == "aa" and st2["branch"] == 2
        assert (st2["i"], st2["j"]) == (o.state.i, o.state.j)
        # the kept memory: same count and the same columns in the same order
        assert st2["nlive"] == len(o.state.dG)
        # g^k of the pass (oracle), g^{k-1} and u^k (loaded): the GPU rounds u_hat = u + g and g to
        # float32 before it forms the difference, and the y part is formed from K x_bar with x_bar
        # stored in float32 (the oracle keeps it in float64)
        g_new, g_old, u_k = o.state.g_prev, st["g_prev"], st["u"]
        bound = 4 * 2.0 ** -24 * (np.abs(u_k) + np.abs(g_new) + np.abs(g_old)) + 1e-30
        xbar = 2.0 * (u_k[:n] + g_new[:n]) - u_k[:n]
        bound[n:] += 4 * 2.0 ** -24 * sigma * (abs(Po.K) @ np.abs(xbar))
        for t, col in zip(st2["live"], o.state.dG):
            assert np.all(np.abs(st2["dG"][t] - col) <= bound)
        kept.append((min(before, 10), st2["nlive"]))
        # gamma of the mix (Cholesky of the Gram on the GPU, QR in the oracle)
        assert st2["nmix"] == len(o.last_gamma)
        gam_o = np.asarray(o.last_gamma)
        np.testing.assert_allclose(st2["gamma"], gam_o, rtol=1e-4, atol=1e-4 * np.abs(gam_o).max())
        ref = np.r_[o.state.x, o.state.y]
        assert entrywise_err(st2["u"], ref, 1e-3) < 1e-5
    g.close()
    print("memory before the filters -> kept:", kept)


def _batch_member():
    lps = lpgen.batch_lps(256, 3)
    return lps[int(np.argmin([q.nnz for q in lps]))]  # 1035 x 2070, 7292 entries


def _solve(lp, tol, precision, max_iter, **kw):
    Po = _scaled(lp, fp32=precision == 0)
    tau = sigma = 0.9 / oracle.power_norm(Po)
    g = P.Solver(lp, precision=precision, ruiz_iters=10, tol=tol, max_iter=max_iter, tau=tau, sigma=sigma, **kw)
    g.solve()
    r = g.result()
    d_row, d_col = g.scaling()
    g.close()
    # the GPU's returned point evaluated by the oracle (variables of the scaled LP)
    ko = oracle.kkt(Po, r["x"] / d_col, r["y"] / d_row)
    return r, ko, Po, tau


@pytest.mark.timeout(600)
@pytest.mark.parametrize("tol", [1e-4, 1e-6])
def test_fp64_objective_of_a_batch_member_matches_the_oracle(tol):
    """Float64 on both sides, so the stopping decisions are taken in the same
    precision: the objectives at relative KKT `tol` agree to 1e-6 (the
    oracle's own objective moves by 1.1e-7 at 1e-4 and 5.7e-7 at 1e-6 when
    its start point is perturbed by 2^-24, on this LP), and both lie within
    2e-6 of the planted optimum."""
    lp = _batch_member()
    kw = dict(variant=1, memory=8, kkt_every=64, dhat_mode=0)
    r, ko, Po, tau = _solve(lp, tol, 1, 200000, **kw)
    ro = oracle.Solver(Po, oracle.Options(tol=tol, max_iter=200000, tau=tau, sigma=tau, **kw)).solve()
    assert r["status"] == ro["status"] == "converged"
    assert r["kkt"] <= tol and ko["kkt"] <= tol * 1.000001
    assert r["primal_obj"] == pytest.approx(ko["pobj"], rel=1e-12, abs=1e-12)
    o_obj = ro["kkt"]["pobj"]
    rel = abs(r["primal_obj"] - o_obj) / (1.0 + abs(o_obj))
    pstar = lp.planted["pstar"]
    print(f"tol {tol}: gpu obj {r['primal_obj']!r} ({r['iters']} passes), oracle obj {o_obj!r} "
          f"({ro['k']} passes), rel diff {rel:.2e}, planted {pstar!r}")
    assert rel <= 1e-6, rel
    for obj in (r["primal_obj"], o_obj):
        assert abs(obj - pstar) / (1.0 + abs(pstar)) <= 2e-6


@pytest.mark.timeout(600)
@pytest.mark.parametrize("tol", [1e-4, 1e-6])
def test_fp32_solve_of_a_batch_member_returns_a_valid_point(tol):
    """Float32 iterates: which pass first passes the KKT test is a float32
    decision.  The oracle with its iterates and memory rounded to float32
    after every pass stops at pass 16,512 at KKT 1e-4 with its objective
    2.6e-3 from the planted optimum, as the GPU does, where the float64
    oracle runs on to pass 123,008 (1.1e-6); several points pass the test
    and each is a correct result.  So: the returned point passes the
    oracle's own KKT test at `tol`, the reported objective is the oracle's
    evaluation at that point, and the objective lies within 5e-3 (KKT 1e-4)
    or 1e-4 (KKT 1e-6) of the planted optimum.  At 1e-6 float32 iterates
    may stall above the tolerance (the emulation does, at 1.6e-4 after
    200,000 passes): a run that reaches the pass limit must still hold a
    point at KKT 1e-3."""
    lp = _batch_member()
    r, ko, Po, tau = _solve(lp, tol, 0, 200000, variant=1, memory=8, kkt_every=64, dhat_mode=0)
    assert r["kkt"] == pytest.approx(ko["kkt"], rel=1e-6, abs=1e-12)
    assert r["primal_obj"] == pytest.approx(ko["pobj"], rel=1e-6, abs=1e-9)
    pstar = lp.planted["pstar"]
    rel = abs(r["primal_obj"] - pstar) / (1.0 + abs(pstar))
    print(f"tol {tol}: {r['status']} after {r['iters']} passes, KKT {r['kkt']:.2e}, obj {r['primal_obj']!r}, "
          f"planted {pstar!r}, rel {rel:.2e}")
    if tol >= 1e-4 or r["status"] == "converged":
        assert r["status"] == "converged" and ko["kkt"] <= tol * 1.01
        assert rel <= (5e-3 if tol >= 1e-4 else 1e-4), rel
    else:
        assert r["status"] == "iter_limit" and ko["kkt"] <= 1e-3


@pytest.mark.timeout(300)
@pytest.mark.parametrize("precision", [0, 1])
def test_mip20k_solved_to_1e4_is_a_valid_point(precision):
    """The 20k x 50k LP solved to relative KKT 1e-4 (the oracle's own solve
    at this size takes too long for a test): the oracle's KKT at the returned
    point passes, the reported objective is the oracle's evaluation there,
    and the objective lies within 5e-3 of the generator's planted optimum
    (measured 1.6e-3 in both precisions: a relative KKT of 1e-4 bounds the
    residuals relative to the norms of q and c, which here are large next
    to the objective)."""
    lp = lpgen.mip_like_lp(1)
    r, ko, Po, tau = _solve(lp, 1e-4, precision, 400000, variant=1, memory=10, kkt_every=64, dhat_mode=0)
    assert r["status"] == "converged", r["status"]
    assert ko["kkt"] <= 1e-4 * 1.01
    assert r["primal_obj"] == pytest.approx(ko["pobj"], rel=1e-6, abs=1e-9)
    pstar = lp.planted["pstar"]
    rel = abs(r["primal_obj"] - pstar) / (1.0 + abs(pstar))
    print(f"precision {precision}: obj {r['primal_obj']!r} after {r['iters']} passes, planted {pstar!r}, "
          f"rel {rel:.2e}")
    assert rel <= 5e-3, rel
