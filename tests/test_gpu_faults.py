"""Failure handling and recovery on the GPU, each condition forced from the
host (every kernel still runs on finite, in-range data or on NaN values,
never on bad indices):

  * checkpoint and resume: a state copied out with aapdhg_get_state and
    restored on a fresh handle continues bit for bit like the uninterrupted
    run (AA and FAA, both loop kernels);
  * a history whose difference columns are zero makes dG^T dG singular with
    eta = 0: the step is a PDHG step, as in the oracle loaded with the same
    state (failed factorisation -> PDHG step, the memory still updated);
  * an infeasible LP ends at the iteration limit with finite iterates, the
    same pass count and AA-step count as the oracle;
  * a NaN planted in the iterate stops the LP with the NUMERICAL status.
"""
import numpy as np
import pytest

import lpgen
import oracle
from _util import entrywise_err, norm_rel

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2508_08062_amd")


@pytest.mark.parametrize("loop_kernel", [0, 1])
@pytest.mark.parametrize("variant", [1, 2])
def test_checkpoint_resume_is_bitwise(variant, loop_kernel):
    lp = lpgen.mip_like_lp(21, m=1500, n=3500, nnz=20000)
    kw = dict(variant=variant, precision=0, memory=8, kkt_every=16, tol=0.0, max_iter=10 ** 6, ruiz_iters=10,
              loop_kernel=loop_kernel)
    a = P.Solver(lp, **kw)
    a.iterate(1)
    a.iterate(40)
    st = a.get_state()
    a.iterate(60)
    end = a.get_state()
    b = P.Solver(lp, **kw)
    b.iterate(1)
    b.set_state(st)
    b.iterate(60)
    got = b.get_state()
    assert (got["k"], got["i"], got["j"]) == (end["k"], end["i"], end["j"])
    np.testing.assert_array_equal(got["u"], end["u"])
    np.testing.assert_array_equal(got["g_prev"], end["g_prev"])
    a.close()
    b.close()


@pytest.mark.parametrize("loop_kernel", [0, 1])
def test_zero_history_takes_the_pdhg_branch(loop_kernel):
    lp = lpgen.tiny_lp(2)
    common = dict(variant=1, memory=3, D=1e300, eta=0.0, dhat_mode=0, beta=1.0, tau=0.05, sigma=0.05,
                  kkt_every=1, tol=0.0, max_iter=10 ** 6)
    g = P.Solver(lp, precision=1, loop_kernel=loop_kernel, **common)
    g.iterate(1)
    g.iterate(5)
    st = g.get_state()
    assert st["nlive"] == 3 and st["i"] == 5  # every step so far accelerated
    for t in st["live"]:
        st["W"][t] -= st["dG"][t]  # W = dU + beta D-hat dG with beta = 1, D-hat = I
        st["dG"][t] = 0.0
    st["G"][:] = 0.0
    st["rhs"][:] = 0.0
    g.set_state(st)
    # the oracle in the same state
    o = oracle.Solver(oracle.Problem.from_lpdata(lp), oracle.Options(**common))
    o.start()
    S = o.state
    n = lp.n
    S.k, S.i, S.j, S.n0 = st["k"], st["i"], st["j"], st["n0"]
    S.x, S.y = st["u"][:n].copy(), st["u"][n:].copy()
    S.u_prev, S.g_prev = st["u_prev"].copy(), st["g_prev"].copy()
    S.dG = [st["dG"][t].copy() for t in st["live"]]
    S.dU = [st["W"][t].copy() for t in st["live"]]
    o.step()
    assert o.last_branch == "pdhg"
    g.iterate(1)
    st2 = g.get_state()
    assert (st2["i"], st2["j"]) == (st["i"], st["j"] + 1) == (o.state.i, o.state.j)
    assert st2["nlive"] == 3  # the memory was still updated
    ref = np.r_[o.state.x, o.state.y]
    assert norm_rel(st2["u"], ref) < 1e-13 and entrywise_err(st2["u"], ref, 1e-3) < 1e-12
    g.close()


def _infeasible_lp():
    # x0 + x1 = 1 and x0 + x1 = 3 with 0 <= x <= 10
    K = np.array([[1.0, 1.0], [1.0, 1.0]])
    rows, cols = np.nonzero(K)
    return lpgen.LPData(m=2, n=2, rowptr=np.array([0, 2, 4], dtype=np.int64), colidx=cols.astype(np.int32),
                        val=K[rows, cols], c=np.array([1.0, 1.0]), q=np.array([1.0, 3.0]), l=np.zeros(2),
                        u=np.full(2, 10.0), rowtype=np.zeros(2, dtype=np.uint8))


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_infeasible_lp_ends_at_the_iteration_limit(variant, precision):
    lp = _infeasible_lp()
    common = dict(variant=variant, memory=5, tau=0.2, sigma=0.2, kkt_every=16, tol=1e-6, max_iter=3000)
    g = P.Solver(lp, precision=precision, **common)
    g.solve()
    r = g.result()
    o = oracle.Solver(oracle.Problem.from_lpdata(lp), oracle.Options(**common))
    ro = o.solve()
    assert r["status"] == ro["status"] == "iter_limit"
    assert r["iters"] == ro["k"] == 3001
    assert r["aa_steps"] == ro["aa_steps"]
    assert np.all(np.isfinite(r["x"])) and np.all(np.isfinite(r["y"]))
    # the dual iterate drifts along the infeasibility ray to |y| ~ 600; in
    # float32 each pass rounds an increment of about 0.4 at that magnitude
    # (ulp 6e-5), and 3000 passes (AA steps among them) accumulate it
    tol = 1e-9 if precision == 1 else 5e-3
    assert norm_rel(r["y"], ro["y"]) < tol and entrywise_err(r["y"], ro["y"], 1.0) < tol
    g.close()


@pytest.mark.parametrize("loop_kernel", [0, 1])
def test_nan_in_the_iterate_stops_with_numerical_status(loop_kernel):
    lp = lpgen.tiny_lp(4)
    g = P.Solver(lp, precision=1, loop_kernel=loop_kernel, kkt_every=8, tol=0.0, max_iter=10 ** 6)
    g.iterate(1)
    g.iterate(10)
    st = g.get_state()
    st["u"][3] = np.nan
    g.set_state(st)
    g.iterate(5)
    st2 = g.get_state()
    assert st2["status"] == 3  # AAPDHG_NUMERICAL
    assert st2["k"] == st["k"]  # stopped at the pass that saw the NaN residual
    r = g.result()
    assert r["status"] == "numerical"
    g.close()
