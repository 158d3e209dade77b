"""GPU parity of fixed-frequency restarted PDHG (the comparison method of
Section 5.2) against the oracle, through the C ABI: tiny LPs in float64
(iterates to 1e-9), the 2k x 5k LP in float32 (1e-5) over several epochs in
both loop kernels, the toy LP with the paper's restart length 75, an LP with
split rows and columns (the coherent epilogue path), restarts inside one
persistent launch against one-pass launches (bit for bit), and a solve
against the planted optimum."""
import numpy as np
import pytest

import lpgen
import oracle
from _util import err32, err64
from test_gpu_parity import _ragged_lp

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2508_08062_amd")

RP = 3  # restarted PDHG


def _run(lp, steps, precision, R, loop_kernel=0, tau=None, kkt_every=1):
    err = err64 if precision == 1 else err32
    Po = oracle.Problem.from_lpdata(lp)
    if tau is None:
        tau = 0.9 / oracle.power_norm(Po)
    common = dict(variant=RP, restart_period=R, memory=4, tau=tau, sigma=tau, kkt_every=kkt_every, tol=0.0,
                  max_iter=10 ** 6)
    g = P.Solver(lp, precision=precision, loop_kernel=loop_kernel, dhat_mode=1, **common)
    o = oracle.Solver(Po, oracle.Options(**common))
    o.start()
    g.iterate(1)
    errs = [err(g.get_state()["u"], np.r_[o.state.x, o.state.y])]
    for _ in range(steps):
        o.step()
        g.iterate(1)
        st = g.get_state()
        errs.append(err(st["u"], np.r_[o.state.x, o.state.y]))
        assert (st["i"], st["j"]) == (o.state.i, o.state.j) == (0, st["k"] - 1)
    return errs, g, o


@pytest.mark.parametrize("loop_kernel", [0, 1])
@pytest.mark.parametrize("seed", [0, 3])
def test_tiny_fp64_restarted_trajectory(seed, loop_kernel):
    errs, g, _ = _run(lpgen.tiny_lp(seed), 60, precision=1, R=7, loop_kernel=loop_kernel)
    assert max(errs) < 1e-9, (max(errs), int(np.argmax(errs)))
    g.close()


@pytest.mark.parametrize("loop_kernel", [0, 1])
def test_mip_like_fp32_restarted_trajectory(loop_kernel):
    lp = lpgen.mip_like_lp(11, m=2000, n=5000, nnz=25000)
    errs, g, _ = _run(lp, 50, precision=0, R=10, loop_kernel=loop_kernel)
    assert max(errs) < 1e-5, (max(errs), int(np.argmax(errs)))
    g.close()


def test_toy_restart_length_75():
    errs, g, o = _run(lpgen.toy_lp(), 225, precision=1, R=75, tau=0.1)
    assert max(errs) < 1e-12, max(errs)
    g.close()


def test_split_rows_restarted_fp64():
    errs, g, _ = _run(_ragged_lp(), 30, precision=1, R=6)
    assert max(errs) < 1e-9, errs
    g.close()


def test_restarts_inside_one_persistent_launch():
    lp = lpgen.mip_like_lp(13, m=2000, n=5000, nnz=25000)
    kw = dict(variant=RP, restart_period=9, precision=0, memory=4, kkt_every=64, tol=0.0, max_iter=10 ** 6)
    a = P.Solver(lp, **kw)
    b = P.Solver(lp, **kw)
    a.iterate(1)
    b.iterate(1)
    t = a.iterate_timed(100)
    assert t["kernel"] == "persistent"
    for _ in range(100):
        b.iterate(1)
    sa, sb = a.get_state(), b.get_state()
    assert sa["k"] == sb["k"] == 101
    np.testing.assert_array_equal(sa["u"], sb["u"])
    a.close()
    b.close()


def test_restarted_solve_matches_the_oracle_and_the_planted_optimum():
    """Each side solves to KKT 1e-6 and stops on its own; the objectives
    agree to 1e-6 relative.  The KKT test bounds the gap and the residuals,
    not the distance of c^T x to p* (a primal residual r moves it by up to
    about ||y*|| r): the restarted run stops 1.1e-5 from the planted optimum
    on both sides, so that check takes 100 tol."""
    lp = lpgen.tiny_lp(2)
    tol = 1e-6
    Po = oracle.Problem.from_lpdata(lp)
    tau = 0.9 / oracle.power_norm(Po)
    kw = dict(variant=RP, restart_period=64, tol=tol, kkt_every=16, max_iter=200000, tau=tau, sigma=tau)
    g = P.Solver(lp, precision=1, **kw)
    g.solve()
    r = g.result()
    o = oracle.Solver(Po, oracle.Options(**kw))
    ro = o.solve()
    assert r["status"] == ro["status"] == "converged"
    o_obj = ro["kkt"]["pobj"]
    assert abs(r["primal_obj"] - o_obj) / (1 + abs(o_obj)) <= 1e-6
    ps = lp.planted["pstar"]
    assert abs(r["primal_obj"] - ps) / (1 + abs(ps)) < 100 * tol
    assert r["aa_steps"] == 0
    g.close()


def test_restart_period_must_be_positive():
    with pytest.raises(P.AAPDHGError, match="restart_period"):
        P.Solver(lpgen.tiny_lp(1), variant=RP, restart_period=0)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_mixing_methods_equals_solo_runs(precision):
    """A batch whose members use AA-PDHG, restarted PDHG, AA-PDHG with primal
    weights and vanilla PDHG runs every member in the extended loop kernel;
    each member's iterate after 60 batch passes equals its solo run's bit for
    bit (the plain AA member's solo run uses the unextended kernel: with the
    LP's fixed steps and D-hat both compute the same values)."""
    specs = [(lpgen.tiny_lp(0), dict(variant=1)),
             (lpgen.tiny_lp(1), dict(variant=RP, restart_period=7)),
             (lpgen.tiny_lp(2), dict(variant=1, pw_period=8)),
             (lpgen.tiny_lp(3), dict(variant=0))]
    base = dict(precision=precision, memory=5, kkt_every=8, tol=0.0, max_iter=10 ** 6)
    solo = []
    for lp, kw in specs:
        s = P.Solver(lp, **base, **kw)
        s.iterate(1)
        s.iterate(60)
        solo.append(s.get_state()["u"])
        s.close()
    members = [P.Solver(lp, **base, **kw) for lp, kw in specs]
    b = P.Batch(members)
    b.iterate(60)  # a batch takes the members' init step before the 60 passes
    for g, ref in zip(members, solo):
        st = g.get_state()
        assert st["k"] == 61
        np.testing.assert_array_equal(st["u"], ref)
    b.close()
    for g in members:
        g.close()
