"""GPU parity at the edges of the input space, against the oracle:
  * the smallest and the largest Anderson memory (m_A = 1 and 16, the widest
    kernel instantiation), AA-PDHG and FAA-PDHG, both loop kernels;
  * an LP whose matrix has no entries (K = 0): the map reduces to projected
    gradient steps on c and the dual stays at its fixed point; the solve
    reaches the box minimum of c^T x."""
import numpy as np
import pytest

import lpgen
import oracle
from _util import err64

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2508_08062_amd")


def _pair(lp, steps, tau, loop_kernel, **kw):
    common = dict(tau=tau, sigma=tau, kkt_every=1, tol=0.0, max_iter=10 ** 6, **kw)
    g = P.Solver(lp, precision=1, loop_kernel=loop_kernel, **common)
    o = oracle.Solver(oracle.Problem.from_lpdata(lp), oracle.Options(**common))
    o.start()
    g.iterate(1)
    errs = []
    for _ in range(steps):
        o.step()
        g.iterate(1)
        st = g.get_state()
        errs.append(err64(st["u"], np.r_[o.state.x, o.state.y]))
        assert (st["i"], st["j"]) == (o.state.i, o.state.j)
    return errs, g


@pytest.mark.parametrize("loop_kernel", [0, 1])
@pytest.mark.parametrize("variant,memory", [(1, 1), (1, 16), (2, 16)])
def test_memory_extremes_fp64(variant, memory, loop_kernel):
    lp = lpgen.tiny_lp(5)
    tau = 0.9 / oracle.power_norm(oracle.Problem.from_lpdata(lp))
    errs, g = _pair(lp, 50, tau, loop_kernel, variant=variant, memory=memory)
    assert max(errs) < 1e-9, (max(errs), int(np.argmax(errs)))
    g.close()


def _empty_matrix_lp():
    m, n = 3, 5
    return lpgen.LPData(m=m, n=n, rowptr=np.zeros(m + 1, dtype=np.int64), colidx=np.zeros(0, dtype=np.int32),
                        val=np.zeros(0), c=np.array([1.0, -2.0, 0.5, -0.25, 0.0]),
                        q=np.array([0.0, 0.0, -1.0]),
                        l=np.array([-1.0, -np.inf, 0.0, -3.0, -np.inf]),
                        u=np.array([2.0, 4.0, np.inf, 1.0, np.inf]),
                        rowtype=np.array([0, 0, 1], dtype=np.uint8))


@pytest.mark.parametrize("loop_kernel", [0, 1])
def test_matrix_without_entries(loop_kernel):
    """The PDHG trajectory is compared pass by pass (AA on this LP solves
    nearly singular systems: its difference columns are collinear, x walks to
    its bounds in equal steps and y never moves, so rounding is amplified by
    1/eta); the AA solve must reach the box minimum."""
    lp = _empty_matrix_lp()
    errs, g = _pair(lp, 30, 0.5, loop_kernel, variant=0, memory=4)
    assert max(errs) < 1e-14, errs
    g.close()
    # the solve: x at the bound c pushes it to, y = 0, objective sum_j min over the box
    s = P.Solver(lp, precision=1, tol=1e-9, kkt_every=1, max_iter=1000, loop_kernel=loop_kernel)
    s.solve()
    r = s.result()
    assert r["status"] == "converged"
    np.testing.assert_allclose(r["x"][:4], [-1.0, 4.0, 0.0, 1.0], atol=1e-9)
    assert r["primal_obj"] == pytest.approx(-1.0 - 8.0 + 0.0 - 0.25, abs=1e-9)
    np.testing.assert_allclose(r["y"], 0.0, atol=1e-12)
    s.close()


def _cycle_difference_lp(m, c):
    # rows x_i - x_{i+1 mod m} = 0: every row sums to zero (K 1 = 0), ||K||_2 = 2 for even m
    K = np.eye(m) - np.roll(np.eye(m), 1, axis=1)
    rows, cols = np.nonzero(K)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rowptr[1:])
    return lpgen.LPData(m=m, n=m, rowptr=rowptr, colidx=cols.astype(np.int32), val=K[rows, cols],
                        c=np.asarray(c, float), q=np.zeros(m), l=np.zeros(m), u=np.full(m, 10.0),
                        rowtype=np.zeros(m, dtype=np.uint8))


@pytest.mark.parametrize("precision", [0, 1])
def test_step_size_when_the_rows_of_K_sum_to_zero(precision):
    """The power iteration starts from the SplitMix64 vector, not a constant
    one (orthogonal to every singular vector of this K with a nonzero
    singular value): tau = 0.9 / ||K||_2 = 0.45, and the solve reaches the
    closed-form optimum (all x_i equal, at the bound the cost pushes them to)."""
    m = 16  # 200 power steps reach ||K|| to 1e-8 here (the gap closes as m grows)
    for c, xstar in ((np.ones(m), 0.0), (-np.ones(m), 10.0)):
        s = P.Solver(_cycle_difference_lp(m, c), precision=precision, tol=1e-6, kkt_every=8, max_iter=20000)
        assert s.dims()["tau"] == pytest.approx(0.45, rel=1e-5)
        s.solve()
        r = s.result()
        assert r["status"] == "converged"
        np.testing.assert_allclose(r["x"], xstar, atol=1e-3)
        s.close()


def test_power_iteration_seed():
    lp = lpgen.tiny_lp(3)
    nrm = oracle.power_norm(oracle.Problem.from_lpdata(lp), iters=5000, rtol=1e-14)
    for seed in (0, 12345):
        s = P.Solver(lp, precision=1, seed=seed, power_iters=2000)
        assert s.dims()["tau"] == pytest.approx(0.9 / nrm, rel=1e-6)
        s.close()
