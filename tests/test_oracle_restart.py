"""Pins of the oracle's fixed-frequency restarted PDHG (the toy comparison
of Section 5.2): special cases that reduce to vanilla PDHG, the epoch
averages on the toy LP in closed form (its PDHG map is affine while x > 0),
and the toy behaviour the paper describes (restarts move the iterate to the
solution far faster than vanilla PDHG)."""
import numpy as np
import pytest

import lpgen
import oracle


def _traj(s, iters):
    s.start()
    out = [np.r_[s.state.x, s.state.y]]
    for _ in range(iters):
        s.step()
        out.append(np.r_[s.state.x, s.state.y])
    return np.array(out)


@pytest.mark.parametrize("R", [1, 1000])
def test_restart_every_iterate_or_never_is_vanilla_pdhg(R):
    P = oracle.Problem.from_lpdata(lpgen.tiny_lp(3))
    base = dict(kkt_every=0, tau=0.05, sigma=0.05)
    a = _traj(oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_PDHG, **base)), 120)
    s = oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_RPDHG, restart_period=R, **base))
    b = _traj(s, 120)
    np.testing.assert_array_equal(a, b)
    assert s.state.i == 0 and s.state.j == s.state.k - 1


@pytest.mark.parametrize("R", [5, 75])
def test_toy_epoch_averages_in_closed_form(R):
    """Toy LP (min 0 s.t. x = 3, x >= 0; tau = sigma = 0.1): while x > 0 one
    PDHG step is z -> A z + b with A = [[1, tau], [-sigma, 1 - 2 sigma tau]],
    b = (0, 3 sigma) (eq. pdhg with c = 0, K = 1, q = 3), fixed point (3, 0).
    Epoch e holds z_{eR+1}, ..., z_{(e+1)R}; its last iterate becomes the
    epoch's average, from which the next epoch starts."""
    t = s_ = 0.1
    A = np.array([[1.0, t], [-s_, 1.0 - 2.0 * s_ * t]])
    zs = np.array([3.0, 0.0])
    P = oracle.Problem.from_lpdata(lpgen.toy_lp())
    o = oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_RPDHG, restart_period=R, kkt_every=0,
                                        tau=t, sigma=s_))
    traj = _traj(o, 3 * R)  # traj[j] = u^{j+1}
    z = np.array([0.0, 0.3])  # u^1 = T u^0 (hand trace of the toy)
    for e in range(3):
        pts = [z]
        for _ in range(R - 1):
            pts.append(zs + A @ (pts[-1] - zs))
        pts = np.array(pts)
        assert np.all(pts[:, 0] + t * pts[:, 1] > 0)  # the projection is inactive
        np.testing.assert_allclose(traj[e * R:(e + 1) * R - 1], pts[:-1], rtol=1e-12, atol=1e-14)
        avg = pts.mean(axis=0)
        np.testing.assert_allclose(traj[(e + 1) * R - 1], avg, rtol=1e-12, atol=1e-14)
        z = zs + A @ (avg - zs)


def test_toy_restarts_reach_the_solution_faster_than_vanilla():
    P = oracle.Problem.from_lpdata(lpgen.toy_lp())
    kw = dict(kkt_every=0, tau=0.1, sigma=0.1)
    r = _traj(oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_RPDHG, restart_period=75, **kw)), 750)
    v = _traj(oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_PDHG, **kw)), 750)
    zs = np.array([3.0, 0.0])
    dr = np.linalg.norm(r[-1] - zs)
    dv = np.linalg.norm(v[-1] - zs)
    assert dr < 0.1 * dv, (dr, dv)
    # restarts are where the distance drops: the epoch ends are closer than the epoch middles
    ends = [np.linalg.norm(r[75 * e - 1] - zs) for e in range(1, 11)]
    assert all(b < a for a, b in zip(ends, ends[1:]))
