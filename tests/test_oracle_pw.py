"""Pins of the oracle's primal-weight update (Alg 7), its D-hat re-blend
(remark on the primal-weight form) and the Iter_AA / c safeguard, against
facts that do not come from the oracle's own formulas: a hand-written PDHG
loop with the weight in geometric-mean form, equivariance of weighted PDHG
under a scaling of the primal variables, the epsilon_zero gate, the memory
reset, and the ordering of the safeguard bounds."""
import math

import numpy as np
import pytest

import lpgen
import oracle


def _problem(seed=3):
    return oracle.Problem.from_lpdata(lpgen.tiny_lp(seed))


def _traj(s, iters):
    s.start()
    out = [np.r_[s.state.x, s.state.y]]
    for _ in range(iters):
        s.step()
        out.append(np.r_[s.state.x, s.state.y])
    return np.array(out)


def test_period_beyond_the_run_changes_nothing():
    P = _problem()
    base = dict(variant=oracle.VARIANT_AA, kkt_every=0, tau=0.05, sigma=0.05, memory=5)
    a = _traj(oracle.Solver(P, oracle.Options(**base)), 40)
    b = _traj(oracle.Solver(P, oracle.Options(**base, pw_period=1000)), 40)
    np.testing.assert_array_equal(a, b)


def test_weighted_pdhg_matches_a_hand_loop():
    """Vanilla PDHG with the weight update: T with tau = gamma/omega,
    sigma = gamma*omega, omega' = (dy/dx)^theta omega^(1-theta) at every U_P-th
    iterate, distances to the iterate of the previous check."""
    P = _problem(5)
    tau = sigma = 0.04
    U, theta, iters = 7, 0.5, 50
    s = oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_PDHG, kkt_every=0, tau=tau, sigma=sigma,
                                        pw_period=U, pw_theta=theta))
    got = _traj(s, iters)
    # the hand loop
    x = np.clip(np.zeros(P.n), P.l, P.u)
    y = np.zeros(P.m)
    A = P.K.toarray()
    gam, om = math.sqrt(tau * sigma), 1.0
    t, sg = tau, sigma

    def T(x, y, t, sg):
        xh = np.clip(x - t * (P.c - A.T @ y), P.l, P.u)
        yh = y + sg * (P.q - A @ (2 * xh - x))  # every row is an equality row
        return xh, yh

    anchor = np.r_[x, y]
    x, y = T(x, y, t, sg)
    want = [np.r_[x, y]]
    omegas = []
    for k in range(1, iters + 1):
        if k % U == 0:
            dx = np.linalg.norm(x - anchor[:P.n])
            dy = np.linalg.norm(y - anchor[P.n:])
            anchor = np.r_[x, y]
            if dx > 1e-10 and dy > 1e-10:
                om = (dy / dx) ** theta * om ** (1 - theta)
                t, sg = gam / om, gam * om
                omegas.append(om)
        x, y = T(x, y, t, sg)
        want.append(np.r_[x, y])
    np.testing.assert_allclose(got, np.array(want), rtol=1e-10, atol=1e-12)
    assert len(omegas) == iters // U
    np.testing.assert_allclose([e[4] for e in s.pw_log], omegas, rtol=1e-12)


def test_weighted_pdhg_is_equivariant_under_primal_scaling():
    """x = s x~ maps the LP to K~ = s K, c~ = s c, bounds / s; PDHG on it with
    gamma / s and omega^0 s follows x^k / s, y^k, and the update keeps
    omega~ = s omega (the weight measures the primal scale)."""
    P = _problem(6)
    sc = 4.0
    Ps = oracle.Problem(P.m, P.n, P.K.indptr, P.K.indices, sc * P.K.data, sc * P.c, P.q, P.l / sc, P.u / sc,
                        P.rowtype)
    kw = dict(variant=oracle.VARIANT_PDHG, kkt_every=0, pw_period=5, pw_theta=0.5)
    a = oracle.Solver(P, oracle.Options(**kw, tau=0.05, sigma=0.05))
    b = oracle.Solver(Ps, oracle.Options(**kw, tau=0.05 / sc, sigma=0.05 / sc, pw_omega0=sc))
    ta, tb = _traj(a, 45), _traj(b, 45)
    n = P.n
    np.testing.assert_allclose(tb[:, :n] * sc, ta[:, :n], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(tb[:, n:], ta[:, n:], rtol=1e-9, atol=1e-12)
    assert len(a.pw_log) == 9 and all(e[3] for e in a.pw_log)
    np.testing.assert_allclose([e[4] for e in b.pw_log], [sc * e[4] for e in a.pw_log], rtol=1e-12)


def test_zero_motion_gate_leaves_weight_and_memory_alone():
    """With every column fixed (l = u) x never moves: dx = 0 <= eps_zero, so no
    update is accepted and AA runs exactly as without the weight update."""
    lp = lpgen.tiny_lp(2)
    P0 = oracle.Problem.from_lpdata(lp)
    fix = np.full(P0.n, 1.5)
    P = oracle.Problem(P0.m, P0.n, P0.K.indptr, P0.K.indices, P0.K.data, P0.c, P0.q, fix, fix, P0.rowtype)
    base = dict(variant=oracle.VARIANT_AA, kkt_every=0, tau=0.05, sigma=0.05, memory=5)
    a = _traj(oracle.Solver(P, oracle.Options(**base)), 40)
    s = oracle.Solver(P, oracle.Options(**base, pw_period=6))
    b = _traj(s, 40)
    np.testing.assert_array_equal(a, b)
    assert len(s.pw_log) == 6 and not any(e[3] for e in s.pw_log)
    assert all(e[1] == 0.0 and e[2] > 0.0 for e in s.pw_log)


def test_accepted_update_resets_memory_and_reblends_dhat():
    P = _problem(7)
    U = 10
    s = oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_AA, kkt_every=0, tau=0.05, sigma=0.05, memory=5,
                                        pw_period=U, dhat_mode=0))
    s.start()
    for _ in range(U - 1):
        s.step()
    assert len(s.state.dU) == 5
    r_prev = float(np.linalg.norm(s.state.g_prev))
    s.step()  # iteration U: update accepted, no pair formed
    assert s.pw_log[-1][3]
    assert len(s.state.dU) == 0
    om = s.omega
    # with D-hat = I the blend is diag(1/omega, omega) for either alpha
    np.testing.assert_allclose(s.Dhat[:P.n], 1.0 / om, rtol=1e-15)
    np.testing.assert_allclose(s.Dhat[P.n:], om, rtol=1e-15)
    alpha = s.pw_log[-1][5]
    assert alpha == (0.1 if s.last_gnorm < r_prev else 0.9)
    s.step()
    assert len(s.state.dU) == 1
    assert s.state.i + s.state.j == s.state.k - 1


def test_dhat_blend_keeps_construction_between_weight_scalings():
    """With the literal D-hat the blended diagonal times the weight scaling
    (omega on the x part, 1/omega on the y part) lies between 1 and D-hat_0,
    at the alpha chosen by the residual test."""
    P = _problem(8)
    s = oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_AA, kkt_every=0, tau=0.05, sigma=0.05, memory=5,
                                        pw_period=9, dhat_mode=1))
    s.start()
    for _ in range(9):
        s.step()
    om, alpha = s.omega, s.pw_log[-1][5]
    d0 = s.Dhat0
    t = np.r_[s.Dhat[:P.n] * om, s.Dhat[P.n:] / om]
    lo, hi = np.minimum(1.0, d0), np.maximum(1.0, d0)
    assert np.all(t >= lo * (1 - 1e-15)) and np.all(t <= hi * (1 + 1e-15))
    # the point on the segment from 1 to D-hat_0 is alpha of the way
    moved = np.abs(d0 - 1.0) > 1e-6
    np.testing.assert_allclose((t[moved] - 1.0) / (d0[moved] - 1.0), alpha, rtol=1e-12)


def test_theta_zero_keeps_the_steps():
    P = _problem(9)
    s = oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_AA, kkt_every=0, tau=0.05, sigma=0.05,
                                        pw_period=5, pw_theta=0.0, pw_dhat=False))
    _traj(s, 30)
    assert all(e[3] for e in s.pw_log)
    assert s.omega == 1.0 and s.opt.tau == 0.05 and s.opt.sigma == 0.05
    np.testing.assert_array_equal(s.Dhat, s.Dhat0)


def test_sg_div_one_is_the_default_safeguard():
    P = _problem(4)
    base = dict(variant=oracle.VARIANT_AA, kkt_every=0, tau=0.05, sigma=0.05, D=2.0)
    a = _traj(oracle.Solver(P, oracle.Options(**base)), 60)
    b = _traj(oracle.Solver(P, oracle.Options(**base, sg_div=1.0)), 60)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("seed", [1, 4, 6])
def test_larger_sg_div_accepts_first_where_the_runs_part(seed):
    """(i/c + 1)^{-(1+eps)} >= (i + 1)^{-(1+eps)} for c >= 1: while the two runs
    agree they take the same branches, and the first step where they differ is
    one that the c = 3 run accelerates and the c = 1 run does not."""
    P = _problem(seed)
    base = dict(variant=oracle.VARIANT_AA, kkt_every=0, tau=0.05, sigma=0.05, D=1.0)
    a = oracle.Solver(P, oracle.Options(**base))
    b = oracle.Solver(P, oracle.Options(**base, sg_div=3.0))
    a.start(); b.start()
    parted = False
    for _ in range(400):
        a.step(); b.step()
        if a.last_branch != b.last_branch:
            assert b.last_branch == "aa" and a.last_branch == "pdhg"
            parted = True
            break
        np.testing.assert_array_equal(np.r_[a.state.x, a.state.y], np.r_[b.state.x, b.state.y])
    assert parted
