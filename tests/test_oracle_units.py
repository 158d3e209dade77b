"""Pins of the CPU oracle against facts fixed by the paper or by mathematics
(hand-derived traces, closed forms, lemmas, a second algorithm)."""
import math

import numpy as np
import pytest

import lpgen
import oracle
from _util import golden, lp_from_dense


# ---------------------------------------------------------------------------
# the toy LP of Section 5.2, traced by hand
# ---------------------------------------------------------------------------

def test_toy_first_steps_match_hand_trace():
    g = golden("toy_lp.json")
    P = oracle.Problem.from_lpdata(lpgen.toy_lp())
    s = oracle.Solver(P, oracle.Options(tau=g["tau"], sigma=g["sigma"], memory=5, D=10.0,
                                        eps_sg=1.0, eta=1e-10, kkt_every=0, max_iter=10))
    st = s.start()
    np.testing.assert_allclose(np.r_[st.x, st.y], g["u1"], atol=1e-15)
    np.testing.assert_allclose(st.g_prev, g["g0"], atol=1e-15)
    xh, yh = oracle.pdhg_map(P, st.x, st.y, g["tau"], g["sigma"])
    np.testing.assert_allclose(np.r_[xh, yh], g["T_u1"], atol=1e-15)
    s.step()
    st = s.state
    np.testing.assert_allclose(st.dU[0], g["dU0"], atol=1e-15)
    np.testing.assert_allclose(st.dG[0], g["dG0"], atol=1e-15)
    np.testing.assert_allclose(st.g_prev, g["g1"], atol=1e-15)
    assert s.last_branch == "aa"
    np.testing.assert_allclose(s.last_gamma[0], g["gamma"], rtol=1e-6)
    np.testing.assert_allclose(np.r_[st.x, st.y], g["u2"], rtol=1e-6)


def test_toy_reaches_optimum_in_a_few_aa_steps():
    # Section 5.2: AA-PDHG reaches (3,0) in a few iterations; while x > 0 the map
    # is affine and AA behaves like GMRES on a 2-dimensional problem.
    g = golden("toy_lp.json")
    P = oracle.Problem.from_lpdata(lpgen.toy_lp())
    res, s = oracle.solve(P, tau=0.1, sigma=0.1, memory=5, tol=1e-10, kkt_every=1, max_iter=20)
    assert res["status"] == "converged"
    assert res["k"] <= 5
    np.testing.assert_allclose(np.r_[res["x"], res["y"]], g["optimum"], atol=1e-9)


# ---------------------------------------------------------------------------
# KKT residual and D-hat: hand-computed cases
# ---------------------------------------------------------------------------

def _kkt_lp():
    g = golden("kkt_cases.json")["lp"]
    return oracle.Problem.from_lpdata(lp_from_dense(g["dense_K"], g["q"], g["c"], g["l"], g["u"], g["rowtype"]))


@pytest.mark.parametrize("case", [0, 1])
def test_kkt_hand_cases(case):
    g = golden("kkt_cases.json")["cases"][case]
    P = _kkt_lp()
    r = oracle.kkt(P, np.array(g["x"], float), np.array(g["y"], float))
    for key in ("pobj", "dobj", "r_g", "r_p", "r_d"):
        assert r[key] == pytest.approx(g[key], rel=1e-14, abs=1e-15), key
    np.testing.assert_allclose(r["lam"], g["lam"], atol=0)
    assert r["kkt"] == pytest.approx(max(g["r_g"], g["r_p"], g["r_d"]), rel=1e-14)


def test_dhat_hand_case():
    g = golden("kkt_cases.json")["dhat"]
    P = _kkt_lp()
    np.testing.assert_allclose(oracle.dhat(P, 1), g["literal"], rtol=1e-15)
    np.testing.assert_allclose(oracle.dhat(P, 2), 1.0 / np.array(g["literal"]), rtol=1e-15)
    np.testing.assert_array_equal(oracle.dhat(P, 0), np.ones(7))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_kkt_zero_at_planted_optimum(seed):
    lp = lpgen.tiny_lp(seed)
    P = oracle.Problem.from_lpdata(lp)
    r = oracle.kkt(P, lp.planted["x"], lp.planted["y"])
    assert r["kkt"] < 1e-12
    assert r["pobj"] == pytest.approx(lp.planted["pstar"], rel=1e-12)


def test_kkt_zero_at_planted_optimum_mixed_bounds():
    lp = lpgen.mip_like_lp(5, m=300, n=700, nnz=3000, fp32=False)
    P = oracle.Problem.from_lpdata(lp)
    r = oracle.kkt(P, lp.planted["x"], lp.planted["y"])
    assert r["kkt"] < 1e-12
    np.testing.assert_allclose(r["lam"], lp.planted["s"], atol=1e-12)


def test_projections():
    P = _kkt_lp()
    x = np.array([-5.0, 5.0, -5.0, 5.0, 7.0])
    np.testing.assert_array_equal(oracle.proj_X(P, x), [-5.0, 2.0, 1.0, 3.0, 7.0])
    np.testing.assert_array_equal(oracle.proj_Y(P, np.array([-1.0, -1.0])), [-1.0, 0.0])
    lam = np.array([1.0, 1.0, -1.0, -1.0, 1.0])
    np.testing.assert_array_equal(oracle.proj_Lambda(P, lam), [0.0, 0.0, 0.0, -1.0, 0.0])


# ---------------------------------------------------------------------------
# the AA update against Alg 1 (standard type-II AA, constrained alpha form)
# ---------------------------------------------------------------------------

def _alg1_alpha(Gcols):
    """argmin ||G alpha|| s.t. sum alpha = 1, by the Lagrange system (a second,
    independent formula for the same least-squares problem)."""
    G = np.stack(Gcols, axis=1)
    k = G.shape[1]
    A = np.zeros((k + 1, k + 1))
    A[:k, :k] = 2.0 * G.T @ G
    A[:k, k] = 1.0
    A[k, :k] = 1.0
    rhs = np.zeros(k + 1)
    rhs[k] = 1.0
    return np.linalg.solve(A, rhs)[:k]


def test_difference_form_equals_alg1_alpha_form():
    # Free variables and equality rows: the projections are inactive and T is
    # affine.  With D-hat = I, beta = 1, eta = 0 and the safeguard always passed,
    # Alg 2's u^{k+1} must equal Alg 1's sum_i alpha_i T(u^i) over the window.
    rng = np.random.default_rng(7)
    m, n = 4, 9
    K = rng.standard_normal((m, n))
    lp = lp_from_dense(K, rng.standard_normal(m), rng.standard_normal(n),
                       ["-inf"] * n, ["inf"] * n, [0] * m)
    P = oracle.Problem.from_lpdata(lp)
    nrm = np.linalg.norm(K, 2)
    mem = 3
    s = oracle.Solver(P, oracle.Options(tau=0.5 / nrm, sigma=0.5 / nrm, memory=mem, D=1e300,
                                        eta=0.0, dhat_mode=0, beta=1.0, kkt_every=0))
    s.start()
    us = [s.state.u_prev, np.r_[s.state.x, s.state.y]]
    gs = [s.state.g_prev]
    for _ in range(8):
        u_k = np.r_[s.state.x, s.state.y]
        s.step()
        assert s.last_branch == "aa"
        gs.append(s.state.g_prev)  # g^k
        mk = min(mem, len(gs) - 1)
        window = list(range(len(gs) - 1 - mk, len(gs)))
        alpha = _alg1_alpha([gs[t] for t in window])
        expect = sum(a * (us[t] + gs[t]) for a, t in zip(alpha, window))
        got = np.r_[s.state.x, s.state.y]
        np.testing.assert_allclose(got, expect, rtol=1e-8, atol=1e-10)
        us.append(got)
        assert np.allclose(u_k, us[-2])


def test_difference_form_equals_alpha_form_with_dhat_and_damping():
    """The same equivalence with a mixing matrix: for D-hat != I (literal
    reading on a dense K with uneven magnitudes) and beta = 0.7, the AA step
    must equal sum_i alpha_i (u^i + beta D-hat g^i), the type-II Anderson
    step with mixing beta D-hat written in Alg 1's constrained form."""
    rng = np.random.default_rng(11)
    m, n = 5, 8
    K = rng.standard_normal((m, n)) * rng.uniform(0.1, 10.0, (m, 1)) * rng.uniform(0.1, 10.0, (1, n))
    lp = lp_from_dense(K, rng.standard_normal(m), rng.standard_normal(n),
                       ["-inf"] * n, ["inf"] * n, [0] * m)
    P = oracle.Problem.from_lpdata(lp)
    nrm = np.linalg.norm(K, 2)
    mem, beta = 3, 0.7
    s = oracle.Solver(P, oracle.Options(tau=0.5 / nrm, sigma=0.5 / nrm, memory=mem, D=1e300,
                                        eta=0.0, dhat_mode=1, beta=beta, kkt_every=0))
    D = s.Dhat
    assert np.ptp(D) > 1.0  # a genuinely non-identity D-hat
    s.start()
    us = [s.state.u_prev, np.r_[s.state.x, s.state.y]]
    gs = [s.state.g_prev]
    for _ in range(6):
        s.step()
        assert s.last_branch == "aa"
        gs.append(s.state.g_prev)
        mk = min(mem, len(gs) - 1)
        window = list(range(len(gs) - 1 - mk, len(gs)))
        alpha = _alg1_alpha([gs[t] for t in window])
        expect = sum(a * (us[t] + beta * D * gs[t]) for a, t in zip(alpha, window))
        got = np.r_[s.state.x, s.state.y]
        np.testing.assert_allclose(got, expect, rtol=1e-7, atol=1e-9)
        us.append(got)


# ---------------------------------------------------------------------------
# vanilla PDHG: firm non-expansiveness (Thm th:pdhg-residual-0)
# ---------------------------------------------------------------------------

def _m_norm_sq(P, g, tau, sigma):
    gx, gy = g[:P.n], g[P.n:]
    return gx @ gx / tau + gy @ gy / sigma + 2.0 * gy @ (P.K @ gx)


@pytest.mark.parametrize("seed", [0, 3])
def test_pdhg_residual_monotone_in_M_norm(seed):
    lp = lpgen.mip_like_lp(seed, m=60, n=150, nnz=700, fp32=False)
    P = oracle.Problem.from_lpdata(lp)
    nrm = np.linalg.norm(lpgen.to_dense(lp), 2)
    tau = sigma = 0.9 / nrm
    s = oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_PDHG, tau=tau, sigma=sigma, kkt_every=0))
    s.start()
    prev = _m_norm_sq(P, s.state.g_prev, tau, sigma)
    assert prev > 0
    for _ in range(400):
        s.step()
        cur = _m_norm_sq(P, s.state.g_prev, tau, sigma)
        assert cur <= prev * (1 + 1e-12) + 1e-300
        prev = cur


# ---------------------------------------------------------------------------
# safeguard and counters (Alg 2; Lemma le-AA-use-inifite)
# ---------------------------------------------------------------------------

def test_D_zero_is_vanilla_pdhg_and_counters_add_up():
    lp = lpgen.tiny_lp(3)
    P = oracle.Problem.from_lpdata(lp)
    a = oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_AA, D=0.0, kkt_every=0, tau=0.05, sigma=0.05))
    b = oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_PDHG, kkt_every=0, tau=0.05, sigma=0.05))
    a.start(); b.start()
    for k in range(60):
        a.step(); b.step()
        np.testing.assert_array_equal(np.r_[a.state.x, a.state.y], np.r_[b.state.x, b.state.y])
        assert a.state.i + a.state.j == a.state.k - 1
    assert a.state.i == 0


def test_infinite_D_always_accelerates_and_counters_add_up():
    lp = lpgen.tiny_lp(4)
    P = oracle.Problem.from_lpdata(lp)
    s = oracle.Solver(P, oracle.Options(D=math.inf, kkt_every=0, tau=0.05, sigma=0.05))
    s.start()
    for _ in range(40):
        s.step()
        assert s.last_branch == "aa"
        assert s.state.i + s.state.j == s.state.k - 1
    assert s.state.j == 0


def test_aa_used_infinitely_often_on_convergent_run():
    lp = lpgen.tiny_lp(0)
    P = oracle.Problem.from_lpdata(lp)
    s = oracle.Solver(P, oracle.Options(D=10.0, kkt_every=0))
    s.start()
    seen = []
    for _ in range(6000):
        s.step()
        seen.append(s.last_branch == "aa")
    # AA steps keep appearing late in the run
    assert any(seen[-1500:])


def test_memory_window_and_singular_history_falls_back():
    # a zero difference column makes dG^T dG + 0 I singular: the step is PDHG
    # (reading: failed factorisation -> PDHG step; memory still updated)
    P = oracle.Problem.from_lpdata(lpgen.tiny_lp(2))
    s = oracle.Solver(P, oracle.Options(D=math.inf, eta=0.0, kkt_every=0, memory=3, tau=0.05, sigma=0.05))
    s.start()
    for _ in range(5):
        s.step()
        assert len(s.state.dU) <= 3
    s.state.dG = [np.zeros_like(c) for c in s.state.dG]
    before_j = s.state.j
    s.step()
    assert s.last_branch == "pdhg" and s.state.j == before_j + 1
    assert len(s.state.dG) == 3


# ---------------------------------------------------------------------------
# FAA filters (Alg 4-6; Lemmas eq:lemma1.51, le:RK-1bound1,
# lem:conditioning_after_stab)
# ---------------------------------------------------------------------------

def _angled_columns(rng, N, m, cs):
    """Columns whose sine against the span of the previous ones is >= cs."""
    F = np.zeros((N, m))
    F[:, 0] = rng.standard_normal(N) * rng.uniform(0.1, 10)
    for i in range(1, m):
        while True:
            v = rng.standard_normal(N) * rng.uniform(0.1, 10)
            Q, _ = np.linalg.qr(F[:, :i])
            perp = v - Q @ (Q.T @ v)
            if np.linalg.norm(perp) / np.linalg.norm(v) >= cs:
                break
        F[:, i] = v
    return F


@pytest.mark.parametrize("seed", range(5))
def test_length_bounds_dominate_columns_of_R_inverse(seed):
    rng = np.random.default_rng(seed)
    cs = 0.2
    F = _angled_columns(rng, 30, 7, cs)
    _, R = np.linalg.qr(F)
    Rinv = np.linalg.inv(R)
    b = oracle.length_bounds(np.linalg.norm(F, axis=0), cs)
    col_sq = np.sum(Rinv ** 2, axis=0)
    assert np.all(col_sq <= b * (1 + 1e-10))
    assert col_sq[0] == pytest.approx(b[0], rel=1e-10)  # b_1 is exact


@pytest.mark.parametrize("cs", [0.2, 0.5])
def test_length_bounds_hold_on_extremal_angles(cs):
    """Three unit columns, each at exactly the smallest allowed sine cs from
    the span of the ones before it, with the off-diagonal part of the third
    turned by theta: R = [[1, ct, -ct sin t], [0, cs, ct cos t], [0, 0, cs]].
    The squared norm of column 3 of R^{-1} then reaches 83% (cs = 0.2) and
    69% (cs = 0.5) of b_3, so the bound is checked where it is close to
    tight."""
    ct = math.sqrt(1.0 - cs * cs)
    worst = 0.0
    for t in np.linspace(-np.pi, np.pi, 721):
        F = np.array([[1.0, ct, -ct * math.sin(t)], [0.0, cs, ct * math.cos(t)], [0.0, 0.0, cs]])
        _, R = np.linalg.qr(F)
        col_sq = np.sum(np.linalg.inv(R) ** 2, axis=0)
        b = oracle.length_bounds(np.linalg.norm(F, axis=0), cs)
        assert np.all(col_sq <= b * (1 + 1e-12))
        worst = max(worst, col_sq[2] / b[2])
    assert worst > 0.5  # the construction does press on the bound


@pytest.mark.parametrize("cs", [0.2, 0.5, 0.9])
def test_length_bound_b2_is_attained(cs):
    """The second bound is tight: with r_11 = ||f_1||, r_12 = ct ||f_2|| and
    r_22 = cs ||f_2|| (ct = sqrt(1 - cs^2), the largest off-diagonal entry the
    angle condition allows), column 2 of R^{-1} has squared norm
    ct^2 / (cs^2 ||f_1||^2) + 1 / (cs^2 ||f_2||^2), which the bound must equal.
    The inverse is taken numerically from the constructed columns."""
    f1, f2 = 3.0, 0.25
    ct = math.sqrt(1.0 - cs * cs)
    F = np.array([[f1, ct * f2], [0.0, cs * f2], [0.0, 0.0]])
    _, R = np.linalg.qr(F)
    col2 = float(np.sum(np.linalg.inv(R)[:, 1] ** 2))
    b = oracle.length_bounds(np.linalg.norm(F, axis=0), cs)
    assert b[1] == pytest.approx(col2, rel=1e-12)


def _entry_bounds(fnorm, cs):
    """The entrywise bounds of Lemma eq:lemma1.51 on |s_ij|, s = R^{-1}, as an
    upper-triangular table (1-based i <= j in the lemma, 0-based here):
    s_11 = 1 / ||f_1||; |s_1j| <= ct (ct + cs)^(j-2) / (||f_1|| cs^(j-1)) for
    j >= 2; s_ii <= 1 / (||f_i|| cs) for i >= 2; and
    |s_ij| <= ct (ct + cs)^(j-i-1) / (||f_i|| cs^(j-i+1)) for 2 <= i < j."""
    ct = math.sqrt(1.0 - cs * cs)
    m = len(fnorm)
    B = np.zeros((m, m))
    for i in range(1, m + 1):
        for j in range(i, m + 1):
            if i == 1 and j == 1:
                v = 1.0 / fnorm[0]
            elif i == 1:
                v = ct * (ct + cs) ** (j - 2) / (fnorm[0] * cs ** (j - 1))
            elif i == j:
                v = 1.0 / (fnorm[i - 1] * cs)
            else:
                v = ct * (ct + cs) ** (j - i - 1) / (fnorm[i - 1] * cs ** (j - i + 1))
            B[i - 1, j - 1] = v
    return B


@pytest.mark.parametrize("cs", [0.05, 0.2, 0.5, 0.9, 1.0])
def test_length_bounds_are_the_squared_entry_bounds_summed(cs):
    """Lemma le:RK-1bound1 bounds the squared norm of column j of R^{-1} by
    b_j; Lemma eq:lemma1.51 bounds each entry s_ij of that column.  The
    column's squared norm is the sum of its squared entries, so b_j must be
    the sum over i <= j of the squared entry bounds, for every j (here up to
    16, the largest memory) and any column norms.  This second formula comes
    from the entrywise lemma, not from the printed b_j, and fixes every power
    of ct, (ct + cs) and cs in b_j."""
    rng = np.random.default_rng(int(cs * 1000))
    for trial in range(4):
        fnorm = rng.uniform(0.05, 20.0, size=16)
        b = oracle.length_bounds(fnorm, cs)
        B = _entry_bounds(fnorm, cs)
        ref = np.sum(B ** 2, axis=0)
        np.testing.assert_allclose(b, ref, rtol=4e-15, atol=0.0)


@pytest.mark.parametrize("cs", [0.2, 0.5, 0.9])
def test_entry_bounds_attained_on_a_bidiagonal_chain(cs):
    """Columns f_1 = ||f_1|| e_1 and, for i >= 2, f_i = ||f_i|| (ct e_{i-1} +
    cs e_i) satisfy the hypotheses of Lemma eq:lemma1.51 with equality in the
    sine condition (each f_i is at sine exactly cs from the span of the ones
    before it, and its cosines with them are ct cs, ct or 0).  Their R is
    bidiagonal, and the diagonal and first superdiagonal of R^{-1} (taken
    numerically) reach the lemma's entry bounds exactly; every other entry
    stays below its bound.  This fixes the powers of cs and the column norm
    each entry bound carries where the bound is attained; the sum identity
    above carries them into b_j."""
    ct = math.sqrt(1.0 - cs * cs)
    m = 7
    fnorm = np.array([3.0, 0.25, 1.5, 0.7, 2.0, 0.4, 1.1])
    F = np.zeros((m + 2, m))
    F[0, 0] = fnorm[0]
    for i in range(1, m):
        F[i - 1, i] = fnorm[i] * ct
        F[i, i] = fnorm[i] * cs
    Q, R = np.linalg.qr(F)
    # the hypotheses hold: sines from the QR, cosines directly
    for i in range(1, m):
        assert abs(R[i, i]) / fnorm[i] >= cs * (1 - 1e-12)
        for k in range(i):
            cosik = abs(F[:, i] @ F[:, k]) / (fnorm[i] * fnorm[k])
            assert cosik <= ct * (1 + 1e-12)
    S = np.abs(np.linalg.inv(R))
    B = _entry_bounds(fnorm, cs)
    iu = np.triu_indices(m)
    assert np.all(S[iu] <= B[iu] * (1 + 1e-12))
    for i in range(m):
        assert S[i, i] == pytest.approx(B[i, i], rel=1e-12)
        if i + 1 < m:
            assert S[i, i + 1] == pytest.approx(B[i, i + 1], rel=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_entry_bounds_hold_for_random_angled_columns(seed):
    """Random columns drawn to satisfy the sine condition with cs, whose
    cosines with earlier columns happen to stay below ct: every entry of
    R^{-1} is within the bound of Lemma eq:lemma1.51."""
    rng = np.random.default_rng(300 + seed)
    cs = 0.3
    ct = math.sqrt(1.0 - cs * cs)
    checked = 0
    while checked < 5:
        F = _angled_columns(rng, 12, 6, cs)
        fn = np.linalg.norm(F, axis=0)
        C = np.abs(F.T @ F) / np.outer(fn, fn)
        if np.any(C[np.triu_indices(6, 1)] > ct):
            continue
        _, R = np.linalg.qr(F)
        S = np.abs(np.linalg.inv(R))
        B = _entry_bounds(fn, cs)
        iu = np.triu_indices(6)
        assert np.all(S[iu] <= B[iu] * (1 + 1e-10))
        checked += 1


@pytest.mark.parametrize("seed", range(5))
def test_angle_filter_survivors_satisfy_angle_condition(seed):
    rng = np.random.default_rng(100 + seed)
    N, m, cs = 25, 8, 0.3
    F = rng.standard_normal((N, m))
    F[:, 3] = F[:, 1] + 0.01 * rng.standard_normal(N)  # nearly dependent columns
    F[:, 6] = 2.0 * F[:, 0] - F[:, 2]
    E = rng.standard_normal((N, m))
    keep = oracle.angle_filter(E, F, cs)
    assert keep[0] == 0
    assert 3 not in keep and 6 not in keep
    Fk = F[:, keep]
    for i in range(1, Fk.shape[1]):
        Q, _ = np.linalg.qr(Fk[:, :i])
        perp = Fk[:, i] - Q @ (Q.T @ Fk[:, i])
        assert np.linalg.norm(perp) / np.linalg.norm(Fk[:, i]) >= cs - 1e-12


@pytest.mark.parametrize("seed", range(5))
def test_length_filter_output_is_conditioned(seed):
    rng = np.random.default_rng(200 + seed)
    cs = 0.2
    F = _angled_columns(rng, 40, 6, cs)
    E = rng.standard_normal((40, 6)) * np.array([1, 1, 1, 1e3, 1e4, 1e5])
    en, fn = np.linalg.norm(E, axis=0), np.linalg.norm(F, axis=0)
    b = oracle.length_bounds(fn, cs)
    kbar = math.sqrt(float(np.sum(en[:3] ** 2) * np.sum(b[:3]))) * 1.0001
    k = oracle.length_filter(en, fn, cs, kbar)
    assert k == 3
    _, R = np.linalg.qr(F[:, :k])
    lhs = np.linalg.norm(E[:, :k], "fro") * np.linalg.norm(np.linalg.inv(R), "fro")
    assert lhs <= kbar
    assert float(np.sum(en[:k] ** 2) * np.sum(b[:k])) <= kbar ** 2
    assert oracle.length_filter(en, fn, cs, 1e-30) == 0  # nothing passes: the loop runs out
    fz = fn.copy(); fz[0] = 0.0
    assert oracle.length_filter(en, fz, cs, 1e150) == 0  # zero newest column never passes
    assert oracle.length_filter(en, fn, cs, 1e300) == 6


def _dist_to_span(F, cols, v):
    """Distance of v from the span of F[:, cols], by least squares (a routine
    other than the QR the filter uses)."""
    if not cols:
        return float(np.linalg.norm(v))
    coef, *_ = np.linalg.lstsq(F[:, cols], v, rcond=None)
    return float(np.linalg.norm(v - F[:, cols] @ coef))


@pytest.mark.parametrize("seed", range(5))
def test_sequential_angle_filter_definition_and_superset(seed):
    """angle_mode 1: every column is kept exactly when its sine against the
    columns kept before it is >= cs (checked by least squares), and every
    column the one-factorisation filter keeps is kept too (its distance from
    a subset of the earlier columns is at least its distance from all of
    them)."""
    rng = np.random.default_rng(300 + seed)
    N, m, cs = 25, 9, 0.3
    F = rng.standard_normal((N, m)) * rng.uniform(0.1, 10, m)
    F[:, 2] = F[:, 1] + 0.05 * rng.standard_normal(N)
    F[:, 5] = F[:, 0] - 0.5 * F[:, 3] + 0.02 * rng.standard_normal(N)
    F[:, 7] = 0.0
    E = rng.standard_normal((N, m))
    seq = oracle.angle_filter(E, F, cs, sequential=True)
    once = oracle.angle_filter(E, F, cs)
    assert set(once) <= set(seq)
    kept = [0]
    for i in range(1, m):
        fn = np.linalg.norm(F[:, i])
        if fn > 0 and _dist_to_span(F, kept, F[:, i]) / fn >= cs:
            kept.append(i)
    assert seq == kept
    assert 7 not in seq


def test_sequential_angle_filter_keeps_a_column_the_single_factorisation_drops():
    """f1 is nearly parallel to f0 (dropped by both); f2 = e2 lies in the span
    of f0 and f1 (dropped by the single factorisation) but is orthogonal to
    f0, the only column kept before it (kept by the sequential reading)."""
    F = np.zeros((4, 3))
    F[0, 0] = 1.0
    F[:, 1] = [1.0, 0.01, 0.0, 0.0]
    F[1, 2] = 1.0
    E = np.eye(4)[:, :3]
    assert oracle.angle_filter(E, F, 0.2) == [0]
    assert oracle.angle_filter(E, F, 0.2, sequential=True) == [0, 2]


def test_angle_filter_modes_agree_on_well_separated_columns():
    rng = np.random.default_rng(7)
    F = _angled_columns(rng, 30, 7, 0.5)
    E = rng.standard_normal((30, 7))
    assert oracle.angle_filter(E, F, 0.4) == list(range(7))
    assert oracle.angle_filter(E, F, 0.4, sequential=True) == list(range(7))


def test_reverse_is_involution():
    E = np.arange(12.0).reshape(3, 4)
    F = -E
    E2, F2 = oracle.reverse(*oracle.reverse(E, F))
    np.testing.assert_array_equal(E2, E)
    np.testing.assert_array_equal(F2, F)
    np.testing.assert_array_equal(oracle.reverse(E, F)[0][:, 0], E[:, -1])


def test_faa_without_filtering_equals_aa_without_regularisation():
    # c_s -> 0 and kappa_bar -> inf keep every column; then R^{-1} Q^T g is the
    # unregularised least-squares solution, i.e. Alg 2 with eta = 0.
    P = oracle.Problem.from_lpdata(lpgen.tiny_lp(1))
    common = dict(D=10.0, kkt_every=0, memory=5, tau=0.05, sigma=0.05)
    a = oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_AA, eta=0.0, **common))
    f = oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_FAA, cs=1e-300, kappa_bar=1e300, **common))
    a.start(); f.start()
    for _ in range(40):
        a.step(); f.step()
        assert a.last_branch == f.last_branch
        np.testing.assert_allclose(np.r_[f.state.x, f.state.y], np.r_[a.state.x, a.state.y],
                                   rtol=1e-7, atol=1e-9)


def test_faa_memory_never_exceeds_limit_and_filters_bind():
    P = oracle.Problem.from_lpdata(lpgen.tiny_lp(0))
    f = oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_FAA, cs=0.5, kappa_bar=1e2, memory=6,
                                        D=math.inf, kkt_every=0))
    f.start()
    sizes = []
    for _ in range(60):
        f.step()
        sizes.append(len(f.state.dU))
        assert len(f.state.dU) <= 6
    assert min(sizes[10:]) < 6  # the filters removed columns


def test_length_filter_floor_reading():
    """Alg 5 when no k passes: the count-down loop runs out (0 columns) or,
    with the floor reading, stops at k = 1; when some k passes both readings
    give that k."""
    rng = np.random.default_rng(11)
    F = _angled_columns(rng, 30, 5, 0.3)
    E = rng.standard_normal((30, 5))
    en, fn = np.linalg.norm(E, axis=0), np.linalg.norm(F, axis=0)
    assert oracle.length_filter(en, fn, 0.3, 1e-30) == 0
    assert oracle.length_filter(en, fn, 0.3, 1e-30, floor=1) == 1
    for kbar in (1e300, 1e3, 10.0):
        assert oracle.length_filter(en, fn, 0.3, kbar, floor=1) == max(1, oracle.length_filter(en, fn, 0.3, kbar))
    assert oracle.length_filter(np.zeros(0), np.zeros(0), 0.3, 1e-30, floor=1) == 0  # no column to keep


def test_faa_floor_one_keeps_the_newest_pair_in_closed_form():
    """kappa-bar so small that no k passes: with m-bar = 1 the FAA step
    mixes the newest pair alone, gamma = <f, g> / <f, f> (one-column least
    squares), u+ = P(u + beta D g - (du + beta D f) gamma); with m-bar = 0
    it is u+ = P(u + beta D g).  Both are written out here from the
    definitions, and the memory after the step holds that one pair or
    nothing."""
    P = oracle.Problem.from_lpdata(lpgen.tiny_lp(2))
    n = P.n
    for floor in (0, 1):
        f = oracle.Solver(P, oracle.Options(variant=oracle.VARIANT_FAA, cs=0.2, kappa_bar=1e-300, memory=5,
                                            D=math.inf, kkt_every=0, dhat_mode=1, beta=0.7, length_floor=floor))
        f.start()
        for _ in range(6):
            f.step()
        S = f.state
        u = np.r_[S.x, S.y]
        # the pair the next step appends, and its residual, from the map itself
        xh, yh = oracle.pdhg_map(P, S.x, S.y, f.opt.tau, f.opt.sigma)
        g = np.r_[xh, yh] - u
        du, dg = u - S.u_prev, g - S.g_prev
        D = f.Dhat
        if floor == 1:
            gam = float(dg @ g) / float(dg @ dg)
            want = u + 0.7 * D * g - (du + 0.7 * D * dg) * gam
        else:
            want = u + 0.7 * D * g
        want = np.r_[oracle.proj_X(P, want[:n]), oracle.proj_Y(P, want[n:])]
        empty0 = f.faa_empty
        f.step()
        assert f.last_branch == "aa"
        np.testing.assert_allclose(np.r_[f.state.x, f.state.y], want, rtol=1e-12, atol=1e-14)
        assert len(f.state.dG) == floor
        assert f.faa_empty == empty0 + (1 - floor)
        if floor == 1:
            np.testing.assert_allclose(f.state.dG[0], dg, rtol=0, atol=0)


# ---------------------------------------------------------------------------
# power iteration and Ruiz equilibration (Sections 5.1, 5.2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 5])
def test_power_norm_matches_svd(seed):
    lp = lpgen.tiny_lp(seed)
    P = oracle.Problem.from_lpdata(lp)
    smax = np.linalg.svd(lpgen.to_dense(lp), compute_uv=False)[0]
    est = oracle.power_norm(P, iters=2000, rtol=1e-14)
    assert est <= smax * (1 + 1e-12)
    assert est >= smax * (1 - 1e-6)


def test_ruiz_equilibrates_and_preserves_the_lp():
    lp = lpgen.mip_like_lp(2, m=80, n=160, nnz=900, fp32=False)
    P = oracle.Problem.from_lpdata(lp)
    S, dr, dc = oracle.ruiz(P, 10)
    Kd = lpgen.to_dense(lp)
    Ks = S.K.toarray()
    np.testing.assert_allclose(Ks, dr[:, None] * Kd * dc[None, :], rtol=1e-13, atol=1e-15)
    rmax = np.abs(Ks).max(axis=1)
    cmax = np.abs(Ks).max(axis=0)
    assert np.all(np.abs(rmax[rmax > 0] - 1) < 0.02)
    assert np.all(np.abs(cmax[cmax > 0] - 1) < 0.02)
    # the planted optimum maps to a KKT point of the scaled LP
    r = oracle.kkt(S, lp.planted["x"] / dc, lp.planted["y"] / dr)
    assert r["kkt"] < 1e-12
    assert r["pobj"] == pytest.approx(lp.planted["pstar"], rel=1e-12)


@pytest.mark.parametrize("seed", [2, 3])
def test_pock_chambolle_bounds_the_norm_and_preserves_the_lp(seed):
    """With alpha = 1 the scaled matrix has ||K~||_2 <= 1: the Schur test with
    weights sqrt(row sums) and sqrt(column sums) bounds it by the product of
    two quantities that are both 1.  The planted optimum stays a KKT point of
    the scaled LP with the same objective (the scaling is a change of
    variables)."""
    lp = lpgen.mip_like_lp(seed, m=80, n=160, nnz=900, fp32=False)
    P = oracle.Problem.from_lpdata(lp)
    S, dr, dc = oracle.pock_chambolle(P, 1.0)
    Kd = lpgen.to_dense(lp)
    Ks = S.K.toarray()
    np.testing.assert_allclose(Ks, dr[:, None] * Kd * dc[None, :], rtol=1e-13, atol=1e-15)
    # the factors are the plain row and column 1-norms
    np.testing.assert_allclose(1.0 / dr ** 2, np.where(np.abs(Kd).sum(1) > 0, np.abs(Kd).sum(1), 1.0), rtol=1e-13)
    np.testing.assert_allclose(1.0 / dc ** 2, np.where(np.abs(Kd).sum(0) > 0, np.abs(Kd).sum(0), 1.0), rtol=1e-13)
    assert np.linalg.norm(Ks, 2) <= 1.0 + 1e-12
    assert np.linalg.norm(Kd, 2) > 1.5  # the bound is not trivially true before scaling
    r = oracle.kkt(S, lp.planted["x"] / dc, lp.planted["y"] / dr)
    assert r["kkt"] < 1e-12
    assert r["pobj"] == pytest.approx(lp.planted["pstar"], rel=1e-12)


def test_ruiz_then_pock_chambolle_composes():
    """Ruiz sweeps followed by the Pock-Chambolle step (the preconditioning of
    Section 5.2): the factors multiply and the norm bound holds after both."""
    lp = lpgen.mip_like_lp(4, m=80, n=160, nnz=900, fp32=False)
    P = oracle.Problem.from_lpdata(lp)
    S1, r1, c1 = oracle.ruiz(P, 10)
    S2, r2, c2 = oracle.pock_chambolle(S1, 1.0)
    Kd = lpgen.to_dense(lp)
    np.testing.assert_allclose(S2.K.toarray(), (r1 * r2)[:, None] * Kd * (c1 * c2)[None, :], rtol=1e-12, atol=1e-15)
    assert np.linalg.norm(S2.K.toarray(), 2) <= 1.0 + 1e-12


# ---------------------------------------------------------------------------
# power-iteration start vector (step size 0.9 / ||K||_2, Section 5.1)
# ---------------------------------------------------------------------------

def test_splitmix64_published_outputs():
    g = golden("splitmix64.json")
    want = [int(h, 16) for h in g["outputs_hex"]]
    got = [int(v) for v in oracle.splitmix64(g["seed"], len(want))]
    assert got == want


def test_power_start_is_uniform_on_minus_one_one():
    v = oracle.power_start(200000, seed=7)
    assert v.min() >= -1.0 and v.max() < 1.0
    assert abs(v.mean()) < 0.01 and abs(v.var() - 1.0 / 3.0) < 0.01
    assert not np.array_equal(v, oracle.power_start(200000, seed=8))


def _cycle_difference_lp(m, c):
    """Rows x_i - x_{i+1 mod m} = 0: every row of K sums to zero, so the
    constant vector is in its null space; K = I - P (P the cyclic shift) has
    eigenvalues 1 - w^k, so ||K||_2 = 2 for even m."""
    K = np.eye(m) - np.roll(np.eye(m), 1, axis=1)
    return lp_from_dense(K, np.zeros(m), c, [0.0] * m, [10.0] * m, [0] * m)


def test_power_norm_finds_the_norm_where_a_constant_start_sees_nothing():
    Po = oracle.Problem.from_lpdata(_cycle_difference_lp(6, np.ones(6)))
    assert oracle.power_norm(Po, v0=np.ones(6)) == 0.0  # K 1 = 0
    assert oracle.power_norm(Po) == pytest.approx(2.0, rel=1e-8)
    s = oracle.Solver(Po, oracle.Options(tol=1e-8, max_iter=20000, kkt_every=1))
    assert s.opt.tau == pytest.approx(0.45, rel=1e-8)
    r = s.solve()
    assert r["status"] == "converged"
    np.testing.assert_allclose(r["x"], 0.0, atol=1e-6)  # all equal (K x = 0), at the bound c pushes to
