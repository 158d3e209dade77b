"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs, element by element.  Tolerances (tests/_util.py):
  * float64 path (err64): every entry to 1e-9 of its own size or of 1e-3 of
    the largest entry, and the vector to 1e-9 in norm (summation order
    differs; AA least-squares conditioning amplifies rounding);
  * float32 path (err32) over the first 50 loop passes: the iterate to 1e-5
    in norm, no entry off by more than 1e-5 of the largest entry, every
    entry to 1e-4 of its own size or of 1/100 of the largest (float32
    storage of data, iterates and history; float64 reductions).  Entries
    near zero are differences of terms of the size of the vector's entries,
    so their float32 rounding is relative to those terms.
"""
import numpy as np
import pytest

import lpgen
import oracle
from _util import entrywise_err, err32, err64, golden, norm_rel

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2508_08062_amd")


def _gpu(lp, **kw):
    return P.Solver(lp, **kw)


def _oracle(lp, **kw):
    return oracle.Solver(oracle.Problem.from_lpdata(lp), oracle.Options(**kw))


def _trajectories(lp, steps, precision, variant=1, memory=5, **kw):
    """Run both sides for `steps` loop passes from the start point and return
    the per-pass iterates and branch counters."""
    Po = oracle.Problem.from_lpdata(lp)
    nrm = oracle.power_norm(Po)
    tau = sigma = 0.9 / nrm
    loop_kernel = kw.pop("loop_kernel", 0)
    gram_mode = kw.pop("gram_mode", 0)
    common = dict(variant=variant, memory=memory, tau=tau, sigma=sigma, kkt_every=kw.pop("kkt_every", 1),
                  tol=kw.pop("tol", 0.0), max_iter=10 ** 6, **kw)
    g = _gpu(lp, precision=precision, loop_kernel=loop_kernel, gram_mode=gram_mode, **common)
    o = _oracle(lp, **common)
    o.start()
    g.iterate(1)
    us_g, us_o, ctr = [], [], []
    st = g.get_state()
    us_g.append(st["u"].copy())
    us_o.append(np.r_[o.state.x, o.state.y])
    for _ in range(steps):
        o.step()
        g.iterate(1)
        st = g.get_state()
        us_g.append(st["u"].copy())
        us_o.append(np.r_[o.state.x, o.state.y])
        ctr.append(((st["i"], st["j"]), (o.state.i, o.state.j)))
    return us_g, us_o, ctr, g, o


# ---------------------------------------------------------------------------

def test_toy_lp_hand_trace_on_gpu():
    gld = golden("toy_lp.json")
    g = _gpu(lpgen.toy_lp(), precision=1, memory=5, tau=0.1, sigma=0.1, kkt_every=1, tol=1e-10, max_iter=50)
    g.iterate(1)
    st = g.get_state()
    np.testing.assert_allclose(st["u"], gld["u1"], atol=1e-15)
    np.testing.assert_allclose(st["u_prev"], [0.0, 0.0], atol=0)
    g.iterate(1)
    st = g.get_state()
    np.testing.assert_allclose(st["u"], gld["u2"], rtol=1e-6)
    assert st["i"] == 1 and st["j"] == 0
    g.solve()
    r = g.result()
    assert r["status"] == "converged" and r["iters"] <= 5
    np.testing.assert_allclose(np.r_[r["x"], r["y"]], gld["optimum"], atol=1e-9)


# (loop_kernel, gram_mode): the persistent kernel; three launches per pass with
# the Gram matrix formed on demand (the default for an LP held to three launches);
# three launches with the per-pass dots
PATHS = [(0, 0), (1, 0), (1, 1)]


@pytest.mark.parametrize("loop_kernel,gram_mode", PATHS)
@pytest.mark.parametrize("seed", [0, 1])
def test_tiny_fp64_trajectory_50(seed, loop_kernel, gram_mode):
    lp = lpgen.tiny_lp(seed)
    ug, uo, ctr, _, _ = _trajectories(lp, 50, precision=1, memory=5, loop_kernel=loop_kernel, gram_mode=gram_mode)
    errs = [err64(a, b) for a, b in zip(ug, uo)]
    assert max(errs) < 1e-9, errs
    for (gi, oi) in ctr:
        assert gi == oi


@pytest.mark.parametrize("loop_kernel,gram_mode", PATHS)
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_mip_like_fp32_trajectory_50(variant, loop_kernel, gram_mode):
    lp = lpgen.mip_like_lp(11, m=2000, n=5000, nnz=25000)
    ug, uo, ctr, _, _ = _trajectories(lp, 50, precision=0, variant=variant, memory=10, loop_kernel=loop_kernel,
                                      gram_mode=gram_mode)
    errs = [err32(a, b) for a, b in zip(ug, uo)]
    assert max(errs) < 1e-5, (max(errs), int(np.argmax(errs)))
    assert ctr[-1][0] == ctr[-1][1]


@pytest.mark.parametrize("loop_kernel", [0, 1])
def test_mip_like_fp32_trajectory_faa_refreshed_angle_filter(loop_kernel):
    """FAA-PDHG in float32 with the refreshed angle filter (angle_mode 1)
    and every step accelerated, so the filter runs on each pass.  Free
    running, the Anderson steps amplify the float32 rounding of the iterates
    pass after pass (measured: 4.6e-6 in norm and 1.5e-5 of the largest
    entry after 50 passes), so the bar is 1e-5 in norm and 1e-4 of the
    largest entry; one pass at a time from the GPU's own state (teacher
    forcing) every entry agrees to 1e-3 of its size or of 1e-3 of the
    largest entry: the right-hand sides <dG_t, g^k> are kept up to date
    with the new float32 difference column (reading 20), whose rounding
    each update adds, and when an Anderson step cuts the residual by a
    large factor that error is large next to <dG_t, g^k> (measured up to
    1e-4 of an entry in one pass).  The standard configurations hold 1e-5
    under teacher forcing (the ragged LP below)."""
    lp = lpgen.mip_like_lp(11, m=2000, n=5000, nnz=25000)
    ug, uo, ctr, g, o = _trajectories(lp, 50, precision=0, variant=2, memory=10, loop_kernel=loop_kernel,
                                      angle_mode=1, cs=0.5, D=1e6)
    assert max(norm_rel(a, b) for a, b in zip(ug, uo)) < 1e-5
    assert max(entrywise_err(a, b, 1.0) for a, b in zip(ug, uo)) < 1e-4
    assert all(g_ == o_ for g_, o_ in ctr), ctr
    _teacher_forced(lp, g, o, 20, 1e-3)


def test_mip_like_fp64_trajectory_faa():
    lp = lpgen.mip_like_lp(12, m=1500, n=3500, nnz=20000, fp32=False)
    ug, uo, ctr, _, _ = _trajectories(lp, 50, precision=1, variant=2, memory=10)
    errs = [err64(a, b) for a, b in zip(ug, uo)]
    assert max(errs) < 1e-8, errs
    assert ctr[-1][0] == ctr[-1][1]


@pytest.mark.parametrize("angle_mode", [0, 1])
def test_faa_filters_removing_columns_on_most_steps_fp64(angle_mode):
    """c_s = 0.8 with every step on the AA branch (D = 1e6): the angle filter
    removes columns on most steps (under both readings of Alg 4, which here
    give different trajectories); the GPU keeps the oracle's memory length
    and iterate pass for pass: to 1e-8 in norm, and every entry to 1e-6 of
    its size or of 1e-3 of the largest entry (the filtered steps amplify
    the float64 rounding of the summation order, measured 7.6e-8)."""
    lp = lpgen.mip_like_lp(12, m=1500, n=3500, nnz=20000, fp32=False)
    tau = 0.9 / oracle.power_norm(oracle.Problem.from_lpdata(lp))
    common = dict(variant=2, memory=10, tau=tau, sigma=tau, kkt_every=1, tol=0.0, max_iter=10 ** 6, cs=0.8,
                  D=1e6, angle_mode=angle_mode)
    g = _gpu(lp, precision=1, **common)
    o = _oracle(lp, **common)
    o.start()
    g.iterate(1)
    errs, lens = [], []
    for _ in range(50):
        o.step()
        g.iterate(1)
        st = g.get_state()
        ref = np.r_[o.state.x, o.state.y]
        errs.append((norm_rel(st["u"], ref), entrywise_err(st["u"], ref, 1e-3)))
        lens.append((len(st["live"]), len(o.state.dG)))
        assert (st["i"], st["j"]) == (o.state.i, o.state.j)
    assert all(a == b for a, b in lens), lens
    assert sum(1 for a, _ in lens[10:] if a < 10) >= 5, lens  # the filter did remove columns
    assert max(e[0] for e in errs) < 1e-8 and max(e[1] for e in errs) < 1e-6, errs
    g.close()


@pytest.mark.parametrize("floor", [0, 1])
def test_faa_length_filter_readings_fp64(floor):
    """kappa-bar so small that the length filter never passes (D large, so
    nearly every step is an FAA step): after an FAA step floor 0 leaves an
    empty memory and floor 1 the newest pair; the GPU follows the oracle
    under both readings, pass for pass, and counts the emptied steps as the
    oracle does."""
    lp = lpgen.mip_like_lp(12, m=1500, n=3500, nnz=20000, fp32=False)
    tau = 0.9 / oracle.power_norm(oracle.Problem.from_lpdata(lp))
    common = dict(variant=2, memory=6, tau=tau, sigma=tau, kkt_every=1, tol=0.0, max_iter=10 ** 6,
                  kappa_bar=1e-30, D=1e6, length_floor=floor)
    g = _gpu(lp, precision=1, **common)
    o = _oracle(lp, **common)
    o.start()
    g.iterate(1)
    faa_steps = 0
    for _ in range(30):
        o.step()
        g.iterate(1)
        st = g.get_state()
        assert err64(st["u"], np.r_[o.state.x, o.state.y]) < 1e-9
        assert (st["i"], st["j"]) == (o.state.i, o.state.j)
        assert len(st["live"]) == len(o.state.dG)
        if o.last_branch == "aa":  # the filters ran: the memory is what the reading keeps
            faa_steps += 1
            assert len(st["live"]) == floor
    assert faa_steps >= 20
    assert g.result()["faa_empty"] == o.faa_empty == (faa_steps if floor == 0 else 0)
    g.close()


def _teacher_forced(lp, g, o, steps, tol):
    """For `steps` loop passes: load the GPU's state into the oracle, let both
    take one pass, compare the next iterates entry by entry (to `tol` of each
    entry's size or of 1e-3 of the largest entry).  Isolates the rounding of
    one pass from its amplification by later passes."""
    errs = []
    for _ in range(steps):
        st = g.get_state()
        S = o.state
        beta = o.opt.beta
        S.k = st["k"]
        S.x, S.y = st["u"][:lp.n].copy(), st["u"][lp.n:].copy()
        S.u_prev, S.g_prev = st["u_prev"].copy(), st["g_prev"].copy()
        S.dG = [st["dG"][t].copy() for t in st["live"]]
        S.dU = [st["W"][t] - beta * o.Dhat * st["dG"][t] for t in st["live"]]
        S.i, S.j, S.n0 = st["i"], st["j"], st["n0"]
        o.step()
        g.iterate(1)
        st2 = g.get_state()
        errs.append(entrywise_err(st2["u"], np.r_[o.state.x, o.state.y], 1e-3))
        assert (st2["i"], st2["j"]) == (o.state.i, o.state.j)
    assert max(errs) < tol, errs
    return errs


@pytest.mark.parametrize("loop_kernel,gram_mode", [(0, 0), (1, 2)])
@pytest.mark.parametrize("variant,cs", [(1, 0.8), (2, 0.8), (2, 0.05)])
def test_gamma_from_the_gram_matches_least_squares_fp64(variant, cs, loop_kernel, gram_mode):
    """The mixing weights against the oracle's, one pass at a time from the
    GPU's own state: the GPU solves the normal equations of its float64 Gram
    (dG^T dG + eta I) gamma = dG^T g (Alg 2) and runs the filters of Alg 4-5
    on that Gram; the oracle factors by Cholesky (AA) or filters and solves by
    Householder QR of dG itself (FAA).  With c_s = 0.8 the angle filter
    removes columns on more than half the steps, so kept columns sit near
    its limit; with 0.05 it keeps nearly all and the length filter (Alg 5)
    holds the memory at six columns.  Both sides keep the same columns and
    gamma agrees to 1e-11 of max(1, |gamma|): the two solutions differ by
    about cond(G) times the float64 rounding, cond(G) stays below 500 on
    these memories (largest with plain AA, whose Gram is never filtered),
    and the largest difference measured is 1.9e-14.  Both ways of forming
    the Gram matrix: updated pass by pass in the persistent kernel, and from
    the stored columns by the Gram launch of the three-launch path."""
    lp = lpgen.mip_like_lp(12, m=1500, n=3500, nnz=20000, fp32=False)
    tau = 0.9 / oracle.power_norm(oracle.Problem.from_lpdata(lp))
    common = dict(variant=variant, memory=10, tau=tau, sigma=tau, kkt_every=1, tol=0.0, max_iter=10 ** 6, cs=cs,
                  D=1e6)
    g = _gpu(lp, precision=1, loop_kernel=loop_kernel, gram_mode=gram_mode, **common)
    o = _oracle(lp, **common)
    o.start()
    g.iterate(1)
    for _ in range(12):  # fill the memory
        o.step()
        g.iterate(1)
    beta = o.opt.beta
    compared, filtered, worst = 0, 0, 0.0
    for _ in range(30):
        st = g.get_state()
        S = o.state
        S.k = st["k"]
        S.x, S.y = st["u"][:lp.n].copy(), st["u"][lp.n:].copy()
        S.u_prev, S.g_prev = st["u_prev"].copy(), st["g_prev"].copy()
        S.dG = [st["dG"][t].copy() for t in st["live"]]
        S.dU = [st["W"][t] - beta * o.Dhat * st["dG"][t] for t in st["live"]]
        S.i, S.j, S.n0 = st["i"], st["j"], st["n0"]
        o.step()
        g.iterate(1)
        st2 = g.get_state()
        assert (st2["i"], st2["j"]) == (o.state.i, o.state.j)
        if o.last_branch != "aa" or len(o.last_gamma) == 0:
            continue
        ref = np.asarray(o.last_gamma)
        assert st2["nmix"] == ref.size
        filtered += ref.size < min(len(st["live"]) + 1, 10)
        worst = max(worst, float(np.max(np.abs(st2["gamma"] - ref)) / max(1.0, float(np.max(np.abs(ref))))))
        compared += 1
    assert compared >= 25
    if variant == 2 and cs == 0.8:
        assert filtered >= 10  # the angle filter removed columns
    assert worst < 1e-11, worst
    assert g.result()["gram_on_demand"] == (gram_mode == 2)
    g.close()


def _ragged_lp():
    # rows longer than one chunk (split into parts with a fix-up), a row long
    # enough for a whole-block reduction, empty rows and empty columns
    rng = np.random.default_rng(5)
    m, n = 40, 30000
    lens = np.full(m, 3)
    lens[0] = 20000   # split row (> 2048 entries): 3 parts
    lens[1] = 1500    # one-row chunk
    lens[2] = 0       # empty row
    rows, cols = [], []
    for i, L in enumerate(lens):
        c = np.sort(rng.choice(n - 100, L, replace=False))  # the last 100 columns stay empty
        rows += [i] * L
        cols += list(c)
    rows, cols = np.array(rows), np.array(cols)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rowptr[1:])
    val = np.round(rng.standard_normal(rows.size) * 8) / 8
    lp = lpgen.LPData(m=m, n=n, rowptr=rowptr, colidx=cols.astype(np.int32), val=val,
                      c=np.round(rng.standard_normal(n) * 8) / 8, q=np.round(rng.standard_normal(m) * 8) / 8,
                      l=np.where(np.arange(n) % 3 == 0, -np.inf, 0.0), u=np.where(np.arange(n) % 2 == 0, np.inf, 2.0),
                      rowtype=(np.arange(m) % 2).astype(np.uint8))
    return lpgen.round_fp32(lp)


def test_long_rows_split_and_empty_rows_and_columns_fp64():
    lp = _ragged_lp()
    ug, uo, ctr, _, _ = _trajectories(lp, 30, precision=1, memory=4)
    errs = [err64(a, b) for a, b in zip(ug, uo)]
    assert max(errs) < 1e-9, errs
    assert ctr[-1][0] == ctr[-1][1]


def test_long_rows_split_and_empty_rows_and_columns_fp32():
    lp = _ragged_lp()
    # free-running on the (non-expansive) PDHG map
    ug, uo, _, _, _ = _trajectories(lp, 50, precision=0, variant=0)
    errs = [err32(a, b) for a, b in zip(ug, uo)]
    assert max(errs) < 1e-5, errs
    # AA-PDHG: one pass at a time from the GPU's own state
    _, _, _, g, o = _trajectories(lp, 3, precision=0, memory=4)
    _teacher_forced(lp, g, o, 30, 1e-5)


def test_columns_longer_than_a_chunk_in_the_primal_pass():
    lp = lpgen.powerlaw_lp(7, m=20000, n=40000, nnz=400000)
    colcnt = np.bincount(lp.colidx, minlength=lp.n)
    assert colcnt.max() > 2048  # exercises the split path of the CSC pass
    ug, uo, _, _, _ = _trajectories(lp, 20, precision=0, memory=6, kkt_every=5)
    errs = [err32(a, b) for a, b in zip(ug, uo)]
    assert max(errs) < 1e-5, errs


def test_kkt_and_lambda_match_oracle_at_returned_iterate():
    lp = lpgen.mip_like_lp(13, m=1000, n=2500, nnz=12000)
    g = _gpu(lp, precision=0, memory=10, tol=1e-4, kkt_every=16, max_iter=3000)
    g.solve()
    r = g.result()
    Po = oracle.Problem.from_lpdata(lp)
    ref = oracle.kkt(Po, r["x"], r["y"])
    for key, gkey in (("pobj", "primal_obj"), ("dobj", "dual_obj"), ("r_g", "r_gap"), ("r_p", "r_pri"),
                      ("r_d", "r_dual")):
        assert r[gkey] == pytest.approx(ref[key], rel=1e-5, abs=1e-7), key
    np.testing.assert_allclose(r["lam"], ref["lam"], rtol=1e-5, atol=1e-5)
    if r["status"] == "converged":
        assert r["kkt"] <= 1e-4


def test_bitwise_repeatable():
    lp = lpgen.mip_like_lp(14, m=3000, n=7000, nnz=40000)
    outs = []
    for _ in range(2):
        g = _gpu(lp, precision=0, memory=10, kkt_every=8, max_iter=200, tol=0.0)
        g.solve()
        outs.append(g.get_state())
    assert np.array_equal(outs[0]["u"], outs[1]["u"])
    assert np.array_equal(outs[0]["dG"], outs[1]["dG"])


def test_batch_member_equals_solo_run():
    lps = [lpgen.mip_like_lp(20 + i, m=m, n=2 * m, nnz=6 * m) for i, m in enumerate((800, 3000, 1500, 5000))]
    kw = dict(precision=0, memory=8, kkt_every=8, max_iter=300, tol=1e-4)
    solo = []
    for lp in lps:
        g = _gpu(lp, **kw)
        g.solve()
        solo.append((g.get_state(), g.result()))
    members = [_gpu(lp, **kw) for lp in lps]
    b = P.Batch(members)
    b.solve()
    for (st, res), g in zip(solo, members):
        st2 = g.get_state()
        assert st2["k"] == st["k"]
        assert np.array_equal(st2["u"], st["u"])
        r2 = g.result()
        assert r2["status"] == res["status"] and r2["kkt"] == res["kkt"]
    b.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_loop_kernels_agree_over_many_passes(precision):
    """The persistent loop kernel and the three-launch passes take the same
    steps (same branches and counters) and reach the same iterate up to
    summation order, over passes that run many AA steps in one launch."""
    lp = lpgen.mip_like_lp(13, m=3000, n=7000, nnz=40000)
    out = []
    for lk in (0, 1):
        g = _gpu(lp, precision=precision, memory=10, kkt_every=16, tol=0.0, max_iter=10 ** 6, loop_kernel=lk)
        g.iterate(1)
        g.iterate(150)
        out.append(g.get_state())
        g.close()
    a, b = out
    assert a["k"] == b["k"] == 151
    assert (a["i"], a["j"]) == (b["i"], b["j"])
    assert norm_rel(a["u"], b["u"]) < (1e-4 if precision == 0 else 1e-9)


@pytest.mark.parametrize("gram_mode", [0, 2])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("variant", [1, 2])
def test_three_launch_passes_then_persistent_passes(precision, variant, gram_mode):
    """With gram_mode 2 the three-launch passes leave the history's Gram
    matrix stale (it is formed only when a step needs it); before the
    persistent kernel, which updates it pass by pass, takes the LP over, a
    refresh forms it.  With gram_mode 0 this LP (which the persistent kernel
    can take alone) keeps the per-pass dots in three launches too.  Either
    way the LP advanced first by three-launch passes (in a batch with a member
    held to them) and then by persistent launches takes the same steps as the
    LP advanced by persistent launches throughout, and reaches the same
    iterate up to summation order; its Gram matrix then equals the dots of its
    history."""
    lp = lpgen.mip_like_lp(13, m=3000, n=7000, nnz=40000)
    other = lpgen.mip_like_lp(14, m=1000, n=2500, nnz=10000)
    kw = dict(precision=precision, variant=variant, memory=10, kkt_every=16, tol=0.0, max_iter=10 ** 6)
    ref = _gpu(lp, loop_kernel=0, **kw)
    ref.iterate(1)
    ref.iterate(150)
    a = ref.get_state()
    ref.close()
    g = _gpu(lp, loop_kernel=0, gram_mode=gram_mode, **kw)
    h = _gpu(other, loop_kernel=1, **kw)
    b = P.Batch([g, h])
    assert b.iterate_timed(80)["kernel"] == "three"  # k = 81 (the first pass is the init step)
    b.close()
    assert g.iterate_timed(70)["kernel"] == "persistent"
    st = g.get_state()
    h.close()
    assert a["k"] == st["k"] == 151
    assert (a["i"], a["j"]) == (st["i"], st["j"]) and a["i"] > 5
    assert norm_rel(a["u"], st["u"]) < (1e-4 if precision == 0 else 1e-9)
    live, G, gp = st["live"], st["G"], st["g_prev"]
    big = max(np.sqrt(G[y, y]) for y in live)
    for x in live:
        for y in live:
            want = float(np.dot(st["dG"][x], st["dG"][y]))
            assert abs(G[x, y] - want) <= 1e-9 * np.sqrt(G[x, x] * G[y, y]) + 1e-300
        # rhs = <dG[x], g^{k-1}>, updated pass by pass since the refresh (float32: the
        # identity adds the dots of the rounded differences)
        upd = 4 * 10 * 2.0 ** -24 * np.sqrt(G[x, x]) * big if precision == 0 else 0.0
        want = float(np.dot(st["dG"][x], gp))
        assert abs(st["rhs"][x] - want) <= 1e-9 * np.sqrt(G[x, x] * float(gp @ gp)) + upd + 1e-300
    g.close()


@pytest.mark.parametrize("tol", [1e-4, 1e-6])
def test_fp64_solve_objective_matches_oracle(tol):
    """Float64 solves to relative KKT `tol` on both sides reach the same
    objective.  The iteration is chaotic at this scale: perturbing the
    oracle's own start point by one ulp moves its stopping pass by hundreds of
    passes and its objective by up to 7e-5 at KKT 1e-4 and 3e-7 at KKT 1e-6
    (relative to 1 + |obj|), so each side is taken at its own stop and the
    objectives must agree to 1e-6 at KKT 1e-6 and to the tolerance at 1e-4.
    Both must lie within the tolerance of the planted optimum."""
    lp = lpgen.tiny_lp(4)
    Po = oracle.Problem.from_lpdata(lp)
    tau = sigma = 0.9 / oracle.power_norm(Po)
    common = dict(variant=1, memory=5, tau=tau, sigma=sigma, kkt_every=8, tol=tol, max_iter=40000)
    g = _gpu(lp, precision=1, **common)
    g.solve()
    r = g.result()
    ro = _oracle(lp, **common).solve()
    assert r["status"] == ro["status"] == "converged"
    assert r["kkt"] <= tol
    o_obj = ro["kkt"]["pobj"]
    assert abs(r["primal_obj"] - o_obj) / (1 + abs(o_obj)) <= (1e-6 if tol <= 1e-6 else tol)
    pstar = lp.planted["pstar"]
    assert abs(r["primal_obj"] - pstar) / (1 + abs(pstar)) < 10 * tol


def test_bounded_waits_give_up_cleanly():
    """Failure handling forced from the host: a wait limit of 1 us makes the
    persistent kernel's waits give up; the launch ends (every wait is
    bounded), the solve reports the error and stops the LP, and the device
    runs the next solve normally."""
    lp = lpgen.tiny_lp(4)
    kw = dict(precision=1, memory=5, kkt_every=8, tol=1e-4, max_iter=20000)
    g = _gpu(lp, wait_limit_us=1, **kw)
    with pytest.raises(P.AAPDHGError) as e:
        g.solve()
    assert e.value.status == P.E_HIP
    assert "timed out" in str(e.value)
    assert g.result()["status"] == "numerical"
    g.close()
    g2 = _gpu(lp, **kw)
    g2.solve()
    r = g2.result()
    assert r["status"] == "converged" and r["kkt"] <= 1e-4
    g2.close()
