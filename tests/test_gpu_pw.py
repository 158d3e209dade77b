"""GPU parity of the primal-weight update (Alg 7), the D-hat re-blend that
follows it (remark on the primal-weight form) and the Iter_AA / c safeguard,
through the C ABI, against the CPU oracle on the same seeded inputs.

Tolerances as for the unweighted path: float64 iterates to 1e-9 relative,
float32 iterates to 1e-5 relative over 50 loop passes; the weight itself
(omega) to 1e-12 in float64 (distances summed in another order, then log and
exp) and 1e-5 in float32 (distances of float32 iterates).  The accept/reject
decisions of the weight checks and the AA/PDHG counters must agree exactly.
"""
import numpy as np
import pytest

import lpgen
import oracle
from _util import err32, err64

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2508_08062_amd")


def _run(lp, steps, precision, loop_kernel, variant=1, memory=5, **kw):
    Po = oracle.Problem.from_lpdata(lp)
    nrm = oracle.power_norm(Po)
    tau = sigma = 0.9 / nrm
    common = dict(variant=variant, memory=memory, tau=tau, sigma=sigma, kkt_every=kw.pop("kkt_every", 1),
                  tol=0.0, max_iter=10 ** 6, **kw)
    g = P.Solver(lp, precision=precision, loop_kernel=loop_kernel, **common)
    o = oracle.Solver(Po, oracle.Options(**common))
    o.start()
    g.iterate(1)
    rows = []
    for _ in range(steps):
        o.step()
        g.iterate(1)
        st = g.get_state()
        w = g.get_weights(anchor=False)
        rows.append(dict(k=st["k"], ug=st["u"].copy(), uo=np.r_[o.state.x, o.state.y], ctr_g=(st["i"], st["j"]),
                         ctr_o=(o.state.i, o.state.j), om_g=w["omega"], om_o=o.omega, w=w,
                         dh_o=o.Dhat.copy(), upd_o=sum(1 for e in o.pw_log if e[3]), nlive=st["nlive"],
                         mem_o=len(o.state.dU)))
    return rows, g, o


def _weight_ref(rows, r, period):
    """The oracle row holding the weight the device holds at row r: the
    device takes the check of iteration k at the end of pass k - 1, the oracle
    at the start of its next step."""
    return rows[r + 1] if rows[r]["k"] % period == 0 else rows[r]


def _dhat_gpu(w, d0, n):
    return np.r_[w["dha"][0] * d0[:n] + w["dhb"][0], w["dha"][1] * d0[n:] + w["dhb"][1]]


@pytest.mark.parametrize("loop_kernel", [0, 1])
@pytest.mark.parametrize("seed", [0, 2])
def test_tiny_fp64_weighted_trajectory(seed, loop_kernel):
    lp = lpgen.tiny_lp(seed)
    rows, g, o = _run(lp, 60, precision=1, loop_kernel=loop_kernel, pw_period=8, pw_theta=0.5)
    n = lp.n
    errs = [err64(r["ug"], r["uo"]) for r in rows]
    assert max(errs) < 1e-9, (max(errs), int(np.argmax(errs)))
    for q, r in enumerate(rows[:-1]):
        ref = _weight_ref(rows, q, 8)
        assert r["ctr_g"] == r["ctr_o"]
        assert r["om_g"] == pytest.approx(ref["om_o"], rel=1e-12)
        assert r["w"]["updates"] == ref["upd_o"]
        assert r["nlive"] == ref["mem_o"]
        np.testing.assert_allclose(_dhat_gpu(r["w"], o.Dhat0, n), r["dh_o"], rtol=1e-12)
    assert rows[-1]["upd_o"] >= 5  # the checks were accepted
    assert any(e[5] == 0.1 for e in o.pw_log) or any(e[5] == 0.9 for e in o.pw_log)
    g.close()


@pytest.mark.parametrize("loop_kernel", [0, 1])
@pytest.mark.parametrize("variant", [1, 2])
def test_mip_like_fp32_weighted_trajectory(variant, loop_kernel):
    lp = lpgen.mip_like_lp(11, m=2000, n=5000, nnz=25000)
    rows, g, o = _run(lp, 50, precision=0, loop_kernel=loop_kernel, variant=variant, memory=10, pw_period=10,
                      pw_theta=0.5)
    errs = [err32(r["ug"], r["uo"]) for r in rows]
    assert max(errs) < 1e-5, (max(errs), int(np.argmax(errs)))
    assert rows[-1]["ctr_g"] == rows[-1]["ctr_o"]
    assert rows[-1]["w"]["updates"] == rows[-1]["upd_o"] >= 3
    assert rows[-1]["om_g"] == pytest.approx(rows[-1]["om_o"], rel=1e-5)
    g.close()


@pytest.mark.parametrize("loop_kernel", [0, 1])
def test_iter_aa_over_c_safeguard(loop_kernel):
    lp = lpgen.tiny_lp(4)
    rows, g, o = _run(lp, 60, precision=1, loop_kernel=loop_kernel, sg_div=3.0, D=1.0)
    errs = [err64(r["ug"], r["uo"]) for r in rows]
    assert max(errs) < 1e-9, errs
    for r in rows:
        assert r["ctr_g"] == r["ctr_o"]
    g.close()


def test_weighted_persistent_launch_equals_single_passes():
    """Weight checks inside one launch of many passes (the benchmark's launch
    form) and at launch boundaries give the same iterates, bit for bit."""
    lp = lpgen.mip_like_lp(13, m=2000, n=5000, nnz=25000)
    kw = dict(variant=1, precision=0, memory=10, kkt_every=64, tol=0.0, max_iter=10 ** 6, pw_period=16)
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
    wa, wb = a.get_weights(), b.get_weights()
    np.testing.assert_array_equal(wa["words"], wb["words"])
    np.testing.assert_array_equal(wa["anchor"], wb["anchor"])
    assert wa["updates"] >= 3
    a.close()
    b.close()


@pytest.mark.parametrize("loop_kernel", [0, 1])
def test_weight_checkpoint_roundtrip(loop_kernel):
    """get_state + get_weights at a point one pass after a weight update, then
    set_state + set_weights on a fresh handle, continue: the same iterates."""
    lp = lpgen.tiny_lp(3)
    kw = dict(variant=1, precision=1, memory=5, kkt_every=1, tol=0.0, max_iter=10 ** 6, pw_period=7,
              loop_kernel=loop_kernel)
    a = P.Solver(lp, **kw)
    a.iterate(1)
    a.iterate(13)  # k = 14: the check at the top of iteration 14 has run
    st, w = a.get_state(), a.get_weights()
    assert st["k"] == 14 and w["updates"] >= 1 and w["flag"] == 1
    a.iterate(20)
    ua = a.get_state()["u"]
    b = P.Solver(lp, **kw)
    b.iterate(1)
    b.set_state(st)
    b.set_weights(w["words"], w["anchor"])
    b.iterate(20)
    np.testing.assert_array_equal(b.get_state()["u"], ua)
    a.close()
    b.close()


def test_weight_state_errors():
    lp = lpgen.tiny_lp(1)
    g = P.Solver(lp, precision=1, memory=5)
    g.iterate(1)
    with pytest.raises(P.AAPDHGError, match="pw_period"):
        g.get_weights(anchor=True)
    w = g.get_weights(anchor=False)
    assert w["omega"] == 1.0 and w["updates"] == 0 and list(w["dha"]) == [1.0, 1.0]
    with pytest.raises(P.AAPDHGError):
        g.set_weights(np.zeros(P.WEIGHT_WORDS))
    g.close()
