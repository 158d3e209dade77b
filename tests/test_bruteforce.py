"""Ground truth on tiny LPs: vertex enumeration agrees with HiGHS, and the
oracle's converged objective agrees with both (a bounded feasible LP with a
vertex attains its optimum at a vertex)."""
import numpy as np
import pytest

import lpgen
import oracle
from _util import brute_force_opt, highs_opt


def _instances(count):
    out = []
    seed = 0
    while len(out) < count:
        lp = lpgen.random_small_lp(seed)
        seed += 1
        h = highs_opt(lp)
        if h is None:
            continue
        b, x = brute_force_opt(lp)
        if b is None:
            continue
        out.append((lp, h, b, x))
    return out


INST = _instances(60)


def test_enough_instances_cover_all_bound_kinds():
    assert len(INST) == 60
    kinds = set()
    for lp, *_ in INST:
        for a, b in zip(lp.l, lp.u):
            kinds.add((bool(np.isfinite(a)), bool(np.isfinite(b))))
    assert kinds == {(True, True), (True, False), (False, True), (False, False)}
    assert any((lp.rowtype == lpgen.ROW_GE).any() for lp, *_ in INST)
    assert any((lp.rowtype == lpgen.ROW_EQ).any() for lp, *_ in INST)


@pytest.mark.parametrize("idx", range(60))
def test_vertex_enumeration_matches_highs(idx):
    lp, h, b, x = INST[idx]
    assert b == pytest.approx(h, rel=1e-7, abs=1e-7)
    r = oracle.kkt(oracle.Problem.from_lpdata(lp), x, np.zeros(lp.m))
    assert r["r_p"] < 1e-9  # the optimal vertex is primal feasible


@pytest.mark.parametrize("idx", range(0, 60, 5))
@pytest.mark.parametrize("variant", [oracle.VARIANT_AA, oracle.VARIANT_FAA, oracle.VARIANT_PDHG])
def test_oracle_reaches_brute_force_optimum(idx, variant):
    lp, h, b, _ = INST[idx]
    P = oracle.Problem.from_lpdata(lp)
    res, _ = oracle.solve(P, variant=variant, memory=5, tol=1e-9, max_iter=200000, kkt_every=10)
    assert res["status"] == "converged", res["kkt"]
    assert res["kkt"]["pobj"] == pytest.approx(b, rel=1e-6, abs=1e-6)
    assert res["kkt"]["dobj"] == pytest.approx(b, rel=1e-6, abs=1e-6)
