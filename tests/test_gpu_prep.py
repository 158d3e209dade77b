"""GPU checks of the scaling of K before the solve (the preconditioning of
Section 5.2: Ruiz sweeps, then a Pock-Chambolle step with alpha = 1), run on
the device by default:
  * Ruiz on the device gives the same bits as Ruiz on the host (same IEEE
    operations on every entry; the maxima are exact in any order), so the
    factors and every later iterate agree bit for bit;
  * the Pock-Chambolle factors equal the oracle's to 1e-13 relative (sums of
    absolute values in another order);
  * the float64 trajectory on the scaled LP matches the oracle's to 1e-9.
"""
import numpy as np
import pytest

import lpgen
import oracle
from _util import err64

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2508_08062_amd")


@pytest.mark.parametrize("precision", [0, 1])
def test_device_ruiz_equals_host_ruiz_bitwise(precision):
    lp = lpgen.powerlaw_lp(7, m=20000, n=40000, nnz=400000)  # long columns and rows
    kw = dict(precision=precision, ruiz_iters=10, memory=6, tol=0.0, max_iter=10 ** 6, kkt_every=8)
    a = P.Solver(lp, prep_device=1, **kw)
    b = P.Solver(lp, prep_device=0, **kw)
    ra, ca = a.scaling()
    rb, cb = b.scaling()
    np.testing.assert_array_equal(ra, rb)
    np.testing.assert_array_equal(ca, cb)
    assert a.dims()["tau"] == b.dims()["tau"]
    a.iterate(1)
    b.iterate(1)
    a.iterate(20)
    b.iterate(20)
    np.testing.assert_array_equal(a.get_state()["u"], b.get_state()["u"])
    a.close()
    b.close()


@pytest.mark.parametrize("prep_device", [1, 0])
def test_pock_chambolle_factors_match_the_oracle(prep_device):
    lp = lpgen.mip_like_lp(5, m=3000, n=7000, nnz=40000, fp32=False)
    g = P.Solver(lp, precision=1, ruiz_iters=10, pock_chambolle=1, prep_device=prep_device)
    dr, dc = g.scaling()
    Po = oracle.Problem.from_lpdata(lp)
    S1, r1, c1 = oracle.ruiz(Po, 10)
    S2, r2, c2 = oracle.pock_chambolle(S1, 1.0)
    np.testing.assert_allclose(dr, r1 * r2, rtol=1e-13)
    np.testing.assert_allclose(dc, c1 * c2, rtol=1e-13)
    # the Schur-test bound on the scaled matrix, through the device's power iteration
    assert g.dims()["tau"] >= 0.9 * (1.0 - 1e-9)
    g.close()


def test_trajectory_on_the_preconditioned_lp_fp64():
    lp = lpgen.mip_like_lp(6, m=1500, n=3500, nnz=20000, fp32=False)
    Po = oracle.Problem.from_lpdata(lp)
    S1, _, _ = oracle.ruiz(Po, 10)
    S2, _, _ = oracle.pock_chambolle(S1, 1.0)
    tau = 0.9 / oracle.power_norm(S2)
    common = dict(variant=1, memory=8, tau=tau, sigma=tau, kkt_every=4, tol=0.0, max_iter=10 ** 6, dhat_mode=1)
    g = P.Solver(lp, precision=1, ruiz_iters=10, pock_chambolle=1, **common)
    o = oracle.Solver(S2, oracle.Options(**common))
    o.start()
    g.iterate(1)
    errs = []
    for _ in range(40):
        o.step()
        g.iterate(1)
        st = g.get_state()
        errs.append(err64(st["u"], np.r_[o.state.x, o.state.y]))
        assert (st["i"], st["j"]) == (o.state.i, o.state.j)
    assert max(errs) < 1e-9, errs
    g.close()


def test_scaling_option_errors():
    with pytest.raises(P.AAPDHGError, match="pock_chambolle"):
        P.Solver(lpgen.tiny_lp(1), pock_chambolle=2)
    with pytest.raises(P.AAPDHGError, match="prep_device"):
        P.Solver(lpgen.tiny_lp(1), prep_device=3)
