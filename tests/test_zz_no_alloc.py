"""aapdhg_iterate_noalloc (the passes of aapdhg_iterate with their scratch in
the library's static device array) against aapdhg_iterate: two calls in a
row on twin handles, the second on a smaller LP, in the persistent loop
kernel and in the three-launch path; the same bits.  An LP whose pass tables
need more scratch than the array holds is refused with a clear error."""
import numpy as np
import pytest

import lpgen

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2508_08062_amd")


def _state(g):
    st = g.get_state()
    return st["k"], st["i"], st["j"], st["u"], st["dG"], st["W"]


@pytest.mark.parametrize("loop_kernel", [0, 1])
def test_noalloc_passes_equal_iterate(loop_kernel):
    big = lpgen.mip_like_lp(1)  # 20k x 50k, 250k entries
    small = lpgen.mip_like_lp(5, m=3000, n=7000, nnz=40000)
    kw = dict(precision=0, variant=1, memory=10, kkt_every=16, ruiz_iters=10, dhat_mode=0, tol=0.0,
              max_iter=10 ** 9, loop_kernel=loop_kernel)
    for lp, passes in ((big, 120), (small, 75)):
        ref = P.Solver(lp, **kw)
        got = P.Solver(lp, **kw)
        ref.iterate(passes)
        got.iterate_noalloc(passes)
        a, b = _state(ref), _state(got)
        assert a[:3] == b[:3] == (passes, a[1], a[2])
        for x, y in zip(a[3:], b[3:]):
            assert np.array_equal(x, y)
        # a second call continues from the state the first left
        ref.iterate(33)
        got.iterate_noalloc(33)
        a, b = _state(ref), _state(got)
        assert a[0] == b[0] == passes + 33
        for x, y in zip(a[3:], b[3:]):
            assert np.array_equal(x, y)
        ra, rb = ref.result(), got.result()
        assert ra["kkt"] == rb["kkt"] and ra["aa_steps"] == rb["aa_steps"]
        ref.close()
        got.close()


def test_noalloc_refuses_an_lp_beyond_the_scratch():
    """6000 rows of 2100 entries: every row is split (one partial-sum record
    of 384 bytes each), 2.3 MB of pass scratch against 2 MiB."""
    rng = np.random.default_rng(0)
    m, n, L = 6000, 10000, 2100
    cols = np.argsort(rng.random((m, n)), axis=1)[:, :L]
    cols.sort(axis=1)
    rowptr = np.arange(m + 1, dtype=np.int64) * L
    lp = lpgen.LPData(m=m, n=n, rowptr=rowptr, colidx=cols.ravel().astype(np.int32),
                      val=np.ones(m * L), c=-np.ones(n), q=np.zeros(m), l=np.zeros(n), u=np.full(n, 1.0),
                      rowtype=np.ones(m, dtype=np.uint8))
    g = P.Solver(lp, precision=0, memory=4, tol=0.0, loop_kernel=1, kkt_every=64)
    with pytest.raises(P.AAPDHGError) as e:
        g.iterate_noalloc(1)
    assert e.value.status == P.E_ARG and "scratch" in str(e.value)
    g.iterate(2)  # the allocating entry point still runs it
    assert g.get_state()["k"] == 2
    g.close()
