"""Seeded generators: determinism, shapes, planted optimum."""
import numpy as np
import pytest

import lpgen


def _same(a, b):
    for f in ("rowptr", "colidx", "val", "c", "q", "l", "u", "rowtype"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))


def test_deterministic_per_seed():
    _same(lpgen.tiny_lp(3), lpgen.tiny_lp(3))
    _same(lpgen.mip_like_lp(9, m=500, n=1200, nnz=6000), lpgen.mip_like_lp(9, m=500, n=1200, nnz=6000))
    a = lpgen.mip_like_lp(9, m=500, n=1200, nnz=6000)
    b = lpgen.mip_like_lp(10, m=500, n=1200, nnz=6000)
    assert not np.array_equal(a.val, b.val)


def _check_csr(lp):
    assert lp.rowptr[0] == 0 and lp.rowptr[-1] == lp.nnz
    assert np.all(np.diff(lp.rowptr) >= 0)
    rows = np.repeat(np.arange(lp.m), np.diff(lp.rowptr))
    key = rows.astype(np.int64) * lp.n + lp.colidx
    assert np.all(np.diff(key) > 0)  # sorted, distinct within rows
    assert lp.colidx.min() >= 0 and lp.colidx.max() < lp.n


def test_tiny_shape():
    lp = lpgen.tiny_lp(0)
    _check_csr(lp)
    assert (lp.m, lp.n, lp.nnz) == (50, 100, 500)
    assert np.sum(lp.planted["x"] == 0.0) == 30
    assert np.all(lp.rowtype == lpgen.ROW_EQ)


def test_mip_like_shape_and_statistics():
    lp = lpgen.mip_like_lp(1)
    _check_csr(lp)
    assert (lp.m, lp.n, lp.nnz) == (20000, 50000, 250000)
    lens = np.diff(lp.rowptr)
    assert lens.max() <= 2000 and lens.min() >= 1
    assert 0.3 < np.mean(lens == 1) < 0.7  # Zipf(1.8): most rows are short
    assert np.mean(lp.rowtype == lpgen.ROW_EQ) == pytest.approx(0.4, abs=1e-3)
    unit = np.mean(np.abs(lp.val) == 1.0)
    assert 0.55 < unit < 0.65
    kinds = np.isfinite(lp.l).astype(int) * 2 + np.isfinite(lp.u)
    for k, frac in ((3, 1 / 3), (2, 1 / 3), (0, 1 / 3)):
        assert np.mean(kinds == k) == pytest.approx(frac, abs=0.02)
    # float32-representable data
    assert np.array_equal(lp.val.astype(np.float32).astype(np.float64), lp.val)


def test_powerlaw_shape_small():
    lp = lpgen.powerlaw_lp(2, m=20000, n=40000, nnz=400000)
    _check_csr(lp)
    assert lp.nnz >= 400000
    colcnt = np.bincount(lp.colidx, minlength=lp.n)
    assert colcnt.max() > 50 * colcnt.mean()  # heavy tail
    assert np.diff(lp.rowptr).min() >= 1


def test_batch_and_serving_shapes():
    shapes = lpgen.batch_shapes(256, 3)
    rows = np.array([s[0] for s in shapes])
    assert rows.min() >= 1000 and rows.max() <= 50000
    rho = np.array([s[2] / s[1] for s in shapes])
    assert rho.min() >= 3 - 1e-9 and rho.max() <= 12 + 1e-9
    req = lpgen.serving_requests(200.0, 10.0, 4)
    assert 1700 < len(req) < 2300
    cols = np.array([r[2] for r in req])
    assert cols.min() >= 1000 and cols.max() <= 500000
