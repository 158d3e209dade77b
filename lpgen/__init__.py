"""Seeded synthetic LP instances.

This module only draws random data and assembles LP instances of the form
(Section 2.1, problem LP-O with K=[G;A], q=[h;b]):

    min c^T x   s.t.  (K x)_i >= q_i  for rows of type GE,
                      (K x)_i  = q_i  for rows of type EQ,
                      l <= x <= u.

It contains none of the solver's arithmetic.  Instances are feasible and
bounded by construction: a primal point x*, a dual point y* and reduced costs
s are drawn first and (c, q) are then chosen so that (x*, y*, s) satisfies the
KKT conditions of the dual pair LP-O / DUAL-2 exactly (in float64, before any
float32 rounding).  The planted optimal value is p* = q^T y* + sum_j l_j s_j.

All draws use numpy.random.Generator(PCG64(seed)) in a fixed order, so an
instance is a pure function of its arguments.

The paper measures on MIPLIB 2017 LP relaxations; those are not available and
nothing here reproduces them.  The shapes, densities and value distributions
below are synthetic stand-ins.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ROW_EQ = 0
ROW_GE = 1


@dataclasses.dataclass
class LPData:
    """An LP in CSR form.  Infinite bounds are stored as +-inf."""

    m: int
    n: int
    rowptr: np.ndarray  # int64 [m+1]
    colidx: np.ndarray  # int32 [nnz], sorted within each row, distinct
    val: np.ndarray  # float64 [nnz]
    c: np.ndarray  # float64 [n]
    q: np.ndarray  # float64 [m]
    l: np.ndarray  # float64 [n]
    u: np.ndarray  # float64 [n]
    rowtype: np.ndarray  # uint8 [m], ROW_EQ or ROW_GE
    planted: dict = dataclasses.field(default_factory=dict)
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def nbytes(self) -> int:
        return int(self.rowptr.nbytes + self.colidx.nbytes + self.val.nbytes + self.c.nbytes
                   + self.q.nbytes + self.l.nbytes + self.u.nbytes + self.rowtype.nbytes)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def round_fp32(lp: LPData) -> LPData:
    """Round the data of an LP to float32-representable float64 values.

    Bounds 0, 1, 10 and +-inf are exact in float32.  The planted point is no
    longer exactly optimal after rounding (it is off by float32 rounding), which
    is recorded in ``planted['rounded']``.
    """
    f = lambda a: a.astype(np.float32).astype(np.float64)
    out = dataclasses.replace(lp, val=f(lp.val), c=f(lp.c), q=f(lp.q), l=f(lp.l), u=f(lp.u),
                              planted=dict(lp.planted))
    out.planted["rounded"] = True
    return out


# --------------------------------------------------------------------------
# sparsity patterns
# --------------------------------------------------------------------------

def _adjust_lengths(rng, lens, total, cap):
    """Add or remove single entries at uniformly random positions until the
    lengths sum to ``total``, keeping every length in [1, cap]."""
    lens = np.minimum(np.maximum(lens.astype(np.int64), 1), cap)
    k = lens.size
    for _ in range(10000):
        diff = int(total - lens.sum())
        if diff == 0:
            return lens
        if diff > 0:
            pick = rng.integers(0, k, diff)
            lens = lens + np.bincount(pick, minlength=k)
            lens = np.minimum(lens, cap)
        else:
            pick = rng.integers(0, k, -diff)
            dec = np.bincount(pick, minlength=k)
            lens = np.maximum(lens - dec, 1)
    raise RuntimeError("could not adjust lengths to the requested total")


def _distinct_positions(rng, lens, width):
    """For segment s of length lens[s], draw lens[s] distinct positions in
    [0, width).  Returns (segment ids, positions), sorted by (segment, pos)."""
    lens = np.asarray(lens, dtype=np.int64)
    offs = np.concatenate(([0], np.cumsum(lens)))
    seg = np.repeat(np.arange(lens.size, dtype=np.int64), lens)
    pos = rng.integers(0, width, seg.size)
    dense = np.nonzero(lens * 8 > width)[0]  # long segments: draw without replacement
    for s in dense:
        pos[offs[s]:offs[s + 1]] = rng.choice(width, int(lens[s]), replace=False)
    key = np.sort(seg * width + pos)
    while True:
        dup = np.nonzero(key[1:] == key[:-1])[0] + 1
        if dup.size == 0:
            break
        # redraw the duplicates, then re-sort only the affected segments
        bad = np.unique(key[dup] // width)
        key[dup] = (key[dup] // width) * width + rng.integers(0, width, dup.size)
        for s in bad:
            a, b = offs[s], offs[s + 1]
            key[a:b] = np.sort(key[a:b])
    return key // width, key % width


def _csr_from_coo(m, rows, cols, vals):
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.argsort(rows * (int(cols.max(initial=0)) + 1) + cols, kind="stable")
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rowptr[1:])
    return rowptr, cols.astype(np.int32), vals.astype(np.float64)


def _mip_values(rng, count):
    """+-1 with probability 0.6, else lognormal(0,1) with a random sign."""
    unit = rng.random(count) < 0.6
    sign = np.where(rng.random(count) < 0.5, -1.0, 1.0)
    mag = np.where(unit, 1.0, rng.lognormal(0.0, 1.0, count))
    return sign * mag


def _spmv(rowptr, colidx, val, x):
    m = rowptr.size - 1
    rows = np.repeat(np.arange(m), np.diff(rowptr))
    return np.bincount(rows, weights=val * x[colidx], minlength=m)


def _spmv_t(rowptr, colidx, val, y, n):
    m = rowptr.size - 1
    rows = np.repeat(np.arange(m), np.diff(rowptr))
    return np.bincount(colidx, weights=val * y[rows], minlength=n)


# --------------------------------------------------------------------------
# planted optimum
# --------------------------------------------------------------------------

def _plant_mixed(rng, m, n, rowptr, colidx, val, eq_frac):
    """Row types, mixed bounds and a planted KKT point for the mixed-structure
    families (the 20k x 50k single LP, batch members, serving requests, and
    the large power-law LP)."""
    rowtype = np.full(m, ROW_GE, dtype=np.uint8)
    n_eq = int(round(eq_frac * m))
    rowtype[rng.permutation(m)[:n_eq]] = ROW_EQ
    kind = rng.integers(0, 3, n)  # 0: [0,1], 1: [0,inf), 2: free
    l = np.where(kind == 2, -np.inf, 0.0)
    u = np.where(kind == 0, 1.0, np.inf)
    lo = np.where(np.isfinite(l), l, -10.0)
    hi = np.where(np.isfinite(u), u, 10.0)
    xs = lo + (hi - lo) * rng.random(n)
    at_lower = np.isfinite(l) & (rng.random(n) < 0.3)
    xs = np.where(at_lower, l, xs)
    kx = _spmv(rowptr, colidx, val, xs)
    ys = np.zeros(m)
    q = kx.copy()
    eq = rowtype == ROW_EQ
    ys[eq] = rng.standard_normal(int(eq.sum()))
    ge_idx = np.nonzero(~eq)[0]
    active = rng.random(ge_idx.size) < 0.5
    ys[ge_idx[active]] = np.abs(rng.standard_normal(int(active.sum())))
    slack_rows = ge_idx[~active]
    q[slack_rows] = kx[slack_rows] - rng.random(slack_rows.size)
    s = np.where(at_lower, rng.random(n), 0.0)
    c = _spmv_t(rowptr, colidx, val, ys, n) + s
    pstar = float(q @ ys + np.sum(np.where(np.isfinite(l), l, 0.0) * s))
    planted = {"x": xs, "y": ys, "s": s, "pstar": pstar}
    return rowtype, l, u, q, c, planted


# --------------------------------------------------------------------------
# instance families
# --------------------------------------------------------------------------

def toy_lp() -> LPData:
    """The two-variable feasibility example of Section 5.2 (eq.
    simple-feasibility): min 0 s.t. x = 3, x >= 0.  Optimum (x, y) = (3, 0)."""
    return LPData(m=1, n=1, rowptr=np.array([0, 1], dtype=np.int64),
                  colidx=np.array([0], dtype=np.int32), val=np.array([1.0]),
                  c=np.array([0.0]), q=np.array([3.0]), l=np.array([0.0]),
                  u=np.array([np.inf]), rowtype=np.array([ROW_EQ], dtype=np.uint8),
                  planted={"x": np.array([3.0]), "y": np.array([0.0]), "s": np.array([0.0]),
                           "pstar": 0.0},
                  name="toy")


def tiny_lp(seed: int, m: int = 50, n: int = 100, nnz: int = 500) -> LPData:
    """Tiny equality-form LP: A (m x n, nnz distinct uniform positions, N(0,1)
    values), 0 <= x <= 10, x* ~ U[0,10] with 30% of entries zero, b = A x*,
    y* ~ N(0,1), c = A^T y* + s with s ~ U[0,1] only where x*_j = 0."""
    rng = _rng(seed)
    while True:
        flat = rng.choice(m * n, nnz, replace=False)
        rows, cols = flat // n, flat % n
        if np.unique(rows).size == m:
            break
    vals = rng.standard_normal(nnz)
    rowptr, colidx, val = _csr_from_coo(m, rows, cols, vals)
    xs = 10.0 * rng.random(n)
    zero = rng.permutation(n)[: int(round(0.3 * n))]
    xs[zero] = 0.0
    b = _spmv(rowptr, colidx, val, xs)
    ys = rng.standard_normal(m)
    s = np.zeros(n)
    s[zero] = rng.random(zero.size)
    c = _spmv_t(rowptr, colidx, val, ys, n) + s
    return LPData(m=m, n=n, rowptr=rowptr, colidx=colidx, val=val, c=c, q=b,
                  l=np.zeros(n), u=np.full(n, 10.0), rowtype=np.full(m, ROW_EQ, dtype=np.uint8),
                  planted={"x": xs, "y": ys, "s": s, "pstar": float(b @ ys)},
                  name=f"tiny_s{seed}")


def mip_like_lp(seed: int, m: int = 20000, n: int = 50000, nnz: int = 250000,
                row_cap: int = 2000, zipf_a: float = 1.8, eq_frac: float = 0.4,
                fp32: bool = True) -> LPData:
    """LP shaped like a presolved MIP relaxation: row lengths Zipf(zipf_a)
    capped at row_cap, adjusted by +-1 at random rows to exactly nnz; columns
    uniform without replacement per row; values +-1 (p=0.6) else lognormal(0,1)
    with random sign; eq_frac equality rows; bounds [0,1], [0,inf), free in
    equal proportion; planted optimum."""
    rng = _rng(seed)
    cap = min(row_cap, n)
    lens = np.minimum(rng.zipf(zipf_a, m), cap)
    lens = _adjust_lengths(rng, lens, nnz, cap)
    rows, cols = _distinct_positions(rng, lens, n)
    vals = _mip_values(rng, rows.size)
    rowptr, colidx, val = _csr_from_coo(m, rows, cols, vals)
    rowtype, l, u, q, c, planted = _plant_mixed(rng, m, n, rowptr, colidx, val, eq_frac)
    lp = LPData(m=m, n=n, rowptr=rowptr, colidx=colidx, val=val, c=c, q=q, l=l, u=u,
                rowtype=rowtype, planted=planted, name=f"mip_{m}x{n}_s{seed}")
    return round_fp32(lp) if fp32 else lp


def powerlaw_lp(seed: int, m: int = 1_000_000, n: int = 2_000_000, nnz: int = 20_000_000,
                zipf_a: float = 2.1, eq_frac: float = 0.4, fp32: bool = True) -> LPData:
    """Large LP with power-law column degrees: degrees min(m, Zipf(zipf_a)),
    adjusted at random columns to exactly nnz; rows uniform without
    replacement per column; values lognormal(0,1.5) with random sign; rows,
    bounds and planted optimum as in ``mip_like_lp``.  No scaling is applied
    here (equilibration is a solver option)."""
    rng = _rng(seed)
    degs = np.minimum(rng.zipf(zipf_a, n), m)
    degs = _adjust_lengths(rng, degs, nnz, m)
    cols, rows = _distinct_positions(rng, degs, m)
    sign = np.where(rng.random(rows.size) < 0.5, -1.0, 1.0)
    vals = sign * rng.lognormal(0.0, 1.5, rows.size)
    rowptr, colidx, val = _csr_from_coo(m, rows, cols, vals)
    del rows, cols, vals
    # an empty row would be a 0 = q or 0 >= q constraint: give it one entry
    empty = np.nonzero(np.diff(rowptr) == 0)[0]
    if empty.size:
        rows = np.repeat(np.arange(m), np.diff(rowptr))
        add_c = rng.integers(0, n, empty.size)
        add_v = np.where(rng.random(empty.size) < 0.5, -1.0, 1.0) * rng.lognormal(0.0, 1.5, empty.size)
        rowptr, colidx, val = _csr_from_coo(m, np.concatenate((rows, empty)),
                                            np.concatenate((colidx.astype(np.int64), add_c)),
                                            np.concatenate((val, add_v)))
    rowtype, l, u, q, c, planted = _plant_mixed(rng, m, n, rowptr, colidx, val, eq_frac)
    lp = LPData(m=m, n=n, rowptr=rowptr, colidx=colidx, val=val, c=c, q=q, l=l, u=u,
                rowtype=rowtype, planted=planted, name=f"powerlaw_{m}x{n}_s{seed}")
    return round_fp32(lp) if fp32 else lp


def batch_shapes(count: int = 256, seed: int = 3, r_lo: int = 1000, r_hi: int = 50000):
    """Shapes of a batch of LPs: rows log-uniform in [r_lo, r_hi], cols = 2 rows,
    nnz per column uniform in [3, 12].  Returns a list of (m, n, nnz, seed)."""
    rng = _rng(seed)
    rows = np.exp(rng.uniform(math.log(r_lo), math.log(r_hi), count)).astype(np.int64)
    rho = rng.uniform(3.0, 12.0, count)
    out = []
    for i in range(count):
        m = int(rows[i])
        n = 2 * m
        out.append((m, n, int(round(rho[i] * n)), seed * 1000 + i))
    return out


def batch_lps(count: int = 256, seed: int = 3, r_lo: int = 1000, r_hi: int = 50000):
    """A batch of mixed-structure LPs with uneven sizes (see ``batch_shapes``)."""
    return [mip_like_lp(s, m=m, n=n, nnz=z) for (m, n, z, s) in batch_shapes(count, seed, r_lo, r_hi)]


def serving_requests(rate: float = 200.0, duration: float = 60.0, seed: int = 4,
                     col_lo: int = 1000, col_hi: int = 500_000, nnz_per_col: float = 5.0):
    """A Poisson request stream: arrival times (seconds) and LP shapes.
    cols ~ lognormal(ln 20000, 1) clipped to [col_lo, col_hi], rows = 0.4 cols,
    nnz = nnz_per_col * cols.  Returns a list of (t_arrival, m, n, nnz, seed)."""
    rng = _rng(seed)
    t = 0.0
    out = []
    i = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        n = int(np.clip(rng.lognormal(math.log(20000.0), 1.0), col_lo, col_hi))
        m = max(1, int(round(0.4 * n)))
        out.append((t, m, n, int(round(nnz_per_col * n)), seed * 100000 + i))
        i += 1
    return out


def random_small_lp(seed: int, n_max: int = 6, m_max: int = 3) -> LPData:
    """A random small LP with mixed row types and all four bound kinds
    (finite box, lower only, upper only, free), for brute-force checks.  Feasible
    by construction (a point x0 inside the bounds satisfies every row)."""
    rng = _rng(seed)
    n = int(rng.integers(2, n_max + 1))
    m = int(rng.integers(1, m_max + 1))
    dense = np.round(rng.standard_normal((m, n)) * 2.0) / 2.0
    dense[rng.random((m, n)) < 0.3] = 0.0
    for i in range(m):
        if not dense[i].any():
            dense[i, rng.integers(0, n)] = 1.0
    kind = rng.integers(0, 4, n)  # 0 box, 1 lower, 2 upper, 3 free
    l = np.where((kind == 0) | (kind == 1), -rng.integers(0, 3, n).astype(float), -np.inf)
    u = np.where((kind == 0) | (kind == 2), rng.integers(1, 4, n).astype(float), np.inf)
    lo = np.where(np.isfinite(l), l, -3.0)
    hi = np.where(np.isfinite(u), u, 3.0)
    x0 = np.round((lo + (hi - lo) * rng.random(n)) * 4.0) / 4.0
    rowtype = np.where(rng.random(m) < 0.5, ROW_EQ, ROW_GE).astype(np.uint8)
    q = dense @ x0 - np.where(rowtype == ROW_GE, np.round(rng.random(m) * 4.0) / 4.0, 0.0)
    c = np.round(rng.standard_normal(n) * 4.0) / 4.0
    rows, cols = np.nonzero(dense)
    rowptr, colidx, val = _csr_from_coo(m, rows, cols, dense[rows, cols])
    return LPData(m=m, n=n, rowptr=rowptr, colidx=colidx, val=val, c=c, q=q, l=l, u=u,
                  rowtype=rowtype, planted={"x_feasible": x0}, name=f"small_s{seed}")


def to_dense(lp: LPData) -> np.ndarray:
    a = np.zeros((lp.m, lp.n))
    rows = np.repeat(np.arange(lp.m), np.diff(lp.rowptr))
    a[rows, lp.colidx] = lp.val
    return a
