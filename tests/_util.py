"""Helpers shared by the tests (not by the oracle or the library)."""
import itertools
import json
import os

import numpy as np

from conftest import GOLDEN


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f, parse_constant=float)


def parse_bound(v):
    if isinstance(v, str):
        return float(v)
    return float(v)


def lp_from_dense(K, q, c, l, u, rowtype):
    """Build an lpgen.LPData from dense data (test fixtures)."""
    import lpgen
    K = np.asarray(K, dtype=float)
    m, n = K.shape
    rows, cols = np.nonzero(K)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rowptr[1:])
    return lpgen.LPData(m=m, n=n, rowptr=rowptr, colidx=cols.astype(np.int32), val=K[rows, cols],
                        c=np.asarray(c, float), q=np.asarray(q, float),
                        l=np.array([parse_bound(v) for v in l]), u=np.array([parse_bound(v) for v in u]),
                        rowtype=np.asarray(rowtype, dtype=np.uint8))


def highs_opt(lp):
    """Optimal value by HiGHS (scipy.optimize.linprog), or None."""
    from scipy.optimize import linprog
    import lpgen
    K = lpgen.to_dense(lp)
    eq = lp.rowtype == lpgen.ROW_EQ
    ge = ~eq
    bounds = [(None if not np.isfinite(a) else a, None if not np.isfinite(b) else b)
              for a, b in zip(lp.l, lp.u)]
    res = linprog(lp.c, A_ub=-K[ge] if ge.any() else None, b_ub=-lp.q[ge] if ge.any() else None,
                  A_eq=K[eq] if eq.any() else None, b_eq=lp.q[eq] if eq.any() else None,
                  bounds=bounds, method="highs")
    return res.fun if res.status == 0 else None


def brute_force_opt(lp, tol=1e-9):
    """Minimum of c^T x over the vertices of the feasible polyhedron, by
    enumerating every choice of n linearly independent active constraints
    (equalities always active).  Returns (value, vertex) or (None, None) when no
    vertex exists.  Only for tiny LPs."""
    import lpgen
    K = lpgen.to_dense(lp)
    n = lp.n
    eq = lp.rowtype == lpgen.ROW_EQ
    A_eq, b_eq = K[eq], lp.q[eq]
    ineq_rows, ineq_rhs = [], []
    for i in np.nonzero(~eq)[0]:
        ineq_rows.append(K[i]); ineq_rhs.append(lp.q[i])
    for j in range(n):
        e = np.zeros(n); e[j] = 1.0
        if np.isfinite(lp.l[j]):
            ineq_rows.append(e); ineq_rhs.append(lp.l[j])
        if np.isfinite(lp.u[j]):
            ineq_rows.append(e.copy()); ineq_rhs.append(lp.u[j])
    ineq_rows = np.array(ineq_rows).reshape(-1, n)
    ineq_rhs = np.array(ineq_rhs)
    need = n - A_eq.shape[0]
    best, best_x = None, None
    if need < 0:
        return None, None
    for S in itertools.combinations(range(ineq_rows.shape[0]), need):
        A = np.vstack([A_eq, ineq_rows[list(S)]]) if need else A_eq
        b = np.concatenate([b_eq, ineq_rhs[list(S)]]) if need else b_eq
        if A.shape[0] != n or abs(np.linalg.det(A)) < 1e-10:
            continue
        x = np.linalg.solve(A, b)
        if np.any(np.abs(A_eq @ x - b_eq) > 1e-7):
            continue
        Kx = K @ x
        if np.any(Kx[~eq] < lp.q[~eq] - 1e-7):
            continue
        if np.any(x < lp.l - 1e-7) or np.any(x > lp.u + 1e-7):
            continue
        v = float(lp.c @ x)
        if best is None or v < best - tol:
            best, best_x = v, x
    return best, best_x


def entrywise_err(got, ref, floor):
    """Largest entry-wise error max_i |got_i - ref_i| / (|ref_i| + floor * max_j |ref_j|):
    a value below rtol means every entry agrees to rtol relative to its own size, or to
    rtol * floor of the vector's largest entry for entries smaller than that."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape
    if ref.size == 0:
        return 0.0
    scale = np.abs(ref) + floor * float(np.abs(ref).max())
    d = np.abs(got - ref)
    return float(np.max(np.where(scale > 0, d / np.where(scale > 0, scale, 1.0), np.where(d > 0, np.inf, 0.0))))


def norm_rel(got, ref):
    """||got - ref||_2 / ||ref||_2."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / max(float(np.linalg.norm(ref)), 1e-300))


def err64(got, ref):
    """Float64 path against the oracle: the larger of the 2-norm relative
    error and the entry-wise error with a floor of 1e-3 of the largest entry."""
    return max(norm_rel(got, ref), entrywise_err(got, ref, 1e-3))


def err32(got, ref):
    """Float32 path against the oracle: the largest of the 2-norm relative
    error, the largest entry error relative to the largest entry (infinity
    norm), and a tenth of the entry-wise error with a floor of 1e-2 of the
    largest entry.  Below 1e-5 it means: the iterate agrees to 1e-5 in norm,
    no entry is off by more than 1e-5 of the largest, and every entry agrees
    to 1e-4 of its own size or of 1/100 of the largest entry."""
    return max(norm_rel(got, ref), entrywise_err(got, ref, 1.0), 0.1 * entrywise_err(got, ref, 1e-2))
