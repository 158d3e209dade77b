"""Serial float64 reference of AA-PDHG / FAA-PDHG for LP.

TEST INFRASTRUCTURE ONLY.  This module is the oracle that the GPU path is
checked against.  Only the test-suite, the package smoke check and the CPU
baseline leg of the benchmark may import it.  It shares no code with the GPU
library and imports nothing from it.

It is written to be read against the paper (arXiv 2508.08062), step by step,
with no blocking, fusion or reordering beyond what the algorithms state.
Library primitives used as single steps: scipy.sparse matrix-vector products,
numpy.linalg.cholesky / solve_triangular / qr, numpy reductions.

Notation follows the paper: u = (x, y), T is one PDHG step (eq. pdhg),
g^k = T u^k - u^k is the fixed-point residual, Delta U / Delta G hold the last
m_k iterate / residual differences (oldest column first), i and j count AA and
PDHG steps, D-hat is the diagonal of Remark se:Dhat_construction.

Every function below is pinned by tests/test_oracle_*.py and
tests/test_bruteforce.py against values and properties the paper and the
mathematics fix.  The paper prints no iteration counts, so the convergence
speed under the D-hat and eta readings below is not compared with it.

Readings of points where the paper is silent or ambiguous (each is an option
where it matters, and the GPU library takes the same reading):
  * D-hat_1 (length n) scales x and D-hat_2 (length m) scales y: the block sizes
    decide (Remark se:Dhat_construction names them the other way round).
  * dhat_mode 1 is the literal square root of the max-abs entry; 2 is its
    reciprocal; 0 is the identity.
  * eta is an absolute Tikhonov shift (Alg 2, AA update line).
  * The KKT test (Remark re:constrcution-termi-con) is evaluated at u^k in
    place of Alg 2's ||g^k|| < tol test, every ``kkt_every`` iterations
    (iterations k with k % kkt_every == 0); u^k is returned.
  * u^0 = (clip(0, l, u), 0).
  * Ties in the safeguard take the AA branch (the test is "<=").
  * A failed Cholesky factorisation or a non-finite gamma makes that step a
    PDHG step; the memory is still updated (Section 3: memory refreshed on both
    branches).
  * FAA: the angle filter factors the reversed Delta G once and judges every
    column against that one factorisation; a column of zero norm, or one past
    the rank bound (m_k > n + m), is dropped.  When no k passes the length
    filter its loop runs out and m-bar = 0: the step keeps no history and
    u_AA = u^k + beta D-hat g^k.  This is the reading under which Lemma
    lem:conditioning_after_stab holds for every output of the filter.  The
    option ``length_floor`` = 1 takes the other reading (the loop stops at
    k = 1, so m-bar = 1 and the newest column is always kept).  The
    filtered columns become the memory that the next difference pair is
    appended to (Section 5, implemented variant).
  * Infinite bounds contribute nothing to the dual objective; the set Lambda
    forces the matching part of lambda to zero (eq. lambda-case).
  * Primal-weight update (Alg 7, optional, ``pw_period`` = U_P > 0): it runs
    at the top of iteration k (k > 0, k % U_P == 0), before T u^k, and
    measures x^k - x^{k-U_P}, y^k - y^{k-U_P} against the iterate of the
    previous check (u^0 for the first).  An accepted update resets the memory;
    the difference pair of iteration k would join residuals of two different
    maps and is not formed, so iteration k has m_k = 0 and its AA step (if the
    safeguard lets it through) is u^k + beta D-hat g^k.  The counters i, j and
    ||g^0|| carry on.  The step sizes are tau = gamma / omega and
    sigma = gamma * omega with gamma = sqrt(tau_0 sigma_0) and, unless given,
    omega^0 = sqrt(sigma_0 / tau_0).
  * D-hat re-blend (remark on the primal-weight form, optional ``pw_dhat``):
    after an accepted update, at iteration k once g^k is known,
    rho_k = (||g^{k-1}|| - ||g^k||) / max(||g^{k-1}||, eps_zero); "decreases
    sufficiently" is rho_k > ``pw_rho`` (default 0), giving alpha = 0.1, else
    alpha = 0.9; D-hat_1, D-hat_2 in R are those of the D-hat construction.
  * Iter_AA / c (supplement, update-D-hat study): the safeguard bound uses
    (i/c + 1) in place of (i + 1), real division; c = ``sg_div`` (default 1).
  * Fixed-frequency restarted PDHG (the toy comparison of Section 5.2, restart
    length 75): PDHG steps; the iterates u^1, u^2, ... are grouped in epochs of
    R = ``restart_period`` consecutive iterates, and the last iterate of each
    epoch is replaced by the epoch's average (the restart point of the cited
    restarted PDHG); the next epoch starts after it.  The paper names the
    scheme but not the restart point.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg
import scipy.sparse

ROW_EQ = 0
ROW_GE = 1

VARIANT_PDHG = 0
VARIANT_AA = 1
VARIANT_FAA = 2
VARIANT_RPDHG = 3  # fixed-frequency restarted PDHG (Section 5.2, the toy comparison)


# ---------------------------------------------------------------------------
# problem data (Section 2.1, LP-O; K = [G; A], q = [h; b])
# ---------------------------------------------------------------------------

class Problem:
    """min c^T x s.t. (Kx)_i >= q_i on GE rows, (Kx)_i = q_i on EQ rows,
    l <= x <= u.  All data float64."""

    def __init__(self, m, n, rowptr, colidx, val, c, q, l, u, rowtype):
        self.m, self.n = int(m), int(n)
        self.K = scipy.sparse.csr_matrix(
            (np.asarray(val, dtype=np.float64), np.asarray(colidx), np.asarray(rowptr)),
            shape=(self.m, self.n))
        self.KT = self.K.T.tocsr()
        self.c = np.asarray(c, dtype=np.float64)
        self.q = np.asarray(q, dtype=np.float64)
        self.l = np.asarray(l, dtype=np.float64)
        self.u = np.asarray(u, dtype=np.float64)
        self.rowtype = np.asarray(rowtype, dtype=np.uint8)
        self.ge = self.rowtype == ROW_GE

    @classmethod
    def from_lpdata(cls, lp):
        return cls(lp.m, lp.n, lp.rowptr, lp.colidx, lp.val, lp.c, lp.q, lp.l, lp.u, lp.rowtype)

    def rounded_fp32(self):
        """The same LP with its data rounded to float32 values (the LP that a
        float32 solver holds)."""
        f = lambda a: a.astype(np.float32).astype(np.float64)
        K = self.K
        return Problem(self.m, self.n, K.indptr, K.indices, f(K.data), f(self.c), f(self.q),
                       f(self.l), f(self.u), self.rowtype)


# ---------------------------------------------------------------------------
# projections (Section 3: X = {l <= x <= u}, Y = R_+^{m1} x R^{m2}; P = diag(P_X, P_Y))
# ---------------------------------------------------------------------------

def proj_X(P: Problem, x):
    return np.minimum(np.maximum(x, P.l), P.u)


def proj_Y(P: Problem, y):
    return np.where(P.ge, np.maximum(y, 0.0), y)


def proj_Lambda(P: Problem, lam):
    """Projection onto Lambda = prod Lambda_i (eq. lambda-case):
    {0} if both bounds are infinite, R_- if only u is finite, R_+ if only l is
    finite, R if both are finite."""
    lf = np.isfinite(P.l)
    uf = np.isfinite(P.u)
    out = lam.copy()
    out = np.where(~lf & ~uf, 0.0, out)
    out = np.where(~lf & uf, np.minimum(out, 0.0), out)
    out = np.where(lf & ~uf, np.maximum(out, 0.0), out)
    return out


# ---------------------------------------------------------------------------
# the fixed-point map T (eq. pdhg; new-fixed-point)
# ---------------------------------------------------------------------------

def pdhg_map(P: Problem, x, y, tau, sigma):
    """One PDHG step:
        x_hat = P_X(x - tau (c - K^T y))
        y_hat = P_Y(y + sigma (q - K (2 x_hat - x)))
    Returns (x_hat, y_hat)."""
    x_hat = proj_X(P, x - tau * (P.c - P.KT @ y))
    y_hat = proj_Y(P, y + sigma * (P.q - P.K @ (2.0 * x_hat - x)))
    return x_hat, y_hat


# ---------------------------------------------------------------------------
# D-hat (Remark se:Dhat_construction)
# ---------------------------------------------------------------------------

def dhat(P: Problem, mode: int = 1):
    """Diagonal of D-hat as one vector of length n + m (x part, then y part)."""
    if mode == 0:
        return np.ones(P.n + P.m)
    absK = abs(P.K)
    colmax = np.asarray(absK.max(axis=0).todense()).ravel()
    rowmax = np.asarray(absK.max(axis=1).todense()).ravel()
    d = np.sqrt(np.maximum(np.concatenate((colmax, rowmax)), 1e-10))
    if mode == 1:
        return d
    if mode == 2:
        return 1.0 / d
    raise ValueError("dhat mode must be 0, 1 or 2")


# ---------------------------------------------------------------------------
# KKT residual (Remark re:constrcution-termi-con, eqs. duality-gap,
# primal-feasi, dual-feasi)
# ---------------------------------------------------------------------------

def kkt(P: Problem, x, y):
    """Relative KKT residual at (x, y) with lambda = P_Lambda(c - K^T y)."""
    w = P.KT @ y
    lam = proj_Lambda(P, P.c - w)
    lam_plus = np.maximum(lam, 0.0)
    lam_minus = np.maximum(-lam, 0.0)
    lf = np.isfinite(P.l)
    uf = np.isfinite(P.u)
    pobj = float(P.c @ x)
    dobj = float(P.q @ y + np.sum(P.l[lf] * lam_plus[lf]) - np.sum(P.u[uf] * lam_minus[uf]))
    r_g = abs(dobj - pobj) / (1.0 + abs(dobj) + abs(pobj))
    res = P.q - P.K @ x  # b - Ax on EQ rows, h - Gx on GE rows
    res = np.where(P.ge, np.maximum(res, 0.0), res)
    r_p = float(np.linalg.norm(res)) / (1.0 + float(np.linalg.norm(P.q)))
    r_d = float(np.linalg.norm(P.c - w - lam)) / (1.0 + float(np.linalg.norm(P.c)))
    return {"pobj": pobj, "dobj": dobj, "r_g": r_g, "r_p": r_p, "r_d": r_d,
            "kkt": max(r_g, r_p, r_d), "lam": lam}


# ---------------------------------------------------------------------------
# step size by power iteration (Section 5.1)
# ---------------------------------------------------------------------------

_SM_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(seed: int, count: int):
    """The first ``count`` outputs of SplitMix64 (Steele, Lea and Flood,
    OOPSLA 2014) started at state ``seed``: output j mixes the state
    seed + (j + 1) * 0x9E3779B97F4A7C15 with two xor-shift-multiply rounds and
    a final xor-shift.  uint64 arithmetic wraps modulo 2^64."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.arange(1, count + 1, dtype=np.uint64) * _SM_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def power_start(n: int, seed: int = 0):
    """Start vector of the power iteration: entry j is 2u - 1 with u the top
    53 bits of SplitMix64 output j as a fraction in [0, 1).  A random start
    reaches the dominant singular vector whatever the sign pattern of K (a
    constant start is orthogonal to it when, say, every row of K sums to
    zero)."""
    u = (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return 2.0 * u - 1.0


def power_norm(P: Problem, iters: int = 200, rtol: float = 1e-8, v0=None, seed: int = 0):
    """Estimate ||K||_2 as sqrt of the dominant eigenvalue of K^T K by power
    iteration.  The start vector is v0 (default: power_start(n, seed))."""
    v = power_start(P.n, seed) if v0 is None else np.asarray(v0, dtype=np.float64).copy()
    v /= np.linalg.norm(v)
    est = 0.0
    for _ in range(iters):
        z = P.KT @ (P.K @ v)
        nz = float(np.linalg.norm(z))
        if nz == 0.0:
            return 0.0
        new = math.sqrt(nz)  # ||K^T K v|| with ||v|| = 1
        v = z / nz
        if est > 0.0 and abs(new - est) <= rtol * new:
            est = new
            break
        est = new
    return est


# ---------------------------------------------------------------------------
# Ruiz equilibration (Section 5.2 preprocessing)
# ---------------------------------------------------------------------------

def ruiz(P: Problem, iters: int = 10):
    """``iters`` sweeps of infinity-norm equilibration.  Each sweep takes the
    row and column max-abs of the current matrix, r_i and s_j, replaces zeros by
    one, and divides entry (i,j) by sqrt(r_i) * sqrt(s_j).  Returns the scaled
    problem and (d_row, d_col) with K_scaled = diag(d_row) K diag(d_col).
    Variables map back as x = d_col * x_s, y = d_row * y_s."""
    K = P.K.copy().astype(np.float64)
    rows = np.repeat(np.arange(P.m), np.diff(K.indptr))
    d_row = np.ones(P.m)
    d_col = np.ones(P.n)
    for _ in range(iters):
        absK = abs(K)
        rmax = np.asarray(absK.max(axis=1).todense()).ravel()
        cmax = np.asarray(absK.max(axis=0).todense()).ravel()
        r = np.sqrt(np.where(rmax > 0.0, rmax, 1.0))
        s = np.sqrt(np.where(cmax > 0.0, cmax, 1.0))
        K.data = K.data / (r[rows] * s[K.indices])
        d_row = d_row / r
        d_col = d_col / s
    scaled = Problem(P.m, P.n, K.indptr, K.indices, K.data, P.c * d_col, P.q * d_row,
                     P.l / d_col, P.u / d_col, P.rowtype)
    return scaled, d_row, d_col


def pock_chambolle(P: Problem, alpha: float = 1.0):
    """Diagonal Pock-Chambolle scaling with parameter alpha (the
    preconditioning of Section 5.2 together with Ruiz): row i is divided by
    sqrt(sum_j |K_ij|^alpha) and column j by sqrt(sum_i |K_ij|^(2 - alpha))
    (zero sums replaced by one), both measured on the matrix as given.
    Returns the scaled problem and (d_row, d_col) as ruiz does."""
    K = P.K.copy().astype(np.float64)
    rows = np.repeat(np.arange(P.m), np.diff(K.indptr))
    a = np.abs(K.data)
    rsum = np.zeros(P.m)
    csum = np.zeros(P.n)
    np.add.at(rsum, rows, a ** alpha)
    np.add.at(csum, K.indices, a ** (2.0 - alpha))
    r = np.sqrt(np.where(rsum > 0.0, rsum, 1.0))
    s = np.sqrt(np.where(csum > 0.0, csum, 1.0))
    K.data = K.data / (r[rows] * s[K.indices])
    d_row = 1.0 / r
    d_col = 1.0 / s
    scaled = Problem(P.m, P.n, K.indptr, K.indices, K.data, P.c * d_col, P.q * d_row,
                     P.l / d_col, P.u / d_col, P.rowtype)
    return scaled, d_row, d_col


# ---------------------------------------------------------------------------
# Anderson pieces
# ---------------------------------------------------------------------------

def aa_gamma(dG, g, eta):
    """gamma = (dG^T dG + eta I)^{-1} dG^T g by Cholesky (Alg 2, AA update).
    Returns None if the factorisation fails or gamma is not finite."""
    A = dG.T @ dG + eta * np.eye(dG.shape[1])
    try:
        L = np.linalg.cholesky(A)
    except np.linalg.LinAlgError:
        return None
    z = scipy.linalg.solve_triangular(L, dG.T @ g, lower=True)
    gamma = scipy.linalg.solve_triangular(L.T, z, lower=False)
    return gamma if np.all(np.isfinite(gamma)) else None


def reverse(E, F):
    """Alg 6: reverse the column order of both matrices."""
    return E[:, ::-1], F[:, ::-1]


def angle_filter(E, F, cs, sequential=False):
    """Alg 4 on matrices whose first column is the newest.  One economy QR of
    F; column i >= 2 is removed when |r_ii| / ||f_i|| < cs.  Returns the kept
    column indices (into the input order).

    ``sequential``: the factor is refreshed after every removal, so column i
    is judged by its distance from the span of the columns kept so far (the
    last diagonal entry of the QR of those columns followed by f_i)."""
    m = F.shape[1]
    if sequential:
        keep = [0]
        for i in range(1, m):
            fn = float(np.linalg.norm(F[:, i]))
            if fn == 0.0 or len(keep) >= F.shape[0]:
                continue
            _, Ri = np.linalg.qr(F[:, keep + [i]], mode="reduced")
            if abs(Ri[-1, -1]) / fn >= cs:
                keep.append(i)
        return keep
    _, R = np.linalg.qr(F, mode="reduced")
    keep = [0]
    for i in range(1, m):
        fn = float(np.linalg.norm(F[:, i]))
        if fn == 0.0 or i >= R.shape[0]:
            continue
        if abs(R[i, i]) / fn >= cs:
            keep.append(i)
    return keep


def length_bounds(fnorm, cs):
    """Upper bounds b_j on ||column j of R^{-1}||^2 (Lemma le:RK-1bound1),
    from the column norms ||f_j|| of F (newest first).  A zero norm gives an
    infinite bound.  b_j equals the sum over i <= j of the squares of
    Lemma eq:lemma1.51's bounds on the entries s_ij of that column."""
    ct = math.sqrt(1.0 - cs * cs)
    m = len(fnorm)
    b = np.zeros(m)
    fnorm = np.asarray(fnorm, dtype=np.float64)  # numpy division: 1/0 -> inf
    for j in range(1, m + 1):  # 1-based as in the lemma
        if j == 1:
            b[0] = 1.0 / fnorm[0] ** 2
            continue
        total = ct ** 2 * (ct + cs) ** (2 * (j - 2)) / (fnorm[0] ** 2 * cs ** (2 * (j - 2)))
        for i in range(2, j):
            total += ct ** 2 * (ct + cs) ** (2 * (j - i - 1)) / (fnorm[i - 1] ** 2 * cs ** (2 * (j - i)))
        total += 1.0 / fnorm[j - 1] ** 2
        b[j - 1] = total / cs ** 2
    return b


def length_filter(enorm, fnorm, cs, kappa_bar, floor=0):
    """Alg 5: the largest k (counting down from m) with
    (sum_{j<=k} e_j^2)(sum_{j<=k} b_j) <= kappa_bar^2.  When no k passes,
    the count-down loop runs out: ``floor`` = 0 returns 0 (nothing kept),
    ``floor`` = 1 returns 1 (the loop read as stopping at k = 1, so the
    newest column is always kept).  A NaN product (0 * inf) does not pass."""
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        b = length_bounds(fnorm, cs)
        m = len(fnorm)
        k = m
        while k >= 1:
            C = float(np.sum(np.asarray(enorm[:k]) ** 2)) * float(np.sum(b[:k]))
            if C <= kappa_bar * kappa_bar:
                break
            k -= 1
    if k < floor and m > 0:
        k = floor
    return k


# ---------------------------------------------------------------------------
# the solver (Alg 2 = AA-PDHG, Alg 3 = FAA-PDHG, and vanilla PDHG)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Options:
    variant: int = VARIANT_AA
    memory: int = 5  # m_A
    D: float = 10.0  # safeguard constant
    eps_sg: float = 1.0  # safeguard exponent epsilon
    beta: float = 1.0
    eta: float = 1e-10
    cs: float = 0.2
    kappa_bar: float = 1e8
    angle_mode: int = 0  # 0: Alg 4 with one factorisation; 1: refreshed after each removal
    length_floor: int = 0  # Alg 5 when no k passes: 0 keeps nothing, 1 keeps the newest column
    tau: float = 0.0  # <= 0: 0.9 / ||K|| by power iteration
    sigma: float = 0.0
    tol: float = 1e-4
    max_iter: int = 1000
    kkt_every: int = 64
    dhat_mode: int = 1
    fpr_stop: bool = False  # Alg 2's literal ||g^k|| < tol test
    sg_div: float = 1.0  # c of the Iter_AA / c safeguard
    # primal-weight update (Alg 7) and D-hat re-blend (remark on the primal-weight form)
    pw_period: int = 0  # U_P; 0 = off
    pw_theta: float = 0.5  # smoothing theta
    pw_eps_zero: float = 1e-10  # epsilon_zero
    pw_omega0: float = 0.0  # omega^0; <= 0: sqrt(sigma / tau)
    pw_dhat: bool = True  # re-blend D-hat after each accepted update
    pw_rho: float = 0.0  # rho_k above this: alpha = 0.1, else 0.9
    restart_period: int = 75  # R of the restarted PDHG variant
    seed: int = 0  # power-iteration start vector (power_start)


@dataclasses.dataclass
class State:
    """Everything the iteration carries from k to k+1."""
    k: int  # index of the current iterate u^k
    x: np.ndarray
    y: np.ndarray
    u_prev: np.ndarray  # u^{k-1} (x then y)
    g_prev: np.ndarray  # g^{k-1}
    dU: list  # columns, oldest first
    dG: list
    i: int = 0  # AA steps taken
    j: int = 0  # PDHG steps taken
    n0: float = 0.0  # ||g^0||
    rsum: np.ndarray = None  # restarted PDHG: sum of the epoch's iterates so far
    rcount: int = 0


class Solver:
    """AA-PDHG / FAA-PDHG / PDHG on a Problem, one iteration per ``step``."""

    def __init__(self, P: Problem, opt: Options):
        self.P = P
        self.opt = dataclasses.replace(opt)
        if self.opt.tau <= 0.0 or self.opt.sigma <= 0.0:
            nrm = power_norm(P, seed=self.opt.seed)
            self.opt.tau = self.opt.sigma = 0.9 / nrm if nrm > 0.0 else 1.0
        self.Dhat = dhat(P, self.opt.dhat_mode)
        self.Dhat0 = self.Dhat.copy()  # D-hat_1, D-hat_2 of the construction
        # primal weight: tau = gamma / omega, sigma = gamma * omega (remark on the primal-weight form)
        self.step_gamma = math.sqrt(self.opt.tau * self.opt.sigma)
        self.omega = self.opt.pw_omega0 if self.opt.pw_omega0 > 0.0 else math.sqrt(self.opt.sigma / self.opt.tau)
        if self.opt.pw_omega0 > 0.0:
            self.opt.tau = self.step_gamma / self.omega
            self.opt.sigma = self.step_gamma * self.omega
        self.pw_log = []  # (k, dx, dy, accepted, omega after, alpha or None)
        self.status = "running"
        self.last_branch = None
        self.last_gamma = None
        self.last_kkt = None
        self.kkt_trace = []  # (k, kkt dict without lambda)
        self.faa_empty = 0  # FAA steps whose filters kept no column

    # -- Alg 2, initialisation ------------------------------------------------
    def start(self):
        P = self.P
        x0 = proj_X(P, np.zeros(P.n))
        y0 = np.zeros(P.m)
        x1, y1 = pdhg_map(P, x0, y0, self.opt.tau, self.opt.sigma)
        u0 = np.concatenate((x0, y0))
        u1 = np.concatenate((x1, y1))
        g0 = u1 - u0
        self.state = State(k=1, x=x1, y=y1, u_prev=u0, g_prev=g0, dU=[], dG=[],
                           n0=float(np.linalg.norm(g0)))
        self.anchor = u0.copy()  # iterate of the last primal-weight check
        if self.opt.variant == VARIANT_RPDHG:
            u1 = self._restart_point(u1)
            self.state.x, self.state.y = u1[:P.n].copy(), u1[P.n:].copy()
        if self.state.n0 == 0.0:
            self.state = dataclasses.replace(self.state, k=0, x=x0, y=y0)
            self.status = "converged"
        return self.state

    # -- Alg 2 / Alg 3, loop body ----------------------------------------------
    def step(self):
        """One pass of the loop body at iteration k.  Returns the status."""
        P, o, S = self.P, self.opt, self.state
        n = P.n
        u = np.concatenate((S.x, S.y))
        reset = self._primal_weight(u) if o.pw_period > 0 else False
        xh, yh = pdhg_map(P, S.x, S.y, o.tau, o.sigma)
        u_hat = np.concatenate((xh, yh))
        g = u_hat - u
        gnorm = float(np.linalg.norm(g))
        self.last_gnorm = gnorm

        # termination test at u^k
        if o.kkt_every > 0 and S.k % o.kkt_every == 0:
            r = kkt(P, S.x, S.y)
            self.last_kkt = r
            self.kkt_trace.append((S.k, {kk: v for kk, v in r.items() if kk != "lam"}))
            if r["kkt"] <= o.tol:
                self.status = "converged"
                return self.status
        if o.fpr_stop and gnorm < o.tol:
            self.status = "converged"
            return self.status

        if reset:
            if o.pw_dhat:
                self._reblend_dhat(float(np.linalg.norm(S.g_prev)), gnorm)
            # the pair (u^k - u^{k-1}, g^k - g^{k-1}) straddles the weight change: not formed
        else:
            # memory update (both branches)
            S.dU.append(u - S.u_prev)
            S.dG.append(g - S.g_prev)
            while len(S.dU) > o.memory:
                S.dU.pop(0)
                S.dG.pop(0)

        u_next = None
        gamma = None
        branch = "pdhg"
        if o.variant in (VARIANT_AA, VARIANT_FAA) and gnorm <= o.D * S.n0 * (S.i / o.sg_div + 1) ** (-(1.0 + o.eps_sg)):
            N = P.n + P.m
            dU = np.stack(S.dU, axis=1) if S.dU else np.zeros((N, 0))
            dG = np.stack(S.dG, axis=1) if S.dG else np.zeros((N, 0))
            if dG.shape[1] == 0:
                gamma = np.zeros(0)  # empty memory: H^k = -beta D-hat
            elif o.variant == VARIANT_AA:
                gamma = aa_gamma(dG, g, o.eta)
            else:
                gamma, dU, dG = self._faa(dU, dG, g)
            if gamma is not None:
                # u_AA = u^k - H^k g^k with
                # H^k = -beta D + (dU + beta D dG) (dG^T dG + eta I)^{-1} dG^T
                Dg = self.Dhat[:, None] * dG
                Hg = -o.beta * self.Dhat * g + (dU + o.beta * Dg) @ gamma
                u_aa = u - Hg
                u_next = np.concatenate((proj_X(P, u_aa[:n]), proj_Y(P, u_aa[n:])))
                branch = "aa"
        if u_next is None:
            u_next = u_hat
            if o.variant == VARIANT_RPDHG:
                u_next = self._restart_point(u_hat)
            S.j += 1
        else:
            S.i += 1
        self.last_branch = branch
        self.last_gamma = gamma
        S.u_prev = u
        S.g_prev = g
        S.x = u_next[:n].copy()
        S.y = u_next[n:].copy()
        S.k += 1
        return self.status

    # -- restarted PDHG: the epoch's iterates and its restart -------------------
    def _restart_point(self, u_new):
        """Adds the new iterate to the epoch; returns it, or the epoch's
        average when it completes the epoch of restart_period iterates."""
        S, R = self.state, self.opt.restart_period
        S.rsum = u_new.copy() if S.rcount == 0 else S.rsum + u_new
        S.rcount += 1
        if S.rcount < R:
            return u_new
        avg = S.rsum / R
        S.rsum, S.rcount = None, 0
        return avg

    # -- Alg 7 (primal-weight update), at the top of iteration k ------------------
    def _primal_weight(self, u):
        """Returns True when the weight was updated (and the memory reset)."""
        P, o, S = self.P, self.opt, self.state
        if not (S.k > 0 and S.k % o.pw_period == 0):
            return False
        n = P.n
        dx = float(np.linalg.norm(u[:n] - self.anchor[:n]))
        dy = float(np.linalg.norm(u[n:] - self.anchor[n:]))
        self.anchor = u.copy()
        if dx > o.pw_eps_zero and dy > o.pw_eps_zero:
            S.dU, S.dG = [], []
            self.omega = math.exp(o.pw_theta * math.log(dy / dx) + (1.0 - o.pw_theta) * math.log(self.omega))
            o.tau = self.step_gamma / self.omega
            o.sigma = self.step_gamma * self.omega
            self.pw_log.append([S.k, dx, dy, True, self.omega, None])
            return True
        self.pw_log.append([S.k, dx, dy, False, self.omega, None])
        return False

    # -- D-hat = (1 - alpha) D_1 + alpha R (remark on the primal-weight form) -----
    def _reblend_dhat(self, r_prev, r_cur):
        o, n = self.opt, self.P.n
        rho = (r_prev - r_cur) / max(r_prev, o.pw_eps_zero)
        alpha = 0.1 if rho > o.pw_rho else 0.9
        w = self.omega
        D1 = np.concatenate((np.full(n, 1.0 / w), np.full(self.P.m, w)))
        R = np.concatenate((self.Dhat0[:n] / w, self.Dhat0[n:] * w))
        self.Dhat = (1.0 - alpha) * D1 + alpha * R
        self.pw_log[-1][5] = alpha

    def _faa(self, dU, dG, g):
        """Alg 3 lines Reverse .. QR: filter the memory, then gamma = R^{-1} Q^T g."""
        o, S = self.opt, self.state
        E, F = reverse(dU, dG)  # newest first
        keep = angle_filter(E, F, o.cs, sequential=o.angle_mode == 1)
        E, F = E[:, keep], F[:, keep]
        mbar = length_filter(np.linalg.norm(E, axis=0), np.linalg.norm(F, axis=0), o.cs, o.kappa_bar,
                             floor=o.length_floor)
        if mbar == 0:
            self.faa_empty += 1
        E, F = E[:, :mbar], F[:, :mbar]
        dU, dG = reverse(E, F)  # oldest first again
        # the filtered columns become the memory
        S.dU = [dU[:, t].copy() for t in range(dU.shape[1])]
        S.dG = [dG[:, t].copy() for t in range(dG.shape[1])]
        if mbar == 0:
            return np.zeros(0), dU, dG
        Q, R = np.linalg.qr(dG, mode="reduced")
        gamma = scipy.linalg.solve_triangular(R, Q.T @ g, lower=False)
        if not np.all(np.isfinite(gamma)):
            return None, dU, dG
        return gamma, dU, dG

    def solve(self, trace=False):
        """Run until convergence or max_iter loop passes.  With ``trace`` the
        iterates u^1, u^2, ... are recorded."""
        self.start()
        self.trace = [np.concatenate((self.state.x, self.state.y))] if trace else None
        iters = 0
        while self.status == "running" and iters < self.opt.max_iter:
            self.step()
            iters += 1
            if trace and self.status == "running":
                self.trace.append(np.concatenate((self.state.x, self.state.y)))
        if self.status == "running":
            self.status = "iter_limit"
        return self.result()

    def result(self):
        S = self.state
        r = kkt(self.P, S.x, S.y)
        return {"status": self.status, "k": S.k, "x": S.x, "y": S.y, "lam": r["lam"],
                "aa_steps": S.i, "pdhg_steps": S.j, "kkt": r}


def solve(P: Problem, **kw):
    """Convenience wrapper: Solver(P, Options(**kw)).solve()."""
    s = Solver(P, Options(**kw))
    return s.solve(), s
