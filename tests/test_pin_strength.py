"""Strength of the oracle's pins.

Each plausible mistake below (a dropped term, a wrong sign, a swapped
operand or index) is planted in a temporary copy of the oracle, never in the
oracle itself; the pin files then run against that copy in a subprocess and
must fail.  The unmodified copy must pass them, so a failure is the planted
mistake's doing.  CPU only."""
import concurrent.futures
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["test_oracle_units.py", "test_bruteforce.py", "test_oracle_pw.py", "test_oracle_restart.py"]
ORACLE = "aapdhg_oracle.py"

# (name, text in the oracle, replacement)
MUTATIONS = [
    ("pdhg: sign of K^T y", "x - tau * (P.c - P.KT @ y)", "x - tau * (P.c + P.KT @ y)"),
    ("pdhg: no extrapolation", "P.K @ (2.0 * x_hat - x)", "P.K @ x_hat"),
    ("pdhg: sigma for tau", "x - tau * (P.c", "x - sigma * (P.c"),
    ("projection onto Y dropped", "np.where(P.ge, np.maximum(y, 0.0), y)", "y"),
    ("Lambda: R- case as R+", "np.where(~lf & uf, np.minimum(out, 0.0), out)",
     "np.where(~lf & uf, np.maximum(out, 0.0), out)"),
    ("KKT: l^T lambda+ dropped", " + np.sum(P.l[lf] * lam_plus[lf])", ""),
    ("KKT: GE residual part", "res = np.where(P.ge, np.maximum(res, 0.0), res)",
     "res = np.where(P.ge, np.minimum(res, 0.0), res)"),
    ("KKT: dual residual without lambda", "np.linalg.norm(P.c - w - lam)", "np.linalg.norm(P.c - w)"),
    ("AA: sign of the beta D g term", "Hg = -o.beta * self.Dhat * g +", "Hg = o.beta * self.Dhat * g +"),
    ("AA: dU term dropped", "(dU + o.beta * Dg) @ gamma", "(o.beta * Dg) @ gamma"),
    ("AA: D-hat left out of the dG term", "Dg = self.Dhat[:, None] * dG", "Dg = dG"),
    ("AA: gamma from dG^T u instead of dG^T g", "gamma = aa_gamma(dG, g, o.eta)", "gamma = aa_gamma(dG, u, o.eta)"),
    ("memory: dG without the previous residual", "S.dG.append(g - S.g_prev)", "S.dG.append(g)"),
    ("memory: keeps one column too many", "while len(S.dU) > o.memory:", "while len(S.dU) > o.memory + 1:"),
    ("safeguard: exponent sign", "** (-(1.0 + o.eps_sg))", "** (1.0 + o.eps_sg)"),
    ("angle filter: test inverted", "if abs(R[i, i]) / fn >= cs:", "if abs(R[i, i]) / fn < cs:"),
    ("length bound: ct for cs in the first term", "/ (fnorm[0] ** 2 * cs ** (2 * (j - 2)))",
     "/ (fnorm[0] ** 2 * ct ** (2 * (j - 2)))"),
    ("length bound: 1 / cs^2 dropped", "b[j - 1] = total / cs ** 2", "b[j - 1] = total"),
    ("length bound: power of (ct + cs) in the first term one higher", "(ct + cs) ** (2 * (j - 2))",
     "(ct + cs) ** (2 * (j - 1))"),
    ("length bound: power of (ct + cs) in the sum one higher", "(ct + cs) ** (2 * (j - i - 1))",
     "(ct + cs) ** (2 * (j - i))"),
    ("length bound: power of cs in the sum one lower", "cs ** (2 * (j - i)))", "cs ** (2 * (j - i - 1)))"),
    ("length bound: norm of the wrong column in the sum", "/ (fnorm[i - 1] ** 2 *", "/ (fnorm[i] ** 2 *"),
    ("length filter: keeps one more", "        k = floor\n    return k", "        k = floor\n    return min(k + 1, m)"),
    ("length filter: floor of one under either reading", "if k < floor and m > 0:\n        k = floor",
     "if k < 1 and m > 0:\n        k = 1"),
    ("power iteration: eigenvalue for norm", "new = math.sqrt(nz)", "new = nz"),
    ("Ruiz: column factor inverted", "        d_col = d_col / s\n", "        d_col = d_col * s\n"),
    ("restart: average over R + 1", "avg = S.rsum / R", "avg = S.rsum / (R + 1)"),
    ("primal weight: ratio inverted", "math.log(dy / dx)", "math.log(dx / dy)"),
    ("primal weight: tau and sigma swapped", "o.tau = self.step_gamma / self.omega\n            o.sigma = self.step_gamma * self.omega",
     "o.tau = self.step_gamma * self.omega\n            o.sigma = self.step_gamma / self.omega"),
    ("D-hat: reciprocal for the literal reading", "    if mode == 1:\n        return d", "    if mode == 1:\n        return 1.0 / d"),
    ("start point: y^0 = 1", "y0 = np.zeros(P.m)", "y0 = np.ones(P.m)"),
    ("KKT: gap relative to the dual objective only", "(1.0 + abs(dobj) + abs(pobj))", "(1.0 + abs(dobj))"),
    ("SplitMix64: second mixing round dropped",
     "z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)", "z = z ^ (z >> np.uint64(27))"),
    ("sequential angle filter against every earlier column", "np.linalg.qr(F[:, keep + [i]], mode=\"reduced\")",
     "np.linalg.qr(F[:, : i + 1], mode=\"reduced\")"),
    ("FAA: memory left newest first", "dU, dG = reverse(E, F)  # oldest first again", "dU, dG = E, F"),
    ("restart: epoch one iterate longer", "if S.rcount < R:", "if S.rcount <= R:"),
    ("D-hat re-blend: alpha cases swapped", "alpha = 0.1 if rho > o.pw_rho else 0.9",
     "alpha = 0.9 if rho > o.pw_rho else 0.1"),
]


def _tree(tmp, mutation):
    """A minimal copy of the repository (oracle, generators, pin files and
    fixtures) with the mutation applied to the oracle copy."""
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(tmp, "oracle"),
                    ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copytree(os.path.join(ROOT, "lpgen"), os.path.join(tmp, "lpgen"),
                    ignore=shutil.ignore_patterns("__pycache__"))
    os.makedirs(os.path.join(tmp, "tests"))
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), os.path.join(tmp, "tests", "golden"))
    for f in PIN_FILES + ["conftest.py", "_util.py"]:
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(tmp, "tests", f))
    if mutation is not None:
        _, old, new = mutation
        path = os.path.join(tmp, "oracle", ORACLE)
        src = open(path).read()
        assert src.count(old) == 1, f"mutation site not unique or missing: {old!r}"
        with open(path, "w") as f:
            f.write(src.replace(old, new))


def _pins_pass(mutation):
    with tempfile.TemporaryDirectory() as tmp:
        _tree(tmp, mutation)
        env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1", OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
                           + [os.path.join("tests", f) for f in PIN_FILES],
                           cwd=tmp, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                           timeout=600)
        return r.returncode == 0, r.stdout[-800:]


@pytest.fixture(scope="module")
def outcomes():
    cases = [None] + MUTATIONS
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        res = list(ex.map(_pins_pass, cases))
    return dict(zip([None] + [m[0] for m in MUTATIONS], res))


def test_unmodified_copy_passes_the_pins(outcomes):
    ok, out = outcomes[None]
    assert ok, out


@pytest.mark.parametrize("name", [m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(outcomes, name):
    ok, out = outcomes[name]
    assert not ok, f"no pin fails when the oracle has the mistake '{name}'"
