"""Python binding of libaapdhg (AA-PDHG / FAA-PDHG for LP on MI355X).

Argument marshalling only: every step of the solver runs in the HIP library
``libaapdhg.so`` built in-tree by ``paper_2508_08062_amd.build``.  Importing
this package does not load the library; the first call does, and it raises
if the library is missing.  There is no CPU fallback.

Entry points mirror include/aapdhg.h:  Solver (aapdhg_create/solve/iterate/
result/get_state/set_state/get_weights/set_weights/destroy; from_device and
result_device for torch CUDA tensors through aapdhg_create_device and
aapdhg_result_device), Batch (aapdhg_batch_*), Server (aapdhg_server_*).
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libaapdhg.so")
MAX_MEMORY = 16
WEIGHT_WORDS = 10

ROW_EQ, ROW_GE = 0, 1
VARIANT_PDHG, VARIANT_AA, VARIANT_FAA, VARIANT_RPDHG = 0, 1, 2, 3
TERM_NAMES = {0: "converged", 1: "iter_limit", 2: "time_limit", 3: "numerical", 4: "running"}
OK, E_ARG, E_NOMEM, E_HIP, E_STATE, PENDING = 0, -1, -2, -3, -4, 1


class Options(C.Structure):
    _fields_ = [("variant", C.c_int32), ("precision", C.c_int32), ("memory", C.c_int32),
                ("D", C.c_double), ("eps_sg", C.c_double), ("beta", C.c_double), ("eta", C.c_double),
                ("cs", C.c_double), ("kappa_bar", C.c_double), ("tau", C.c_double), ("sigma", C.c_double),
                ("tol", C.c_double), ("max_iter", C.c_int64), ("time_limit_s", C.c_double),
                ("kkt_every", C.c_int32), ("dhat_mode", C.c_int32), ("ruiz_iters", C.c_int32),
                ("power_iters", C.c_int32), ("epoch", C.c_int32), ("chunks_per_block", C.c_int32),
                ("loop_kernel", C.c_int32), ("wait_limit_us", C.c_int32), ("pw_period", C.c_int32),
                ("pw_theta", C.c_double), ("pw_eps_zero", C.c_double), ("pw_omega0", C.c_double),
                ("pw_rho", C.c_double), ("sg_div", C.c_double), ("pw_dhat", C.c_int32),
                ("restart_period", C.c_int32), ("prep_device", C.c_int32), ("pock_chambolle", C.c_int32),
                ("angle_mode", C.c_int32), ("seed", C.c_uint64), ("length_floor", C.c_int32),
                ("graph", C.c_int32), ("autotune", C.c_int32), ("gram_mode", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("term", C.c_int32), ("gram_on_demand", C.c_int32), ("iters", C.c_int64),
                ("aa_steps", C.c_int64), ("pdhg_steps", C.c_int64), ("primal_obj", C.c_double),
                ("dual_obj", C.c_double), ("r_gap", C.c_double), ("r_pri", C.c_double),
                ("r_dual", C.c_double), ("kkt", C.c_double), ("gnorm", C.c_double),
                ("g0norm", C.c_double), ("solve_seconds", C.c_double), ("step_tau", C.c_double),
                ("step_sigma", C.c_double), ("omega", C.c_double), ("pw_updates", C.c_int64),
                ("faa_empty", C.c_int64)]

    def to_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_ if not name.startswith("reserved")}
        d["status"] = TERM_NAMES.get(self.term, str(self.term))
        return d


EXPORTS = [
    "aapdhg_default_options", "aapdhg_create", "aapdhg_solve", "aapdhg_wait", "aapdhg_iterate",
    "aapdhg_iterate_noalloc",
    "aapdhg_iterate_timed",
    "aapdhg_reset",
    "aapdhg_result", "aapdhg_create_device", "aapdhg_result_device", "aapdhg_get_state", "aapdhg_set_state",
    "aapdhg_get_weights", "aapdhg_set_weights",
    "aapdhg_get_dims", "aapdhg_get_scaling",
    "aapdhg_destroy", "aapdhg_last_error", "aapdhg_batch_create", "aapdhg_batch_solve",
    "aapdhg_batch_iterate", "aapdhg_batch_iterate_timed", "aapdhg_batch_result", "aapdhg_batch_destroy", "aapdhg_server_start", "aapdhg_server_submit",
    "aapdhg_server_poll", "aapdhg_server_stats", "aapdhg_server_stop",
]

_lib = None
# Every open handle, so that the ones a program leaves open are destroyed by an
# exit hook while the HIP runtime is still up (Python runs it before the
# process's C exit handlers), never by a finaliser during interpreter teardown.
_open = {"server": weakref.WeakSet(), "batch": weakref.WeakSet(), "solver": weakref.WeakSet()}
_P = C.c_void_p
_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)


def lib():
    """Load libaapdhg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2508_08062_amd.build`")
    L = C.CDLL(LIB_PATH)
    L.aapdhg_default_options.argtypes = [C.POINTER(Options)]
    L.aapdhg_default_options.restype = None
    L.aapdhg_create.argtypes = [C.c_int32, C.c_int32, C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                _dp, _dp, _dp, _dp, _dp, C.POINTER(C.c_uint8), C.POINTER(Options), C.POINTER(_P)]
    L.aapdhg_solve.argtypes = [_P, _P]
    L.aapdhg_wait.argtypes = [_P]
    L.aapdhg_iterate.argtypes = [_P, _P, C.c_int64]
    L.aapdhg_iterate_noalloc.argtypes = [_P, _P, C.c_int64]
    L.aapdhg_iterate_timed.argtypes = [_P, _P, C.c_int64, _dp]
    L.aapdhg_reset.argtypes = [_P, _P]
    L.aapdhg_result.argtypes = [_P, _dp, _dp, _dp, C.POINTER(Info)]
    L.aapdhg_create_device.argtypes = [C.c_int32, C.c_int32, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P,
                                       C.POINTER(Options), _P, C.POINTER(_P)]
    L.aapdhg_result_device.argtypes = [_P, _P, _P, _P, C.POINTER(Info), _P]
    L.aapdhg_get_state.argtypes = [_P, _dp, _dp, _dp, _dp, _dp, _i64p, _dp]
    L.aapdhg_set_state.argtypes = [_P, _dp, _dp, _dp, _dp, _dp, _i64p, _dp]
    L.aapdhg_get_weights.argtypes = [_P, _dp, _dp]
    L.aapdhg_set_weights.argtypes = [_P, _dp, _dp]
    L.aapdhg_get_dims.argtypes = [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int64), _dp, _dp]
    L.aapdhg_get_scaling.argtypes = [_P, _dp, _dp]
    L.aapdhg_destroy.argtypes = [_P]
    L.aapdhg_last_error.argtypes = [_P]
    L.aapdhg_last_error.restype = C.c_char_p
    L.aapdhg_batch_create.argtypes = [C.c_int32, C.POINTER(_P), C.POINTER(_P)]
    L.aapdhg_batch_solve.argtypes = [_P, _P]
    L.aapdhg_batch_iterate.argtypes = [_P, _P, C.c_int64]
    L.aapdhg_batch_iterate_timed.argtypes = [_P, _P, C.c_int64, _dp]
    L.aapdhg_batch_result.argtypes = [_P, C.c_int32, _dp, _dp, _dp, C.POINTER(Info)]
    L.aapdhg_batch_destroy.argtypes = [_P]
    L.aapdhg_server_start.argtypes = [C.c_size_t, C.c_int32, C.POINTER(Options), _P, _P, C.POINTER(_P)]
    L.aapdhg_server_submit.argtypes = [_P, C.c_int32, C.c_int32, C.c_int64, C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int32), _dp, _dp, _dp, _dp, _dp, C.POINTER(C.c_uint8),
                                       C.POINTER(C.c_uint64)]
    L.aapdhg_server_poll.argtypes = [_P, C.c_uint64, C.POINTER(Info), _dp, _dp, _dp, _dp]
    L.aapdhg_server_stats.argtypes = [_P, _i64p]
    L.aapdhg_server_stop.argtypes = [_P]
    for name in EXPORTS:
        fn = getattr(L, name)
        if name not in ("aapdhg_default_options", "aapdhg_last_error"):
            fn.restype = C.c_int
    _lib = L
    return L


class AAPDHGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"aapdhg error {status}: {msg}")
        self.status = status


def _check(status, handle=None):
    if status not in (OK, PENDING):
        msg = lib().aapdhg_last_error(handle).decode(errors="replace")
        raise AAPDHGError(status, msg)
    return status


def default_options(**kw) -> Options:
    o = Options()
    lib().aapdhg_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _stream(stream):
    """A hipStream_t as void*: None (default stream), an int handle, or a torch stream."""
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _lp_arrays(lp):
    """Contiguous arrays of an LP given as an object with m, n, rowptr, colidx,
    val, c, q, l, u, rowtype attributes."""
    arrs = dict(rowptr=np.ascontiguousarray(lp.rowptr, dtype=np.int64),
                colidx=np.ascontiguousarray(lp.colidx, dtype=np.int32),
                val=_f64(lp.val), c=_f64(lp.c), q=_f64(lp.q), l=_f64(lp.l), u=_f64(lp.u),
                rowtype=np.ascontiguousarray(lp.rowtype, dtype=np.uint8))
    return arrs


def _timing(ms):
    if ms[0] == 1.0:
        return {"kernel": "persistent", "launch_ms": float(ms[1]), "passes": int(ms[2])}
    return {"kernel": "three", "primal": float(ms[1]), "dual": float(ms[2]), "mix": float(ms[3])}


class Solver:
    """One LP on the GPU (aapdhg_create ... aapdhg_destroy)."""

    def __init__(self, lp, options: Options | None = None, **kw):
        L = lib()
        opt = options if options is not None else default_options(**kw)
        a = _lp_arrays(lp)
        self._keep = a
        self.m, self.n = int(lp.m), int(lp.n)
        h = C.c_void_p()
        st = L.aapdhg_create(self.m, self.n, int(a["rowptr"][-1]), _ptr(a["rowptr"], C.c_int64),
                             _ptr(a["colidx"], C.c_int32), _ptr(a["val"], C.c_double), _ptr(a["c"], C.c_double),
                             _ptr(a["q"], C.c_double), _ptr(a["l"], C.c_double), _ptr(a["u"], C.c_double),
                             _ptr(a["rowtype"], C.c_uint8), C.byref(opt), C.byref(h))
        _check(st, None)
        self.h = h
        self.options = opt
        self.memory = int(opt.memory)
        _open["solver"].add(self)

    @classmethod
    def from_device(cls, m, n, rowptr, colidx, val, c, q, l, u, rowtype, stream=None,
                    options: Options | None = None, **kw):
        """Create from device tensors (torch, contiguous): rowptr int64[m+1],
        colidx int32[nnz], val/c/q/l/u float64, rowtype uint8[m]
        (aapdhg_create_device).  The copies run on `stream`, by default
        torch's current stream, so they follow the work that produced the
        tensors."""
        import torch
        L = lib()
        if stream is None:
            stream = torch.cuda.current_stream()
        opt = options if options is not None else default_options(**kw)
        ts = (rowptr, colidx, val, c, q, l, u, rowtype)
        want = (torch.int64, torch.int32, torch.float64, torch.float64, torch.float64, torch.float64,
                torch.float64, torch.uint8)
        for t, dt in zip(ts, want):
            if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
                raise ValueError("device inputs must be contiguous CUDA tensors of the documented dtypes")
        sizes = (m + 1, colidx.numel(), colidx.numel(), n, m, n, n, m)
        if any(t.numel() != k for t, k in zip(ts, sizes)):
            raise ValueError("device input lengths do not match m, n and nnz")
        self = cls.__new__(cls)
        self.m, self.n = int(m), int(n)
        self._keep = ts
        h = C.c_void_p()
        _check(L.aapdhg_create_device(self.m, self.n, int(colidx.numel()), *[C.c_void_p(t.data_ptr()) for t in ts],
                                      C.byref(opt), _stream(stream), C.byref(h)), None)
        self.h = h
        self.options = opt
        self.memory = int(opt.memory)
        _open["solver"].add(self)
        return self

    def result_device(self, stream=None):
        """x, y, lambda as float64 CUDA tensors written by the library
        (aapdhg_result_device) on `stream` (by default torch's current
        stream, where they were allocated), and the info dictionary."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        x = torch.empty(self.n, dtype=torch.float64, device="cuda")
        y = torch.empty(self.m, dtype=torch.float64, device="cuda")
        lam = torch.empty(self.n, dtype=torch.float64, device="cuda")
        info = Info()
        _check(lib().aapdhg_result_device(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                          C.c_void_p(lam.data_ptr()), C.byref(info), _stream(stream)), self.h)
        return {"x": x, "y": y, "lam": lam, **info.to_dict()}

    def close(self):
        if getattr(self, "h", None):
            lib().aapdhg_destroy(self.h)
            self.h = None

    def __del__(self):
        if lib is not None:  # module globals are gone during interpreter teardown
            self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def solve(self, stream=None, wait=True):
        """aapdhg_solve (asynchronous); with `wait` the call also waits for
        the solve to finish (aapdhg_wait)."""
        _check(lib().aapdhg_solve(self.h, _stream(stream)), self.h)
        if wait:
            self.wait()
        return self

    def wait(self):
        """Wait for a solve in flight (aapdhg_wait)."""
        _check(lib().aapdhg_wait(self.h), self.h)
        return self

    def iterate(self, iters: int, stream=None):
        _check(lib().aapdhg_iterate(self.h, _stream(stream), int(iters)), self.h)
        return self

    def iterate_noalloc(self, iters: int, stream=None):
        """The passes of iterate() with the pass scratch in the library's
        static device array (aapdhg_iterate_noalloc): no allocation."""
        _check(lib().aapdhg_iterate_noalloc(self.h, _stream(stream), int(iters)), self.h)
        return self

    def iterate_timed(self, iters: int, stream=None):
        """`iters` loop passes with HIP events around the launches (see
        aapdhg_iterate_timed): the persistent kernel's launch time, or the mean
        milliseconds of the primal, dual and mix launches."""
        ms = np.zeros(4)
        _check(lib().aapdhg_iterate_timed(self.h, _stream(stream), int(iters), _ptr(ms, C.c_double)), self.h)
        return _timing(ms)

    def reset(self, stream=None):
        _check(lib().aapdhg_reset(self.h, _stream(stream)), self.h)
        return self

    def result(self):
        x = np.empty(self.n)
        y = np.empty(self.m)
        lam = np.empty(self.n)
        info = Info()
        _check(lib().aapdhg_result(self.h, _ptr(x, C.c_double), _ptr(y, C.c_double), _ptr(lam, C.c_double),
                                   C.byref(info)), self.h)
        return {"x": x, "y": y, "lam": lam, **info.to_dict()}

    def dims(self):
        m, n, nnz = C.c_int32(), C.c_int32(), C.c_int64()
        tau, sigma = C.c_double(), C.c_double()
        _check(lib().aapdhg_get_dims(self.h, C.byref(m), C.byref(n), C.byref(nnz), C.byref(tau),
                                     C.byref(sigma)), self.h)
        return {"m": m.value, "n": n.value, "nnz": nnz.value, "tau": tau.value, "sigma": sigma.value}

    def scaling(self):
        dr, dc = np.empty(self.m), np.empty(self.n)
        _check(lib().aapdhg_get_scaling(self.h, _ptr(dr, C.c_double), _ptr(dc, C.c_double)), self.h)
        return dr, dc

    def get_state(self):
        N = self.m + self.n
        M = self.memory
        st = {"u": np.empty(N), "u_prev": np.empty(N), "g_prev": np.empty(N),
              "dG": np.empty(M * N), "W": np.empty(M * N),
              "meta": np.zeros(8 + 2 * MAX_MEMORY, dtype=np.int64),
              "gram": np.zeros(MAX_MEMORY * MAX_MEMORY + 3 * MAX_MEMORY + 2)}
        _check(lib().aapdhg_get_state(self.h, _ptr(st["u"], C.c_double), _ptr(st["u_prev"], C.c_double),
                                      _ptr(st["g_prev"], C.c_double), _ptr(st["dG"], C.c_double),
                                      _ptr(st["W"], C.c_double), _ptr(st["meta"], C.c_int64),
                                      _ptr(st["gram"], C.c_double)), self.h)
        st["dG"] = st["dG"].reshape(M, N)
        st["W"] = st["W"].reshape(M, N)
        meta = st["meta"]
        nmix = int(meta[7])
        st.update(k=int(meta[0]), status=int(meta[1]), i=int(meta[2]), j=int(meta[3]), nlive=int(meta[4]),
                  newslot=int(meta[5]), branch=int(meta[6]), nmix=nmix,
                  live=[int(v) for v in meta[8:8 + int(meta[4])]],
                  mixslot=[int(v) for v in meta[8 + MAX_MEMORY:8 + MAX_MEMORY + nmix]])
        g = st["gram"]
        S = MAX_MEMORY
        st["G"] = g[:S * S].reshape(S, S)
        st["rhs"] = g[S * S:S * S + S]
        st["du2"] = g[S * S + S:S * S + 2 * S]
        st["n0"] = float(g[S * S + 2 * S])
        st["gnorm"] = float(g[S * S + 2 * S + 1])
        st["gamma"] = g[S * S + 2 * S + 2:S * S + 2 * S + 2 + nmix].copy()
        return st

    def get_weights(self, anchor=True):
        """Primal-weight state: omega, gamma, tau, sigma, D-hat coefficients
        (a_x, a_y, b_x, b_y), accepted updates, the reset flag and (when the
        update is on) the anchor iterate."""
        w = np.zeros(WEIGHT_WORDS)
        anc = np.empty(self.m + self.n) if anchor else None
        _check(lib().aapdhg_get_weights(self.h, _ptr(anc, C.c_double) if anchor else None,
                                        _ptr(w, C.c_double)), self.h)
        out = {"omega": w[0], "gamma": w[1], "tau": w[2], "sigma": w[3], "dha": w[4:6].copy(),
               "dhb": w[6:8].copy(), "updates": int(w[8]), "flag": int(w[9]), "words": w}
        if anchor:
            out["anchor"] = anc
        return out

    def set_weights(self, words, anchor=None):
        w = _f64(words)
        anc = _f64(anchor) if anchor is not None else None
        _check(lib().aapdhg_set_weights(self.h, _ptr(anc, C.c_double) if anc is not None else None,
                                        _ptr(w, C.c_double)), self.h)
        return self

    def set_state(self, st):
        dG = _f64(st["dG"]).ravel()
        W = _f64(st["W"]).ravel()
        u, up, gp = _f64(st["u"]), _f64(st["u_prev"]), _f64(st["g_prev"])
        meta = np.ascontiguousarray(st["meta"], dtype=np.int64)
        gram = _f64(st["gram"])
        _check(lib().aapdhg_set_state(self.h, _ptr(u, C.c_double), _ptr(up, C.c_double), _ptr(gp, C.c_double),
                                      _ptr(dG, C.c_double), _ptr(W, C.c_double), _ptr(meta, C.c_int64),
                                      _ptr(gram, C.c_double)), self.h)
        return self


class Batch:
    """Many LPs advanced by the same launches (aapdhg_batch_*)."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        arr = (C.c_void_p * len(self.solvers))(*[s.h for s in self.solvers])
        h = C.c_void_p()
        _check(lib().aapdhg_batch_create(len(self.solvers), arr, C.byref(h)), None)
        self.h = h
        _open["batch"].add(self)

    def solve(self, stream=None):
        _check(lib().aapdhg_batch_solve(self.h, _stream(stream)), None)
        return self

    def iterate(self, iters, stream=None):
        _check(lib().aapdhg_batch_iterate(self.h, _stream(stream), int(iters)), None)
        return self

    def iterate_timed(self, iters: int, stream=None):
        ms = np.zeros(4)
        _check(lib().aapdhg_batch_iterate_timed(self.h, _stream(stream), int(iters), _ptr(ms, C.c_double)), None)
        return _timing(ms)

    def result(self, i):
        """Member i's result (aapdhg_batch_result)."""
        s = self.solvers[i] if 0 <= i < len(self.solvers) else None
        x, y, lam = (np.empty(s.n), np.empty(s.m), np.empty(s.n)) if s else (None, None, None)
        info = Info()
        _check(lib().aapdhg_batch_result(self.h, int(i), _ptr(x, C.c_double) if s else None,
                                         _ptr(y, C.c_double) if s else None, _ptr(lam, C.c_double) if s else None,
                                         C.byref(info)), None)
        return {"x": x, "y": y, "lam": lam, **info.to_dict()}

    def results(self):
        return [self.result(i) for i in range(len(self.solvers))]

    def close(self):
        if getattr(self, "h", None):
            lib().aapdhg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        if lib is not None:  # module globals are gone during interpreter teardown
            self.close()


class Server:
    """Continuous-batching request loop (aapdhg_server_*)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int, options: Options | None = None,
                 compute_stream=None, copy_stream=None, **kw):
        """compute_stream / copy_stream: torch streams (or hipStream_t ints)
        for the epochs and for admitting requests; None lets the server
        create its own."""
        opt = options if options is not None else default_options(**kw)
        h = C.c_void_p()
        _check(lib().aapdhg_server_start(int(hbm_budget_bytes), int(max_slots), C.byref(opt),
                                         _stream(compute_stream), _stream(copy_stream), C.byref(h)), None)
        self.h = h
        self._dims = {}
        _open["server"].add(self)

    def submit(self, lp) -> int:
        a = _lp_arrays(lp)
        t = C.c_uint64()
        _check(lib().aapdhg_server_submit(self.h, int(lp.m), int(lp.n), int(a["rowptr"][-1]),
                                          _ptr(a["rowptr"], C.c_int64), _ptr(a["colidx"], C.c_int32),
                                          _ptr(a["val"], C.c_double), _ptr(a["c"], C.c_double),
                                          _ptr(a["q"], C.c_double), _ptr(a["l"], C.c_double),
                                          _ptr(a["u"], C.c_double), _ptr(a["rowtype"], C.c_uint8),
                                          C.byref(t)), None)
        self._dims[t.value] = (int(lp.m), int(lp.n))
        return t.value

    def poll(self, ticket: int, want_solution: bool = True):
        """None while pending; a result dict once finished (then the ticket is released)."""
        m, n = self._dims[ticket]
        x = np.empty(n) if want_solution else None
        y = np.empty(m) if want_solution else None
        info = Info()
        ta, td = C.c_double(), C.c_double()
        st = lib().aapdhg_server_poll(self.h, ticket, C.byref(info),
                                      _ptr(x, C.c_double) if want_solution else None,
                                      _ptr(y, C.c_double) if want_solution else None, C.byref(ta), C.byref(td))
        _check(st, None)
        if st == PENDING:
            return None
        del self._dims[ticket]
        return {"x": x, "y": y, "t_admit": ta.value, "t_done": td.value, **info.to_dict()}

    def stats(self):
        s = np.zeros(6, dtype=np.int64)
        _check(lib().aapdhg_server_stats(self.h, _ptr(s, C.c_int64)), None)
        keys = ["submitted", "admitted", "finished", "resident", "epochs", "resident_bytes"]
        return dict(zip(keys, (int(v) for v in s)))

    def close(self):
        if getattr(self, "h", None):
            lib().aapdhg_server_stop(self.h)
            self.h = None

    def __del__(self):
        if lib is not None:  # module globals are gone during interpreter teardown
            self.close()


def close_all():
    """Destroy every handle still open: servers (their worker threads stop
    first), then batches, then solvers.  Runs at interpreter exit."""
    for kind in ("server", "batch", "solver"):
        for obj in list(_open[kind]):
            obj.close()


atexit.register(close_all)
