"""The device-memory entry points against the host ones:
  * a problem created from torch CUDA tensors (aapdhg_create_device) is the
    problem created from the same arrays in host memory: same scaling, same
    step sizes and, pass for pass, the same iterate bits;
  * results written to device memory (aapdhg_result_device) equal the host
    results bit for bit (the same float64 products and quotients), in both
    precisions, on the default stream and on a caller's stream;
  * the host-side argument checks of the device create."""
import numpy as np
import pytest

import lpgen

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2508_08062_amd")
torch = pytest.importorskip("torch")


def _dev(lp):
    t = torch.from_numpy
    return (t(lp.rowptr).cuda(), t(lp.colidx).cuda(), t(lp.val).cuda(), t(lp.c).cuda(), t(lp.q).cuda(),
            t(lp.l).cuda(), t(lp.u).cuda(), t(lp.rowtype).cuda())


@pytest.mark.parametrize("precision", [0, 1])
def test_device_create_equals_host_create(precision):
    lp = lpgen.mip_like_lp(3, m=2000, n=5000, nnz=30000, fp32=False)
    kw = dict(precision=precision, ruiz_iters=10, memory=6, tol=0.0, max_iter=10 ** 6, kkt_every=8)
    a = P.Solver(lp, **kw)
    b = P.Solver.from_device(lp.m, lp.n, *_dev(lp), **kw)
    for ua, ub in zip(a.scaling(), b.scaling()):
        np.testing.assert_array_equal(ua, ub)
    assert a.dims() == b.dims()
    for k in (1, 30):
        a.iterate(k)
        b.iterate(k)
    np.testing.assert_array_equal(a.get_state()["u"], b.get_state()["u"])
    a.close()
    b.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("own_stream", [False, True])
def test_device_result_equals_host_result(precision, own_stream):
    lp = lpgen.mip_like_lp(4, m=1500, n=4000, nnz=20000, fp32=False)
    s = P.Solver(lp, precision=precision, ruiz_iters=10, tol=1e-4, max_iter=2000, kkt_every=16)
    s.solve()
    h = s.result()
    stream = torch.cuda.Stream() if own_stream else None
    d = s.result_device(stream=stream)
    (stream or torch.cuda.current_stream()).synchronize()
    for key in ("x", "y", "lam"):
        np.testing.assert_array_equal(d[key].cpu().numpy(), h[key])
    for key in ("status", "iters", "kkt", "primal_obj", "dual_obj", "omega"):
        assert d[key] == h[key], key
    s.close()


def test_device_result_before_any_solve_is_a_state_error():
    lp = lpgen.tiny_lp(2)
    s = P.Solver.from_device(lp.m, lp.n, *_dev(lp))
    with pytest.raises(P.AAPDHGError, match="no solve"):
        s.result_device()
    s.close()


def test_device_create_argument_errors():
    lp = lpgen.tiny_lp(2)
    ts = _dev(lp)
    with pytest.raises(ValueError):  # host tensor where device memory is documented
        P.Solver.from_device(lp.m, lp.n, torch.from_numpy(lp.rowptr), *ts[1:])
    with pytest.raises(ValueError):  # wrong dtype
        P.Solver.from_device(lp.m, lp.n, ts[0].to(torch.int32), *ts[1:])


def _raw_create(m, n, nnz, ptrs):
    import ctypes as C
    L = P.lib()
    h = C.c_void_p()
    st = L.aapdhg_create_device(m, n, nnz, *[C.c_void_p(p) for p in ptrs], C.byref(P.default_options()), None,
                                C.byref(h))
    msg = L.aapdhg_last_error(None).decode()
    if h.value:
        L.aapdhg_destroy(h)
    return st, msg


def test_device_create_checks_in_the_library():
    """The library's own checks, below the binding: sizes, host memory, and a
    buffer shorter than the sizes imply (found from the allocation's range,
    before any copy)."""
    lp = lpgen.tiny_lp(2)
    ts = _dev(lp)
    ptrs = [t.data_ptr() for t in ts]
    nnz = int(lp.rowptr[-1])
    st, msg = _raw_create(0, lp.n, nnz, ptrs)
    assert st == P.E_ARG and "m and n" in msg
    host = [lp.rowptr.ctypes.data] + ptrs[1:]
    st, msg = _raw_create(lp.m, lp.n, nnz, host)
    assert st == P.E_ARG and "not device memory" in msg
    st, msg = _raw_create(lp.m, lp.n, 1 << 30, ptrs)  # 8 GiB of values in a small allocation
    assert st == P.E_ARG and "allocation ends" in msg
    st, msg = _raw_create(lp.m, lp.n, nnz, ptrs)
    assert st == P.OK, msg
