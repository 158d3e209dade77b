"""The C-ABI library loads and exports every entry point that include/aapdhg.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

from conftest import ROOT


def _declared():
    with open(os.path.join(ROOT, "include", "aapdhg.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aapdhg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("aapdhg_create", "aapdhg_solve", "aapdhg_result", "aapdhg_destroy",
                 "aapdhg_batch_create", "aapdhg_server_start"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2508_08062_amd as P
    L = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(P.EXPORTS) == _declared()


def _c_layout(struct, fields, tmp_path):
    """sizeof and offsetof of a struct of aapdhg.h, from a C program built with gcc."""
    src = tmp_path / "probe.c"
    body = "".join(f'printf("%zu ", offsetof({struct}, {f}));' for f in fields)
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"aapdhg.h\"\n"
                   f"int main(void){{printf(\"%zu \", sizeof({struct}));{body}return 0;}}\n")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return [int(v) for v in out]


@pytest.mark.parametrize("struct", ["aapdhg_options", "aapdhg_info"])
def test_ctypes_structs_match_the_header(struct, tmp_path):
    import paper_2508_08062_amd as P
    cls = P.Options if struct == "aapdhg_options" else P.Info
    fields = [f for f, _ in cls._fields_]
    size, *offs = _c_layout(struct, fields, tmp_path)
    assert size == ctypes.sizeof(cls)
    assert offs == [getattr(cls, f).offset for f in fields]


def test_default_options():
    import paper_2508_08062_amd as P
    o = P.default_options()
    assert (o.variant, o.precision, o.memory) == (1, 0, 10)
    assert (o.D, o.eps_sg, o.beta, o.eta, o.cs, o.kappa_bar, o.tol) == (10.0, 1.0, 1.0, 1e-10, 0.2, 1e8, 1e-4)
    assert (o.max_iter, o.kkt_every, o.dhat_mode, o.power_iters, o.epoch) == (100000, 64, 1, 200, 256)


def test_invalid_input_is_rejected_without_a_gpu_call():
    import numpy as np
    import lpgen
    import paper_2508_08062_amd as P
    lp = lpgen.tiny_lp(0)
    bad = lpgen.LPData(**{**lp.__dict__, "rowtype": np.full(lp.m, 7, dtype=np.uint8)})
    with pytest.raises(P.AAPDHGError) as e:
        P.Solver(bad, precision=1)
    assert e.value.status == P.E_ARG and "row_type" in str(e.value)
    bad = lpgen.LPData(**{**lp.__dict__, "colidx": lp.colidx + 1000})
    with pytest.raises(P.AAPDHGError) as e:
        P.Solver(bad, precision=1)
    assert "out of range" in str(e.value)
    with pytest.raises(P.AAPDHGError):
        P.Solver(lp, memory=17)


@pytest.mark.parametrize("opts,needle", [
    (dict(pw_period=-1), "pw_period"),
    (dict(pw_period=10, pw_theta=1.5), "pw_theta"),
    (dict(pw_period=10, pw_eps_zero=0.0), "pw_eps_zero"),
    (dict(pw_dhat=2), "pw_dhat"),
    (dict(sg_div=0.0), "sg_div"),
    (dict(variant=3, restart_period=0), "restart_period"),
    (dict(variant=4), "variant"),
    (dict(prep_device=3), "prep_device"),
    (dict(pock_chambolle=2), "pock_chambolle"),
    (dict(angle_mode=2), "angle_mode"),
])
def test_invalid_method_options_are_rejected_without_a_gpu_call(opts, needle):
    """The options of the primal-weight update, the Iter_AA / c safeguard,
    restarted PDHG and the scaling are validated before any device work."""
    import lpgen
    import paper_2508_08062_amd as P
    with pytest.raises(P.AAPDHGError) as e:
        P.Solver(lpgen.tiny_lp(0), precision=1, **opts)
    assert e.value.status == P.E_ARG and needle in str(e.value)


def test_method_option_defaults():
    import paper_2508_08062_amd as P
    o = P.default_options()
    assert (o.pw_period, o.pw_theta, o.pw_eps_zero, o.pw_omega0, o.pw_rho, o.pw_dhat) == (0, 0.5, 1e-10, 0.0, 0.0, 1)
    assert (o.sg_div, o.restart_period, o.prep_device, o.pock_chambolle, o.angle_mode, o.seed) == (1.0, 75, 2, 0, 0, 0)
