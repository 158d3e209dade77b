"""Host-side logic of the benchmark script (no GPU): the algorithmic byte
model, the HBM-traffic lookup keyed by the kernel sources, and the guard
against runs on more than one GPU."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# the 1M x 2M benchmark LP, memory 10
N_COL, M_ROW, NNZ, MEM = 2_000_000, 1_000_000, 20_000_000, 10


def test_bytes_model_scales_with_the_matrix_and_the_memory():
    base = bench._bytes_model(N_COL, M_ROW, NNZ, MEM, 0.0, dots=False)
    more = bench._bytes_model(N_COL, M_ROW, NNZ + 1000, MEM, 0.0, dots=False)
    # each pass streams the matrix once: a 4-byte value and a 4-byte index per entry
    assert more["primal"] - base["primal"] == 8 * 1000
    assert more["dual"] - base["dual"] == 8 * 1000
    # both SpMV products read the matrix and one vector entry per row or column
    assert more["spmv"] - base["spmv"] == 16 * 1000
    # the per-pass Gram row reads the M - 1 kept history columns (4 bytes per
    # element); on demand the Gram launch reads the M columns and g instead
    dots = bench._bytes_model(N_COL, M_ROW, NNZ, MEM, 0.0, dots=True)
    assert dots["primal"] - base["primal"] == (MEM - 1) * 4 * N_COL
    assert dots["dual"] - base["dual"] == (MEM - 1) * 4 * M_ROW
    assert dots["gram"] == 0 and base["gram"] == (MEM + 1) * 4 * (N_COL + M_ROW)
    # KKT passes gather x^k beside x_bar in the dual pass
    kkt = bench._bytes_model(N_COL, M_ROW, NNZ, MEM, 1.0, dots=False)
    assert kkt["dual"] - base["dual"] == 4 * N_COL


def test_bytes_model_matches_the_figures_the_roofline_quotes():
    b = bench._bytes_model(N_COL, M_ROW, NNZ, MEM, 0.0, dots=False)
    assert b["primal"] == 268_000_004
    assert b["spmv"] == 344_000_000
    assert bench._bytes_model(N_COL, M_ROW, NNZ, MEM, 0.0, dots=True)["primal"] == 340_000_004


def test_committed_traffic_summary_belongs_to_the_committed_kernels():
    """The bench line's roofline.traffic comes from the committed counter
    summary only while the kernel sources are the ones it was taken on."""
    with open(os.path.join(ROOT, "profiles", "traffic_powerlaw1m.json")) as f:
        t = json.load(f)
    assert t["kernel_source_hash"] == bench._src_hash()
    primal = bench._traffic("powerlaw1m", "primal", 1)
    assert primal == t["kernels"]["primal"]["hbm_bytes_per_pass"]
    # the dual launch's events bracket the panel kernel and the decisions too
    dual = bench._traffic("powerlaw1m", "dual", 1)
    ks = t["kernels"]
    assert dual == ks["dual"]["hbm_bytes_per_pass"] + ks["panel"]["hbm_bytes_per_pass"] + \
        ks["decide"]["hbm_bytes_per_pass"]
    assert bench._traffic("powerlaw1m", "primal", 7) == 7 * primal


def test_traffic_is_null_for_other_kernel_sources(monkeypatch):
    monkeypatch.setattr(bench, "_src_hash", lambda: "0000000000000000")
    assert bench._traffic("powerlaw1m", "primal", 1) is None
    assert bench._traffic("no_such_workload", "primal", 1) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
