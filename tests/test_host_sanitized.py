"""The host library (host.cpp, server.cpp) built with AddressSanitizer and
UBSan against a CPU stand-in of the HIP runtime (tests/hostcheck/hip_stub.cpp)
and driven through the C ABI (tests/hostcheck/driver.cpp): validation, CSR and
CSC building, row orders, chunk, split-row, panel and launch tables, the
no-allocation pass scratch layout, checkpoints, the device-memory entry
points, batches and the server's admission and retirement, on ragged, empty,
long-row, long-column and invalid LPs.  The stand-in's kernels do nothing, so
only host logic is checked: no out-of-bounds access, use after free,
undefined behaviour or leak, and every call returns what it should."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2508_08062_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "hostcheck")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


@pytest.mark.timeout(600)
def test_host_library_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the HIP headers are missing")
    common = ["-std=c++17", "-O1", "-g"] + SAN + ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", CSRC,
                                                  "-I", os.path.join(ROOT, "include")]
    objs = []
    for src in (os.path.join(CSRC, "host.cpp"), os.path.join(CSRC, "server.cpp"), os.path.join(CSRC, "tuner.cpp"),
                os.path.join(HERE, "hip_stub.cpp"), os.path.join(HERE, "driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([gxx] + common + ["-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    exe = str(tmp_path / "hostcheck")
    r = subprocess.run([gxx] + SAN + ["-o", exe] + objs + ["-lpthread"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    # verify_asan_link_order=0: the process environment may preload a library ahead of the runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=500, cwd=str(tmp_path))
    assert r.returncode == 0 and "hostcheck ok" in r.stdout, (r.stdout[-2000:] + r.stderr[-6000:])
