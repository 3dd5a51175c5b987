"""Host-only checks of the library's index arithmetic under AddressSanitizer and
UBSan: the tile walk of full and symmetric GEMM grids (every tile exactly once for
every grid and band height), the norm-partial slot of a tile, the XCD renumbering of
blocks, the batched task tables, the learned guess's acceptance rule and the 3 x 3
label solve.  The same header code runs on the device; here it is compiled for the
host only (hipcc --offload-host-only), so no GPU is needed."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and not shutil.which("hipcc"), reason="needs hipcc")
def test_index_arithmetic_sanitized(tmp_path):
    exe = tmp_path / "index_check"
    cmd = [HIPCC, "--offload-host-only", "-x", "hip", "-std=c++17", "-O1", "-g",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2404_19163_amd", "csrc"),
           os.path.join(ROOT, "tests", "host", "index_check.hip"), "-o", str(exe)]
    cc = subprocess.run(cmd, capture_output=True, text=True)
    assert cc.returncode == 0, cc.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    assert run.stdout.startswith("ok "), run.stdout
    assert int(run.stdout.split()[1]) > 100000
