"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

The planner (`csrc/plan.cpp`: fixed-point cells, the (tile, cell) order inside each block, work items, patch
slots, the J = 8 gridder's row spans, reduction chunks) and the float64 tables (`csrc/tables.cpp`) are plain
host code.  They are compiled here with g++ on their own, together with `tests/host/plan_check.cpp`, with both
sanitizers and no recovery, and the check runs its seeded workloads: any out-of-bounds access, leak, signed
overflow, bad shift or broken plan invariant ends it with a non-zero status.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1502_05037_amd", "csrc")
ROCM_INC = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INC), reason="needs g++ and the ROCm headers")
def test_planner_and_tables_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "plan_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM_INC}", f"-I{CSRC}",
           os.path.join(ROOT, "tests", "host", "plan_check.cpp"), os.path.join(CSRC, "plan.cpp"),
           os.path.join(CSRC, "tables.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.strip().splitlines()[-1] == "ok"
    assert "runtime error" not in r.stderr
