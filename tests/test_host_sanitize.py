"""The library's pure host code (launch planning and the SP2-ACC schedule of
Alg. 3) built with AddressSanitizer and UndefinedBehaviorSanitizer on the
host side only, and run over random and edge-case inputs by
tests/host_check.cpp, which checks exact coverage of every tile and K slice
by the work plan and the ranges of the schedule. No GPU is used."""
import os
import shlex
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# host-side sanitizers only (the device code of these files is not built
# with them)
SAN = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined " \
      "-Xarch_host -fno-sanitize-recover=all"


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc not available")
def test_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_check")
    csrc = os.path.join(ROOT, "paper_1507_02087_amd", "csrc")
    cmd = ([HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950"] + shlex.split(SAN) +
           ["-I", os.path.join(ROOT, "include"), "-I", csrc,
            os.path.join(ROOT, "tests", "host_check.cpp"),
            "-x", "hip", os.path.join(csrc, "host_plan.hip"),
            os.path.join(csrc, "schedule.hip"), "-o", exe])
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert r.stdout.strip() == "ok"
