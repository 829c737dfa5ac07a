"""The host code that builds the projector geometry (build_tables_host),
compiled with the address and undefined-behaviour sanitizers on the host
side only and run over periodic, Bloch, self-overlapping, ragged,
zero-boundary and atom-free geometries plus a rejected descriptor
(tests/host_check/tables_check.hip states the invariants it checks). No
device call is made, so this runs without a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not (os.path.exists(HIPCC) or shutil.which("hipcc")), reason="hipcc not found")
def test_table_builder_under_host_sanitizers(tmp_path):
    exe = str(tmp_path / "tables_check")
    csrc = os.path.join(ROOT, "paper_2310_14776_amd", "csrc")
    cmd = [HIPCC if os.path.exists(HIPCC) else shutil.which("hipcc"), "--offload-arch=gfx950",
           "-O1", "-g", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(csrc, "tables.hip"), os.path.join(ROOT, "tests", "host_check", "tables_check.hip"),
           "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stdout + b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    print(out)
    assert r.returncode == 0, out
    assert "all checks passed" in out
    assert "runtime error" not in out and "AddressSanitizer" not in out
