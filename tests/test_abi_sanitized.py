"""The C-ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(the host half of the library instrumented with -Xarch_host; its device code
as always): tests/sanitize_abi.cpp drives the parameter validation and state
layout of every precision, collision form and g rounding mode, the batch head
size, the error strings and every entry point's rejection of null,
misaligned or undersized arguments.  No GPU is needed: every call it makes
returns before any device work."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1810_09299_amd", "csrc")


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_abi_host_code_is_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_abi")
    cmd = ["hipcc", "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           os.path.join(CSRC, "lbm_axi.hip"), os.path.join(CSRC, "lbm_axi_batch.hip"),
           os.path.join(HERE, "sanitize_abi.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=900)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
    assert "0 failing checks" in r.stdout
