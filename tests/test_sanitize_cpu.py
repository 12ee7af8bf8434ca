"""The library's host-only code (instance validation and entry selectors,
chordal extension and maximal cliques, data scaling) built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer and run on valid and invalid
inputs by tests/sanitize_driver.cpp.  No device code is built or run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1707_05058_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    srcs = [os.path.join(HERE, "sanitize_driver.cpp")] + [
        os.path.join(CSRC, f) for f in ("sdp_validate.cpp", "sdp_pattern.cpp", "sdp_scale.cpp")]
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "Sanitizer" not in out and "runtime error" not in out, out
    assert "0 failed checks" in r.stdout
