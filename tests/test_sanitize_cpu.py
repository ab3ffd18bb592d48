"""The library's host-only source and the C oracle under AddressSanitizer and
UndefinedBehaviorSanitizer (g++, CPU only): tests/sanitize_main.cpp drives
codebook construction, the reference encoder, stream layout and the oracle's
encoders and decoders over random and edge-case inputs, and both sides must
agree.  Any sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="needs gcc/g++")
def test_host_code_under_asan_ubsan(tmp_path):
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
    oracle_o = str(tmp_path / "hdref.o")
    subprocess.check_call(["gcc", "-std=c11", "-c", os.path.join(ROOT, "oracle", "hdref.c"), "-o", oracle_o] + san)
    exe = str(tmp_path / "sanitize_main")
    subprocess.check_call(["g++", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "sanitize_main.cpp"),
                           os.path.join(ROOT, "paper_2201_09118_amd", "csrc", "hd_host.cpp"), oracle_o,
                           "-o", exe] + san)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "0 failures" in r.stdout
