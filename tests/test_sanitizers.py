"""Host code built with AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only, no device code): the trace replayer, the max-trace-length split, the
agreement, the trace finder and the Algorithm 1 driver (against a stand-in
for the analysis server), and the C oracle.  Each driver must exit cleanly
with no sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2406_18111_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _build_and_run(cmd, exe, tmp_path):
    r = subprocess.run(cmd + ["-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    p = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=ENV)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out, out[-4000:]
    return out


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_library_code_under_asan_ubsan(tmp_path):
    srcs = [os.path.join(CSRC, "replayer.cpp"), os.path.join(CSRC, "auto.cpp"),
            os.path.join(HERE, "fake_server.cpp"), os.path.join(HERE, "host_driver.cpp")]
    # tracer.hip holds host code only; compiled here as plain C++
    cmd = ["g++", "-std=c++17"] + SAN + ["-I" + os.path.join(ROOT, "include"), "-pthread"] + srcs + \
          ["-x", "c++", os.path.join(CSRC, "tracer.hip")]
    out = _build_and_run(cmd, tmp_path / "host_driver", tmp_path)
    assert "host driver ok" in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_c_oracle_under_asan_ubsan(tmp_path):
    cmd = ["gcc", "-std=c11"] + SAN + [os.path.join(ROOT, "oracle", "findrepeats_ref.c"),
                                       os.path.join(HERE, "oracle_driver.c")]
    out = _build_and_run(cmd, tmp_path / "oracle_driver", tmp_path)
    assert "oracle driver ok" in out
