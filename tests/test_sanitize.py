"""CPU sanitizer builds: the oracle under AddressSanitizer + UndefinedBehaviorSanitizer, and the library's
threaded host runtime (mesh topology, patching, element order and colour order, LDS working-set count,
work-unit segments, patch-local index structures) under ASan + UBSan and under ThreadSanitizer, each driven
by a harness in tests/sanitize/ that also checks the structures' invariants. g++/gcc only: no GPU code is
built with a sanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_SRC = [os.path.join(ROOT, "paper_2509_00406_amd", "csrc", f)
            for f in ("host_mesh.cpp", "host_patch.cpp", "host_layout.cpp")]
HIP_INC = os.environ.get("ROCM_PATH", "/opt/rocm") + "/include"


def build_and_run(tmp_path, name, cmd):
    exe = str(tmp_path / name)
    subprocess.run(cmd + ["-o", exe], check=True, cwd=ROOT, capture_output=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "Sanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_oracle_asan_ubsan(tmp_path):
    out = build_and_run(tmp_path, "oracle_asan", [
        "gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
        "-fno-omit-frame-pointer", "-fopenmp", "-Ioracle", "oracle/oracle.c", "tests/sanitize/oracle_driver.c",
        "-lm"])
    assert "oracle checks passed" in out


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(HIP_INC), reason="g++ or HIP headers missing")
@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_host_runtime_sanitized(tmp_path, san):
    flags = ["-fsanitize=" + san] + (["-fno-sanitize-recover=all", "-fno-omit-frame-pointer"] if san != "thread"
                                     else [])
    out = build_and_run(tmp_path, "host_" + san.split(",")[0], [
        "g++", "-std=c++17", "-O1", "-g", *flags, "-D__HIP_PLATFORM_AMD__", "-I" + HIP_INC, "-Iinclude",
        "-Ipaper_2509_00406_amd/csrc", *HOST_SRC, "tests/sanitize/host_driver.cpp", "-pthread"])
    assert "host runtime checks passed" in out
