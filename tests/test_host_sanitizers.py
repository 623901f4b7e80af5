"""Address- and undefined-behaviour-sanitizer build of the host construction code
(butterfly factorization, peeling, skeletonization, the plan file format), run on
small problems of every phase: no memory error, leak or undefined behaviour may be
reported.  GPU code is not part of this sanitizer build (host sources with g++ only)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2105_02995_amd", "csrc")
SOURCES = ["la.cpp", "stages.cpp", "butterfly.cpp", "hif1d.cpp", "hif2d.cpp", "build.cpp"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_construction_is_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES],
           os.path.join(ROOT, "tests", "native", "host_check.cpp"), "-lpthread", "-o", exe]
    b = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600)
    assert b.returncode == 0, b.stdout[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe, str(tmp_path)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=600, env=env)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-4000:]
    assert "host check ok" in r.stdout
    assert "runtime error" not in r.stdout
