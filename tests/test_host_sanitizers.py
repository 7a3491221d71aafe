"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only).  Every source of the library is compiled with the sanitizers on
its host side only (-Xarch_host before each -fsanitize=; the device code is
built as usual and never runs here) and linked into tests/host_sanitize_driver.cpp,
which runs the host-only paths: planning and workspace sizes for random
shapes, the batch schedule builder and its simulation, the serving admission
policy and arena, and argument validation.  Any sanitizer report fails the
run."""
import glob
import os
import shutil
import subprocess
import tempfile
import concurrent.futures as cf

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2309_09072_amd", "csrc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
FLAGS = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-w"]


@pytest.mark.slow
def test_host_code_under_sanitizers():
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    tmp = tempfile.mkdtemp(prefix="lcs_san_")
    try:
        srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
        srcs.append(os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"))

        def compile_one(src):
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            r = subprocess.run(["hipcc", *FLAGS, *SAN, "-c", src, "-o", obj],
                               capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-3000:]
            return obj

        with cf.ThreadPoolExecutor(max_workers=min(6, len(srcs))) as ex:
            objs = list(ex.map(compile_one, srcs))
        exe = os.path.join(tmp, "driver")
        r = subprocess.run(["hipcc", "--offload-arch=gfx950", *SAN, *objs, "-o", exe],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0 and "ERROR: AddressSanitizer" not in r.stderr \
            and "runtime error" not in r.stderr, r.stderr[-5000:]
        assert r.stdout.strip().endswith("ok")
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
