"""The host planner under the address + undefined-behaviour sanitizers and the
thread sanitizer: plan.cpp, host_math.cpp and tune.cpp are built with g++ into
a CPU program (tests/sanitize/driver.cpp; kernel launchers replaced by
tests/sanitize/stubs.cpp) that plans every window family and precision over
uniform, clustered, edge and single-node sets, through the dry-run entry point
and the NFFT planner.  Any sanitizer report fails the test.  Plans with at
least 2^15 points per side build their two sides on two threads; the thread
run adds four planner threads on top.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2107_02671_amd", "csrc")
SOURCES = [os.path.join(CSRC, s) for s in ("plan.cpp", "host_math.cpp", "tune.cpp")] + [
    os.path.join(HERE, "sanitize", "stubs.cpp"), os.path.join(HERE, "sanitize", "driver.cpp")]
ROCM = "/opt/rocm"

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(os.path.join(ROCM, "include")),
                                reason="needs g++ and the ROCm headers")


def _build(tmp, flags):
    common = ["-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-D__HIP_PLATFORM_AMD__",
              f"-I{ROCM}/include", *flags]

    def comp(src):
        obj = os.path.join(tmp, os.path.basename(src) + ".o")
        r = subprocess.run(["g++", *common, "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(comp, SOURCES))
    exe = os.path.join(tmp, "driver")
    r = subprocess.run(["g++", *common, *objs, f"-L{ROCM}/lib", "-lamdhip64", "-lpthread", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _run(exe, *args, env=None):
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=600,
                       env={**os.environ, **(env or {})})
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR:" not in out and "runtime error" not in out and "WARNING: ThreadSanitizer" not in out, out[-4000:]
    assert "refused " in out, out[-2000:]   # some combinations are refused by design (2 m >= n)


def test_planner_address_and_undefined_behaviour(tmp_path):
    exe = _build(str(tmp_path), ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"])
    _run(exe, env={"ASAN_OPTIONS": "detect_leaks=1"})


def test_planner_threads(tmp_path):
    exe = _build(str(tmp_path), ["-fsanitize=thread"])
    _run(exe, "threads", env={"TSAN_OPTIONS": "halt_on_error=1"})
