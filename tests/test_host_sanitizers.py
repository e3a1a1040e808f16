"""The planner and argument validation under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; no GPU needed).

The library's host source is rebuilt with the sanitizers on its host pass,
linked with the kernel objects of the regular build and driven through
``psatd_plan_describe`` (which makes no HIP call) by
``tests/host_asan/plan_describe_driver.cpp``: every supported 2D length pair,
3D shapes up to the full workload sizes, ragged batched patch lists, every
source form, path, stencil order and kernel-choice flag, and the invalid
arguments with their documented status codes.  Any sanitizer report fails the
run (halt_on_error), as does any case with the wrong status.
"""

import os
import subprocess

import pytest

from paper_1608_05739_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(B.BUILD, "host_sanitizers")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.fixture(scope="module")
def driver():
    kernel_objs = [os.path.join(B.BUILD, os.path.splitext(s)[0] + ".o")
                   for s in B.SOURCES if s != "api.cpp"]
    missing = [o for o in kernel_objs if not os.path.exists(o)]
    if missing:
        pytest.fail(f"{missing} not built; run __graft_entry__.build()")
    os.makedirs(OUT, exist_ok=True)
    hipcc = B.hipcc()
    flags = [f for f in B.common_flags() if f not in ("-O3",)] + ["-O1", "-g"]
    api = os.path.join(OUT, "api.o")
    _run([hipcc] + flags + SAN + ["-c", os.path.join(B.CSRC, "api.cpp"), "-o", api])
    drv = os.path.join(OUT, "driver.o")
    _run([hipcc, "-x", "c++", "-O1", "-g", "-std=c++17", "-I", os.path.join(B.ROOT, "include")]
         + SAN + ["-c", os.path.join(HERE, "host_asan", "plan_describe_driver.cpp"), "-o", drv])
    exe = os.path.join(OUT, "plan_describe_driver")
    _run([hipcc, f"--offload-arch={B.ARCH}"] + SAN + [drv, api] + kernel_objs + ["-o", exe])
    return exe


def test_planner_under_address_and_ub_sanitizers(driver):
    env = dict(os.environ)
    # the HIP runtime keeps process-lifetime allocations; leaks are not checked
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=600)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "Sanitizer" not in r.stderr, tail
    assert r.stdout.strip().endswith("0 failed"), tail
