"""Host-only tests of the serving scheduler behind a fake executor (no GPU).

``tests/native/sched_test.cpp`` drives ``csrc/scheduler.cpp`` (admission under
the budget, FIFO batching of mixed sizes, slot reuse, overlapping
batches, launch and allocation fault injection with status codes and no
leak, many submitting threads). It is built three ways: plain, under
AddressSanitizer + UndefinedBehaviorSanitizer (g++) and under
ThreadSanitizer (ROCm's host clang++, whose runtime intercepts the
condition-variable waits libstdc++ uses). Nothing here touches HIP.
"""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2112_10603_amd", "csrc")
SRCS = [os.path.join(ROOT, "tests", "native", "sched_test.cpp"),
        os.path.join(CSRC, "scheduler.cpp"), os.path.join(CSRC, "fault.cpp")]


def _clang():
    c = "/opt/rocm/llvm/bin/clang++"
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.tsan-x86_64.a")
    return c if os.path.exists(c) and rt else None


VARIANTS = {
    "plain": (lambda: shutil.which("g++"), ["-O2"]),
    "asan_ubsan": (lambda: shutil.which("g++"),
                   ["-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined"]),
    "tsan": (_clang, ["-O1", "-fsanitize=thread"]),
}


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_scheduler_host(variant, tmp_path):
    find, flags = VARIANTS[variant]
    cxx = find()
    if cxx is None:
        pytest.skip(f"no compiler with {variant} support")
    exe = str(tmp_path / f"sched_{variant}")
    cmd = [cxx, "-std=c++17", "-g", "-Wall", *flags, f"-I{CSRC}", *SRCS, "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ)
    env.pop("FFV_FAULT", None)
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    env["ASAN_OPTIONS"] = "detect_leaks=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "all passed" in r.stdout
    assert "WARNING" not in r.stderr, r.stderr[-6000:]
