"""The library's host code under AddressSanitizer and ThreadSanitizer (CPU only).

runtime.cpp and types.cpp -- everything of libmpixs except the kernels -- are
built with g++ against a test-only recording stand-in for the HIP runtime and
the kernel launchers (tests/host_src/hipstub/, tests/host_src/hipstub.cpp),
and a threaded driver (tests/host_src/threads_driver.cpp) runs the
concurrent patterns of the benchmarks and tests through the C ABI: a 32-rank
uneven batch through the plain enqueue path, 16-rank enqueued allreduces,
one-shot groups, persistent batches (allocated and static), wildcard
receives from racing senders, the host-synchronised calls, stream and
communicator create/free cycles with block recycling, and datatypes made and
freed from many threads.  Both builds must finish with no sanitizer report.
The one suppression (tests/host_src/lsan.supp) is the documented retention
of freed datatypes' descriptions.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "paper_2208_13707_amd", "csrc", f) for f in ("runtime.cpp", "types.cpp")]
SRC += [os.path.join(ROOT, "tests", "host_src", f) for f in ("hipstub.cpp", "threads_driver.cpp")]
INC = ["-I", os.path.join(ROOT, "tests", "host_src", "hipstub"), "-I", os.path.join(ROOT, "include")]


def build(tmp_path, san):
    exe = tmp_path / f"threads_{san}"
    cmd = (["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={san}", "-fno-omit-frame-pointer"]
           + INC + SRC + ["-lpthread", "-o", str(exe)])
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


@pytest.mark.parametrize("san", ["address", "thread"])
def test_threaded_patterns_are_clean(tmp_path, san):
    exe = build(tmp_path, san)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    env["LSAN_OPTIONS"] = "suppressions=" + os.path.join(ROOT, "tests", "host_src", "lsan.supp")
    env["TSAN_OPTIONS"] = "halt_on_error=0:second_deadlock_stack=1"
    r = subprocess.run([str(exe), "2"], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "ok (" in r.stdout, out[-6000:]
    assert "ERROR: AddressSanitizer" not in out and "ERROR: LeakSanitizer" not in out, out[-6000:]
    assert "WARNING: ThreadSanitizer" not in out, out[-6000:]
