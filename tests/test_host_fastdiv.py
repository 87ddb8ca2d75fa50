"""The copy kernels' invariant-divisor division equals integer division
(host build of the same header, CPU only)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_fastdiv_matches_integer_division(tmp_path):
    exe = tmp_path / "fastdiv_test"
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(HERE, "host_src", "fastdiv_test.cpp"),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok")
