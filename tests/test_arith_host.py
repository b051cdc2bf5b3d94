"""The kernels' integer arithmetic (division by a 2^64 reciprocal, execution
times, Q32 utilisation, Lemma 2 closed form), compiled as host code with g++
and checked against 128-bit reference expressions on the CPU."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_kernel_arithmetic_on_host(tmp_path):
    exe = tmp_path / "arith_check"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2105_10312_amd", "csrc"),
                           os.path.join(ROOT, "tests", "cpp", "arith_check.cpp"), "-o", str(exe)])
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr
