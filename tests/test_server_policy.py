"""The shot server's admission policy (csrc/server_policy.hpp, host code
without HIP) driven by a fake executor on the CPU: budget, running cap,
first-in first-out order, when retired memory is freed, completion.  The
simulation (tests/cpp/server_policy_sim.cpp) is compiled with the host C++
compiler and run; it prints "ok" or the failed check."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_admission_policy_simulation(tmp_path):
    exe = str(tmp_path / "server_policy_sim")
    src = os.path.join(HERE, "cpp", "server_policy_sim.cpp")
    inc = os.path.join(ROOT, "paper_1608_08658_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I", inc, src, "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(out.stdout)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr
