"""Host policies kept free of HIP so that they run on the CPU, each checked by
a small program under tests/cpp compiled with the host C++ compiler (it
prints "ok" or the failed check):

* the shot server's admission (csrc/server_policy.hpp), driven by a fake
  executor: budget, running cap, first-in first-out order, when retired
  memory is freed, completion;
* the autotuner's choice of launch shape (csrc/tune_policy.hpp): ties within
  1% settled by the longer z-chunk, then the faster."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _run_check(tmp_path, name):
    exe = str(tmp_path / name)
    src = os.path.join(HERE, "cpp", name + ".cpp")
    inc = os.path.join(ROOT, "paper_1608_08658_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I", inc, src, "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(out.stdout)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_admission_policy_simulation(tmp_path):
    _run_check(tmp_path, "server_policy_sim")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_launch_shape_choice(tmp_path):
    _run_check(tmp_path, "tune_policy_check")
