"""Host-only check of the long-first task numbering of the Cholesky step
launches (csrc/inla_internal.h, compiled here with g++ against the HIP
headers; no GPU): a bijection onto the decoder's tasks for every tile count
up to 40 and both step forms."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2204_04678_amd", "csrc")
HIP_INC = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(HIP_INC),
                    reason="needs g++ and the HIP headers")
def test_step_task_numbering_is_a_bijection(tmp_path):
    exe = tmp_path / "step_split_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I" + HIP_INC, "-I" + CSRC,
                    os.path.join(HERE, "native", "step_split_check.cpp"), "-o", str(exe)], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "step split checks passed" in res.stdout
