"""Host-only unit test of the key under which the library replays a captured
evaluation graph (csrc/graph_key.h, compiled here with g++; no GPU)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2204_04678_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_graph_key_refuses_other_models(tmp_path):
    exe = tmp_path / "graph_key_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I" + CSRC,
                    os.path.join(HERE, "native", "graph_key_check.cpp"), "-o", str(exe)],
                   check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "graph key checks passed" in res.stdout
