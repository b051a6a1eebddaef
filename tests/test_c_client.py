"""A plain C program against include/uvadmm.h and libuvadmm.so: it builds
and links on the CPU; on a GPU it solves a small LP to its known optimum,
reads the run's residual history and solves again on the same handle with
a new right-hand side."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c_client", "solve_lp.c")
PKG = os.path.join(ROOT, "paper_2203_05027_amd")


def _build(tmp_path):
    exe = str(tmp_path / "solve_lp")
    subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-I", os.path.join(ROOT, "include"), SRC,
                    "-o", exe, "-L", PKG, "-luvadmm", f"-Wl,-rpath,{PKG}", "-lm"], check=True)
    return exe


def test_c_client_builds_and_links(tmp_path):
    exe = _build(tmp_path)
    assert os.path.exists(exe)


@pytest.mark.gpu
def test_c_client_solves_on_the_gpu(tmp_path):
    exe = _build(tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "status 1" in r.stdout
