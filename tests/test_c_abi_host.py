"""The library used from plain C (no Python, no torch): tests/c_abi_host.c is
compiled with gcc against include/opflux.h and libopflux.so and run on the
host (host-only context: declarations, plan, verification, error paths)."""
import os
import shutil
import subprocess

import pytest

import paper_1403_7209_amd as pk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_c_program_against_the_abi(tmp_path):
    lib = pk.LIB_PATH
    assert os.path.exists(lib), "libopflux.so is not built"
    exe = tmp_path / "c_abi_host"
    libdir = os.path.dirname(lib)
    cmd = ["gcc", "-std=c99", "-O1", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c_abi_host.c"), "-o", str(exe), lib,
           f"-Wl,-rpath,{libdir}"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "ok"
