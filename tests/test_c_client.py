"""The C ABI from plain C (no Python, no GPU): tests/c_client/client.c is
compiled with gcc as C99 against include/p2m.h, linked with libp2m.so, and
run on a host-only handle."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2605_00429_amd")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_c99_client(tmp_path):
    lib = os.path.join(PKG, "libp2m.so")
    assert os.path.exists(lib), "libp2m.so is not built"
    exe = str(tmp_path / "client")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_client", "client.c"), "-o", exe, "-L", PKG, "-lp2m",
                    f"-Wl,-rpath,{PKG}", "-lm"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "ok"
