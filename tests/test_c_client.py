"""CPU: the C ABI used from plain C.  tests/c/client.c is compiled with gcc against include/pspec.h,
linked with libpspec.so and run; it exercises the entry points that need no GPU."""
import os
import shutil
import subprocess

import pytest

from paper_2605_26975_amd import pspec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_client_links_and_runs(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lib = pspec.LIB_PATH
    if not os.path.exists(lib):
        pytest.skip("libpspec.so is not built")
    exe = str(tmp_path / "client")
    # no HIP headers: pspec.h declares the stream type opaquely
    cmd = ["gcc", "-std=c99", "-O1", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c", "client.c"), lib, "-o", exe, f"-Wl,-rpath,{os.path.dirname(lib)}"]
    subprocess.run(cmd, check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    print(out)
    assert "rcm bandwidth 1" in out
    assert "project n=0 -> 1" in out
    assert "kmeans d=40 -> 2" in out
    assert "graph_create no workspace -> 1" in out
    assert "graph_create small workspace -> 4" in out
    assert "graph workspace k=65: 0 bytes" in out
    gws = int(out.split("graph workspace n=8000000 nnz=95998824 k=16: ")[1].split()[0])
    assert 400e6 < gws < 1e9  # the bound from (n, nnz, k_max) alone; an exact size is usually far smaller
    ws = int(out.split("dense workspace k=16: ")[1].split()[0])
    assert ws >= 2 * 1024 * 16 * 16 * 8
