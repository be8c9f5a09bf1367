"""GPU: the C ABI from plain C on the device (tests/c/gpu_client.c): HIP runtime allocations, a graph
handle and F_p in FP64, against the C oracle, with no Python between the caller and the library."""
import os
import shutil
import subprocess

import pytest

import oracle as orc
from paper_2605_26975_amd import pspec

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_client_on_the_gpu(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lib, olib = pspec.LIB_PATH, orc.LIB
    if not os.path.exists(olib):
        orc.build()
    print("[case] gpu C client", flush=True)
    exe = str(tmp_path / "gpu_client")
    cmd = ["gcc", "-std=c99", "-O1", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", "/opt/rocm/include", os.path.join(ROOT, "tests", "c", "gpu_client.c"), lib, olib,
           "-L/opt/rocm/lib", "-lamdhip64", "-lm", "-o", exe,
           f"-Wl,-rpath,{os.path.dirname(lib)}:{os.path.dirname(olib)}:/opt/rocm/lib"]
    subprocess.run(cmd, check=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(res.stdout, res.stderr)
    assert res.returncode == 0 and "ok" in res.stdout
