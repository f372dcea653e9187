"""The C ABI from plain C: tests/c/compress_log2d.c includes only include/blr_tag.h and the HIP
runtime API, links libblrtag.so, and compresses, applies and measures a 2D log-kernel matrix.
The build runs on the CPU (C99, all warnings as errors); running it needs the GPU."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "compress_log2d.c")
LIBDIR = os.path.join(ROOT, "paper_2501_05528_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _build(tmp_path):
    if not os.path.exists(os.path.join(LIBDIR, "libblrtag.so")):
        pytest.fail("libblrtag.so is not built")
    exe = str(tmp_path / "compress_log2d")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{ROCM}/include", f"-I{ROOT}/include", "-o", exe, SRC, f"-L{LIBDIR}", "-lblrtag",
           f"-L{ROCM}/lib", "-lamdhip64", "-lm", f"-Wl,-rpath,{LIBDIR}", f"-Wl,-rpath,{ROCM}/lib"]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    return exe


def test_c_example_builds(tmp_path):
    assert os.path.exists(_build(tmp_path))


@pytest.mark.gpu
def test_c_example_runs(tmp_path):
    exe = _build(tmp_path)
    print("[gpu-case] plain C compress_log2d", flush=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=180)
    print(res.stdout, res.stderr, flush=True)
    assert res.returncode == 0, (res.returncode, res.stdout, res.stderr)
    assert "rel fro error" in res.stdout
