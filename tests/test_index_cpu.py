"""CPU: the index arithmetic that places a batch's 64-output chunks in the
caller's arrays (paper_2410_05408_amd/csrc/gl_index.h, used by the window,
classification, averaging and fused kernels), built for the host and walked
over every block of the window launch, every chunk and every output with
bounds assertions.  On a shared time grid the outputs of set s start at
s * n_times while its times start at 0; a kernel that read times at the
output index would run (n_sets - 1) * n_times * 8 bytes past the grid for the
last set, which is what the multi-set shapes below would catch."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIP_INC = "/opt/rocm/include"


@pytest.fixture(scope="module")
def index_check(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None or not os.path.exists(os.path.join(HIP_INC, "hip", "hip_runtime.h")):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path_factory.mktemp("idx") / "gl_index_check")
    subprocess.run([cxx, "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", HIP_INC,
                    "-I", os.path.join(ROOT, "paper_2410_05408_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "gl_index_check.cpp"), "-o", exe], check=True)
    return exe


def run(exe, *args):
    r = subprocess.run([exe, *map(str, args)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    tag, n = r.stdout.split()
    assert tag == "ok"
    return int(n)


@pytest.mark.parametrize("n_sets,n_times", [(48, 3000), (4096, 3000), (1, 1000), (7, 1), (3, 64),
                                            (5, 65), (2, 1024 + 63), (512, 65536)])
def test_shared_grid_indices_in_bounds(index_check, n_sets, n_times):
    assert run(index_check, "shared", n_sets, n_times) == n_sets * n_times


def test_csr_indices_in_bounds(index_check):
    lens = [0, 1, 63, 64, 65, 127, 200, 0, 0, 4097, 1]
    assert run(index_check, "csr", *lens) == sum(lens)
    rng = np.random.default_rng(4)
    lens = np.floor(np.exp(rng.uniform(np.log(200), np.log(20000), 600))).astype(int)
    assert run(index_check, "csr", *lens) == int(lens.sum())

