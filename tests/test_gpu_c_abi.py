"""The boundary used from plain C, without PyTorch: a C99 program allocates
device memory with the HIP runtime's C API, builds a plan, solves and copies
the potential back; the result is compared with the oracle's literal Eq. 10
algorithm element by element (FP64 tolerance)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from helpers import TOL, log, rel_l2, rel_max

pytestmark = pytest.mark.gpu

C_SOLVE = r"""
#include <stdio.h>
#include <stdlib.h>
#include <hip/hip_runtime_api.h>
#include "pipe_poisson.h"
#define NX 9
#define NY 7
#define NZ 12
int main(int argc, char** argv) {
    if (argc != 3) return 10;
    const size_t n = (size_t)NX * NY * NZ;
    double* h = (double*)malloc(n * sizeof(double));
    FILE* f = fopen(argv[1], "rb");
    if (!f || fread(h, sizeof(double), n, f) != n) return 11;
    fclose(f);
    pipe_plan_t plan = 0;
    pipe_status_t st = pipe_green_plan(NX, NY, NZ, 1.0 / 10, 1.2 / 8, 0.08, 1.0, 1.2,
                                       PIPE_GREEN_IGF_Z | PIPE_PREC_FP64, &plan);
    if (st != PIPE_OK) { fprintf(stderr, "plan: %s\n", pipe_last_error()); return 12; }
    pipe_plan_info_t info;
    if (pipe_plan_info(plan, &info) != PIPE_OK) return 13;
    void *rho = 0, *phi = 0, *ws = 0;
    if (hipMalloc(&rho, n * sizeof(double)) != hipSuccess) return 14;
    if (hipMalloc(&phi, n * sizeof(double)) != hipSuccess) return 14;
    if (hipMalloc(&ws, info.workspace_bytes) != hipSuccess) return 14;
    if (hipMemcpy(rho, h, n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return 15;
    st = pipe_poisson_solve(plan, rho, phi, ws, 0);
    if (st != PIPE_OK) { fprintf(stderr, "solve: %s\n", pipe_last_error()); return 16; }
    if (hipMemcpy(h, phi, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return 17;
    f = fopen(argv[2], "wb");
    if (!f || fwrite(h, sizeof(double), n, f) != n) return 18;
    fclose(f);
    hipFree(rho); hipFree(phi); hipFree(ws);
    pipe_plan_destroy(plan);
    free(h);
    return 0;
}
"""


def test_solve_from_a_c_program(tmp_path):
    from oracle import fourterm
    from paper_1111_4971_amd import pipe
    cc = shutil.which("gcc") or shutil.which("cc")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if cc is None or not os.path.exists(os.path.join(rocm, "include", "hip", "hip_runtime_api.h")):
        pytest.skip("no C compiler or HIP headers")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    libdir = os.path.dirname(pipe.LIB_PATH)
    src, exe = tmp_path / "solve.c", tmp_path / "solve"
    src.write_text(C_SOLVE)
    # the HIP runtime's C header selects its AMD back end from this macro
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(root, "include"),
                        "-I", os.path.join(rocm, "include"), str(src), "-L", libdir, "-lpipe",
                        "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath," + libdir,
                        "-Wl,-rpath," + os.path.join(rocm, "lib"), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    rho = np.random.default_rng(31).standard_normal((9, 7, 12))
    rho.tofile(tmp_path / "rho.bin")
    log("C program solve 9x7x12 IGF FP64")
    r = subprocess.run([str(exe), str(tmp_path / "rho.bin"), str(tmp_path / "phi.bin")], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stderr)
    got = np.fromfile(tmp_path / "phi.bin").reshape(rho.shape)
    ref = fourterm.solve(rho, 1.0 / 10, 1.2 / 8, 0.08, 1.0, 1.2, 18, 14, 1)
    assert rel_l2(got, ref) <= TOL["fp64"] and rel_max(got, ref) <= TOL["fp64"]
