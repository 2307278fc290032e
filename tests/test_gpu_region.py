"""Meshes covering a sub-region of the pipe cross-section (pipe_green_plan_region).

Sec. 5 of the paper: when the beam is thin, only a small transverse area
around it needs a mesh; the Green function is still that of the whole pipe.
Checked against the oracle's Eq. 10 with the offset, and against a full
mesh of the same spacing with the charge confined to the sub-region.
"""
import numpy as np
import pytest

from helpers import TOL, gpu_solve, log, oracle_input, rel_l2, rel_max

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape,offset", [((6, 5, 9), (0.23, 0.41)), ((13, 10, 20), (0.05, 0.0)),
                                          ((9, 16, 12), (0.31, 0.17))])
def test_region_matches_eq10_oracle(torch_cuda, kind, prec, shape, offset):
    from oracle import fourterm
    from paper_1111_4971_amd import pipe
    nx, ny, nz = shape
    a, b = 1.4, 1.2
    hx, hy, hz = 0.045, 0.05, 0.08
    x0, y0 = offset
    rho = np.random.default_rng(nx * 7 + ny).standard_normal(shape)
    log("region %s kind=%d shape=%s offset=%s" % (prec, kind, shape, offset))
    plan = pipe.GreenPlan(nx, ny, nz, hx, hy, hz, a, b, kind=kind, precision=prec, mx=2 * nx + 5,
                          my=2 * ny + 3, offset=offset)
    assert (plan.info.x0, plan.info.y0) == offset
    got = gpu_solve(plan, rho)
    ref = fourterm.solve(oracle_input(rho, prec), hx, hy, hz, a, b, 2 * nx + 5, 2 * ny + 3, kind, x0=x0, y0=y0)
    assert rel_l2(got, ref) <= TOL[prec] and rel_max(got, ref) <= TOL[prec]


def test_region_equals_full_mesh_restricted(torch_cuda):
    """A 24x20x64 sub-region at node offset (40, 9) of a full-aperture 96x64x64 mesh."""
    from paper_1111_4971_amd import pipe
    NX, NY, nz = 96, 64, 64
    a, b = 1.0, 0.7
    hx, hy, hz = a / (NX + 1), b / (NY + 1), 0.03
    k0, l0, nx, ny = 40, 9, 24, 20
    rng = np.random.default_rng(61)
    rho = rng.standard_normal((nx, ny, nz))
    full = np.zeros((NX, NY, nz))
    full[k0:k0 + nx, l0:l0 + ny] = rho
    log("region vs full mesh")
    pf = pipe.GreenPlan(NX, NY, nz, hx, hy, hz, a, b, kind=1, precision="fp64", mx=2 * NX, my=2 * NY)
    ps = pipe.GreenPlan(nx, ny, nz, hx, hy, hz, a, b, kind=1, precision="fp64", mx=2 * NX, my=2 * NY,
                        offset=(k0 * hx, l0 * hy))
    ref = gpu_solve(pf, full)[k0:k0 + nx, l0:l0 + ny]
    got = gpu_solve(ps, rho)
    assert rel_l2(got, ref) <= 1e-12 and rel_max(got, ref) <= 1e-12
