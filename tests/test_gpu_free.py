"""Free-space Hockney plans (pipe_free_plan, Eq. 3-5) and the mixed-direction
3-D transform (pipe_fft3d, Sec. 5 and Eq. 6).

Free-space solves are compared with the oracle's Eq. 5 (itself pinned to the
direct sum of Eq. 4), the point-charge response, the adjoint identity, mixed
batches, and the pipe solver's free-space limit.  The 3-D transform is
compared with numpy for every direction string, in and out of place, and
used to check Eq. 6 on the GPU.
"""
import math

import numpy as np
import pytest

from helpers import TOL, gpu_solve, log, oracle_input, rel_l2, rel_max

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape,h,g0,L", [((9, 7, 12), (0.1, 0.12, 0.08), 0.0, None),
                                          ((16, 10, 24), (0.05, 0.07, 0.04), 25.0, None),
                                          ((20, 13, 40), (0.03, 0.03, 0.06), 40.0, (48, 32, 96)),
                                          ((5, 6, 7), (0.2, 0.2, 0.2), 3.0, (12, 12, 16)),
                                          ((14, 5, 20), (0.04, 0.1, 0.05), 9.0, (27, 9, 54)),
                                          ((40, 18, 60), (0.02, 0.05, 0.03), 11.0, (81, 36, 144)),
                                          ((1, 1, 1), (0.1, 0.1, 0.1), 4.0, None),
                                          ((3, 1, 2), (0.1, 0.2, 0.3), 4.0, None)])
def test_free_matches_eq5_oracle(torch_cuda, prec, shape, h, g0, L):
    from oracle import free
    from paper_1111_4971_amd import pipe
    rho = np.random.default_rng(sum(shape)).standard_normal(shape)
    log("free %s shape=%s L=%s" % (prec, shape, L))
    plan = pipe.FreePlan(*shape, *h, g0, precision=prec, L=L)
    assert plan.info.kind & 0x0F == pipe.FREE and plan.info.norm == 1.0
    got = gpu_solve(plan, rho)
    ref = free.solve_fft(oracle_input(rho, prec), h, g0, L)
    assert rel_l2(got, ref) <= TOL[prec] and rel_max(got, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_free_spectra_are_the_transform_of_eq5_green_array(torch_cuda, prec):
    """The plan keeps one value per orbit: the forward 3-D DFT of the zero-padded
    1/r array (real, as the array is even in every dimension); the spectra copy
    returns it as plane 0 and zeros in planes 1..8."""
    from oracle import free
    from paper_1111_4971_amd import pipe
    shape, h, g0 = (9, 7, 12), (0.1, 0.12, 0.08), 5.0
    log("free spectra %s" % prec)
    plan = pipe.FreePlan(*shape, *h, g0, precision=prec, L=(24, 16, 32))
    i = plan.info
    tab, nyq = (t.double().cpu().numpy() for t in plan.spectra())
    full = np.concatenate([tab, nyq[..., None]], axis=3)        # kz = 0 .. lz/2
    S = np.fft.fftn(free.green_array(shape, (i.lx, i.ly, i.lz), h, g0))
    ref = S[:i.lx // 2 + 1, :i.ly // 2 + 1, :i.lz // 2 + 1]
    assert np.max(np.abs(ref.imag)) <= 1e-12 * np.max(np.abs(ref))
    tol = 1e-13 if prec == "fp64" else 1e-6
    assert np.max(np.abs(full[0] - ref.real)) <= tol * np.max(np.abs(ref))
    assert not np.any(full[1:])


def test_free_point_charge(torch_cuda):
    """rho = delta / (hx hy hz) at node c gives phi = 1/r, and g0 at c."""
    from paper_1111_4971_amd import pipe
    h = (0.1, 0.15, 0.12)
    shape = (12, 9, 16)
    c = (5, 3, 11)
    rho = np.zeros(shape)
    rho[c] = 1.0 / np.prod(h)
    log("free point charge")
    got = gpu_solve(pipe.FreePlan(*shape, *h, 17.0), rho)
    i, j, k = np.meshgrid(*(np.arange(n) - cc for n, cc in zip(shape, c)), indexing="ij")
    r = np.sqrt((i * h[0]) ** 2 + (j * h[1]) ** 2 + (k * h[2]) ** 2)
    ref = np.where(r > 0, 1.0 / np.where(r > 0, r, 1.0), 17.0)
    assert np.max(np.abs(got - ref)) <= 1e-12 * ref.max()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_free_adjoint_identity(torch_cuda, prec):
    torch = torch_cuda
    from paper_1111_4971_amd import pipe
    shape = (14, 11, 19)
    rng = np.random.default_rng(8)
    plan = pipe.FreePlan(*shape, 0.05, 0.06, 0.07, 30.0, precision=prec)
    x = torch.tensor(rng.standard_normal(shape), device="cuda", dtype=plan.dtype)
    y = torch.tensor(rng.standard_normal(shape), device="cuda", dtype=plan.dtype)
    log("free adjoint %s" % prec)
    ax, aty = plan.solve(x).double(), plan.adjoint(y).double()
    lhs, rhs = float((ax * y.double()).sum()), float((x.double() * aty).sum())
    assert abs(lhs - rhs) <= 10 * TOL[prec] * float(ax.norm() * y.double().norm())


def test_free_and_pipe_plans_in_one_batch(torch_cuda):
    torch = torch_cuda
    from paper_1111_4971_amd import pipe
    rng = np.random.default_rng(9)
    plans = [pipe.FreePlan(16, 12, 20, 0.05, 0.05, 0.1, 20.0),
             pipe.GreenPlan(16, 12, 20, 1.0 / 17, 1.0 / 13, 0.1, 1.0, 1.0, kind=pipe.IGF_Z),
             pipe.FreePlan(9, 9, 9, 0.1, 0.1, 0.1, 10.0)]
    rhos = [torch.tensor(rng.standard_normal(p.shape), device="cuda") for p in plans]
    log("free + pipe batch")
    outs = pipe.Batch(plans).solve(rhos)
    torch.cuda.synchronize()
    for p, r, o in zip(plans, rhos, outs):
        ref = p.solve(r)
        assert rel_max(o.cpu().numpy(), ref.cpu().numpy()) <= 1e-14


def test_pipe_solver_tends_to_the_free_space_solver(torch_cuda):
    """A point charge at the centre of ever wider square pipes (point Green
    function, modes up to 40 a / (pi h)): away from its own plane, 4 pi^2
    phi_pipe - phi_free tends to a constant image potential C(a) in (-3/a,
    -0.5/a), and the remainder falls roughly like a^-3 (Sec. 2's Green function
    against Eq. 3; the 4 pi^2 undoes the normalisation of Eq. 9)."""
    from paper_1111_4971_amd import pipe
    n, h, c = 8, 0.1, 4
    rho = np.zeros((n, n, n))
    rho[c, c, c] = 1.0 / h ** 3
    free_phi = gpu_solve(pipe.FreePlan(n, n, n, h, h, h, 0.0), rho)
    away = np.abs(np.arange(n) - c) >= 1
    resid = []
    for a in (2.0, 4.0, 8.0):
        M = int(40 * a / (math.pi * h)) + 1
        x0 = a / 2 - (c + 1) * h
        log("pipe -> free limit a=%g modes=%d" % (a, M))
        plan = pipe.GreenPlan(n, n, n, h, h, h, a, a, kind=pipe.POINT, mx=M, my=M, offset=(x0, x0))
        d = (4 * math.pi ** 2 * gpu_solve(plan, rho) - free_phi)[:, :, away]
        assert -3.0 / a < d.mean() < -0.5 / a
        resid.append(np.max(np.abs(d - d.mean())))
        plan.close()
    assert resid[1] < resid[0] / 5 and resid[2] < resid[1] / 5


DIRS = ["fff", "bbb", "fbf", "bfb", "ffb", "bbf", "fbb", "bff"]


def _numpy_mixed(a, dirs):
    for axis, d in enumerate(dirs):
        a = np.fft.fft(a, axis=axis) if d == "f" else np.fft.ifft(a, axis=axis) * a.shape[axis]
    return a


@pytest.mark.parametrize("dirs", DIRS)
@pytest.mark.parametrize("shape", [(8, 12, 16), (24, 8, 48), (64, 32, 128), (384, 8, 768), (768, 8, 384), (27, 36, 81), (9, 144, 54)])
def test_fft3d_matches_numpy(torch_cuda, dirs, shape):
    torch = torch_cuda
    from paper_1111_4971_amd import pipe
    rng = np.random.default_rng(len(dirs) + sum(shape))
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = _numpy_mixed(a, dirs)
    log("fft3d %s %s" % (dirs, shape))
    for dt, tol in ((torch.complex128, 1e-12), (torch.complex64, 1e-5)):
        x = torch.tensor(a, device="cuda", dtype=dt)
        got = pipe.fft3d(x, dirs).cpu().numpy()
        assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))
        y = pipe.fft3d(x, dirs, out=x).cpu().numpy()            # in place
        assert np.array_equal(y, got)


def test_eq6_on_the_gpu(torch_cuda):
    """Eq. 6 with the GPU transforms: a y correlation, x and z convolutions."""
    torch = torch_cuda
    from paper_1111_4971_amd import pipe
    rng = np.random.default_rng(12)
    nx, ny, nz = 5, 4, 6
    L = (12, 8, 12)
    rho = rng.standard_normal((nx, ny, nz))
    Gf = rng.standard_normal((2 * nx - 1, 2 * ny - 1, 2 * nz - 1))   # [d_x + nx-1, s_y, d_z + nz-1]
    ref = np.zeros((nx, ny, nz))
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                ref[i, j, k] = np.sum(rho * Gf[i - np.arange(nx)[:, None, None] + nx - 1,
                                               j + np.arange(ny)[None, :, None],
                                               k - np.arange(nz)[None, None, :] + nz - 1])
    garr = np.zeros(L)
    for p in range(-(nx - 1), nx):
        for q in range(-(nz - 1), nz):
            garr[p % L[0], :2 * ny - 1, q % L[2]] = Gf[p + nx - 1, :, q + nz - 1]
    pad = np.zeros(L)
    pad[:nx, :ny, :nz] = rho
    log("eq6 on gpu")
    r = pipe.fft3d(torch.tensor(pad, device="cuda", dtype=torch.complex128), "fff")
    g = pipe.fft3d(torch.tensor(garr, device="cuda", dtype=torch.complex128), "fbf")
    out = pipe.fft3d(r * g, "bfb").cpu().numpy() / np.prod(L)
    assert np.max(np.abs(out[:nx, :ny, :nz].real - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.fixture(scope="module")
def three_bunch():
    from paper_1111_4971_amd import workloads
    return workloads.three_bunch_cic()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_free_benchmark_mesh_full_field(torch_cuda, three_bunch, prec):
    """The bench's free-space leg: 128 x 128 x 512 three-bunch charge, G(0) = 0,
    against the oracle's Eq. 5 on the whole field."""
    from oracle import free
    from paper_1111_4971_amd import pipe
    wl = three_bunch
    h = (wl.hx, wl.hy, wl.hz)
    log("free 128x128x512 %s" % prec)
    got = gpu_solve(pipe.FreePlan(wl.nx, wl.ny, wl.nz, *h, 0.0, precision=prec), wl.rho)
    log("free 128x128x512 %s: oracle" % prec)
    ref = free.solve_fft(oracle_input(wl.rho, prec), h, 0.0)
    assert rel_l2(got, ref) <= TOL[prec] and rel_max(got, ref) <= TOL[prec]
