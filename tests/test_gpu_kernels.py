"""GPU unit tests of the pieces of the hot path, each against the oracle or numpy.

* the batched FFT engine (every supported length, both precisions and directions,
  zero-padded input) against numpy.fft;
* the on-mesh Green table (Eq. 9 / Eq. 16 at the distances the four terms need)
  against the oracle's mode sum;
* the compressed Green spectra against the oracle's literal Eq. 10 transforms.
"""
import numpy as np
import pytest

from helpers import log, rel_l2

pytestmark = pytest.mark.gpu

# every transform length the library supports: each 2^p 3^q in [8, 1024]
def _smooth23(n):
    for p in (2, 3):
        while n % p == 0:
            n //= p
    return n == 1


LENGTHS = [n for n in range(8, 1025) if _smooth23(n)]
assert len(LENGTHS) == 36


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fft_lines_all_lengths(torch_cuda, prec):
    torch = torch_cuda
    from paper_1111_4971_amd import pipe
    rng = np.random.default_rng(1)
    cdt = torch.complex128 if prec == "fp64" else torch.complex64
    tol = 1e-14 if prec == "fp64" else 3e-7
    for n in LENGTHS:
        for n_in in sorted({n, n // 2 + 1, 1}):
            for direction in (-1, 1):
                log("fft_lines %s len=%d n_in=%d dir=%d" % (prec, n, n_in, direction))
                x = rng.standard_normal((7, n_in)) + 1j * rng.standard_normal((7, n_in))
                xt = torch.from_numpy(x).to(device="cuda", dtype=cdt)
                y = pipe.fft_lines(xt, n, direction).cpu().numpy()
                xp = np.zeros((7, n), complex)
                xp[:, :n_in] = x
                ref = np.fft.fft(xp, axis=1) if direction < 0 else np.fft.ifft(xp, axis=1) * n
                err = float(np.linalg.norm(y - ref) / np.linalg.norm(ref))
                assert err <= tol, (n, n_in, direction, err)


def _small_plan(kind, prec, nx=7, ny=5, nz=9, a=1.0, b=1.3, keep=True, **kw):
    from paper_1111_4971_amd import pipe
    hx, hy = a / (nx + 1), 0.9 * b / (ny + 1)
    return pipe.GreenPlan(nx, ny, nz, hx, hy, 0.11, a, b, kind=kind, precision=prec,
                          keep_green=keep, **kw), (nx, ny, nz, hx, hy, 0.11, a, b)


def table_distances(n, h, x0=0.0):
    """The rows of the plan's Green table: differences p h (p < n), then sums 2 x0 + (p + 2) h."""
    return np.concatenate([np.arange(n) * h, 2.0 * x0 + (np.arange(2 * n - 1) + 2) * h])


@pytest.mark.parametrize("kind", [0, 1])
def test_green_table_matches_oracle_small(torch_cuda, kind):
    from oracle import green
    log("green table small kind=%d" % kind)
    plan, (nx, ny, nz, hx, hy, hz, a, b) = _small_plan(kind, "fp64", mx=13, my=9)
    got = plan.green_table().cpu().numpy()
    ref = green.R_table(table_distances(nx, hx), table_distances(ny, hy), np.arange(nz), hz, a, b, 13, 9, kind)
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("kind", [0, 1])
def test_green_table_with_offset_matches_oracle(torch_cuda, kind):
    from oracle import green
    from paper_1111_4971_amd import pipe
    nx, ny, nz, a, b = 6, 5, 7, 1.0, 1.3
    hx, hy, x0, y0 = 0.1, 0.12, 0.17, 0.31
    log("green table offset kind=%d" % kind)
    plan = pipe.GreenPlan(nx, ny, nz, hx, hy, 0.1, a, b, kind=kind, precision="fp64", mx=13, my=9,
                          keep_green=True, offset=(x0, y0))
    got = plan.green_table().cpu().numpy()
    ref = green.R_table(table_distances(nx, hx, x0), table_distances(ny, hy, y0), np.arange(nz), 0.1, a, b,
                        13, 9, kind)
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_gpu_igf_kernel_matches_golden_quadrature(torch_cuda):
    """One mode (m = n = 1) on a 1 x 1 x 21 mesh: the table's R(0, 0, r hz) is
    g_z(kappa_11, r hz) / (2 pi a b kappa_11), so the GPU's FP64 Eq. 15 form is
    checked directly against the 40-digit quadrature values of
    tests/golden/igf_gz_quadrature.txt (hz = x / kappa_11 for each tabulated x)."""
    import math
    import os
    from paper_1111_4971_amd import pipe
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "igf_gz_quadrature.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    a = b = 1.0
    kap = math.pi * math.sqrt(2.0)
    for xs in sorted({r[0] for r in rows}, key=float):
        x = float(xs)
        log("igf golden x=%s" % xs)
        plan = pipe.GreenPlan(1, 1, 21, 0.5, 0.5, x / kap, a, b, kind=pipe.IGF_Z, precision="fp64",
                              mx=1, my=1, keep_green=True)
        got = plan.green_table().cpu().numpy()[0, 0] * (2.0 * math.pi * a * b * kap)
        plan.close()
        for rx, n, v in rows:
            if rx == xs:
                assert abs(got[int(n)] - float(v)) <= 1e-13 * float(v), (xs, n, got[int(n)], v)


@pytest.mark.parametrize("which", ["plain_fp64_32cubed", "igf_long_bunch"])
def test_green_table_matches_oracle_full_size(torch_cuda, which):
    from oracle import green
    from paper_1111_4971_amd import pipe, workloads
    wl = getattr(workloads, which)()
    log("green table %s" % which)
    plan = pipe.GreenPlan(wl.nx, wl.ny, wl.nz, wl.hx, wl.hy, wl.hz, wl.a, wl.b, kind=wl.kind,
                          precision="fp64", mx=wl.mx, my=wl.my, keep_green=True)
    got = plan.green_table().cpu().numpy()
    ref = green.R_table(table_distances(wl.nx, wl.hx), table_distances(wl.ny, wl.hy),
                        np.arange(wl.nz), wl.hz, wl.a, wl.b, wl.mx, wl.my, wl.kind)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert err <= 1e-13, err


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_spectra_match_oracle_transforms(torch_cuda, kind, prec):
    from oracle import fourterm
    log("spectra kind=%d %s" % (kind, prec))
    plan, (nx, ny, nz, hx, hy, hz, a, b) = _small_plan(kind, prec, mx=13, my=9)
    i = plan.info
    L = (i.lx, i.ly, i.lz)
    tab, nyq = (t.double().cpu().numpy() for t in plan.spectra())
    S = fourterm.green_spectra((nx, ny, nz), L, (hx, hy, hz), (a, b, 13, 9), kind)
    kx, ky, nh = i.lx // 2 + 1, i.ly // 2 + 1, i.lz // 2
    full = np.concatenate([tab, nyq[..., None]], axis=3)        # kz = 0 .. lz/2
    # The oracle holds Eq. 10's mixed-direction transforms (F^fff, F^fbf, F^bff,
    # F^bbf); the plan stores plain forward transforms.  A backward transform
    # along a dimension is the forward one at the reflected index, so
    # T_cr(kx,ky) = S_cr(kx,-ky), T_rc(kx,ky) = S_rc(-kx,ky), T_rr(kx,ky) = S_rr(-kx,-ky).
    px = np.arange(kx)
    py = np.arange(ky)
    mx_ = (i.lx - px) % i.lx
    my_ = (i.ly - py) % i.ly
    cc = S[0][np.ix_(px, py)][..., :nh + 1]
    cr = S[1][np.ix_(px, my_)][..., :nh + 1]
    rc = S[2][np.ix_(mx_, py)][..., :nh + 1]
    rr = S[3][np.ix_(mx_, my_)][..., :nh + 1]
    rr2 = S[3][np.ix_(px, my_)][..., :nh + 1]                 # T_rr(-kx, ky)
    ref = np.empty_like(full)
    ref[0] = cc.real
    ref[1], ref[2] = cr.real, cr.imag
    ref[3], ref[4] = rc.real, rc.imag
    ref[5], ref[6] = rr.real, rr.imag
    ref[7], ref[8] = rr2.real, rr2.imag
    scale = np.max(np.abs(ref))
    tol = 1e-13 if prec == "fp64" else 1e-6
    assert np.max(np.abs(full - ref)) <= tol * scale
    # the discarded parts really are zero: T_cc is real
    assert np.max(np.abs(cc.imag)) <= 1e-13 * scale
