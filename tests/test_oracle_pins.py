"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each check is a closed form, a
textbook routine, brute force, an invariant of the pipe problem, or a second
algorithm that shares no arithmetic with the first.
"""
import math
import os

import numpy as np
import pytest

from oracle import conv1d, direct, fourterm, green, gradient, igf_quad, modespace

POINT, IGF = green.POINT, green.IGF_Z


def rel_l2(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


# ---------------------------------------------------------------- Appendix (A.1-A.9)

@pytest.mark.parametrize("J,K,extra", [(5, 5, 0), (7, 4, 0), (6, 6, 3), (9, 3, 1)])
def test_appendix_conv_matches_numpy_convolve(J, K, extra):
    rng = np.random.default_rng(100 + J + K)
    r = rng.standard_normal(K)
    xs = rng.standard_normal(J + K - 1)             # x_m, m = -(K-1)..J-1
    x = lambda m: xs[m + K - 1]
    N = J + K - 1 + extra
    got = conv1d.conv_fft(r, x, J, N).real
    # numpy.convolve(r, xs)[j + K - 1] = sum_k r_k xs[j + K - 1 - k] = sum_k r_k x_{j-k}
    ref = np.convolve(r, xs)[K - 1:K - 1 + J]
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.allclose(conv1d.conv_direct(r, x, J), ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("J,K,extra", [(5, 5, 0), (7, 4, 0), (6, 6, 3), (4, 8, 2)])
def test_appendix_corr_matches_numpy_correlate(J, K, extra):
    rng = np.random.default_rng(200 + J + K)
    r = rng.standard_normal(K)
    xs = rng.standard_normal(J + K - 1)             # x_m, m = 0..J+K-2
    x = lambda m: xs[m]
    N = J + K - 1 + extra
    got = conv1d.corr_fft(r, x, J, N).real
    # numpy.correlate(xs, r, 'valid')[j] = sum_k xs[j + k] r_k  (real input)
    ref = np.correlate(xs, r, mode='full')[K - 1:K - 1 + J]
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.allclose(conv1d.corr_direct(r, x, J), ref, rtol=0, atol=1e-13)


def test_appendix_padding_too_short_wraps():
    """N < J + K - 1 aliases: the padding rule of the Appendix is not vacuous."""
    rng = np.random.default_rng(3)
    J = K = 6
    r = rng.standard_normal(K)
    xs = rng.standard_normal(J + K - 1)
    x = lambda m: xs[m + K - 1]
    ref = np.convolve(r, xs)[K - 1:K - 1 + J]
    with pytest.raises(ValueError):
        conv1d.conv_fft(r, x, J, J + K - 2)


# ---------------------------------------------------------------- IGF kernel (Eq. 13-15)

@pytest.mark.parametrize("x", [1e-6, 1e-3, 0.05, 0.3, 1.0, 4.0, 30.0, 300.0])
@pytest.mark.parametrize("r", [0, 1, 2, 5, 50])
def test_igf_rewrite_matches_quadrature_of_eq14(x, r):
    hz = 0.2
    kap = x / hz
    got = green.gz_igf(np.array([kap]), np.array([r]), hz)[0, 0]
    ref = float(igf_quad.gz_quad(kap, r * hz, hz))
    exact = float(igf_quad.gz_exact(kap, r * hz, hz))
    assert abs(exact - ref) <= 1e-25 * abs(ref)       # Eq. 15 is the integral of Eq. 14
    if ref < 1e-300:
        assert got < 1e-290
    else:
        # e^{-kappa |w|} has condition number ~kappa |w|: one rounding of its
        # argument moves it by that many ulps
        cond = 1.0 + x * (r + 1)
        assert abs(got - ref) <= 4e-15 * cond * abs(ref), (got, ref)


def igf_golden():
    """(x, n, g_z) rows of tests/golden/igf_gz_quadrature.txt (40-digit quadrature, hz = 1)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "igf_gz_quadrature.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    return [(float(x), int(n), float(v)) for x, n, v in rows]


def test_igf_rewrite_matches_golden_quadrature():
    """The cancellation-free Eq. 15 of the oracle against the stored quadrature values,
    from x = kappa hz = 1e-8 (where the printed Eq. 15 loses all digits) to x = 40."""
    rows = igf_golden()
    assert len(rows) >= 50
    for x, n, v in rows:
        got = float(green.gz_igf(np.array(x), np.array([n]), 1.0)[0])
        assert abs(got - v) <= 1e-14 * v, (x, n, got, v)


def test_igf_literal_eq15_agrees_where_it_is_accurate():
    hz = 0.1
    kap = np.array([3.0, 10.0, 40.0])
    r = np.arange(0, 8)
    assert np.allclose(green.gz_igf_eq15(kap, r, hz), green.gz_igf(kap, r, hz), rtol=1e-13, atol=0)


@pytest.mark.parametrize("x", [1e-4, 0.01, 0.3, 2.0, 15.0])
def test_igf_partition_of_unity(x):
    """sum_k h g(k h) = integral of e^{-kappa|w|} = 2/kappa (hats sum to one)."""
    hz = 0.05
    kap = x / hz
    nmax = int(60.0 / x) + 5
    r = np.arange(-nmax, nmax + 1)
    s = math.fsum(hz * green.gz_igf(np.array([kap]), r, hz)[0])
    assert abs(s - 2.0 / kap) <= 2e-14 * (2.0 / kap)


def test_igf_tends_to_point_kernel_as_cells_shrink():
    kap, w = 5.0, 0.3
    errs = []
    for n in (10, 100, 1000):
        hz = w / n
        g = green.gz_igf(np.array([kap]), np.array([n]), hz)[0, 0]
        errs.append(abs(g - math.exp(-kap * w)))
    # second-order in hz: 10x finer cell -> ~100x smaller difference
    assert errs[1] < errs[0] / 50 and errs[2] < errs[1] / 50


# ---------------------------------------------------------------- Green function (Eq. 7-9)

def test_R_table_matches_plain_loops():
    a, b, mx, my = 1.3, 0.7, 7, 5
    u = np.array([0.0, 0.11, 0.9, 2.1])
    v = np.array([0.05, 0.6, 1.3])
    hz = 0.07
    r = np.array([0, 1, 3])
    tab = green.R_table(u, v, r, hz, a, b, mx, my, POINT)
    for iu, uu in enumerate(u):
        for iv, vv in enumerate(v):
            for ir, rr in enumerate(r):
                assert abs(tab[iu, iv, ir] - green.R_point(uu, vv, rr * hz, a, b, mx, my)) <= 1e-15


def test_R_is_even_and_2a_periodic():
    a, b, mx, my = 1.0, 1.7, 9, 6
    u = np.array([0.13, 0.7])
    v = np.array([0.21, 1.1])
    r = np.array([2])
    t0 = green.R_table(u, v, r, 0.1, a, b, mx, my, IGF)
    assert np.allclose(green.R_table(-u, v, r, 0.1, a, b, mx, my, IGF), t0, rtol=1e-14, atol=1e-15)
    assert np.allclose(green.R_table(u, -v, r, 0.1, a, b, mx, my, IGF), t0, rtol=1e-14, atol=1e-15)
    assert np.allclose(green.R_table(u + 2 * a, v, r, 0.1, a, b, mx, my, IGF), t0, rtol=1e-12, atol=1e-14)
    assert np.allclose(green.R_table(u, v, -r, 0.1, a, b, mx, my, IGF), t0, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("kind", [POINT, IGF])
def test_eq8_four_terms_equal_four_times_eq7(kind):
    """Eq. 8 (with Eq. 9's prefactor) is exactly 4x Eq. 7 as printed: sin A sin B identity."""
    rng = np.random.default_rng(7)
    a, b = 1.2, 0.8
    x, xp = rng.uniform(0, a, 3), rng.uniform(0, a, 2)
    y, yp = rng.uniform(0, b, 2), rng.uniform(0, b, 3)
    r = np.array([0, 1, 4])
    g8 = green.G_four_term(x, xp, y, yp, r, 0.05, a, b, 11, 9, kind)
    g7 = green.G_sine_series(x, xp, y, yp, r, 0.05, a, b, 11, 9, kind)
    assert np.allclose(g8, 4.0 * g7, rtol=1e-12, atol=1e-14)


def test_green_vanishes_on_the_walls():
    a, b = 1.1, 0.9
    xp, yp = np.array([0.3, 0.77]), np.array([0.2, 0.5])
    r = np.array([0, 2])
    for x in (0.0, a):
        g = green.G_four_term(np.array([x]), xp, np.array([0.4]), yp, r, 0.1, a, b, 15, 15, IGF)
        assert np.max(np.abs(g)) <= 1e-13
    for y in (0.0, b):
        g = green.G_four_term(np.array([0.4]), xp, np.array([y]), yp, r, 0.1, a, b, 15, 15, POINT)
        assert np.max(np.abs(g)) <= 1e-13


def test_free_space_limit_of_the_pipe_green_function():
    """Far from the walls 4 pi^2 G -> 1/r + C(a) (Eq. 3 up to the dropped 4 pi and
    a constant image potential); the residual shape decays with the pipe size."""
    hz = 0.1
    resid = []
    for a in (2.0, 4.0, 8.0):
        M = int(40 * a / (math.pi * hz)) + 1
        x0 = a / 2
        xs = x0 + np.array([0.0, 0.1, 0.2])
        r = np.array([1, 2, 3])
        G = green.G_four_term(xs, np.array([x0]), xs, np.array([x0]), r, hz, a, a, M, M, POINT)
        G = G[:, 0, :, 0, :]
        dx = (xs - x0)[:, None, None]
        dy = (xs - x0)[None, :, None]
        dz = (r * hz)[None, None, :]
        diff = 4 * math.pi ** 2 * G - 1.0 / np.sqrt(dx ** 2 + dy ** 2 + dz ** 2)
        resid.append(np.max(np.abs(diff - diff.mean())))
        # constant image term is O(1/a) and negative (opposite-sign images)
        assert -3.0 / a < diff.mean() < -0.5 / a
    # residual after removing the constant falls roughly like a^-3
    assert resid[1] < resid[0] / 5 and resid[2] < resid[1] / 5


# ---------------------------------------------------------------- whole solve: three algorithms

CASES = [
    # (nx, ny, nz, full aperture?, a, b, mx, my)
    (3, 2, 3, True, 1.0, 1.0, 6, 4),
    (5, 4, 6, True, 1.3, 0.8, 10, 8),
    (4, 5, 7, False, 1.0, 1.4, 9, 7),
    (6, 3, 5, True, 2.0, 1.0, 13, 5),
]


def _mesh(nx, ny, full, a, b):
    if full:
        return a / (nx + 1), b / (ny + 1)
    return 0.8 * a / (nx + 1), 0.9 * b / (ny + 1)


def test_O1_vectorised_equals_python_loops():
    rng = np.random.default_rng(11)
    rho = rng.standard_normal((3, 2, 3))
    hx, hy = 1.0 / 4, 1.0 / 3
    got = direct.solve(rho, hx, hy, 0.2, 1.0, 1.0, 5, 4, POINT)
    ref = direct.solve_python_loops(rho, hx, hy, 0.2, 1.0, 1.0, 5, 4)
    assert rel_l2(got, ref) <= 1e-14


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("kind", [POINT, IGF])
def test_O1_O2_O3_agree(case, kind):
    nx, ny, nz, full, a, b, mx, my = case
    hx, hy = _mesh(nx, ny, full, a, b)
    hz = 0.13
    rng = np.random.default_rng(nx * 100 + ny * 10 + nz + kind)
    rho = rng.standard_normal((nx, ny, nz))
    o1 = direct.solve(rho, hx, hy, hz, a, b, mx, my, kind)
    o2 = fourterm.solve(rho, hx, hy, hz, a, b, mx, my, kind)
    assert rel_l2(o2, o1) <= 1e-13
    if full:
        o3 = modespace.solve(rho, hx, hy, hz, a, b, mx, my, kind)
        assert rel_l2(o3, o1) <= 1e-13


@pytest.mark.parametrize("kind", [POINT, IGF])
def test_O2_is_invariant_under_pad_length(kind):
    nx, ny, nz = 5, 4, 6
    a, b = 1.0, 1.2
    hx, hy = a / 6, b / 5
    rng = np.random.default_rng(5)
    rho = rng.standard_normal((nx, ny, nz))
    base = fourterm.solve(rho, hx, hy, 0.1, a, b, 9, 8, kind)
    for L in [(9, 7, 11), (10, 8, 12), (13, 11, 15), (16, 9, 20)]:
        got, imag = fourterm.solve(rho, hx, hy, 0.1, a, b, 9, 8, kind, L=L, return_imag=True)
        assert rel_l2(got, base) <= 1e-13
        assert imag <= 1e-13 * np.max(np.abs(base))
    with pytest.raises(ValueError):
        fourterm.solve(rho, hx, hy, 0.1, a, b, 9, 8, kind, L=(8, 8, 12))


@pytest.mark.slow
def test_brute_force_sub_case_8cubed():
    """The 8x8x8 sub-case: h = 1/9, hz = 0.05, 64 x 64 modes, point kernel."""
    rng = np.random.default_rng(11)
    n = 8
    h = 1.0 / 9
    rho = rng.standard_normal((n, n, n))
    o1 = direct.solve(rho, h, h, 0.05, 1.0, 1.0, 64, 64, POINT)
    o2 = fourterm.solve(rho, h, h, 0.05, 1.0, 1.0, 64, 64, POINT)
    o3 = modespace.solve(rho, h, h, 0.05, 1.0, 1.0, 64, 64, POINT)
    assert rel_l2(o2, o1) <= 1e-13 and rel_l2(o3, o1) <= 1e-13


# ---------------------------------------------------------------- invariants of the pipe operator

@pytest.mark.parametrize("kind", [POINT, IGF])
def test_wall_nodes_carry_zero_potential(kind):
    """Mesh with n nodes whose last node lies on the wall X = a (h = a/n)."""
    nx, ny, nz = 6, 5, 4
    a, b = 1.0, 0.7
    hx, hy = a / nx, b / ny                       # X_{nx-1} = a, Y_{ny-1} = b
    rng = np.random.default_rng(21)
    rho = rng.standard_normal((nx, ny, nz))
    phi = fourterm.solve(rho, hx, hy, 0.1, a, b, 20, 20, kind)
    scale = np.max(np.abs(phi))
    assert np.max(np.abs(phi[-1])) <= 1e-13 * scale
    assert np.max(np.abs(phi[:, -1])) <= 1e-13 * scale
    o1 = direct.solve(rho, hx, hy, 0.1, a, b, 20, 20, kind)
    assert np.max(np.abs(o1[-1])) <= 1e-13 * scale


@pytest.mark.parametrize("kind", [POINT, IGF])
def test_reflection_symmetry(kind):
    nx, ny, nz = 6, 5, 4
    a, b = 1.0, 1.5
    hx, hy = a / (nx + 1), b / (ny + 1)
    rng = np.random.default_rng(22)
    rho = rng.standard_normal((nx, ny, nz))
    A = lambda r: fourterm.solve(r, hx, hy, 0.1, a, b, 12, 10, kind)
    base = A(rho)
    assert rel_l2(A(rho[::-1]), base[::-1]) <= 1e-13
    assert rel_l2(A(rho[:, ::-1]), base[:, ::-1]) <= 1e-13
    assert rel_l2(A(rho[:, :, ::-1]), base[:, :, ::-1]) <= 1e-13


@pytest.mark.parametrize("kind", [POINT, IGF])
def test_operator_is_symmetric_and_linear(kind):
    nx, ny, nz = 5, 4, 6
    a, b = 1.0, 1.3
    hx, hy = 0.9 * a / (nx + 1), b / (ny + 1)
    rng = np.random.default_rng(23)
    r1, r2 = rng.standard_normal((2, nx, ny, nz))
    A = lambda r: fourterm.solve(r, hx, hy, 0.1, a, b, 10, 8, kind)
    lhs, rhs = np.sum(A(r1) * r2), np.sum(r1 * A(r2))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    al, be = 0.7, -2.3
    assert rel_l2(A(al * r1 + be * r2), al * A(r1) + be * A(r2)) <= 1e-13


@pytest.mark.parametrize("kind", [POINT, IGF])
def test_single_sine_mode_closed_form(kind):
    nx, ny, nz = 7, 6, 9
    a, b = 1.0, 1.4
    hx, hy = a / (nx + 1), b / (ny + 1)
    hz = 0.11
    X, Y = green.node_coords(nx, ny, hx, hy)
    f = np.random.default_rng(24).standard_normal(nz)
    sx, sy = np.sin(np.pi * X / a), np.sin(np.pi * Y / b)
    rho = sx[:, None, None] * sy[None, :, None] * f[None, None, :]
    phi = fourterm.solve(rho, hx, hy, hz, a, b, 2 * nx, 2 * ny, kind)
    prof = modespace.single_mode_response(f, hz, a, b, kind, 2 * nx, 2 * ny)
    ref = sx[:, None, None] * sy[None, :, None] * prof[None, None, :]
    assert rel_l2(phi, ref) <= 1e-13


@pytest.mark.parametrize("kind", [POINT, IGF])
def test_single_tabulated_array_on_a_wall_node_grid(kind):
    """The statement after Eq. 10 (one R array transformed four ways) holds on a
    mesh whose nodes include the walls; it reproduces the direct sum there."""
    N, Ny, nz = 6, 5, 4
    h = 0.2
    rng = np.random.default_rng(25)
    rho = np.zeros((N + 1, Ny + 1, nz))
    rho[1:N, 1:Ny] = rng.standard_normal((N - 1, Ny - 1, nz))
    got = fourterm.single_array_wall_grid(rho, h, N, Ny, 0.1, 14, 12, kind)
    # interior nodes i = 1..N-1 are the (i+1) h mesh with n = N - 1 nodes, a = N h
    ref = direct.solve(rho[1:N, 1:Ny], h, h, 0.1, N * h, Ny * h, 14, 12, kind)
    assert rel_l2(got[1:N, 1:Ny], ref) <= 1e-13
    assert np.max(np.abs(got[0])) <= 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(got[N])) <= 1e-12 * np.max(np.abs(ref))


def test_gradient_oracle_matches_finite_differences():
    nx, ny, nz = 4, 3, 5
    a, b = 1.0, 1.0
    hx, hy = a / 5, b / 4
    rng = np.random.default_rng(26)
    rho = rng.standard_normal((nx, ny, nz))
    tgt = rng.standard_normal((nx, ny, nz)) * 0.01
    A = lambda r: fourterm.solve(r, hx, hy, 0.2, a, b, 8, 6, IGF)
    g = gradient.grad(A, rho, tgt)
    eps = 1e-3
    for idx in [(0, 0, 0), (2, 1, 3), (3, 2, 4)]:
        e = np.zeros_like(rho)
        e[idx] = eps
        lp = gradient.loss(rho + e, A(rho + e), tgt)
        lm = gradient.loss(rho - e, A(rho - e), tgt)
        assert abs((lp - lm) / (2 * eps) - g[idx]) <= 1e-8 * np.max(np.abs(g))


def test_sampled_direct_sum_equals_full_direct_sum():
    rng = np.random.default_rng(27)
    nx, ny, nz = 5, 4, 6
    a, b = 1.0, 1.2
    hx, hy = 0.9 * a / (nx + 1), b / (ny + 1)
    rho = rng.standard_normal((nx, ny, nz))
    for kind in (POINT, IGF):
        full = direct.solve(rho, hx, hy, 0.1, a, b, 9, 7, kind)
        pts = [(0, 0, 0), (4, 3, 5), (2, 1, 3), (1, 2, 0)]
        got = direct.solve_at(rho, pts, hx, hy, 0.1, a, b, 9, 7, kind)
        assert np.allclose(got, [full[p] for p in pts], rtol=1e-13, atol=1e-15 * np.max(np.abs(full)))


# ---------------------------------------------------------------- transverse sub-region mesh (Sec. 5)

@pytest.mark.parametrize("kind", [POINT, IGF])
def test_offset_mesh_equals_full_mesh_restricted(kind):
    """A mesh offset by (k0 h, l0 h) is the block k0.., l0.. of the full mesh with the
    same spacing: with charge only in that block both give the same potential there."""
    nx, ny, nz = 4, 3, 5
    k0, l0 = 2, 1
    NX, NY = 8, 6
    a, b = (NX + 1) * 0.1, (NY + 1) * 0.12
    hx, hy = 0.1, 0.12
    rng = np.random.default_rng(51)
    rho = rng.standard_normal((nx, ny, nz))
    full = np.zeros((NX, NY, nz))
    full[k0:k0 + nx, l0:l0 + ny] = rho
    ref = fourterm.solve(full, hx, hy, 0.1, a, b, 11, 9, kind)[k0:k0 + nx, l0:l0 + ny]
    got2 = fourterm.solve(rho, hx, hy, 0.1, a, b, 11, 9, kind, x0=k0 * hx, y0=l0 * hy)
    got1 = direct.solve(rho, hx, hy, 0.1, a, b, 11, 9, kind, x0=k0 * hx, y0=l0 * hy)
    assert rel_l2(got2, ref) <= 1e-13 and rel_l2(got1, ref) <= 1e-13


@pytest.mark.parametrize("kind", [POINT, IGF])
def test_offset_mesh_centred_is_mirror_symmetric(kind):
    nx, ny, nz = 5, 4, 6
    a, b = 1.0, 1.2
    hx, hy = 0.1, 0.11
    x0, y0 = (a - (nx + 1) * hx) / 2, (b - (ny + 1) * hy) / 2
    rng = np.random.default_rng(52)
    rho = rng.standard_normal((nx, ny, nz))
    A = lambda r: fourterm.solve(r, hx, hy, 0.1, a, b, 13, 11, kind, x0=x0, y0=y0)
    base = A(rho)
    assert rel_l2(A(rho[::-1].copy()), base[::-1]) <= 1e-13
    assert rel_l2(A(rho[:, ::-1].copy()), base[:, ::-1]) <= 1e-13


# ---------------------------------------------------------------- neighbouring-plane sums (Eq. 17-18)

@pytest.mark.parametrize("kind", [POINT, IGF])
def test_band_limits_of_the_z_sum(kind):
    """band = nz - 1 is the full sum; band = 0 decouples the planes (Eq. 17): each
    plane is its own one-plane problem; Eq. 10 with the banded Green array equals
    the banded direct sum."""
    nx, ny, nz = 5, 4, 6
    a, b = 1.0, 1.2
    hx, hy, hz = 0.9 * a / (nx + 1), b / (ny + 1), 0.1
    rng = np.random.default_rng(71)
    rho = rng.standard_normal((nx, ny, nz))
    full = direct.solve(rho, hx, hy, hz, a, b, 9, 8, kind)
    assert rel_l2(direct.solve(rho, hx, hy, hz, a, b, 9, 8, kind, band=nz - 1), full) <= 1e-15
    b0 = direct.solve(rho, hx, hy, hz, a, b, 9, 8, kind, band=0)
    planes = np.stack([fourterm.solve(rho[:, :, k:k + 1], hx, hy, hz, a, b, 9, 8, kind)[:, :, 0]
                       for k in range(nz)], axis=2)
    assert rel_l2(b0, planes) <= 1e-13
    for band in (0, 1, 2):
        d = direct.solve(rho, hx, hy, hz, a, b, 9, 8, kind, band=band)
        f = fourterm.solve(rho, hx, hy, hz, a, b, 9, 8, kind, band=band)
        assert rel_l2(f, d) <= 1e-13


# ---------------------------------------------------------------- free space (Eq. 3-5)

def test_free_direct_equals_python_loops():
    from oracle import free
    rng = np.random.default_rng(81)
    rho = rng.standard_normal((3, 2, 4))
    h = (0.3, 0.5, 0.2)
    assert rel_l2(free.solve_direct(rho, h, 2.5), free.solve_python_loops(rho, h, 2.5)) <= 1e-14


@pytest.mark.parametrize("shape,L", [((4, 3, 5), None), ((5, 4, 3), (9, 7, 5)), ((6, 2, 7), (16, 6, 20))])
def test_free_eq5_fft_equals_direct_sum(shape, L):
    """Eq. 5 with any padding L >= 2n - 1 reproduces the direct sum of Eq. 4 (Appendix A.8)."""
    from oracle import free
    rng = np.random.default_rng(sum(shape))
    rho = rng.standard_normal(shape)
    h = (0.11, 0.07, 0.13)
    assert rel_l2(free.solve_fft(rho, h, 3.0, L), free.solve_direct(rho, h, 3.0)) <= 1e-13


def test_free_point_charge_gives_the_green_function():
    """A unit point charge (rho = delta / (hx hy hz)) at node c: phi = G(i - c) exactly,
    with the supplied self value at c."""
    from oracle import free
    h = (0.2, 0.3, 0.25)
    rho = np.zeros((5, 4, 6))
    c = (2, 1, 4)
    rho[c] = 1.0 / (h[0] * h[1] * h[2])
    phi = free.solve_fft(rho, h, 7.0)
    i, j, k = np.meshgrid(np.arange(5) - c[0], np.arange(4) - c[1], np.arange(6) - c[2], indexing="ij")
    r = np.sqrt((i * h[0]) ** 2 + (j * h[1]) ** 2 + (k * h[2]) ** 2)
    ref = np.where(r > 0, 1.0 / np.where(r > 0, r, 1.0), 7.0)
    assert np.max(np.abs(phi - ref)) <= 1e-12 * np.max(ref)


def test_free_green_of_a_far_charge_is_coulomb():
    """Far from a compact charge the potential is Q / r to leading order (the
    dipole vanishes for a charge symmetric about its centre)."""
    from oracle import free
    h = (0.1, 0.1, 0.1)
    rho = np.zeros((3, 3, 40))
    rho[:, :, :3] = 1.0                       # a 3x3x3 block at the near end, centre (1, 1, 1)
    Q = rho.sum() * h[0] * h[1] * h[2]
    phi = free.solve_fft(rho, h, 0.0)
    r = (np.arange(40) - 1) * h[2]
    far = slice(30, 40)
    assert np.max(np.abs(phi[1, 1, far] * r[far] / Q - 1.0)) <= 2e-3


@pytest.mark.parametrize("dirs", ["fff", "bbb", "fbf", "bfb", "ffb", "bbf", "fbb", "bff"])
def test_mixed_fft_directions(dirs):
    """Each dimension's transform is the DFT matrix W^{jk} ('f') or W^{-jk} ('b'),
    W = e^{-2 pi i/N}, applied along that axis (Eq. A.4), unscaled."""
    from oracle import free
    rng = np.random.default_rng(3)
    shape = (4, 6, 8)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = a.copy()
    for axis, (n, d) in enumerate(zip(shape, dirs)):
        m = np.exp((-2j if d == "f" else 2j) * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
        ref = np.moveaxis(np.tensordot(m, np.moveaxis(ref, axis, 0), axes=(1, 0)), 0, axis)
    assert np.max(np.abs(free.mixed_fft(a, dirs) - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_eq6_correlation_in_y_by_mixed_directions():
    """Eq. 6: sum rho[i',j',k'] G[i-i', j+j', k-k'] = F^bfb{(F^fff rho)(F^fbf G)} / (Lx Ly Lz),
    with the y slots of G holding the sums j + j' (Appendix A.9)."""
    from oracle import free
    rng = np.random.default_rng(12)
    nx, ny, nz = 4, 3, 5
    rho = rng.standard_normal((nx, ny, nz))
    Gf = rng.standard_normal((2 * nx - 1, 2 * ny - 1, 2 * nz - 1))   # G[d_x + nx-1, s_y, d_z + nz-1]
    L = (2 * nx, 2 * ny, 2 * nz)
    direct_sum = np.zeros((nx, ny, nz))
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                for a in range(nx):
                    for b in range(ny):
                        for c in range(nz):
                            direct_sum[i, j, k] += rho[a, b, c] * Gf[i - a + nx - 1, j + b, k - c + nz - 1]
    garr = np.zeros(L)
    for p in range(-(nx - 1), nx):
        for s in range(2 * ny - 1):
            for q in range(-(nz - 1), nz):
                garr[p % L[0], s, q % L[2]] = Gf[p + nx - 1, s, q + nz - 1]
    pad = np.zeros(L)
    pad[:nx, :ny, :nz] = rho
    out = free.mixed_fft(free.mixed_fft(pad, 'fff') * free.mixed_fft(garr, 'fbf'), 'bfb') / np.prod(L)
    assert np.max(np.abs(out[:nx, :ny, :nz].real - direct_sum)) <= 1e-12 * np.max(np.abs(direct_sum))
