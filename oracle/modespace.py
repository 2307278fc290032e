"""O3: an independent solve in the sine eigenbasis of the pipe (oracle; test infrastructure only).

Eq. 7 writes the pipe Green function as a double series over products of
sines.  On a mesh that spans the full aperture, (n_x + 1) h_x = a and
(n_y + 1) h_y = b, node i sits at X_i = (i+1) a/(n_x+1), so

    sin(m pi X_i / a) = +/- s_mu(i),   s_mu(i) = sin(pi mu (i+1) / (n_x + 1)),

where mu in [1, n_x] is m folded modulo 2(n_x+1) (m = +/-mu), and modes with
m = 0 or n_x + 1 (mod 2(n_x+1)) vanish on every node.  The sign appears twice
and cancels.  The discrete operator is therefore diagonal in the DST-I basis:

    phi = h_x h_y h_z S_x^T [ K_{mu nu} *_z (S_x rho S_y^T) ] S_y,
    K_{mu nu}(w) = 4/(2 pi a b) sum_{m -> mu, n -> nu} g(kappa_mn, w) / kappa_mn,

with *_z a linear (open) convolution along z.  The factor 4 and prefactor
1/(2 pi a b) give the normalisation of Eq. 8 with R from Eq. 9 (Eq. 7 as
printed is one quarter of it).  This shares nothing with the FFT
convolution/correlation algorithm of Eq. 10 and agrees with it to rounding.
"""
import numpy as np
import scipy.signal as ssig

from . import green


def _fold(M, n):
    """Map modes m = 1..M to DST index mu-1 in [0, n) or -1 (vanishing on the nodes)."""
    N1 = n + 1
    out = np.full(M, -1, dtype=np.int64)
    for m in range(1, M + 1):
        q = m % (2 * N1)
        if q == 0 or q == N1:
            continue
        mu = q if q < N1 else 2 * N1 - q
        out[m - 1] = mu - 1
    return out


def dst_matrix(n):
    """S[mu-1, i] = sin(pi mu (i+1) / (n+1)), mu = 1..n, i = 0..n-1."""
    mu = np.arange(1, n + 1, dtype=np.float64)
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.sin(np.pi * np.outer(mu, i) / (n + 1))


def mode_kernel(nx, ny, nz, hz, a, b, mx, my, kind):
    """K[mu, nu, d] for d = r + (nz-1), r = -(nz-1)..(nz-1)."""
    kap = green.kappa(a, b, mx, my)
    r = np.arange(0, nz)
    d = green.gz(kind, kap, r, hz) / kap[..., None]          # (mx, my, nz)
    fx, fy = _fold(mx, nx), _fold(my, ny)
    Px = np.zeros((nx, mx))
    Py = np.zeros((ny, my))
    Px[fx[fx >= 0], np.nonzero(fx >= 0)[0]] = 1.0
    Py[fy[fy >= 0], np.nonzero(fy >= 0)[0]] = 1.0
    K = np.einsum('am,mnr,bn->abr', Px, d, Py, optimize=True) * (4.0 / (2.0 * np.pi * a * b))
    return np.concatenate([K[:, :, :0:-1], K], axis=2)       # mirror to r < 0 (K even in w)


def full_aperture(nx, ny, hx, hy, a, b, rtol=1e-12):
    return abs((nx + 1) * hx - a) <= rtol * a and abs((ny + 1) * hy - b) <= rtol * b


def solve(rho, hx, hy, hz, a, b, mx, my, kind, z_method=None):
    """phi for rho of shape (nx, ny, nz) on a full-aperture mesh, FP64."""
    rho = np.asarray(rho, dtype=np.float64)
    nx, ny, nz = rho.shape
    if not full_aperture(nx, ny, hx, hy, a, b):
        raise ValueError("the mode-space oracle needs (nx+1) hx = a and (ny+1) hy = b")
    Sx, Sy = dst_matrix(nx), dst_matrix(ny)
    K = mode_kernel(nx, ny, nz, hz, a, b, mx, my, kind)      # (nx, ny, 2nz-1)
    rt = np.einsum('ai,ijk->ajk', Sx, rho, optimize=True)
    rt = np.einsum('bj,ajk->abk', Sy, rt, optimize=True)      # (nx, ny, nz)
    if z_method is None:
        z_method = 'direct' if nz <= 64 else 'fft'
    if z_method == 'direct':
        psi = np.zeros_like(rt)
        kp = np.arange(nz)
        for k in range(nz):
            psi[:, :, k] = np.sum(K[:, :, k - kp + nz - 1] * rt, axis=2)
    else:
        full = ssig.fftconvolve(K, rt, mode='full', axes=2)
        psi = full[:, :, nz - 1:2 * nz - 1]
    phi = np.einsum('ai,abk->ibk', Sx, psi, optimize=True)
    phi = np.einsum('bj,ibk->ijk', Sy, phi, optimize=True)
    return hx * hy * hz * phi


def single_mode_response(f, hz, a, b, kind, mx, my):
    """Closed form for rho = sin(pi X/a) sin(pi Y/b) f(z) on a full-aperture mesh.

    The (1,1) sine mode is an eigenvector of the transverse operator.  Only
    m = 1 contributes (its aliases 2(n_x+1) -/+ 1, ... are absent when
    mx <= 2 n_x, and likewise in y), with
    sum_i sin^2(pi (i+1)/(n+1)) = (n+1)/2:
        phi = sin sin * h_x h_y h_z (n_x+1)(n_y+1)/4 * 4/(2 pi a b)
              * sum_{k'} g(kappa_11,(k-k') h_z)/kappa_11 f_{k'}
            = sin sin * h_z / (2 pi kappa_11) * sum_{k'} g f_{k'}
    (using h_x (n_x+1) = a, h_y (n_y+1) = b).  Returns the z profile.
    """
    f = np.asarray(f, dtype=np.float64)
    nz = f.size
    k11 = np.pi * np.sqrt(1.0 / a ** 2 + 1.0 / b ** 2)
    r = np.arange(-(nz - 1), nz)
    g = green.gz(kind, np.array([k11]), r, hz)[0]
    prof = np.array([np.sum(g[k - np.arange(nz) + nz - 1] * f) for k in range(nz)])
    return hz / (2.0 * np.pi * k11) * prof
