"""Free-space (isolated) Poisson solve by Hockney's zero-padded FFT convolution (oracle; test infrastructure only).

Sec. 1, Eq. 3-5: with the 4 pi (and epsilon_0) dropped, the isolated Green
function is G(u, v, w) = 1 / sqrt(u^2 + v^2 + w^2) and the discretised
potential (Eq. 4 with G depending on differences only) is

    phi[i,j,k] = hx hy hz sum_{i',j',k'} rho[i',j',k'] G((i-i') hx, (j-j') hy, (k-k') hz).

G is singular at zero separation and the paper does not say what the grid
value there is; the caller supplies it (``g0``).  Eq. 5 computes the same
sum as hx hy hz F^bbb{ (F^fff rho) (F^fff G) } with both arrays zero-padded
(Appendix, Eq. A.3: convolution slot m of a length-L array holds distance
m for |m| <= n - 1, the other slots zero; any L >= 2n - 1 will do) and the
1/(Lx Ly Lz) of the final transform (Eq. A.4).
"""
import numpy as np
import scipy.fft as sfft

from .fourterm import _F3


def green_value(p, q, r, h, g0):
    """G at the grid distance (p hx, q hy, r hz); g0 where all three vanish."""
    hx, hy, hz = h
    p, q, r = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (p, q, r)))
    d2 = (p * hx) ** 2 + (q * hy) ** 2 + (r * hz) ** 2
    out = np.full(d2.shape, float(g0))
    nz = d2 > 0
    out[nz] = 1.0 / np.sqrt(d2[nz])
    return out


def solve_direct(rho, h, g0):
    """The sum of the module docstring, over all pairs (O(n^2) memory per plane pair)."""
    rho = np.asarray(rho, dtype=np.float64)
    nx, ny, nz = rho.shape
    di = np.subtract.outer(np.arange(nx), np.arange(nx))
    dj = np.subtract.outer(np.arange(ny), np.arange(ny))
    phi = np.zeros_like(rho)
    for k in range(nz):
        for kp in range(nz):
            G = green_value(di[:, None, :, None], dj[None, :, None, :], k - kp, h, g0)   # (i, j, i', j')
            phi[:, :, k] += np.einsum('ijab,ab->ij', G, rho[:, :, kp])
    return h[0] * h[1] * h[2] * phi


def solve_python_loops(rho, h, g0):
    """The same sum in plain Python loops (tiny meshes only)."""
    nx, ny, nz = rho.shape
    hx, hy, hz = h
    phi = np.zeros((nx, ny, nz))
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                s = 0.0
                for a in range(nx):
                    for b in range(ny):
                        for c in range(nz):
                            if (i, j, k) == (a, b, c):
                                g = g0
                            else:
                                g = 1.0 / ((((i - a) * hx) ** 2 + ((j - b) * hy) ** 2 + ((k - c) * hz) ** 2) ** 0.5)
                            s += rho[a, b, c] * g
                phi[i, j, k] = hx * hy * hz * s
    return phi


def green_array(shape, L, h, g0):
    """The zero-padded Green array of Eq. 5: slot (m, n, l) holds G at distance
    (m hx, n hy, l hz) for |m| <= nx - 1 etc. (indices modulo L), zero elsewhere."""
    out = np.zeros(L)
    idx = []
    for n, Ld in zip(shape, L):
        m = np.arange(-(n - 1), n)
        idx.append((m % Ld, m))
    (px, mx), (py, my), (pz, mz) = idx
    out[np.ix_(px, py, pz)] = green_value(mx[:, None, None], my[None, :, None], mz[None, None, :], h, g0)
    return out


def solve_fft(rho, h, g0, L=None):
    """Eq. 5: hx hy hz F^bbb{(F^fff rho)(F^fff G)} / (Lx Ly Lz) on the physical nodes."""
    rho = np.asarray(rho, dtype=np.float64)
    shape = rho.shape
    if L is None:
        L = tuple(2 * n for n in shape)
    if any(Ld < 2 * n - 1 for Ld, n in zip(L, shape)):
        raise ValueError("padded length must be at least 2n-1 in every dimension")
    pad = np.zeros(L, dtype=np.complex128)
    pad[:shape[0], :shape[1], :shape[2]] = rho
    spec = _F3(pad, 'fff') * _F3(green_array(shape, L, h, g0).astype(np.complex128), 'fff')
    out = _F3(spec, 'bbb') / (L[0] * L[1] * L[2])
    return h[0] * h[1] * h[2] * out[:shape[0], :shape[1], :shape[2]].real


def mixed_fft(a, dirs):
    """Unscaled 3-D DFT with a direction per dimension: 'f' sums a_n W^{nk},
    'b' sums a_n W^{-nk}, W = e^{-2 pi i / N} (Eq. A.4's conventions)."""
    a = np.asarray(a, dtype=np.complex128)
    for axis, d in enumerate(dirs):
        a = sfft.fft(a, axis=axis) if d == 'f' else sfft.ifft(a, axis=axis, norm='forward')
    return a
