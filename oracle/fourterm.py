"""O2: the paper's four-term FFT algorithm, Eq. 10, taken literally (oracle; test infrastructure only).

phi/(h_x h_y h_z) = F^bbb{(F^fff rho)(F^fff R_cc)} - F^bfb{(F^fff rho)(F^fbf R_cr)}
                  - F^fbb{(F^fff rho)(F^bff R_rc)} + F^ffb{(F^fff rho)(F^bbf R_rr)}

Conventions (Appendix, Eq. A.4 and A.9):
* forward transform  F^f: sum_n a_n W^{nk},  W = e^{-2 pi i / N}  (numpy ``fft``);
* backward transform F^b: sum_n a_n W^{-nk}, unscaled            (N * numpy ``ifft``);
* the 1/N of Eq. A.4 is carried by the final transform only, whatever its direction.

Green arrays (Appendix, Eq. A.3 and the correlation remark A.9), per dimension
with n physical nodes padded to length N >= 2n - 1:
* convolution slot m in [-(n-1), n-1] holds the Green value at distance
  X_i - X_i' = m h; the remaining slots are zero; the array is N-periodic;
* correlation slot m in [0, 2n-2] holds the value at X_i + X_i' = (m + 2) h
  (0-based nodes at (i+1) h); the remaining slots are zero.
z is always a convolution.  Unlike the single tabulated array of the paper's
discussion after Eq. 10, each term gets its own array: on a mesh whose nodes
sit at (i+1) h inside the walls, the convolution and correlation distances
are not one periodic sequence (see ``single_array_wall_grid`` for the grid on
which the single-array statement holds).
"""
import os

import numpy as np
import scipy.fft as sfft

from . import green

# FFT threads: the host's thread budget where one is set, else every core
_WORKERS = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1


def _F(a, axis, direction):
    """Unscaled 1-D transform along ``axis``: 'f' -> W^{+nk}, 'b' -> W^{-nk}."""
    if direction == 'f':
        return sfft.fft(a, axis=axis, workers=_WORKERS)
    return sfft.ifft(a, axis=axis, norm='forward', workers=_WORKERS)


def _F3(a, dirs):
    for axis, d in enumerate(dirs):
        a = _F(a, axis, d)
    return a


def conv_slots(n, N, h):
    """Distances held by the convolution slots of a length-N periodic array; NaN = zero slot."""
    d = np.full(N, np.nan)
    for m in range(-(n - 1), n):
        d[m % N] = m * h
    return d


def corr_slots(n, N, h, x0=0.0):
    """Distances held by the correlation slots, X_i + X_i' = 2 x0 + (m+2) h with
    m = i + i' (nodes at x0 + (i+1) h); NaN = zero slot."""
    d = np.full(N, np.nan)
    for m in range(0, 2 * n - 1):
        d[m] = 2.0 * x0 + (m + 2) * h
    return d


def green_array(shape, L, h, geom, kind, x_corr, y_corr, offset=(0.0, 0.0), band=None):
    """xi_ab[p, q, r] for one term of Eq. 10, zero in unused slots (and, with
    band = N, zero for z distances beyond N planes: Eq. 18)."""
    nx, ny, nz = shape
    Lx, Ly, Lz = L
    hx, hy, hz = h
    a, b, mx, my = geom
    ux = corr_slots(nx, Lx, hx, offset[0]) if x_corr else conv_slots(nx, Lx, hx)
    vy = corr_slots(ny, Ly, hy, offset[1]) if y_corr else conv_slots(ny, Ly, hy)
    rz = np.zeros(Lz, dtype=np.int64)
    okz = np.zeros(Lz, dtype=bool)
    for m in range(-(nz - 1), nz):
        if band is not None and abs(m) > band:
            continue
        rz[m % Lz] = m
        okz[m % Lz] = True
    okx, oky = ~np.isnan(ux), ~np.isnan(vy)
    tab = green.R_table(ux[okx], vy[oky], rz[okz], hz, a, b, mx, my, kind)
    xi = np.zeros((Lx, Ly, Lz))
    xi[np.ix_(okx, oky, okz)] = tab
    return xi


TERMS = (
    # (sign, x correlation?, y correlation?, Green directions, final directions)
    (+1.0, False, False, 'fff', 'bbb'),
    (-1.0, False, True, 'fbf', 'bfb'),
    (-1.0, True, False, 'bff', 'fbb'),
    (+1.0, True, True, 'bbf', 'ffb'),
)


def green_spectra(shape, L, h, geom, kind, offset=(0.0, 0.0), band=None):
    """The four mixed-direction transforms of the Green arrays (the stored, reused spectra)."""
    out = []
    for sign, xc, yc, gdir, fdir in TERMS:
        xi = green_array(shape, L, h, geom, kind, xc, yc, offset, band)
        out.append(_F3(xi.astype(np.complex128), gdir))
    return out


def solve(rho, hx, hy, hz, a, b, mx, my, kind, L=None, spectra=None, return_imag=False, x0=0.0, y0=0.0,
          band=None):
    """Eq. 10: phi on the physical nodes for rho of shape (nx, ny, nz), FP64.

    L = (Lx, Ly, Lz) defaults to (2nx, 2ny, 2nz); any L >= 2n - 1 per axis is
    valid (Appendix, Eq. A.3 and the remark on N >= M).  (x0, y0) offsets the
    mesh inside the pipe (node i at x0 + (i+1) hx); only the correlation
    slots see it.  band = N keeps only z distances |k - k'| <= N (Eq. 18).
    """
    rho = np.asarray(rho, dtype=np.float64)
    nx, ny, nz = rho.shape
    if L is None:
        L = (2 * nx, 2 * ny, 2 * nz)
    Lx, Ly, Lz = L
    if Lx < 2 * nx - 1 or Ly < 2 * ny - 1 or Lz < 2 * nz - 1:
        raise ValueError("padded length must be at least 2n-1 in every dimension")
    if spectra is None:
        spectra = green_spectra(rho.shape, L, (hx, hy, hz), (a, b, mx, my), kind, (x0, y0), band)
    pad = np.zeros((Lx, Ly, Lz), dtype=np.complex128)
    pad[:nx, :ny, :nz] = rho
    rho_hat = _F3(pad, 'fff')
    del pad
    acc = np.zeros((nx, ny, nz), dtype=np.complex128)
    for (sign, xc, yc, gdir, fdir), spec in zip(TERMS, spectra):
        t = _F3(rho_hat * spec, fdir) / (Lx * Ly * Lz)
        acc += sign * t[:nx, :ny, :nz]
        del t
    phi = hx * hy * hz * acc
    if return_imag:
        return phi.real, np.max(np.abs(phi.imag))
    return phi.real


def single_array_wall_grid(rho, h, a_cells, b_cells, hz, mx, my, kind):
    """The paper's statement after Eq. 10 that one tabulated R serves all four terms.

    Grid with nodes ON the walls: x_i = i h for i = 0..Nx (Nx h = a), y likewise,
    padded length 2Nx in x and 2Ny in y, 2nz in z.  One array
    R(p h_x, q h_y, c(r) h_z), p in [0, 2Nx), q in [0, 2Ny), is transformed the
    four ways of Eq. 10; the 2a-periodicity and evenness of R make its slots
    hold both the difference and the sum distances.  rho has shape
    (Nx+1, Ny+1, nz) with zero on the wall nodes.
    """
    rho = np.asarray(rho, dtype=np.float64)
    Nx1, Ny1, nz = rho.shape
    Nx, Ny = Nx1 - 1, Ny1 - 1
    a, b = a_cells * h, b_cells * h
    assert Nx == a_cells and Ny == b_cells
    Lx, Ly, Lz = 2 * Nx, 2 * Ny, 2 * nz
    u = np.arange(Lx) * h
    v = np.arange(Ly) * h
    r = np.array([m if m <= Lz // 2 else m - Lz for m in range(Lz)])
    R = green.R_table(u, v, r, hz, a, b, mx, my, kind).astype(np.complex128)
    pad = np.zeros((Lx, Ly, Lz), dtype=np.complex128)
    pad[:Nx1 - 1, :Ny1 - 1, :nz] = rho[:Nx, :Ny]   # the node at x = a carries no charge
    rho_hat = _F3(pad, 'fff')
    acc = np.zeros((Lx, Ly, Lz), dtype=np.complex128)
    for sign, xc, yc, gdir, fdir in TERMS:
        acc += sign * _F3(rho_hat * _F3(R, gdir), fdir)
    acc /= (Lx * Ly * Lz)
    return (h * h * hz * acc[:Nx1, :Ny1, :nz]).real
