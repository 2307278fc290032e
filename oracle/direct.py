"""O1: the discretised Green integral, summed directly (oracle; test infrastructure only).

phi[i,j,k] = h_x h_y h_z sum_{i',j',k'} rho[i',j',k'] G(X_i, X_i', Y_j, Y_j', (k-k') h_z)

This is the Eq. 4 discretisation of Eq. 1 with the pipe Green function of
Eq. 8 (R from Eq. 9, or R_int from Eq. 16 for the z-integrated kind).  It is
the plain definition of the result the FFT algorithm (Eq. 10) reproduces in
the physical region (Appendix, Eq. A.8 and the remark after it).
"""
import numpy as np

from . import green


def _unique_table(vals):
    uniq, inv = np.unique(vals, return_inverse=True)
    return uniq, inv.reshape(vals.shape)


def green_tensor(nx, ny, nz, hx, hy, hz, a, b, mx, my, kind, x0=0.0, y0=0.0):
    """G[i, i', j, j', d] for d = (k - k') + (nz - 1), from the node coordinates.

    Each distinct transverse distance is evaluated once by ``green.R_table``.
    """
    X, Y = green.node_coords(nx, ny, hx, hy, x0, y0)
    um = np.subtract.outer(X, X)
    up = np.add.outer(X, X)
    vm = np.subtract.outer(Y, Y)
    vp = np.add.outer(Y, Y)
    u_vals, u_inv = _unique_table(np.stack([um, up]))
    v_vals, v_inv = _unique_table(np.stack([vm, vp]))
    r = np.arange(-(nz - 1), nz)
    tab = green.R_table(u_vals, v_vals, r, hz, a, b, mx, my, kind)   # (U, V, 2nz-1)
    # tab[u_inv[s], :, :][:, v_inv[t]] for the four sign combinations of Eq. 8.
    def term(su, sv):
        t = tab[u_inv[su]]                   # (nx, nx, V, R)
        t = t[:, :, v_inv[sv]]               # (nx, nx, ny, ny, R)
        return t
    return term(0, 0) - term(0, 1) - term(1, 0) + term(1, 1)


def solve(rho, hx, hy, hz, a, b, mx, my, kind, x0=0.0, y0=0.0, band=None):
    """Direct O(n^2) sum of the definition above.  rho has shape (nx, ny, nz), FP64;
    the mesh may be offset by (x0, y0) inside the pipe (node i at x0 + (i+1) hx).

    band = N restricts the z sum to |k - k'| <= N (Eq. 17 for N = 0, Eq. 18 in
    general: the neighbouring-plane approximation when the z-kernel is
    negligible beyond N planes); None keeps every plane."""
    rho = np.asarray(rho, dtype=np.float64)
    nx, ny, nz = rho.shape
    G = green_tensor(nx, ny, nz, hx, hy, hz, a, b, mx, my, kind, x0, y0)
    if band is not None:
        d = np.arange(-(nz - 1), nz)
        G[..., np.abs(d) > band] = 0.0
    phi = np.empty_like(rho)
    kp = np.arange(nz)
    for k in range(nz):
        Gk = G[..., k - kp + (nz - 1)]                     # (nx, nx, ny, ny, nz) over k'
        phi[:, :, k] = np.einsum('iajbc,abc->ij', Gk, rho)
    return hx * hy * hz * phi


def solve_at(rho, points, hx, hy, hz, a, b, mx, my, kind, x0=0.0, y0=0.0):
    """The same direct sum, evaluated only at the listed output nodes (i, j, k).

    For full-size meshes: the mode factor g(kappa_mn, w)/kappa_mn is computed
    once for every z distance, then for each listed node R is summed over the
    modes at the distances X_i -/+ X_i', Y_j -/+ Y_j' that node needs, and the
    node's potential is a plain weighted sum over all source cells.
    """
    rho = np.asarray(rho, dtype=np.float64)
    nx, ny, nz = rho.shape
    X, Y = green.node_coords(nx, ny, hx, hy, x0, y0)
    r = np.arange(-(nz - 1), nz)
    d = green.mode_coefficients(r, hz, a, b, mx, my, kind)     # (mx, my, 2nz-1)
    kp = np.arange(nz)
    out = []
    for (i, j, k) in points:
        u = np.concatenate([X[i] - X, X[i] + X])
        v = np.concatenate([Y[j] - Y, Y[j] + Y])
        dk = d[:, :, k - kp + (nz - 1)]                         # (mx, my, nz) over k'
        tab = green.R_from_coefficients(u, v, dk, a, b)          # (2nx, 2ny, nz)
        g = tab[:nx, :ny] - tab[:nx, ny:] - tab[nx:, :ny] + tab[nx:, ny:]
        out.append(hx * hy * hz * float(np.sum(g * rho)))
    return np.array(out)


def solve_python_loops(rho, hx, hy, hz, a, b, mx, my):
    """Point Green function only: every sum as a plain Python loop (tiny cases).

    Uses ``green.R_point`` (math.fsum over modes) for each of the four terms of
    Eq. 8 and each source/observer pair.
    """
    rho = np.asarray(rho, dtype=np.float64)
    nx, ny, nz = rho.shape
    X = [(i + 1) * hx for i in range(nx)]
    Y = [(j + 1) * hy for j in range(ny)]
    phi = np.zeros_like(rho)
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                acc = 0.0
                for ip in range(nx):
                    for jp in range(ny):
                        for kp in range(nz):
                            w = (k - kp) * hz
                            g = (green.R_point(X[i] - X[ip], Y[j] - Y[jp], w, a, b, mx, my)
                                 - green.R_point(X[i] - X[ip], Y[j] + Y[jp], w, a, b, mx, my)
                                 - green.R_point(X[i] + X[ip], Y[j] - Y[jp], w, a, b, mx, my)
                                 + green.R_point(X[i] + X[ip], Y[j] + Y[jp], w, a, b, mx, my))
                            acc += rho[ip, jp, kp] * g
                phi[i, j, k] = hx * hy * hz * acc
    return phi
