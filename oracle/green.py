"""Green functions of the open rectangular pipe (oracle; test infrastructure only).

Plain FP64 numpy.  Sections and equations refer to Ryne, "On FFT-based
convolutions and correlations, with application to solving Poisson's equation
in an open rectangular pipe" (arXiv:1111.4971).
"""
import math

import numpy as np

POINT = 0   # ordinary (point-sampled) Green function, Eq. 9
IGF_Z = 1   # Green function integrated in z against hat functions, Eq. 16


def kappa(a, b, mx, my):
    """kappa_mn = pi * sqrt((m/a)^2 + (n/b)^2), m = 1..mx, n = 1..my (Sec. 2, after Eq. 7).

    Returns an (mx, my) array.
    """
    m = np.arange(1, mx + 1, dtype=np.float64)
    n = np.arange(1, my + 1, dtype=np.float64)
    return np.pi * np.sqrt((m[:, None] / a) ** 2 + (n[None, :] / b) ** 2)


def gz_point(kap, r, hz):
    """z-factor of the ordinary Green function: exp(-kappa |w|), w = r*hz (Eq. 7, 9)."""
    w = np.abs(np.asarray(r, dtype=np.float64)) * hz
    return np.exp(-np.multiply.outer(kap, w))


def gz_igf_eq15(kap, r, hz):
    """Eq. 15 exactly as printed, w = r*hz with integer r.

    g_z(w) = [2 hz kappa delta_{w,0} + e^{-kappa|w+hz|} - 2 e^{-kappa|w|}
              + e^{-kappa|w-hz|}] / (hz kappa)^2.

    Loses about log10(1/(kappa hz)^2) digits to cancellation; kept to pin the
    rewritten form ``gz_igf`` where both are accurate.
    """
    r = np.asarray(r)
    w = r.astype(np.float64) * hz
    k = np.asarray(kap, dtype=np.float64)[..., None]
    delta = (r == 0).astype(np.float64)
    num = (2.0 * hz * k * delta + np.exp(-k * np.abs(w + hz))
           - 2.0 * np.exp(-k * np.abs(w)) + np.exp(-k * np.abs(w - hz)))
    return num / (hz * k) ** 2


def _g0_series(x):
    """2 (x - 1 + e^{-x}) / x^2 by its Taylor series 2 sum_{j>=0} (-x)^j / (j+2)!  (x < 0.5)."""
    out = np.zeros_like(x)
    term = np.full_like(x, 1.0)          # (-x)^j
    fact = 2.0                           # (j+2)!
    for j in range(30):
        out += term / fact
        term = term * (-x)
        fact *= (j + 3)
    return 2.0 * out


def gz_igf(kap, r, hz):
    """Eq. 15 rewritten without cancellation (same function, exact algebra).

    With x = kappa*hz and integer r (w = r*hz):
      r = 0:   g = 2 (x - 1 + e^{-x}) / x^2
               (series below x = 0.5, else x + expm1(-x) directly);
      |r| >= 1: the bracket equals e^{-kappa|w|} (e^{x} - 2 + e^{-x})
               = e^{-kappa|w|} (2 sinh(x/2))^2, so
               g = e^{-kappa|w|} (2 sinh(x/2) / x)^2.
    For x > 600 the sinh form would overflow and the equivalent
    e^{-x(|r|-1)} ((1 - e^{-x})/x)^2 is used.
    Returns an array of shape kap.shape + r.shape.
    """
    r = np.abs(np.asarray(r))
    k = np.asarray(kap, dtype=np.float64)
    x = (k * hz)[..., None] * np.ones(r.shape)
    rr = np.broadcast_to(r, x.shape).astype(np.float64)
    out = np.empty_like(x)
    zero = rr == 0
    small = zero & (x < 0.5)
    big0 = zero & ~small
    out[small] = _g0_series(x[small])
    xb = x[big0]
    out[big0] = 2.0 * (xb + np.expm1(-xb)) / xb ** 2
    far = ~zero
    xf, rf = x[far], rr[far]
    mid = xf <= 600.0
    res = np.empty_like(xf)
    res[mid] = np.exp(-xf[mid] * rf[mid]) * (2.0 * np.sinh(0.5 * xf[mid]) / xf[mid]) ** 2
    xh = xf[~mid]
    res[~mid] = np.exp(-xh * (rf[~mid] - 1.0)) * ((-np.expm1(-xh)) / xh) ** 2
    out[far] = res
    return out


def gz(kind, kap, r, hz):
    """z-factor of R (POINT, Eq. 9) or R_int (IGF_Z, Eq. 16) for integer distances r."""
    if kind == POINT:
        return gz_point(kap, r, hz)
    if kind == IGF_Z:
        return gz_igf(kap, r, hz)
    raise ValueError("unknown Green kind %r" % (kind,))


def mode_coefficients(r, hz, a, b, mx, my, kind):
    """D[m, n, t] = g(kappa_mn, r_t hz) / (2 pi a b kappa_mn): the (u, v)-independent factor of Eq. 9/16."""
    kap = kappa(a, b, mx, my)
    return gz(kind, kap, np.atleast_1d(np.asarray(r)), hz) / kap[..., None] / (2.0 * np.pi * a * b)


def R_from_coefficients(u, v, d, a, b):
    """sum_{m,n} cos(m pi u/a) cos(n pi v/b) D[m, n, t] for the tensor grid u x v x t."""
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    v = np.atleast_1d(np.asarray(v, dtype=np.float64))
    mx, my, nr = d.shape
    m = np.arange(1, mx + 1, dtype=np.float64)
    n = np.arange(1, my + 1, dtype=np.float64)
    cx = np.cos(np.pi * np.multiply.outer(u, m) / a)
    cy = np.cos(np.pi * np.multiply.outer(v, n) / b)
    out = np.empty((u.size, v.size, nr))
    for t in range(nr):
        out[:, :, t] = cx @ d[:, :, t] @ cy.T
    return out


def R_table(u, v, r, hz, a, b, mx, my, kind):
    """R(u, v, r*hz) (Eq. 9) or R_int (Eq. 16) on the tensor grid u x v x r.

    R(u,v,w) = 1/(2 pi a b) sum_{m<=mx, n<=my} kappa_mn^{-1}
               cos(m pi u / a) cos(n pi v / b) g(kappa_mn, w).

    The double sum over modes is done as two matrix products per r
    (a library primitive; no reordering of the definition beyond summing m
    and n in turn).  Returns shape (len(u), len(v), len(r)).
    """
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    v = np.atleast_1d(np.asarray(v, dtype=np.float64))
    r = np.atleast_1d(np.asarray(r))
    kap = kappa(a, b, mx, my)
    m = np.arange(1, mx + 1, dtype=np.float64)
    n = np.arange(1, my + 1, dtype=np.float64)
    cx = np.cos(np.pi * np.multiply.outer(u, m) / a)          # (U, mx)
    cy = np.cos(np.pi * np.multiply.outer(v, n) / b)          # (V, my)
    d = gz(kind, kap, r, hz) / kap[..., None] / (2.0 * np.pi * a * b)   # (mx, my, Rr)
    out = np.empty((u.size, v.size, r.size))
    for t in range(r.size):
        out[:, :, t] = cx @ d[:, :, t] @ cy.T
    return out


def R_point(u, v, w, a, b, mx, my):
    """Eq. 9 at one point, by plain loops over the modes with math.fsum (tiny mx, my only)."""
    terms = []
    for m in range(1, mx + 1):
        for n in range(1, my + 1):
            k = math.pi * math.sqrt((m / a) ** 2 + (n / b) ** 2)
            terms.append(math.cos(m * math.pi * u / a) * math.cos(n * math.pi * v / b)
                         * math.exp(-k * abs(w)) / k)
    return math.fsum(terms) / (2.0 * math.pi * a * b)


def G_four_term(x, xp, y, yp, r, hz, a, b, mx, my, kind):
    """Pipe Green function as the four R terms of Eq. 8 (arguments are 1-D arrays).

    G = R(x-x', y-y') - R(x-x', y+y') - R(x+x', y-y') + R(x+x', y+y'), all at w = r*hz.
    Returns shape (len(x), len(xp), len(y), len(yp), len(r)).
    """
    x, xp, y, yp = (np.atleast_1d(np.asarray(t, dtype=np.float64)) for t in (x, xp, y, yp))
    um = np.subtract.outer(x, xp).ravel()
    up = np.add.outer(x, xp).ravel()
    vm = np.subtract.outer(y, yp).ravel()
    vp = np.add.outer(y, yp).ravel()
    u_all = np.concatenate([um, up])
    v_all = np.concatenate([vm, vp])
    tab = R_table(u_all, v_all, r, hz, a, b, mx, my, kind)
    nu, nv = um.size, vm.size
    g = (tab[:nu, :nv] - tab[:nu, nv:] - tab[nu:, :nv] + tab[nu:, nv:])
    return g.reshape(x.size, xp.size, y.size, yp.size, -1)


def G_sine_series(x, xp, y, yp, r, hz, a, b, mx, my, kind):
    """Eq. 7 as printed (prefactor 1/(2 pi a b)), with g(kappa, w) in place of e^{-kappa|w|}.

    sum_{m,n} kappa^{-1} sin(m pi x/a) sin(m pi x'/a) sin(n pi y/b) sin(n pi y'/b) g / (2 pi a b).
    By sin A sin B = (cos(A-B) - cos(A+B))/2 in x and in y this is exactly one
    quarter of ``G_four_term``: the printed prefactors of Eq. 7 and Eq. 9 are
    mutually inconsistent by that factor.
    """
    x, xp, y, yp = (np.atleast_1d(np.asarray(t, dtype=np.float64)) for t in (x, xp, y, yp))
    kap = kappa(a, b, mx, my)
    m = np.arange(1, mx + 1, dtype=np.float64)
    n = np.arange(1, my + 1, dtype=np.float64)
    sx = np.sin(np.pi * np.multiply.outer(x, m) / a)
    sxp = np.sin(np.pi * np.multiply.outer(xp, m) / a)
    sy = np.sin(np.pi * np.multiply.outer(y, n) / b)
    syp = np.sin(np.pi * np.multiply.outer(yp, n) / b)
    d = gz(kind, kap, r, hz) / kap[..., None] / (2.0 * np.pi * a * b)
    return np.einsum('im,jm,kn,ln,mnr->ijklr', sx, sxp, sy, syp, d)


def node_coords(nx, ny, hx, hy, x0=0.0, y0=0.0):
    """Transverse node positions X_i = x0 + (i+1) h_x, Y_j = y0 + (j+1) h_y (0-based i, j).

    x0 = y0 = 0 is the mesh anchored one cell inside the walls x = 0, y = 0;
    a positive offset places the mesh on a sub-region of the cross-section
    (Sec. 5: only the region around the beam needs to be meshed)."""
    return (x0 + np.arange(1, nx + 1, dtype=np.float64) * hx,
            y0 + np.arange(1, ny + 1, dtype=np.float64) * hy)
