"""High-precision quadrature of the IGF defining integral, Eq. 13-14 (oracle; test infrastructure only).

Inside cell k the density is the linear interpolant of Eq. 13.  Collecting the
coefficient of one nodal value rho_k (it appears in cells k-1 and k) gives a
unit-height hat of half-width h_z centred on z_k, so the z-kernel that
multiplies h_z rho_k in the discrete sum is

    g_z(w) = (1/h_z) int_{-h_z}^{h_z} (1 - |s|/h_z) e^{-kappa |w - s|} ds,   w = z - z_k,

which Eq. 15 states in closed form.  Evaluated with mpmath at 40 digits,
splitting the interval where the integrand has kinks (s = -h, 0, h and s = w)
and into pieces no wider than about 2/kappa.
"""
import mpmath as mp


def gz_quad(kappa, w, hz, dps=40):
    with mp.workdps(dps):
        k = mp.mpf(kappa)
        h = mp.mpf(hz)
        w = mp.mpf(w)
        # the integrand varies on the scale 1/kappa: subdivide so that each
        # piece spans at most ~2/kappa, plus the kinks
        nsub = max(4, int(mp.ceil(k * h)))
        grid = {-h + 2 * h * t / nsub for t in range(nsub + 1)}
        pts = sorted(grid | {mp.mpf(0)} | ({w} if -h < w < h else set()))
        # scale by the integrand's largest exponential so that mpmath's
        # absolute error tolerance acts as a relative one
        d0 = max(mp.mpf(0), abs(w) - h)
        f = lambda s: (1 - abs(s) / h) * mp.exp(-k * (abs(w - s) - d0))
        val = mp.quad(f, pts)
        return val / h * mp.exp(-k * d0)


def gz_exact(kappa, w, hz, dps=40):
    """Eq. 15 evaluated in mpmath (no cancellation at 40 digits)."""
    with mp.workdps(dps):
        k = mp.mpf(kappa)
        h = mp.mpf(hz)
        w = mp.mpf(w)
        delta = 1 if w == 0 else 0
        num = (2 * h * k * delta + mp.e ** (-k * abs(w + h)) - 2 * mp.e ** (-k * abs(w))
               + mp.e ** (-k * abs(w - h)))
        return num / (h * k) ** 2
