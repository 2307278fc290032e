"""Seeded synthetic charge densities for the open-pipe Poisson solve.

These generators hold none of the solver's arithmetic: they only lay out
meshes and draw charge distributions.  Both the GPU path and the CPU oracle
consume what they return.  The bunch shapes follow the paper's numerical
example (Sec. 4: Gaussian bunches inside a rectangular pipe, modes m, n
truncated); sizes and seeds are fixed per workload so that every run sees the
same values.

Conventions: rho has shape (nx, ny, nz), C-order with z fastest, FP64.
Node i sits at X_i = (i+1) h_x, node j at Y_j = (j+1) h_y; in z the grid is
centred, Z_k = (k - (nz-1)/2) h_z.  "Unit charge" means h_x h_y h_z sum(rho) = 1.
"""
import dataclasses
import math
import os

import numpy as np

POINT, IGF_Z = 0, 1


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    hx: float
    hy: float
    hz: float
    a: float
    b: float
    kind: int
    mx: int
    my: int
    rho: np.ndarray = dataclasses.field(repr=False, default=None)
    notes: dict = dataclasses.field(default_factory=dict)

    @property
    def shape(self):
        return (self.nx, self.ny, self.nz)

    def geometry(self):
        return dict(hx=self.hx, hy=self.hy, hz=self.hz, a=self.a, b=self.b,
                    mx=self.mx, my=self.my, kind=self.kind)


def coords(nx, ny, nz, hx, hy, hz):
    X = np.arange(1, nx + 1, dtype=np.float64) * hx
    Y = np.arange(1, ny + 1, dtype=np.float64) * hy
    Z = (np.arange(nz, dtype=np.float64) - 0.5 * (nz - 1)) * hz
    return X, Y, Z


def _unit_charge(rho, hx, hy, hz):
    return rho / (hx * hy * hz * rho.sum())


def _add_noise(rho, rng, level=1e-3):
    return rho + level * rho.max() * rng.random(rho.shape)


def gaussian(nx, ny, nz, hx, hy, hz, centre, sigma):
    X, Y, Z = coords(nx, ny, nz, hx, hy, hz)
    gx = np.exp(-0.5 * ((X - centre[0]) / sigma[0]) ** 2)
    gy = np.exp(-0.5 * ((Y - centre[1]) / sigma[1]) ** 2)
    gz = np.exp(-0.5 * ((Z - centre[2]) / sigma[2]) ** 2)
    return gx[:, None, None] * gy[None, :, None] * gz[None, None, :]


def random_field(shape, seed):
    """Plain standard-normal field, for parity tests on arbitrary shapes."""
    return np.random.default_rng(seed).standard_normal(shape)


def plain_fp64_32cubed(seed=1):
    """32^3 mesh in a 1 x 1 pipe, point Green function, 64 x 64 modes.

    Gaussian at (0.5, 0.5, 0), sigma (0.15, 0.15, 0.4), unit charge plus
    1e-3 uniform noise.
    """
    n, h, hz = 32, 1.0 / 33, 0.05
    rng = np.random.default_rng(seed)
    rho = _unit_charge(gaussian(n, n, n, h, h, hz, (0.5, 0.5, 0.0), (0.15, 0.15, 0.4)), h, h, hz)
    return Workload("plain_fp64_32cubed", n, n, n, h, h, hz, 1.0, 1.0, POINT, 64, 64,
                    _add_noise(rho, rng))


def plain_fp64_8cubed(seed=11):
    """8^3 sub-case of the 32^3 workload (h = 1/9), small enough for the direct sum."""
    n, h, hz = 8, 1.0 / 9, 0.05
    rng = np.random.default_rng(seed)
    rho = _unit_charge(gaussian(n, n, n, h, h, hz, (0.5, 0.5, 0.0), (0.15, 0.15, 0.4)), h, h, hz)
    return Workload("plain_fp64_8cubed", n, n, n, h, h, hz, 1.0, 1.0, POINT, 64, 64,
                    _add_noise(rho, rng))


def igf_long_bunch(seed=2):
    """64 x 64 x 256 in a 2 x 1 pipe, IGF, 128 x 128 modes.

    Uniform elliptical cross-section ((x-1.3)/0.4)^2 + ((y-0.4)/0.25)^2 <= 1,
    Gaussian in z with sigma_z = 3 over +-4 sigma_z, unit charge + 1e-3 noise.
    """
    nx, ny, nz = 64, 64, 256
    a, b = 2.0, 1.0
    hx, hy, hz = a / (nx + 1), b / (ny + 1), 24.0 / (nz - 1)
    X, Y, Z = coords(nx, ny, nz, hx, hy, hz)
    ell = (((X[:, None] - 1.3) / 0.4) ** 2 + ((Y[None, :] - 0.4) / 0.25) ** 2 <= 1.0).astype(float)
    rho = ell[:, :, None] * np.exp(-0.5 * (Z / 3.0) ** 2)[None, None, :]
    rng = np.random.default_rng(seed)
    rho = _add_noise(_unit_charge(rho, hx, hy, hz), rng)
    return Workload("igf_long_bunch", nx, ny, nz, hx, hy, hz, a, b, IGF_Z, 128, 128, rho)


def _cic_weights(px, py, pz, nx, ny, nz, hx, hy, hz):
    """Cloud-in-cell (trilinear) node indices and weights of unit-weight particles.

    Particles outside the node box are dropped.  Returns (index, weight) arrays
    holding the 8 corner contributions of every kept particle.
    """
    X0, Y0 = hx, hy
    Z0 = -0.5 * (nz - 1) * hz
    tx, ty, tz = (px - X0) / hx, (py - Y0) / hy, (pz - Z0) / hz
    keep = (tx >= 0) & (tx < nx - 1) & (ty >= 0) & (ty < ny - 1) & (tz >= 0) & (tz < nz - 1)
    tx, ty, tz = tx[keep], ty[keep], tz[keep]
    ix, iy, iz = tx.astype(np.int64), ty.astype(np.int64), tz.astype(np.int64)
    fx, fy, fz = tx - ix, ty - iy, tz - iz
    base = (ix * ny + iy) * nz + iz
    m = base.size
    idx = np.empty(8 * m, dtype=np.int64)
    wts = np.empty(8 * m)
    c = 0
    for dx, wx in ((0, 1.0 - fx), (1, fx)):
        for dy, wy in ((0, 1.0 - fy), (1, fy)):
            wxy = wx * wy
            for dz, wz in ((0, 1.0 - fz), (1, fz)):
                idx[c * m:(c + 1) * m] = base + ((dx * ny + dy) * nz + dz)
                wts[c * m:(c + 1) * m] = wxy * wz
                c += 1
    return idx, wts


def three_bunch_cic(nx=128, ny=128, nz=512, seed=3, max_particles=1 << 28, target_peak=1.0e4):
    """128 x 128 x 512 in a 1 x 1 pipe, IGF, 256 x 256 modes; h = 1/129, z in +-10.

    Sum of three Gaussian sub-bunches (sigma_x, sigma_y ~ U[0.05, 0.2],
    sigma_z ~ U[0.5, 2.0], centres x, y ~ U[0.35, 0.65], z ~ U[-2, 2],
    weights ~ U[0.5, 1.5]) sampled with N_p macroparticles, N_p set so the
    densest node expects ~1e4 hits (1 % Poisson noise), at most 2^28, and
    deposited by cloud-in-cell; scaled to unit charge.
    """
    a = b = 1.0
    hx, hy = a / (nx + 1), b / (ny + 1)
    hz = 20.0 / (nz - 1)
    rng = np.random.default_rng(seed)
    sig = np.stack([rng.uniform(0.05, 0.2, 3), rng.uniform(0.05, 0.2, 3), rng.uniform(0.5, 2.0, 3)], 1)
    cen = np.stack([rng.uniform(0.35, 0.65, 3), rng.uniform(0.35, 0.65, 3), rng.uniform(-2.0, 2.0, 3)], 1)
    w = rng.uniform(0.5, 1.5, 3)
    w = w / w.sum()
    # expected hits at the densest node of the analytic mixture
    peak = 0.0
    for c in range(3):
        dens = w[c] / ((2 * math.pi) ** 1.5 * np.prod(sig[c]))
        mix = sum(w[d] / ((2 * math.pi) ** 1.5 * np.prod(sig[d]))
                  * math.exp(-0.5 * np.sum(((cen[c] - cen[d]) / sig[d]) ** 2)) for d in range(3))
        peak = max(peak, mix, dens)
    n_p = int(min(max_particles, math.ceil(target_peak / (peak * hx * hy * hz))))
    counts = rng.multinomial(n_p, w)
    # Chunks of at most 2^20 particles, each drawn from its own child stream of
    # the seed (SeedSequence.spawn), generated in worker threads and
    # accumulated in chunk order, so the result does not depend on timing.
    chunk = 1 << 20
    jobs = []
    for c in range(3):
        left = int(counts[c])
        while left > 0:
            jobs.append((c, min(chunk, left)))
            left -= jobs[-1][1]
    streams = np.random.SeedSequence(seed).spawn(len(jobs))

    def draw(j):
        c, m = jobs[j]
        g = np.random.default_rng(streams[j])
        p = g.standard_normal((3, m)) * sig[c][:, None] + cen[c][:, None]
        return _cic_weights(p[0], p[1], p[2], nx, ny, nz, hx, hy, hz)

    import concurrent.futures
    import torch
    acc = torch.zeros(nx * ny * nz, dtype=torch.float64)
    kept = 0
    workers = min(8, os.cpu_count() or 1)
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        for idx, wts in ex.map(draw, range(len(jobs))):
            acc.index_add_(0, torch.from_numpy(idx), torch.from_numpy(wts))
            kept += idx.size // 8
    rho = acc.numpy()
    rho = rho.reshape(nx, ny, nz)
    peak_hits = float(rho.max())
    rho = _unit_charge(rho, hx, hy, hz)
    notes = dict(n_particles=n_p, deposited=kept, peak_node_hits=peak_hits,
                 peak_rel_noise=1.0 / math.sqrt(max(peak_hits, 1.0)),
                 sigma=sig.tolist(), centre=cen.tolist(), weight=w.tolist())
    return Workload("three_bunch_cic", nx, ny, nz, hx, hy, hz, a, b, IGF_Z, 2 * nx, 2 * ny, rho, notes)


def learnable_bunch(seed=5):
    """128 x 128 x 256 in a 1 x 1 pipe, IGF, 256 x 256 modes, h = 1/129, z in +-2.

    Returns (workload with the initial density, target density): initial
    Gaussian at (0.5, 0.5, 0), sigma (0.15, 0.15, 0.5); the target density is
    the same bunch shifted to (0.55, 0.47, 0.25).
    """
    nx, ny, nz = 128, 128, 256
    h = 1.0 / 129
    hz = 4.0 / (nz - 1)
    rho0 = _unit_charge(gaussian(nx, ny, nz, h, h, hz, (0.5, 0.5, 0.0), (0.15, 0.15, 0.5)), h, h, hz)
    rhot = _unit_charge(gaussian(nx, ny, nz, h, h, hz, (0.55, 0.47, 0.25), (0.15, 0.15, 0.5)), h, h, hz)
    wl = Workload("learnable_bunch", nx, ny, nz, h, h, hz, 1.0, 1.0, IGF_Z, 256, 256, rho0)
    return wl, rhot


BATCH_SHAPES = ((32, 32, 32), (48, 48, 96), (64, 64, 128), (96, 96, 192))


def batch_manifest(count=96, seed=4):
    """Draws for the batched workload: per solve a shape from BATCH_SHAPES,
    pipe a, b ~ U[0.8, 2.0], h = a/(n+1), sigma_z ~ U[0.2, 1.0],
    h_z = 8 sigma_z/(nz - 1), Gaussian centre x ~ U[0.2a, 0.8a],
    y ~ U[0.2b, 0.8b], z = 0, sigma = (0.1a, 0.1b, sigma_z); IGF, modes (2nx, 2ny)."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        nx, ny, nz = BATCH_SHAPES[int(rng.integers(len(BATCH_SHAPES)))]
        a, b = rng.uniform(0.8, 2.0), rng.uniform(0.8, 2.0)
        sz = rng.uniform(0.2, 1.0)
        cx, cy = rng.uniform(0.2 * a, 0.8 * a), rng.uniform(0.2 * b, 0.8 * b)
        out.append(dict(index=s, nx=nx, ny=ny, nz=nz, a=a, b=b, hx=a / (nx + 1), hy=b / (ny + 1),
                        hz=8.0 * sz / (nz - 1), centre=(cx, cy, 0.0), sigma=(0.1 * a, 0.1 * b, sz),
                        kind=IGF_Z, mx=2 * nx, my=2 * ny))
    return out


def batch_member(d):
    rho = gaussian(d["nx"], d["ny"], d["nz"], d["hx"], d["hy"], d["hz"], d["centre"], d["sigma"])
    rho = _unit_charge(rho, d["hx"], d["hy"], d["hz"])
    return Workload("batch_%d" % d["index"], d["nx"], d["ny"], d["nz"], d["hx"], d["hy"], d["hz"],
                    d["a"], d["b"], d["kind"], d["mx"], d["my"], rho)


def accuracy_study_bunch(n, nz, sigma_z, a=4.0, kind=IGF_Z, modes=20):
    """The numerical example of Sec. 4 (lengths in cm): pipe a = b = 4, modes
    m, n = 1..20, Gaussian with sigma_x = sigma_y = 0.15 a = 0.6 and the given
    sigma_z, centred on the pipe axis, set to zero outside the 3-sigma
    ellipsoid.  Transverse mesh: n nodes at X_i = (i+1) a/n (the last node on
    the wall), so the axis x = a/2 is node n/2 - 1; z spans +-3 sigma_z with nz
    nodes.  Returns the workload and the on-axis node index (i, j)."""
    b = a
    hx = hy = a / n
    hz = 6.0 * sigma_z / (nz - 1)
    X, Y, Z = coords(n, n, nz, hx, hy, hz)
    sx = sy = 0.15 * a
    q = (((X - a / 2) / sx) ** 2)[:, None, None] + (((Y - b / 2) / sy) ** 2)[None, :, None] \
        + ((Z / sigma_z) ** 2)[None, None, :]
    rho = np.exp(-0.5 * q) * (q <= 9.0)
    wl = Workload("accuracy_study_n%d_nz%d_sz%g" % (n, nz, sigma_z), n, n, nz, hx, hy, hz, a, b, kind,
                  modes, modes, rho)
    return wl, (n // 2 - 1, n // 2 - 1)


def gaussian_bunch(nx, ny, nz, modes=256, seed=6):
    """A smooth bunch on any mesh, for timing and profiling other sizes than the
    benchmark's: pipe 1 x 1, h = 1/(n+1), z over +-10 (hz = 20/(nz-1)), IGF,
    modes min(2n, `modes`) per dimension; Gaussian at (0.5, 0.45, 0.3) with
    sigma (0.1, 0.12, 2.0), unit charge plus 1e-3 uniform noise (seeded)."""
    hx, hy, hz = 1.0 / (nx + 1), 1.0 / (ny + 1), 20.0 / (nz - 1)
    rho = gaussian(nx, ny, nz, hx, hy, hz, (0.5, 0.45, 0.3), (0.1, 0.12, 2.0))
    rho = _add_noise(_unit_charge(rho, hx, hy, hz), np.random.default_rng(seed))
    return Workload("gaussian_bunch_%dx%dx%d" % (nx, ny, nz), nx, ny, nz, hx, hy, hz, 1.0, 1.0, IGF_Z,
                    min(2 * nx, modes), min(2 * ny, modes), rho)
