"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package holds no arithmetic of the method: it only builds velocity
models, source and receiver positions and random vectors. Both the HIP path
and the oracle receive these arrays as inputs.

The paper's own models exist only in figures (the 1D well model and the 2D
true model of its Examples section), so synthetic models of the same kind
stand in for them:

* ``model_1d_layers``    1D, 1001 nodes, h = 5 m, three layers
                         1500/2200/3000 m/s, source at the first node, 10 Hz;
* ``model_2d_lens``      2D 201 x 201, h = 10 m, 2000 m/s background with a
                         Gaussian anomaly (sigma 300 m, +-800 m/s), 5 Hz;
* ``model_2d_layered``   2D 401 x 801, h = 10 m, eight horizontal layers
                         1500-4500 m/s with a smooth seeded random
                         perturbation (5 % rms, 200 m correlation), 64
                         surface shots, frequencies 3/5/8/12 Hz;
* ``model_fwi``          2D 301 x 601, h = 10 m, three units 1800/2600/3500 m/s
                         split by two dipping interfaces plus a seeded
                         elliptical low-velocity lens; starting model = the
                         true slowness smoothed with a 400 m Gaussian; 32
                         surface shots, 151 surface receivers, 3-12 Hz;
* ``model_3d_layered``   3D (nz, ny, nx) box, h = 20 m, horizontal layers
                         1500-4500 m/s with a smooth seeded random
                         perturbation (5 % rms, 200 m correlation), shots on
                         the surface plane (Eq. (1) with d = 3);
* ``serving_request``    one request of a serving stream: square grid of
                         side 129, 257 or 513 (h = 10 m), layered model with
                         a Gaussian anomaly, one frequency from U(2, 15) Hz,
                         1-32 surface shots; ``poisson_arrivals`` gives the
                         arrival times;
* ``gardner_density``    a density field for Eq. (1) that follows the
                         velocity model: Gardner's rule rho ~ c^(1/4),
                         relative to the density at the slowest velocity
                         (dimensionless, 1 to about 1.3 over 1500-4500 m/s).
"""

import numpy as np
from scipy.ndimage import gaussian_filter


class Workload(dict):
    """A dict with attribute access: velocity c, slowness m, h, freqs, ..."""

    __getattr__ = dict.__getitem__


def model_1d_layers(n=1001, h=5.0):
    """Three equal layers over [0, (n-1) h]; an interface node carries the mean
    of the squared slowness of its two sides."""
    c1, c2, c3 = 1500.0, 2200.0, 3000.0
    i1, i2 = n // 3, (2 * n) // 3
    m = np.empty(n)
    m[:i1] = 1 / c1
    m[i1 + 1:i2] = 1 / c2
    m[i2 + 1:] = 1 / c3
    m[i1] = np.sqrt(0.5 * (1 / c1 ** 2 + 1 / c2 ** 2))
    m[i2] = np.sqrt(0.5 * (1 / c2 ** 2 + 1 / c3 ** 2))
    return Workload(name=f"1d-3layer-{n}", m=m, c=1 / m, h=h, shape=(n,),
                    freqs=[10.0], alpha=0.01, src=[0], beta=(1.0, 0.5), tol=1e-10)


def model_2d_lens(n=201, h=10.0, sign=-1.0):
    """Gaussian velocity anomaly 2000 + sign*800*exp(-r^2/(2*300^2)) m/s,
    centred in the square; one source at the middle of the surface row."""
    x = np.arange(n) * h
    z = np.arange(n) * h
    cx = cz = 0.5 * (n - 1) * h
    Z, X = np.meshgrid(z, x, indexing="ij")
    r2 = (X - cx) ** 2 + (Z - cz) ** 2
    c = 2000.0 + sign * 800.0 * np.exp(-r2 / (2 * 300.0 ** 2))
    src = [0 * n + (n - 1) // 2]
    return Workload(name=f"2d-lens{'-' if sign < 0 else '+'}-{n}", m=1 / c, c=c, h=h,
                    shape=(n, n), freqs=[5.0], alpha=0.01, src=src,
                    beta=(1.0, 0.5), levels=4, nu=(2, 2), wj=0.8, tol=1e-8)


def model_2d_layered(nz=401, nx=801, h=10.0, seed=0, nshots=64,
                     freqs=(3.0, 5.0, 8.0, 12.0)):
    """Eight horizontal layers 1500-4500 m/s (each 50 cells thick, the last to
    the bottom) times (1 + p), p a Gaussian-filtered white-noise field
    (covariance length 200 m), scaled to 5 % rms and clipped to +-15 %.
    Shots on the surface row at ix = 22 + 12 k (k < 64 for the full grid;
    spread evenly otherwise)."""
    layer_v = np.linspace(1500.0, 4500.0, 8)
    iz = np.arange(nz)
    c = np.repeat(layer_v[np.minimum(iz // 50, 7)][:, None], nx, axis=1)
    rng = np.random.default_rng(seed)
    p = gaussian_filter(rng.standard_normal((nz, nx)), sigma=200.0 / (h * np.sqrt(2.0)))
    p *= 0.05 / np.sqrt(np.mean(p ** 2))
    p = np.clip(p, -0.15, 0.15)
    c = c * (1.0 + p)
    if nx == 801 and nshots == 64:
        ix = 22 + 12 * np.arange(64)
    else:
        ix = np.round(np.linspace(0.03 * (nx - 1), 0.97 * (nx - 1), nshots)).astype(int)
    src = [int(i) for i in ix]  # surface row iz = 0: flat index = ix
    return Workload(name=f"2d-layered-{nz}x{nx}", m=1 / c, c=c, h=h, shape=(nz, nx),
                    freqs=list(freqs), alpha=0.01, src=src, beta=(1.0, 0.5), tol=1e-8)


def model_3d_layered(nz=65, ny=65, nx=65, h=20.0, seed=0, nshots=8, freqs=(2.0, 4.0), nlayers=6):
    """Horizontal layers 1500-4500 m/s (nlayers of equal thickness in z)
    times (1 + p), p a Gaussian-filtered white-noise field (covariance length
    200 m), scaled to 5 % rms and clipped to +-15 %. Shots on the surface
    plane iz = 0 at (iy, ix) spread over the central 60 % of each axis."""
    layer_v = np.linspace(1500.0, 4500.0, nlayers)
    iz = np.arange(nz)
    lz = np.minimum(iz * nlayers // nz, nlayers - 1)
    c = np.broadcast_to(layer_v[lz][:, None, None], (nz, ny, nx)).copy()
    rng = np.random.default_rng(seed)
    p = gaussian_filter(rng.standard_normal((nz, ny, nx)), sigma=200.0 / (h * np.sqrt(2.0)))
    p *= 0.05 / np.sqrt(np.mean(p ** 2))
    p = np.clip(p, -0.15, 0.15)
    c = c * (1.0 + p)
    k = int(np.ceil(np.sqrt(nshots)))
    ys = np.round(np.linspace(0.2 * (ny - 1), 0.8 * (ny - 1), k)).astype(int)
    xs = np.round(np.linspace(0.2 * (nx - 1), 0.8 * (nx - 1), k)).astype(int)
    src = [(0, int(ys[i // k]), int(xs[i % k])) for i in range(nshots)]
    return Workload(name=f"3d-layered-{nz}x{ny}x{nx}", m=1 / c, c=c, h=h, shape=(nz, ny, nx),
                    freqs=list(freqs), alpha=0.01, src=src, beta=(1.0, 0.5), tol=1e-8)


def model_fwi(nz=301, nx=601, h=10.0, seed=0):
    """True and starting models of a Gauss-Newton FWI test. Interfaces: depth
    800 m -> 1200 m and 2000 m -> 1600 m linearly across x; units 1800, 2600
    and 3500 m/s; a lens (-300 m/s, semi-axes 600 m in x and 150 m in z,
    centre drawn from the seed inside the middle unit). Shots at
    ix = 21 + 18 k (k < 32), receivers at ix = 4 r (r < 151), all on the
    surface row, for the full grid; spread evenly on smaller grids."""
    rng = np.random.default_rng(seed)
    x = np.arange(nx) * h
    z = np.arange(nz) * h
    Z, X = np.meshgrid(z, x, indexing="ij")
    L = (nx - 1) * h
    d1 = (800.0 + 400.0 * X / L) * (nz - 1) * h / 3000.0
    d2 = (2000.0 - 400.0 * X / L) * (nz - 1) * h / 3000.0
    c = np.where(Z < d1, 1800.0, np.where(Z < d2, 2600.0, 3500.0))
    xc = rng.uniform(0.35, 0.65) * L
    zc = 0.5 * (d1 + d2)[0, int(round(xc / h))] + rng.uniform(-0.05, 0.05) * (nz - 1) * h
    ax, az = 600.0 * L / 6000.0, 150.0 * (nz - 1) * h / 3000.0
    c = np.where(((X - xc) / ax) ** 2 + ((Z - zc) / az) ** 2 <= 1.0, c - 300.0, c)
    m_true = 1.0 / c
    m_start = gaussian_filter(m_true, sigma=400.0 / h, mode="nearest")
    if nx == 601:
        src = [21 + 18 * k for k in range(32)]
        rec = [4 * r for r in range(151)]
    else:
        src = [int(i) for i in np.round(np.linspace(0.035 * (nx - 1), 0.965 * (nx - 1), 32))]
        rec = [int(i) for i in np.round(np.linspace(0, nx - 1, min(151, nx)))]
    return Workload(name=f"fwi-{nz}x{nx}", m=m_true, m_start=m_start, c=c, h=h, shape=(nz, nx),
                    freqs=[3.0, 4.0, 6.0, 8.0, 10.0, 12.0], alpha=0.01, src=src, rec=rec, lam=1e-3,
                    beta=(1.0, 0.5), tol=1e-8)


def gardner_density(m):
    """Density of the same shape as the slowness m, (c / c_min)^(1/4) with c = 1/m."""
    c = 1.0 / np.asarray(m, dtype=np.float64)
    return (c / c.min()) ** 0.25


def random_vectors(nvec, size, seed):
    """complex128 [nvec, size] with independent standard normal parts."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nvec, size)) + 1j * rng.standard_normal((nvec, size))


def smooth_random_vectors(nvec, shape, seed, sigma=3.0):
    """Smooth complex fields (Gaussian-filtered noise), flattened, [nvec, size]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nvec):
        re = gaussian_filter(rng.standard_normal(shape), sigma)
        im = gaussian_filter(rng.standard_normal(shape), sigma)
        out.append((re + 1j * im).ravel())
    return np.array(out)


def serving_request(rid, sides=(129, 257, 513), h=10.0):
    """Request ``rid`` of a serving stream (seeded by rid): side from
    ``sides``, four layers from 1500 m/s down to 1500-3500 m/s, plus a
    Gaussian anomaly (+-20 %, radius 5-15 % of the side) at a random point;
    frequency U(2, 15) Hz (at least 10 nodes per wavelength, c >= 1500 m/s
    and h = 10 m); nrhs U{1..32} shots on the surface row."""
    rng = np.random.default_rng(1000 + rid)
    n = int(sides[rng.integers(0, len(sides))])
    iz = np.arange(n)
    bottom = rng.uniform(2500.0, 3500.0)
    layer_v = np.linspace(1500.0, bottom, 4)
    c = np.repeat(layer_v[np.minimum(iz * 4 // n, 3)][:, None], n, axis=1)
    z0, x0 = rng.uniform(0.3, 0.8) * (n - 1), rng.uniform(0.2, 0.8) * (n - 1)
    rad = rng.uniform(0.05, 0.15) * (n - 1)
    Z, X = np.meshgrid(iz, iz, indexing="ij")
    c = c * (1.0 + rng.uniform(-0.2, 0.2) * np.exp(-((Z - z0) ** 2 + (X - x0) ** 2) / (2 * rad ** 2)))
    c = np.maximum(c, 1500.0)
    nrhs = int(rng.integers(1, 33))
    src = sorted(int(i) for i in rng.choice(np.arange(2, n - 2), size=nrhs, replace=False))
    return Workload(name=f"serve-{rid}-{n}", m=1 / c, c=c, h=h, shape=(n, n),
                    freqs=[float(rng.uniform(2.0, 15.0))], alpha=0.01, src=src, beta=(1.0, 0.5), tol=1e-8)


def poisson_arrivals(count, rate, seed=0):
    """Arrival times (s) of ``count`` requests at ``rate`` per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
