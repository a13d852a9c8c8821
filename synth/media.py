"""Seeded procedural media (FP64 generation, rounded once to FP32).

Recipes (the paper's own datasets -- the procedural nebula, the point source,
the checkerboard -- are not available, so these stand in with the same kind of
structure):

* value noise: a 32-bit integer hash of the lattice corner (x, y, z, seed)
  gives a uniform value in [0, 1); cell values are trilinear interpolations of
  the corner values at the cell centre; the lattice wraps, so the noise tiles.
* fBm: sum over octaves o = 0..4 of gain^o * noise(base * lacunarity^o)
  (lacunarity 2, gain 1/2), normalised to [0, 1] by its min and max.
* blobs: Gaussian bumps exp(-|R^T (x - c)|^2_{S^-1} / 2) with random rotation R
  and per-axis standard deviations S.

Grids are indexed [z, y, x] (x fastest), cell centres at ((i + 1/2)/n).
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np

_M32 = np.uint64(0xFFFFFFFF)


def _hash32(v):
    """lowbias32 integer hash (C. Wellons), on uint64 arrays holding 32-bit values."""
    v = np.asarray(v, dtype=np.uint64) & _M32
    v ^= v >> np.uint64(16)
    v = (v * np.uint64(0x7FEB352D)) & _M32
    v ^= v >> np.uint64(15)
    v = (v * np.uint64(0x846CA68B)) & _M32
    v ^= v >> np.uint64(16)
    return v


def _corner_values(ix, iy, iz, seed):
    h = _hash32(np.uint64(seed & 0xFFFFFFFF) + np.uint64(0x9E3779B9))
    h = _hash32(h ^ np.asarray(iz, dtype=np.uint64))
    h = _hash32(h ^ np.asarray(iy, dtype=np.uint64))
    h = _hash32(h ^ np.asarray(ix, dtype=np.uint64))
    return h.astype(np.float64) / 4294967296.0


def value_noise(dims, freq, seed):
    """Trilinear value noise with ``freq`` lattice periods across the domain."""
    nx, ny, nz = dims
    axes = []
    for n in (nx, ny, nz):
        u = (np.arange(n) + 0.5) / n * freq
        i0 = np.floor(u).astype(np.int64)
        axes.append((i0 % freq, (i0 + 1) % freq, u - i0))
    (x0, x1, tx), (y0, y1, ty), (z0, z1, tz) = axes
    out = np.zeros((nz, ny, nx))
    for zi, wz in ((z0, 1 - tz), (z1, tz)):
        for yi, wy in ((y0, 1 - ty), (y1, ty)):
            for xi, wx in ((x0, 1 - tx), (x1, tx)):
                v = _corner_values(xi[None, None, :], yi[None, :, None], zi[:, None, None], seed)
                out += v * (wz[:, None, None] * wy[None, :, None] * wx[None, None, :])
    return out


def fbm(dims, seed, octaves=5, base_freq=4, lacunarity=2, gain=0.5):
    """Fractional Brownian motion of value noise, normalised to [0, 1]."""
    f = np.zeros((dims[2], dims[1], dims[0]))
    amp = 1.0
    freq = base_freq
    for o in range(octaves):
        f += amp * value_noise(dims, freq, seed * 7919 + o)
        amp *= gain
        freq *= lacunarity
    lo, hi = f.min(), f.max()
    return (f - lo) / (hi - lo) if hi > lo else np.zeros_like(f)


def _cell_centres(dims):
    nx, ny, nz = dims
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) / nz, (np.arange(ny) + 0.5) / ny,
                          (np.arange(nx) + 0.5) / nx, indexing="ij")
    return x, y, z


def gaussian_blob(dims, centre, std, rot=None):
    """exp(-0.5 * sum_i (e_i . (x - c))^2 / std_i^2) at the cell centres
    (unit-cube coordinates); ``std`` is a scalar or 3 per-axis values."""
    x, y, z = _cell_centres(dims)
    d = np.stack([x - centre[0], y - centre[1], z - centre[2]], axis=-1)
    if rot is not None:
        d = d @ np.asarray(rot)
    s = np.broadcast_to(np.asarray(std, dtype=np.float64), (3,))
    return np.exp(-0.5 * np.sum((d / s) ** 2, axis=-1))


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                     [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                     [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


@dataclass
class Medium:
    """One synthetic problem: cell-centred FP32 fields, indexed [z, y, x]."""
    name: str
    order: int
    dims: tuple
    sigma_t: np.ndarray
    albedo: np.ndarray
    g: float
    sigma_t_min: float
    q00: List[np.ndarray] = field(default_factory=list)   # one emission field per RHS
    bc: object = 0                                         # 0 vacuum, 1 periodic, 2 Neumann, or one per axis
    h: float = 0.0                                         # cell size (0: 1 / n_x)

    def __post_init__(self):
        # scalars are FP32 inputs like the fields
        self.g = float(np.float32(self.g))
        self.sigma_t_min = float(np.float32(self.sigma_t_min))

    @property
    def nrhs(self):
        return len(self.q00)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def config_p1_homogeneous(n=16):
    """P1, n^3, sigma_t = 10, albedo 0.9, isotropic, Q^{00} = 1 in the central 2^3 cells."""
    dims = (n, n, n)
    q = np.zeros((n, n, n))
    c = n // 2
    q[c - 1:c + 1, c - 1:c + 1, c - 1:c + 1] = 1.0
    return Medium("p1_homogeneous_%d" % n, 1, dims, _f32(np.full((n, n, n), 10.0)),
                  _f32(np.full((n, n, n), 0.9)), 0.0, 0.0, [_f32(q)])


def config_p3_fbm(n=64, seed=1, order=3, sigma_t_min=1.0, g=0.3, nrhs=1):
    """P3, n^3: sigma_t = 50 * fBm, albedo ~ U[0.8, 0.99] per cell, HG g = 0.3,
    emission a Gaussian blob of std 4 cells at a seeded centre (nrhs > 1: more
    blobs at further seeded centres, one per right-hand side)."""
    rng = np.random.default_rng(seed)
    dims = (n, n, n)
    st = 50.0 * fbm(dims, seed)
    alb = rng.uniform(0.8, 0.99, size=(n, n, n))
    qs = []
    for _ in range(nrhs):
        c = rng.uniform(0.3, 0.7, size=3)
        qs.append(_f32(gaussian_blob(dims, c, 4.0 / n)))
    return Medium("p%d_fbm_%d_s%d" % (order, n, seed), order, dims, _f32(st), _f32(alb), g, sigma_t_min, qs)


def config_p3_train(n=64, seed=1000, nrhs=8, order=3, sigma_t_min=1.0, g=0.3):
    """Training media for the learned guess: the P3 fBm medium with its
    extinction scale drawn per medium (sigma_t = S * fBm, S ~ U[25, 200]) and
    emission of mixed widths per right-hand side: a single-cell point source
    (one in four) or a Gaussian blob of std U[0.7, 4] cells."""
    rng = np.random.default_rng(seed)
    dims = (n, n, n)
    scale = rng.uniform(25.0, 200.0)
    st = scale * fbm(dims, seed)
    alb = rng.uniform(0.8, 0.99, size=(n, n, n))
    qs = []
    for _ in range(nrhs):
        if rng.uniform() < 0.25:
            q = np.zeros((n, n, n))
            i = rng.integers(n // 4, 3 * n // 4, size=3)
            q[i[2], i[1], i[0]] = 1.0
        else:
            c = rng.uniform(0.3, 0.7, size=3)
            q = gaussian_blob(dims, c, rng.uniform(0.7, 4.0) / n)
        qs.append(_f32(q))
    return Medium("p%d_train_%d_s%d" % (order, n, seed), order, dims, _f32(st), _f32(alb), g, sigma_t_min, qs)


def config_p5_nebula(n=128, seed=3, g=0.0, order=5, sigma_t_min=1.0, nblobs=32):
    """P5, n^3 nebula: (sum of 32 anisotropic Gaussian blobs) * fBm, scaled to
    sigma_t in [0, 200]; albedo 0.95; emission Q^{00} = 1 in 2 seeded cells."""
    rng = np.random.default_rng(seed)
    dims = (n, n, n)
    dens = np.zeros((n, n, n))
    for _ in range(nblobs):
        c = rng.uniform(0.2, 0.8, size=3)
        s = rng.uniform(0.04, 0.15, size=3)
        w = rng.uniform(0.3, 1.0)
        dens += w * gaussian_blob(dims, c, s, _random_rotation(rng))
    dens *= fbm(dims, seed)
    dens /= dens.max()
    q = np.zeros((n, n, n))
    for _ in range(2):
        i = rng.integers(n // 4, 3 * n // 4, size=3)
        q[i[2], i[1], i[0]] = 1.0
    return Medium("p%d_nebula_%d_s%d_g%g" % (order, n, seed, g), order, dims, _f32(200.0 * dens),
                  _f32(np.full((n, n, n), 0.95)), g, sigma_t_min, [_f32(q)])


def config_batch(seed=7, nmedia=48, nrhs=8, sizes=(32, 48, 64, 96), orders=(1, 3, 5, 7),
                 sigma_t_min=1.0):
    """Batch: media with seeded sizes and orders, fBm sigma_t in [0, 100],
    albedo 0.9, g = 0, each with ``nrhs`` random Gaussian emission blobs."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(nmedia):
        n = int(rng.choice(sizes))
        order = int(rng.choice(orders))
        dims = (n, n, n)
        st = 100.0 * fbm(dims, seed * 1000 + i)
        qs = []
        for _ in range(nrhs):
            c = rng.uniform(0.25, 0.75, size=3)
            s = rng.uniform(2.0, 6.0) / n
            qs.append(_f32(gaussian_blob(dims, c, s)))
        out.append(Medium("batch%d_p%d_%d" % (i, order, n), order, dims, _f32(st),
                          _f32(np.full((n, n, n), 0.9)), 0.0, sigma_t_min, qs))
    return out


def config_uniform_periodic(n=8, order=3, sigma_t=5.0, albedo=0.8, g=0.4, q=1.0, dims=None):
    """Uniform medium and uniform isotropic emission on a periodic grid."""
    dims = dims or (n, n, n)
    shp = (dims[2], dims[1], dims[0])
    return Medium("uniform_periodic", order, dims, _f32(np.full(shp, sigma_t)), _f32(np.full(shp, albedo)),
                  g, 0.0, [_f32(np.full(shp, q))], bc=1)


def config_small(order, dims, seed=0, sigma_range=(0.5, 20.0), albedo_range=(0.5, 0.99), g=0.3,
                 sigma_t_min=0.5, bc=0, nrhs=1):
    """Small heterogeneous medium with i.i.d. random cells (tests)."""
    rng = np.random.default_rng(seed)
    shp = (dims[2], dims[1], dims[0])
    st = rng.uniform(*sigma_range, size=shp)
    alb = rng.uniform(*albedo_range, size=shp)
    qs = [_f32(rng.uniform(0.0, 1.0, size=shp)) for _ in range(nrhs)]
    return Medium("small_p%d_%dx%dx%d_s%d" % ((order,) + tuple(dims) + (seed,)), order, tuple(dims),
                  _f32(st), _f32(alb), g, sigma_t_min, qs, bc=bc)


def checkerboard_blocks():
    """Block kinds of the 7 x 7 checkerboard (lattice) problem, indexed
    [block_y, block_x]: 1 = purely absorbing (sigma_a = 10), 2 = the
    isotropic unit source (purely scattering), 0 = purely scattering
    (sigma_s = 1).  Absorbers sit on the blocks (i, j) of the inner 5 x 5 with
    i + j even, the central block holds the source instead."""
    kind = np.zeros((7, 7), dtype=np.int64)
    for j in range(1, 6):
        for i in range(1, 6):
            if (i + j) % 2 == 0:
                kind[j, i] = 1
    kind[3, 3] = 2
    return kind


def config_checkerboard(order, n=71, size=7.0):
    """2D checkerboard: a size x size domain of unit blocks on n x n cells
    (a cell takes the block containing its centre), z-invariant (one
    z-periodic cell), vacuum in x and y, isotropic scattering.  Absorbing
    blocks: sigma_t = 10, albedo 0; other blocks: sigma_t = 1, albedo 1;
    Q^{0,0} = 1 in the central block."""
    kind = checkerboard_blocks()
    h = size / n
    c = (np.arange(n) + 0.5) * h
    b = np.minimum(np.floor(c).astype(np.int64), int(size) - 1)
    k2 = kind[b[:, None], b[None, :]]                     # [y, x]
    st = np.where(k2 == 1, 10.0, 1.0)[None]
    alb = np.where(k2 == 1, 0.0, 1.0)[None]
    q = (k2 == 2).astype(np.float64)[None]
    return Medium("checkerboard_p%d_%d" % (order, n), order, (n, n, 1), _f32(st), _f32(alb), 0.0, 0.0, [_f32(q)],
                  bc=(0, 0, 1), h=h)


def config_point_source(order, n=80, sigma_t=8.0, albedo=0.9, g=0.0):
    """Point source in a homogeneous medium: n^3 cells of size 1/n, sigma_t =
    8, albedo 0.9, isotropic scattering, Q^{0,0} = 1 in the central 2^3 cells
    (n even), vacuum boundary."""
    if n % 2:
        raise ValueError("the point source needs an even n")
    q = np.zeros((n, n, n))
    c = n // 2
    q[c - 1:c + 1, c - 1:c + 1, c - 1:c + 1] = 1.0
    return Medium("point_source_p%d_%d" % (order, n), order, (n, n, n), _f32(np.full((n, n, n), sigma_t)),
                  _f32(np.full((n, n, n), albedo)), g, 0.0, [_f32(q)])
