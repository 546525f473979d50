"""Seeded synthetic scenes for confocal NLOS reconstruction.

This module is the only code shared by the FP64 oracle, the tests and the
benchmark.  It holds none of the reconstruction method's arithmetic: it draws
hidden volumes, scan masks and photon noise from seeded generators, and nothing
else.  Turning a hidden volume into a clean transient measurement needs the
forward operator, which each side applies with its own implementation; this
module only adds noise to a clean signal it is handed.

Geometry conventions (the paper fixes none of them; see the grid reading in the
design notes):

* scan point (i, j), i, j in [0, n), sits at x_i = (i + 1/2) W / n - W / 2 on the
  wall (same for y with the wall height);
* depth / time bin k in [0, m) covers the one-way distance [k, k + 1) * R / m,
  with R = m * c * dt / 2;
* volumes are C-order float arrays ``[n][n][m]`` with the depth/time axis fastest;
* masks are uint8 ``[n][n]``, 1 = scan point measured.

Workload shapes follow the paper's experiments (Section 5): a 1 m wall with
32 ps bins (Bowling, Section 5.2.1), 16 ps bins with 512 bins (the SU scene),
and a 2 m wall (the Stanford outdoor/teaser scenes).  The scenes themselves are
drawn here; no dataset item is reproduced.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

C_LIGHT = 299792458.0  # m/s


@dataclasses.dataclass
class Scene:
    name: str
    n: int
    m: int
    wall_w: float          # metres
    wall_h: float          # metres
    bin_ps: float          # picoseconds
    u_true: np.ndarray     # float64 [n][n][m], albedo
    mask: np.ndarray       # uint8 [n][n]
    peak: float            # mean photons in the brightest bin
    background: float      # mean photons per bin added uniformly
    seed: int

    @property
    def range_m(self) -> float:
        return self.m * C_LIGHT * (self.bin_ps * 1e-12) / 2.0

    @property
    def shape(self):
        return (self.n, self.n, self.m)


# ----------------------------------------------------------------------------
# masks
# ----------------------------------------------------------------------------

def random_mask(n: int, kept: int, rng: np.random.Generator) -> np.ndarray:
    """Exactly ``kept`` of n*n scan points, chosen uniformly without replacement."""
    idx = rng.choice(n * n, size=kept, replace=False)
    mask = np.zeros(n * n, dtype=np.uint8)
    mask[idx] = 1
    return mask.reshape(n, n)


def strided_dropout_mask(n: int, stride: int, keep_frac: float,
                         rng: np.random.Generator) -> np.ndarray:
    """Regular ``stride`` grid with an exact fraction of its points dropped."""
    grid = [(i, j) for i in range(0, n, stride) for j in range(0, n, stride)]
    kept = int(round(len(grid) * keep_frac))
    sel = rng.choice(len(grid), size=kept, replace=False)
    mask = np.zeros((n, n), dtype=np.uint8)
    for s in sel:
        i, j = grid[s]
        mask[i, j] = 1
    return mask


def density_mask(n: int, density: float, rng: np.random.Generator) -> np.ndarray:
    kept = max(1, int(round(n * n * density)))
    return random_mask(n, kept, rng)


# ----------------------------------------------------------------------------
# hidden-volume primitives
# ----------------------------------------------------------------------------

def _lateral_index(x: np.ndarray, wall: float, n: int) -> np.ndarray:
    return np.floor((x + wall / 2.0) / wall * n).astype(np.int64)


def _depth_index(z: np.ndarray, rng_m: float, m: int) -> np.ndarray:
    return np.floor(z / rng_m * m).astype(np.int64)


def _splat(u: np.ndarray, i, j, k, albedo: float) -> None:
    n0, n1, m = u.shape
    ok = (i >= 0) & (i < n0) & (j >= 0) & (j < n1) & (k >= 0) & (k < m)
    i, j, k = i[ok], j[ok], k[ok]
    u[i, j, k] = np.maximum(u[i, j, k], albedo)


def add_planar_rect(u: np.ndarray, rng: np.random.Generator, size_lo=3, size_hi=8,
                    depth_lo_frac=0.25, depth_hi_frac=0.9) -> None:
    """Axis-aligned rectangle, one voxel thick, facing the wall."""
    n0, n1, m = u.shape
    w = int(rng.integers(size_lo, size_hi + 1))
    h = int(rng.integers(size_lo, size_hi + 1))
    w, h = min(w, n0), min(h, n1)
    i0 = int(rng.integers(0, n0 - w + 1))
    j0 = int(rng.integers(0, n1 - h + 1))
    k0 = int(rng.integers(int(math.ceil(depth_lo_frac * m)), int(math.floor(depth_hi_frac * m)) + 1))
    k0 = min(k0, m - 1)
    alb = float(rng.uniform(0.5, 1.0))
    u[i0:i0 + w, j0:j0 + h, k0] = np.maximum(u[i0:i0 + w, j0:j0 + h, k0], alb)


def add_ellipsoid_shell(u: np.ndarray, rng: np.random.Generator, wall_w: float, wall_h: float,
                        rng_m: float, samples: int = 20000, axis_lo=0.05, axis_hi=0.15,
                        lateral_frac=0.3, depth_lo=0.3, depth_hi=0.8) -> None:
    n0, n1, m = u.shape
    cx = rng.uniform(-lateral_frac * wall_w, lateral_frac * wall_w)
    cy = rng.uniform(-lateral_frac * wall_h, lateral_frac * wall_h)
    cz = rng.uniform(depth_lo * rng_m, depth_hi * rng_m)
    ax, ay, az = rng.uniform(axis_lo, axis_hi, size=3)
    alb = float(rng.uniform(0.5, 1.0))
    d = rng.standard_normal((samples, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    x = cx + ax * d[:, 0]
    y = cy + ay * d[:, 1]
    z = cz + az * d[:, 2]
    _splat(u, _lateral_index(x, wall_w, n0), _lateral_index(y, wall_h, n1),
           _depth_index(z, rng_m, m), alb)


# A 5x7 block letter of this project's own drawing ("N", for NLOS).
_LETTER_N = np.array([
    [1, 0, 0, 0, 1],
    [1, 1, 0, 0, 1],
    [1, 1, 0, 0, 1],
    [1, 0, 1, 0, 1],
    [1, 0, 0, 1, 1],
    [1, 0, 0, 1, 1],
    [1, 0, 0, 0, 1],
], dtype=np.uint8)


def add_letter_patch(u: np.ndarray, rng: np.random.Generator, wall_w: float, wall_h: float,
                     rng_m: float, height_m: float = 0.3) -> None:
    """Planar block letter, ~height_m tall, at a random depth, facing the wall."""
    n0, n1, m = u.shape
    rows, cols = _LETTER_N.shape
    cell = height_m / rows
    width_m = cell * cols
    cx = rng.uniform(-0.5 * wall_w + width_m / 2, 0.5 * wall_w - width_m / 2)
    cy = rng.uniform(-0.5 * wall_h + height_m / 2, 0.5 * wall_h - height_m / 2)
    z = rng.uniform(0.3 * rng_m, 0.8 * rng_m)
    alb = float(rng.uniform(0.5, 1.0))
    k = int(np.floor(z / rng_m * m))
    xs = (np.arange(n0) + 0.5) * wall_w / n0 - wall_w / 2
    ys = (np.arange(n1) + 0.5) * wall_h / n1 - wall_h / 2
    for i, x in enumerate(xs):
        c = int(np.floor((x - (cx - width_m / 2)) / cell))
        if c < 0 or c >= cols:
            continue
        for j, y in enumerate(ys):
            r = int(np.floor(((cy + height_m / 2) - y) / cell))
            if 0 <= r < rows and _LETTER_N[r, c]:
                u[i, j, k] = max(u[i, j, k], alb)


# ----------------------------------------------------------------------------
# noise
# ----------------------------------------------------------------------------

def poisson_counts(clean: np.ndarray, peak: float, background: float,
                   rng: np.random.Generator) -> np.ndarray:
    """Scale ``clean`` so its maximum is ``peak`` mean photons, add a uniform
    background of ``background`` photons per bin, draw Poisson counts."""
    clean = np.asarray(clean, dtype=np.float64)
    mx = float(clean.max())
    scale = peak / mx if mx > 0 else 0.0
    lam = np.clip(clean * scale, 0.0, None) + background
    return rng.poisson(lam).astype(np.float64)


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

def scene_small(seed: int = 101) -> Scene:
    """16x16 scan grid over a 1 m x 1 m wall, 128 bins of 32 ps, 50% random
    mask, three planar patches, 50 photons at the peak bin."""
    n, m, wall, bin_ps = 16, 128, 1.0, 32.0
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = random_mask(n, n * n // 2, rng)
    u = np.zeros((n, n, m))
    for _ in range(3):
        add_planar_rect(u, rng)
    return Scene("16x16x128", n, m, wall, wall, bin_ps, u, mask, 50.0, 0.0, seed)


def scene_medium(seed: int = 201) -> Scene:
    """64x64 scan grid over a 0.7 m wall, 512 bins of 16 ps, 25% random mask,
    five ellipsoid shells and a letter patch, 10 photons at the peak plus a
    uniform background at 1% of the peak."""
    n, m, wall, bin_ps = 64, 512, 0.7, 16.0
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = random_mask(n, n * n // 4, rng)
    u = np.zeros((n, n, m))
    rng_m = m * C_LIGHT * bin_ps * 1e-12 / 2
    for _ in range(5):
        add_ellipsoid_shell(u, rng, wall, wall, rng_m)
    add_letter_patch(u, rng, wall, wall, rng_m)
    return Scene("64x64x512", n, m, wall, wall, bin_ps, u, mask, 10.0, 0.1, seed)


def scene_large(seed: int = 301) -> Scene:
    """128x128 scan grid over a 2 m wall, 1024 bins of 16 ps, stride-2 grid
    with 50% dropout (12.5% of points), planes and ellipsoids, 5 photons."""
    n, m, wall, bin_ps = 128, 1024, 2.0, 16.0
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = strided_dropout_mask(n, 2, 0.5, rng)
    u = np.zeros((n, n, m))
    rng_m = m * C_LIGHT * bin_ps * 1e-12 / 2
    for _ in range(3):
        add_planar_rect(u, rng, size_lo=12, size_hi=40, depth_lo_frac=0.3, depth_hi_frac=0.8)
    for _ in range(3):
        add_ellipsoid_shell(u, rng, wall, wall, rng_m, samples=60000,
                            axis_lo=0.1, axis_hi=0.3)
    return Scene("128x128x1024", n, m, wall, wall, bin_ps, u, mask, 5.0, 0.0, seed)


def scene_custom(n: int, m: int, seed: int, wall: float = 1.0, bin_ps: float = 32.0,
                 density: float = 0.5, n_planes: int = 2, n_shells: int = 1,
                 peak: float = 20.0, background: float = 0.0) -> Scene:
    """Generic small scene for tests and uneven-size mixes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = density_mask(n, density, rng)
    u = np.zeros((n, n, m))
    rng_m = m * C_LIGHT * bin_ps * 1e-12 / 2
    lo = max(1, n // 8)
    hi = max(lo, n // 2)
    for _ in range(n_planes):
        add_planar_rect(u, rng, size_lo=lo, size_hi=hi)
    for _ in range(n_shells):
        add_ellipsoid_shell(u, rng, wall, wall, rng_m, samples=4000,
                            axis_lo=0.05 * wall, axis_hi=0.15 * wall)
    return Scene(f"{n}x{n}x{m}", n, m, wall, wall, bin_ps, u, mask, peak, background, seed)


def random_volume(shape, seed: int, dtype=np.float64) -> np.ndarray:
    """Dense U(0,1) volume for operator-level parity."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random(shape).astype(dtype)


def random_signed(shape, seed: int, dtype=np.float64) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape).astype(dtype)
