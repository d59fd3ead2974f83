"""Seeded synthetic inputs for the zd-tree k-NN workloads.

This module only draws random numbers (numpy PCG64 ``default_rng``); it holds
none of the method's arithmetic.  Both the GPU tests / benchmark and the CPU
oracle take their inputs from here.  Every generator returns float64 arrays
of shape (n, d), row-major.

The paper's own generators (uniform cube / square, points on a sphere,
Plummer, Kuzmin) are not available; these stand in for its uniform 2D / 3D
sets, its sphere-surface set and its two skewed sets (Section 4, "Test
data"); the skewed ones are drawn from the published densities of the
Plummer sphere and the Kuzmin disk by inverting their cumulative mass.
"""
from __future__ import annotations

import numpy as np

UNIT2 = (np.zeros(2), np.ones(2))
UNIT3 = (np.zeros(3), np.ones(3))


def uniform(n: int, dim: int, seed: int) -> np.ndarray:
    """n points uniform in [0,1)^dim."""
    return np.random.default_rng(seed).random((n, dim))


# -- the benchmark workloads --------------------------------------------------

def uniform2d_10k(n: int = 10_000, seed: int = 0) -> np.ndarray:
    """2D uniform in [0,1)^2, leaf size 16, all-points k=10."""
    return uniform(n, 2, seed)


def uniform3d_10m_updates(n: int = 10_000_000, m: int = 1_000_000):
    """3D uniform build set P (seed 0), insert batch Q (seed 1, ids n..n+m-1),
    delete ids D: m distinct ids drawn from all n+m after the insert (seed 2)."""
    P = uniform(n, 3, 0)
    Q = uniform(m, 3, 1)
    D = np.random.default_rng(2).choice(n + m, m, replace=False).astype(np.int32)
    return P, Q, D


def spheres_10m(n: int = 10_000_000, n_spheres: int = 64, noise: float = 1e-4,
                 background: float = 0.01, seed: int = 0) -> np.ndarray:
    """Points on n_spheres sphere surfaces (radius log-uniform in [0.01, 0.2],
    centres uniform in [0,1)^3) with Gaussian radial noise, plus a uniform
    background fraction; shuffled."""
    rng = np.random.default_rng(seed)
    centres = rng.random((n_spheres, 3))
    radii = np.exp(rng.uniform(np.log(0.01), np.log(0.2), n_spheres))
    nb = int(round(n * background))
    ns = n - nb
    which = rng.integers(0, n_spheres, ns)
    v = rng.normal(size=(ns, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = radii[which] + rng.normal(0.0, noise, ns)
    pts = centres[which] + v * r[:, None]
    bg = rng.random((nb, 3))
    allp = np.concatenate([pts, bg])
    return allp[rng.permutation(n)]


def _unit_directions(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def plummer(n: int, seed: int = 0, a: float = 0.01, x_max: float = 0.999,
            centre=(0.5, 0.5, 0.5)) -> np.ndarray:
    """Plummer sphere of scale radius a: density proportional to
    (1 + r^2/a^2)^(-5/2), so the mass inside radius r is the fraction
    X = r^3 / (r^2 + a^2)^(3/2) and r = a / sqrt(X^(-2/3) - 1).  X is drawn
    uniform in (0, x_max] (x_max < 1 truncates the unbounded halo), the
    direction uniform on the sphere."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, x_max, n)
    X = np.maximum(X, 1e-300)
    r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    return np.asarray(centre)[None, :] + _unit_directions(rng, n) * r[:, None]


def kuzmin(n: int, seed: int = 0, a: float = 0.01, x_max: float = 0.999,
           centre=(0.5, 0.5, 0.5)) -> np.ndarray:
    """Kuzmin disk of scale length a in the plane z = centre_z: surface
    density proportional to (R^2 + a^2)^(-3/2), so the mass inside radius R
    is the fraction X = 1 - a / sqrt(R^2 + a^2) and
    R = a * sqrt(1 / (1 - X)^2 - 1).  X is drawn uniform in [0, x_max]
    (x_max < 1 truncates the heavy tail), the angle uniform."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, x_max, n)
    R = a * np.sqrt(1.0 / (1.0 - X) ** 2 - 1.0)
    th = rng.uniform(0.0, 2.0 * np.pi, n)
    c = np.asarray(centre, dtype=np.float64)
    out = np.empty((n, 3))
    out[:, 0] = c[0] + R * np.cos(th)
    out[:, 1] = c[1] + R * np.sin(th)
    out[:, 2] = c[2]
    return out


def forest_4096_clouds(n_clouds: int = 4096, min_size: int = 1000, max_size: int = 65536,
                seed: int = 0):
    """Independent 3D clouds, sizes log-uniform in [min_size, max_size], each a
    Gaussian mixture of 1..8 equal-weight components (sigma in [0.02, 0.1],
    means uniform in [0,1)^3).  Returns (points (N, 3), offsets int64 [C+1])."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(np.log(min_size), np.log(max_size), n_clouds)))
    sizes = sizes.astype(np.int64)
    offsets = np.zeros(n_clouds + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    out = np.empty((int(offsets[-1]), 3))
    for c in range(n_clouds):
        m = int(rng.integers(1, 9))
        counts = rng.multinomial(int(sizes[c]), [1.0 / m] * m)
        means = rng.random((m, 3))
        sig = rng.uniform(0.02, 0.1, m)
        parts = [means[j] + sig[j] * rng.normal(size=(counts[j], 3)) for j in range(m)]
        out[offsets[c]:offsets[c + 1]] = np.concatenate(parts)
    return out, offsets


def uniform3d_1m_rounds(n: int = 1_000_000, rounds: int = 10, frac: float = 0.01,
                   n_fd: int = 1000):
    """Differentiable workload: P (seed 0); finite-difference sample of
    (point id, coordinate) pairs (seed 1); per round r = 1..rounds an insert
    batch (seed 10+r) and a delete-draw generator (seed 20+r)."""
    P = uniform(n, 3, 0)
    rng = np.random.default_rng(1)
    fd = np.stack([rng.integers(0, n, n_fd), rng.integers(0, 3, n_fd)], axis=1)
    m = int(round(n * frac))
    inserts = [uniform(m, 3, 10 + r) for r in range(1, rounds + 1)]
    delete_rngs = [np.random.default_rng(20 + r) for r in range(1, rounds + 1)]
    return P, fd, inserts, delete_rngs, m


# -- small adversarial inputs for parity tests -------------------------------

def grid_points(shape, scale_exp: int = 4, seed: int = 0) -> np.ndarray:
    """All points of an integer grid, scaled by 2^-scale_exp (exactly
    representable, so squared distances are exact and ties abound), in a
    seeded random order."""
    axes = [np.arange(s, dtype=np.float64) for s in shape]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, len(shape))
    g = g * 2.0 ** (-scale_exp)
    return g[np.random.default_rng(seed).permutation(g.shape[0])]


def lattice_1d(n: int, dim: int, scale_exp: int = 3) -> np.ndarray:
    """Points i * 2^-scale_exp on the first axis, i = 0..n-1, in id order."""
    p = np.zeros((n, dim))
    p[:, 0] = np.arange(n, dtype=np.float64) * 2.0 ** (-scale_exp)
    return p


def with_duplicates(n: int, dim: int, n_distinct: int, seed: int) -> np.ndarray:
    """n points drawn (with repetition) from n_distinct random locations."""
    rng = np.random.default_rng(seed)
    base = rng.random((n_distinct, dim))
    return base[rng.integers(0, n_distinct, n)]


def collinear(n: int, dim: int, seed: int) -> np.ndarray:
    """n random points on a segment through the unit cube."""
    rng = np.random.default_rng(seed)
    t = rng.random(n)
    a = rng.random(dim)
    b = rng.random(dim)
    return a[None, :] + t[:, None] * (b - a)[None, :]


def clustered_small(n: int, dim: int, seed: int) -> np.ndarray:
    """A few tight Gaussian clusters plus some uniform background."""
    rng = np.random.default_rng(seed)
    m = 4
    centres = rng.random((m, dim))
    which = rng.integers(0, m, n)
    p = centres[which] + rng.normal(0.0, 1e-3, (n, dim))
    bg = rng.random(n) < 0.05
    p[bg] = rng.random((int(bg.sum()), dim))
    return p
