"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module draws random numbers and nothing else: it holds none of the
spherical-harmonics arithmetic, so neither the oracle nor the HIP path depends
on the other through it.  Every generator works in float64 with
``numpy.random.default_rng(seed)`` and returns arrays the caller may cast.

The paper times its kernels on "10 000 / 100 000 points" without stating their
distribution (Sec. III, Tables I-III); the distributions below stand in for
them and are listed with their seeds in the design notes.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "standard_normal_points",
    "shell_points",
    "precision_stress_points",
    "csr_environments",
    "standard_normal",
    "SEEDS",
]

# One seed per workload so that every consumer draws the same inputs.
SEEDS = {
    "plain_cpu": 1,        # N=1000, l_max=4, float64
    "plain_gpu": 2,        # N=1e6, l_max=8
    "plain_gpu_grad": 12,  # upstream gradient for the l_max=8 workload
    "diff": 3,             # N=4e6, l_max=6, ball 0.5..5
    "batched": 4,          # 20 000 environments
    "precision": 5,        # l_max=32 stress mix
}


def standard_normal_points(n: int, seed: int) -> np.ndarray:
    """``n`` points with iid N(0,1) Cartesian coordinates, shape [n,3], float64."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((int(n), 3))


def _isotropic_directions(rng: np.random.Generator, n: int) -> np.ndarray:
    d = rng.standard_normal((n, 3))
    nrm = np.sqrt((d * d).sum(axis=1, keepdims=True))
    # a zero draw has probability 0; guard anyway so no NaN reaches a test
    nrm[nrm == 0] = 1.0
    d[(d == 0).all(axis=1)] = (0.0, 0.0, 1.0)
    return d / nrm


def shell_points(n: int, r_min: float, r_max: float, seed: int,
                 rng: np.random.Generator | None = None) -> np.ndarray:
    """Points uniform in volume inside the shell r_min <= r <= r_max.

    Direction: a normalised Gaussian vector.  Radius: the inverse CDF of the
    r^2 density, r = (U (r_max^3 - r_min^3) + r_min^3)^(1/3).
    """
    rng = np.random.default_rng(seed) if rng is None else rng
    d = _isotropic_directions(rng, int(n))
    u = rng.random(int(n))
    r = np.cbrt(u * (r_max ** 3 - r_min ** 3) + r_min ** 3)
    return d * r[:, None]


def precision_stress_points(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """The l_max=32 stress mix: half on the unit sphere, a quarter within
    10^U(-12,-3) of the z axis, a quarter at radii 10^U(-6,3).

    Returns ``(xyz, cls)`` with ``cls`` 0 = unit sphere, 1 = near pole,
    2 = wide radius range.
    """
    rng = np.random.default_rng(seed)
    n = int(n)
    n_sph = n // 2
    n_pole = n // 4
    n_rad = n - n_sph - n_pole
    sph = _isotropic_directions(rng, n_sph)
    ex = rng.uniform(-12.0, -3.0, size=(n_pole, 2))
    sg = rng.choice([-1.0, 1.0], size=(n_pole, 3))
    pole = np.empty((n_pole, 3))
    pole[:, 0] = sg[:, 0] * 10.0 ** ex[:, 0]
    pole[:, 1] = sg[:, 1] * 10.0 ** ex[:, 1]
    pole[:, 2] = sg[:, 2]
    rad = _isotropic_directions(rng, n_rad) * (10.0 ** rng.uniform(-6.0, 3.0, size=n_rad))[:, None]
    xyz = np.concatenate([sph, pole, rad], axis=0)
    cls = np.concatenate([np.zeros(n_sph, np.int8), np.ones(n_pole, np.int8),
                          np.full(n_rad, 2, np.int8)])
    return xyz, cls


def csr_environments(n_env: int, lo: int, hi: int, r_min: float, r_max: float,
                     seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Neighbour lists for ``n_env`` atomic environments.

    Neighbour counts are uniform integers in [lo, hi]; the neighbour vectors
    are uniform in the shell r_min..r_max.  Returns ``(xyz [Ntot,3],
    offsets int64 [n_env+1])`` with offsets[0] = 0 and offsets[-1] = Ntot.
    """
    rng = np.random.default_rng(seed)
    counts = rng.integers(lo, hi + 1, size=int(n_env))
    offsets = np.zeros(int(n_env) + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    xyz = shell_points(int(offsets[-1]), r_min, r_max, seed, rng=rng)
    return xyz, offsets


def standard_normal(shape, seed: int) -> np.ndarray:
    """iid N(0,1) array of the given shape (upstream gradients and the like)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape)


def gaussian_radial_basis(xyz: np.ndarray, l_max: int, n_max: int, r_cut: float) -> np.ndarray:
    """Radial values ``R[j, l, n]`` for the expansion of environments: Gaussians
    of width r_cut/n_max centred on n_max evenly spaced radii in [0, r_cut],
    times a cosine cutoff that vanishes at r_cut, damped by 1/(1+l) so that
    every degree gets its own function.  An input of the expansion (the
    paper leaves the radial basis open), float64 [N, l_max+1, n_max]."""
    P = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    r = np.sqrt((P * P).sum(1))
    mu = np.linspace(0.0, r_cut, n_max)
    w = r_cut / n_max
    g = np.exp(-((r[:, None] - mu[None, :]) / w) ** 2)                  # [N, n]
    fc = np.where(r < r_cut, 0.5 * (np.cos(np.pi * r / r_cut) + 1.0), 0.0)
    damp = 1.0 / (1.0 + np.arange(l_max + 1))
    return (g * fc[:, None])[:, None, :] * damp[None, :, None]
