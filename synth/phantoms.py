"""Seeded phantoms: overlapping uniform ellipsoids and Gaussian "atoms".

Object model (paper Section 2): complex refractive index n = 1 + delta + i*beta,
monomorphous objects beta = sigma*delta with constant sigma.  Coordinates are
physical (metres), relative to the rotation centre, which sits at the centre
of the reconstruction cube.

Draw order inside one generator (fixed so that seeds are stable):
centres, then semi-axes, then orientations (uniform SO(3) from normalised
Gaussian quaternions), then values.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def _uniform_in_ball(rng: np.random.Generator, count: int, radius: float) -> np.ndarray:
    """`count` points uniform in the ball of `radius` (direction x radius^(1/3))."""
    g = rng.standard_normal((count, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    r = radius * rng.random(count) ** (1.0 / 3.0)
    return g * r[:, None]


def _quaternion_to_matrix(q: np.ndarray) -> np.ndarray:
    """Rotation matrices [k,3,3] from unit quaternions [k,4] = (w, x, y, z)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    m = np.empty((q.shape[0], 3, 3))
    m[:, 0, 0] = 1 - 2 * (y * y + z * z)
    m[:, 0, 1] = 2 * (x * y - w * z)
    m[:, 0, 2] = 2 * (x * z + w * y)
    m[:, 1, 0] = 2 * (x * y + w * z)
    m[:, 1, 1] = 1 - 2 * (x * x + z * z)
    m[:, 1, 2] = 2 * (y * z - w * x)
    m[:, 2, 0] = 2 * (x * z - w * y)
    m[:, 2, 1] = 2 * (y * z + w * x)
    m[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return m


@dataclass
class EllipsoidPhantom:
    """Sum of uniform ellipsoids; overlaps add.

    centres [k,3] (m), axes [k,3] semi-axes (m), rot [k,3,3] whose columns are
    the principal directions, delta [k] real decrement, sigma = beta/delta.
    """
    centres: np.ndarray
    axes: np.ndarray
    rot: np.ndarray
    delta: np.ndarray
    sigma: float

    @property
    def beta(self) -> np.ndarray:
        return self.sigma * self.delta


@dataclass
class BlobPhantom:
    """Sum of isotropic Gaussians delta0 * exp(-|r-c|^2 / (2 s^2)) ("atoms")."""
    centres: np.ndarray
    width: float
    delta0: float
    sigma: float


def draw_ellipsoids(seed: int, count: int, n_vox: int, voxel: float,
                    delta_range: tuple[float, float], sigma: float,
                    axis_range: tuple[float, float] = (0.05, 0.2),
                    support: float = 0.45) -> EllipsoidPhantom:
    """`count` ellipsoids inside the ball of radius support*N*voxel.

    Semi-axes are U[axis_range] * N * voxel; centres are drawn in the ball of
    radius (support - axis_range[1]) * N * voxel so that |c| + a_max stays
    inside the support ball whatever axes are drawn next.  delta ~ U[range]
    (pass a negative range for X-ray decrements).
    """
    rng = np.random.default_rng(seed)
    edge = n_vox * voxel
    centres = _uniform_in_ball(rng, count, (support - axis_range[1]) * edge)
    axes = rng.uniform(axis_range[0], axis_range[1], size=(count, 3)) * edge
    q = rng.standard_normal((count, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    rot = _quaternion_to_matrix(q)
    lo, hi = delta_range
    delta = rng.uniform(lo, hi, size=count)
    return EllipsoidPhantom(centres, axes, rot, delta, float(sigma))


def draw_blobs(seed: int, n_vox: int, voxel: float, density_per_m3: float,
               width: float, delta0: float, sigma: float = 0.0,
               support: float = 0.45, count: int | None = None) -> BlobPhantom:
    """Gaussian atoms uniform in the ball of radius support*N*voxel.

    The count is density x ball volume (rounded) unless given explicitly.
    """
    rng = np.random.default_rng(seed)
    radius = support * n_vox * voxel
    if count is None:
        count = int(round(density_per_m3 * 4.0 / 3.0 * np.pi * radius ** 3))
    centres = _uniform_in_ball(rng, count, radius)
    return BlobPhantom(centres, float(width), float(delta0), float(sigma))
