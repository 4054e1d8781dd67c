"""Scan geometries: unit illumination directions and the detector frames used to
simulate the images.

A view is described by its illumination direction d (unit, the beam travels
along +d) and the detector's row axis v (unit, perpendicular to d).  The
column axis is u = v x d, so (u, v, d) is right handed.  Object rotation about
the y axis by theta gives d = (sin t, 0, cos t), v = y, u = (cos t, 0, -sin t)
(paper eq. 9 rotates the object about y).
"""
from __future__ import annotations

import numpy as np


def single_axis(n: int, span_deg: float = 180.0, offset_deg: float = 0.0) -> np.ndarray:
    """n directions uniform over [offset, offset+span) rotating about y."""
    th = np.deg2rad(offset_deg + span_deg * np.arange(n) / n)
    return np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], axis=1)


def single_axis_jitter(seed: int, n: int, span_deg: float = 180.0,
                       tilt_deg: float = 5.0) -> np.ndarray:
    """Uniform single-axis angles plus a tilt tau ~ U[-tilt, tilt] out of the
    xz plane: d = (cos tau sin t, sin tau, cos tau cos t)."""
    rng = np.random.default_rng(seed)
    th = np.deg2rad(span_deg * np.arange(n) / n)
    tau = np.deg2rad(rng.uniform(-tilt_deg, tilt_deg, size=n))
    return np.stack([np.cos(tau) * np.sin(th), np.sin(tau), np.cos(tau) * np.cos(th)], axis=1)


def uniform_sphere(seed: int, n: int) -> np.ndarray:
    """n pseudo-random directions uniform on the unit sphere."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def detector_frames(dirs: np.ndarray) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Detector axes (u, v, d) for each direction.

    v is the projection of the lab y axis onto the detector plane (the lab x
    axis when d is within 1e-6 of +-y); u = v x d.
    """
    d = np.asarray(dirs, dtype=np.float64)
    ref = np.tile(np.array([0.0, 1.0, 0.0]), (d.shape[0], 1))
    near_pole = np.linalg.norm(np.cross(ref, d), axis=1) < 1e-6
    ref[near_pole] = np.array([1.0, 0.0, 0.0])
    v = ref - np.sum(ref * d, axis=1, keepdims=True) * d
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    u = np.cross(v, d)
    return u, v, d
