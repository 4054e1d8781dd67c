"""Seeded synthetic inputs: phantoms, scan geometries and forward-simulated images.

This package is shared input plumbing.  It simulates the *measurement* (the
forward problem: projection approximation with Fresnel propagation, or the
first-Born Ewald-sphere model) and contains none of the reconstruction
arithmetic.  Both the FP64 oracle and the HIP path consume what it produces;
neither is imported here.
"""
from .phantoms import EllipsoidPhantom, BlobPhantom, draw_ellipsoids, draw_blobs
from .scan import single_axis, single_axis_jitter, uniform_sphere, detector_frames
from .forward import (project_fresnel_images, born_images, voxelize)
from .workloads import WORKLOADS, Workload, make_workload

__all__ = [
    "EllipsoidPhantom", "BlobPhantom", "draw_ellipsoids", "draw_blobs",
    "single_axis", "single_axis_jitter", "uniform_sphere", "detector_frames",
    "project_fresnel_images", "born_images", "voxelize",
    "WORKLOADS", "Workload", "make_workload",
]
