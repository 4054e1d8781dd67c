"""Named synthetic workloads shaped like the paper's regimes.

Each workload is a reconstruction problem: volume edge N (voxels), detector
edge M, depth planes K, n views, voxel = pixel size, wavelength, distance R
from the rotation-centre plane to the detector, sigma = beta/delta, the
Tikhonov epsilon of eq. (11) and the density-weight mode.  `make_workload`
draws the phantom and simulates the images (float64; callers cast to float32
for the device and hand the same float32 values to the oracle).

Seeds: numpy default_rng(220609151 + index) for the phantom, +1000 for scan
jitter / random directions.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from . import forward, phantoms, scan

SEED_BASE = 220609151


@dataclass(frozen=True)
class Workload:
    name: str
    index: int
    n_vox: int
    n_views: int
    voxel: float
    wavelength: float
    dist: float
    sigma: float
    epsilon: float
    weight_mode: str          # "ramp_axis" | "ramp_iso" | "sampling"
    ewald: int = 1
    n_pix: int = 0            # 0 -> n_vox
    n_planes: int = 0         # 0 -> n_vox
    span_deg: float = 180.0
    geometry: str = "axis"    # "axis" | "axis_jitter" | "sphere"
    image_model: str = "fresnel"  # "fresnel" (projection approx) | "born" (eq. 8)
    phantom: str = "ellipsoids"   # "ellipsoids" | "blobs"
    n_ellipsoids: int = 10
    delta_range: tuple = (1e-7, 1e-6)
    blob_width: float = 0.75e-10
    blob_delta0: float = 5e-5
    blob_density: float = 40.0 / 1000.0 * 1e30   # atoms per m^3 (40 per 1000 A^3)
    blob_count: int | None = None
    eps_sampling: float = 1e-3
    i_in: float = 1.0

    @property
    def M(self) -> int:
        return self.n_pix or self.n_vox

    @property
    def K(self) -> int:
        return self.n_planes or self.n_vox

    @property
    def updates(self) -> int:
        """Voxel-angle updates of one reconstruction: N^3 * n."""
        return self.n_vox ** 3 * self.n_views

    def scaled(self, **kw) -> "Workload":
        return replace(self, **kw)


WORKLOADS = {
    # CT/PCT limit: 64^3, 1 um voxels, 10 ellipsoids delta~U[1e-7,1e-6], beta = delta/100,
    # 90 views over [0,180), lambda 0.1 nm, R 0.1 m, projection approximation + Fresnel.
    "ct_pct_64": Workload("ct_pct_64", 0, 64, 90, 1e-6, 1e-10, 0.1, 0.01, 1e-3, "ramp_axis",
                          span_deg=180.0, image_model="fresnel", phantom="ellipsoids",
                          n_ellipsoids=10, delta_range=(1e-7, 1e-6)),
    # DT with Ewald curvature: 128^3, 1 A voxels, lambda 0.0197 A (DOF ~25 A), Gaussian atoms
    # at 40 per 1000 A^3, 180 views over [0,180), first-Born eq. (8), defocus 500 A.
    "dt_ewald_128": Workload("dt_ewald_128", 1, 128, 180, 1e-10, 0.0197e-10, 500e-10, 0.0, 1e-3,
                             "ramp_axis", span_deg=180.0, image_model="born", phantom="blobs"),
    # Mixed-precision regime: 256^3, 20 nm voxels, lambda 1 nm, 360 views over [0,180) with
    # +-5 deg tilt jitter, 30 X-ray ellipsoids (delta < 0, sigma = -0.1), first-Born images.
    "xray_jitter_256": Workload("xray_jitter_256", 2, 256, 360, 20e-9, 1e-9, 5e-6, -0.1, 1e-3,
                                "sampling", geometry="axis_jitter", image_model="born",
                                phantom="ellipsoids", n_ellipsoids=30, delta_range=(-1e-5, -1e-6)),
}


def make_dirs(w: Workload) -> np.ndarray:
    if w.geometry == "axis":
        return scan.single_axis(w.n_views, w.span_deg)
    if w.geometry == "axis_jitter":
        return scan.single_axis_jitter(SEED_BASE + w.index + 1000, w.n_views, w.span_deg)
    if w.geometry == "sphere":
        return scan.uniform_sphere(SEED_BASE + w.index + 1000, w.n_views)
    raise ValueError(w.geometry)


def make_phantom(w: Workload):
    seed = SEED_BASE + w.index
    if w.phantom == "ellipsoids":
        return phantoms.draw_ellipsoids(seed, w.n_ellipsoids, w.n_vox, w.voxel,
                                        w.delta_range, w.sigma)
    if w.phantom == "blobs":
        return phantoms.draw_blobs(seed, w.n_vox, w.voxel, w.blob_density, w.blob_width,
                                   w.blob_delta0, w.sigma, count=w.blob_count)
    raise ValueError(w.phantom)


def make_workload(w: Workload, device: str | None = None):
    """(phantom, dirs [n,3], dist [n], images float64 [n,M,M])."""
    ph = make_phantom(w)
    dirs = make_dirs(w)
    dist = np.full(w.n_views, w.dist)
    if w.image_model == "fresnel":
        imgs = forward.project_fresnel_images(ph, dirs, w.M, w.voxel, w.wavelength, dist, w.i_in)
    elif w.image_model == "born":
        imgs = forward.born_images(ph, dirs, w.M, w.voxel, w.wavelength, dist, w.sigma,
                                   w.i_in, device=device)
    else:
        raise ValueError(w.image_model)
    return ph, dirs, dist, imgs


# Batched uneven jobs: 64 independent reconstructions in the CT/PCT regime of ct_pct_64,
# volume edges drawn from {64, 96, 128, 160, 192} (M = K = N), view counts from
# {60, ..., 240}; jobs 0-31 are single-axis scans over [0,180) with the axis ramp,
# jobs 32-63 directions uniform on the sphere with sampling-matrix weights.
BATCH_SIZES = (64, 96, 128, 160, 192)


def batch_jobs(count: int = 64, seed: int = SEED_BASE + 3, sizes=BATCH_SIZES, views=(60, 240)):
    """Job table of the batched workload: a list of Workloads (phantom seed per job)."""
    rng = np.random.default_rng(seed)
    n_vox = rng.choice(np.asarray(sizes), size=count)
    n_views = rng.integers(views[0], views[1] + 1, size=count)
    base = WORKLOADS["ct_pct_64"]
    jobs = []
    for j in range(count):
        axis = j < count // 2
        jobs.append(base.scaled(name=f"batch_job{j}", index=100 + j, n_vox=int(n_vox[j]), n_views=int(n_views[j]),
                                geometry="axis" if axis else "sphere",
                                weight_mode="ramp_axis" if axis else "sampling"))
    return jobs
