"""Seeded small problems shared by the GPU parity tests and smoke().

Every problem is described once; the oracle and the HIP path receive the same
float32 images (the oracle reads them as float64) and the same geometry.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from synth import forward, phantoms, scan


@dataclass
class Problem:
    name: str
    n_vox: int
    n_pix: int
    n_planes: int
    voxel: float
    wavelength: float
    sigma: float
    epsilon: float
    ewald: int
    weight_mode: str
    dirs: np.ndarray
    dist: np.ndarray
    images: np.ndarray            # float32 [n, M, M]
    vaxes: np.ndarray | None = None
    i_in: float = 1.0             # flat-field intensity the images were made with
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.dirs.shape[0]

    def oracle_geometry(self):
        import oracle
        return oracle.Geometry(self.n_vox, self.n_pix, self.n_planes if self.ewald else 1, self.voxel,
                               self.wavelength, self.sigma, self.epsilon, ewald=self.ewald,
                               weight_mode=self.weight_mode, i_in=self.i_in)

    def params(self, **kw):
        from paper_2206_09151_amd import tomo
        return tomo.Params(n_vox=self.n_vox, n_angles=self.n, voxel_size=self.voxel,
                           wavelength=self.wavelength, sigma=self.sigma, epsilon=self.epsilon,
                           n_pix=self.n_pix, n_planes=self.n_planes if self.ewald else 0, ewald=self.ewald,
                           weight_mode=self.weight_mode, i_in=self.i_in, **kw)


def _born(seed, n_vox, n_pix, dx, lam, dirs, dist, sigma, width=1.2, count=20, i_in=1.0):
    ph = phantoms.draw_blobs(seed, n_vox, dx, 0.0, width * dx, 2e-5, sigma=sigma, count=count, support=0.4)
    return forward.born_images(ph, dirs, n_pix, dx, lam, dist, sigma, i_in).astype(np.float32)


def pole_directions(seed: int, n: int) -> np.ndarray:
    """Directions with the detector-frame rule's special cases: exactly +y and -y, one
    within 1e-7 of +y (still taken as a pole), one 2e-6 away (not a pole), then
    directions uniform on the sphere."""
    e = 1e-7
    near = np.array([[e, np.sqrt(1 - e * e), 0.0], [0.0, np.sqrt(1 - 4e-12), -2e-6]])
    fixed = np.vstack([[0.0, 1.0, 0.0], [0.0, -1.0, 0.0], near])
    return np.vstack([fixed, scan.uniform_sphere(seed, n - len(fixed))])


def make(name: str) -> Problem:
    dx = 1e-10
    if name == "axis32":
        n, N, M, K = 24, 32, 32, 32
        dirs = scan.single_axis(n, 180.0)
        dist = np.full(n, 50e-10)
        lam, sig = 0.2e-10, 0.1
        imgs = _born(11, N, M, dx, lam, dirs, dist, sig)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_axis", dirs, dist, imgs)
    if name == "ragged44":
        n, N, M, K = 13, 44, 48, 44
        dirs = scan.single_axis(n, 360.0, offset_deg=7.0)
        dist = np.linspace(40e-10, 60e-10, n)
        lam, sig = 0.1e-10, -0.2
        imgs = _born(12, N, M, dx, lam, dirs, dist, sig)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_axis", dirs, dist, imgs)
    if name == "sphere45":
        n, N, M, K = 11, 45, 48, 45
        dirs = scan.uniform_sphere(13, n)
        dist = np.full(n, 30e-10)
        lam, sig = 0.1e-10, 0.0
        imgs = _born(13, N, M, dx, lam, dirs, dist, sig)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_iso", dirs, dist, imgs)
    if name == "sphere70":
        # 70 directions on the sphere, all in one gridding launch (box origins are formed for
        # 64 views at a time)
        n, N, M, K = 70, 20, 24, 20
        dirs = scan.uniform_sphere(15, n)
        dist = np.full(n, 30e-10)
        lam, sig = 0.1e-10, 0.0
        imgs = _born(15, N, M, dx, lam, dirs, dist, sig)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_iso", dirs, dist, imgs)
    if name == "pct64":
        n, N, M = 30, 64, 64
        dirs = scan.single_axis(n, 180.0)
        dist = np.full(n, 0.1)
        lam, sig, px = 1e-10, 0.01, 1e-6
        ph = phantoms.draw_ellipsoids(14, 6, N, px, (1e-8, 5e-8), sig)
        imgs = forward.project_fresnel_images(ph, dirs, M, px, lam, dist).astype(np.float32)
        return Problem(name, N, M, 1, px, lam, sig, 1e-3, 0, "ramp_axis", dirs, dist, imgs)
    if name == "sampling32":
        n, N, M, K = 16, 32, 32, 32
        dirs = scan.single_axis_jitter(15, n, 180.0, 5.0)
        dist = np.full(n, 50e-10)
        lam, sig = 0.1e-10, -0.1
        imgs = _born(15, N, M, dx, lam, dirs, dist, sig)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "sampling", dirs, dist, imgs)
    if name == "oddk16":
        n, N, M, K = 5, 16, 16, 9
        dirs = scan.single_axis(n, 180.0, offset_deg=3.0)
        dist = np.full(n, 20e-10)
        lam, sig = 0.3e-10, 0.2
        imgs = _born(16, N, M, dx, lam, dirs, dist, sig, count=6)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_axis", dirs, dist, imgs)
    if name == "narrow48":
        # detector narrower than the volume (M < N): voxel rows beyond the detector get nothing
        n, N, M, K = 9, 48, 32, 48
        dirs = scan.single_axis(n, 180.0, offset_deg=5.0)
        dist = np.full(n, 40e-10)
        lam, sig = 0.1e-10, 0.1
        imgs = _born(25, N, M, dx, lam, dirs, dist, sig, count=24)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_axis", dirs, dist, imgs)
    if name == "m80":
        n, N, M, K = 4, 80, 80, 80
        dirs = scan.single_axis(n, 180.0)
        dist = np.full(n, 60e-10)
        lam, sig = 0.05e-10, 0.0
        imgs = _born(17, N, M, dx, lam, dirs, dist, sig, count=40)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_axis", dirs, dist, imgs)
    if name == "m96":
        n, N, M, K = 3, 96, 96, 96
        dirs = scan.single_axis(n, 180.0)
        dist = np.full(n, 60e-10)
        lam, sig = 0.05e-10, 0.0
        imgs = _born(18, N, M, dx, lam, dirs, dist, sig, count=40)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_axis", dirs, dist, imgs)
    if name == "vaxes32":
        n, N, M, K = 6, 32, 32, 32
        dirs = scan.uniform_sphere(19, n)
        rng = np.random.default_rng(1019)
        vax = rng.standard_normal((n, 3))
        dist = np.full(n, 40e-10)
        lam, sig = 0.1e-10, 0.3
        imgs = _born(19, N, M, dx, lam, dirs, dist, sig)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_iso", dirs, dist, imgs, vaxes=vax)
    if name == "m256":
        # 256-pixel detector (2 x 2 block-split FFT path) over a small volume, single axis
        n, N, M, K = 6, 48, 256, 48
        dirs = scan.single_axis(n, 180.0, offset_deg=11.0)
        dist = np.full(n, 80e-10)
        lam, sig = 0.05e-10, -0.1
        imgs = _born(20, N, M, dx, lam, dirs, dist, sig, count=30)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_axis", dirs, dist, imgs)
    if name == "m256sph":
        # 256-pixel detector, directions on the sphere (general trilinear path), odd K
        n, N, M, K = 5, 40, 256, 41
        dirs = scan.uniform_sphere(21, n)
        dist = np.full(n, 80e-10)
        lam, sig = 0.05e-10, 0.2
        imgs = _born(21, N, M, dx, lam, dirs, dist, sig, count=30)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_iso", dirs, dist, imgs)
    if name == "m160":
        # 160-pixel detector (direct 160-point transforms, 40 values per thread), odd K
        n, N, M, K = 5, 40, 160, 41
        dirs = scan.single_axis(n, 180.0, offset_deg=4.0)
        dist = np.full(n, 70e-10)
        lam, sig = 0.05e-10, 0.1
        imgs = _born(23, N, M, dx, lam, dirs, dist, sig, count=24)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_axis", dirs, dist, imgs)
    if name == "m192":
        # 192-pixel detector (direct 192-point transforms, 48 values per thread), tilted frames
        n, N, M, K = 4, 48, 192, 48
        dirs = scan.uniform_sphere(24, n)
        dist = np.full(n, 70e-10)
        lam, sig = 0.05e-10, -0.2
        imgs = _born(24, N, M, dx, lam, dirs, dist, sig, count=24)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_iso", dirs, dist, imgs)
    if name == "n256":
        # 256^3 Fourier grid (largest inverse-FFT size), few views
        n, N, M, K = 4, 256, 256, 8
        dirs = scan.uniform_sphere(22, n)
        dist = np.full(n, 80e-10)
        lam, sig = 0.05e-10, -0.1
        imgs = _born(22, N, M, dx, lam, dirs, dist, sig, count=30)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_iso", dirs, dist, imgs)
    if name == "iin32":
        # flat field I_in = 0.7; sampling-matrix weights and curvature keep the q = 0 term,
        # so a dropped or inverted I_in changes the result
        n, N, M, K = 12, 32, 32, 32
        dirs = scan.single_axis_jitter(26, n, 180.0, 5.0)
        dist = np.full(n, 50e-10)
        lam, sig = 0.1e-10, 0.0
        imgs = _born(26, N, M, dx, lam, dirs, dist, sig, i_in=0.7)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "sampling", dirs, dist, imgs, i_in=0.7)
    if name == "m256iin":
        # I_in = 0.7 on the 256-pixel detector path
        n, N, M, K = 4, 40, 256, 40
        dirs = scan.single_axis_jitter(27, n, 180.0, 5.0)
        dist = np.full(n, 80e-10)
        lam, sig = 0.05e-10, 0.0
        imgs = _born(27, N, M, dx, lam, dirs, dist, sig, count=24, i_in=0.7)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "sampling", dirs, dist, imgs, i_in=0.7)
    if name == "pole24":
        # illumination along +-y and within 1e-6 of it: the frame takes lab x as reference
        n, N, M, K = 8, 24, 32, 24
        dirs = pole_directions(28, n)
        dist = np.full(n, 40e-10)
        lam, sig = 0.1e-10, 0.1
        imgs = _born(28, N, M, dx, lam, dirs, dist, sig, count=12)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_iso", dirs, dist, imgs)
    if name == "m128":
        # the headline detector size (radix 16 x 8 FFT) at the full volume, few views
        n, N, M, K = 4, 128, 128, 128
        dirs = scan.single_axis(n, 180.0, offset_deg=9.0)
        dist = np.full(n, 60e-10)
        lam, sig = 0.0197e-10, 0.0
        imgs = _born(29, N, M, dx, lam, dirs, dist, sig, count=60)
        return Problem(name, N, M, K, dx, lam, sig, 1e-3, 1, "ramp_axis", dirs, dist, imgs)
    raise KeyError(name)


def smooth_sizes(lo: int = 16, hi: int = 256) -> list:
    """Every M = 2^a 3^b 5^c in [lo, hi]: the detector sizes the library supports."""
    out = []
    for m in range(lo, hi + 1):
        r = m
        for f in (2, 3, 5):
            while r % f == 0:
                r //= f
        if r == 1:
            out.append(m)
    return out


def size_problem(m: int, n: int = 3) -> Problem:
    """A small problem on an M-pixel detector: a volume of edge N = min(M, 40) or one less
    (so that both parities of M - N occur), 12 depth planes, n views (3 unless given) --
    single-axis with the axis ramp for even M, directions on the sphere with the isotropic
    ramp for odd M."""
    dx = 1e-10
    n_vox = min(m, 40) - (m % 4 == 2)
    if m % 2 == 0:
        dirs = scan.single_axis(n, 180.0, offset_deg=5.0 + m % 7)
        mode = "ramp_axis"
    else:
        dirs = scan.uniform_sphere(300 + m, n)
        mode = "ramp_iso"
    dist = np.full(n, 60e-10)
    lam, sig = 0.05e-10, 0.1
    imgs = _born(300 + m, n_vox, m, dx, lam, dirs, dist, sig, count=16)
    return Problem(f"size{m}" if n == 3 else f"size{m}x{n}", n_vox, m, 12, dx, lam, sig, 1e-3, 1, mode, dirs, dist,
                   imgs)


def fourier_size_problem(n: int) -> Problem:
    """The Fourier-space form on an n^3 grid (N = M = n), 3 views on the sphere."""
    dx = 1e-10
    dirs = scan.uniform_sphere(500 + n, 3)
    dist = np.full(3, 60e-10)
    lam, sig = 0.05e-10, 0.1
    imgs = _born(500 + n, n, n, dx, lam, dirs, dist, sig, count=16)
    return Problem(f"fsize{n}", n, n, 8, dx, lam, sig, 1e-3, 1, "ramp_iso", dirs, dist, imgs)


SMALL = ["axis32", "ragged44", "sphere45", "pct64", "sampling32", "oddk16", "m80", "m96", "vaxes32",
         "m256", "m256sph", "m160", "m192", "narrow48", "iin32", "m256iin", "pole24", "m128"]
