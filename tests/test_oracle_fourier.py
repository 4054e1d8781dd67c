"""Pins of the Fourier-space form of the oracle (3D gridding of eq. 11 / eq. 12,
sampling matrix, NSR filter, inverse 3D transform).

The closed forms come from geometry where the gridding is exact: a view along a
grid axis with the detector and the volume on the same lattice (N = M) and no
curvature puts every detector frequency on a grid vertex with weight one, so the
3D inverse transform must reduce to a 2D inverse DFT (numpy.fft.ifft2) of the
filtered image spectrum, constant along the beam.  The bracket itself is pinned
by the eq. 10 / 13 / 14 / 15 tests of the real-space form.
"""
import numpy as np
import pytest

import oracle
from synth import forward, phantoms, scan

RNG = np.random.default_rng(2206_09152)


def _images(n_views, m, seed):
    rng = np.random.default_rng(seed)
    return np.exp(0.05 * rng.standard_normal((n_views, m, m)))


def _geo(n, lam=1e-10, sigma=-0.3, ewald=0, eps_s=1e-14):
    return oracle.Geometry(n, n, n, 1e-10, lam, sigma, 1e-3, ewald=ewald, weight_mode="sampling",
                           eps_sampling=eps_s)


def _filtered_plane(img, dist, geo):
    """Re IDFT2[C H G] of one image (numpy.fft), H from the pinned bracket."""
    m = geo.n_pix
    q = np.fft.fftfreq(m) / geo.voxel
    q2 = q[:, None] ** 2 + q[None, :] ** 2
    chi = np.pi * geo.wavelength * dist * q2 - np.arctan(geo.sigma)
    c = geo.wavelength / (4 * np.pi * np.sqrt(1 + geo.sigma ** 2))
    g = np.fft.fft2(np.log(img))
    return g, c * oracle.ctf_bracket(chi, geo.epsilon, geo.ewald)


@pytest.mark.parametrize("n", [15, 16])
@pytest.mark.parametrize("variant", [11, 12])
def test_single_view_on_grid_reduces_to_2d_inverse_dft(n, variant):
    """Text after eq. 11 (each sample spread over eight vertices with weights summing
    to one): on-grid samples keep their value, S = 1 (Hermitian halves), and the 3D
    inverse transform of a slab k_z = 0 is the 2D inverse DFT at every depth, scaled
    by the slab thickness 1/(N Delta)."""
    geo = _geo(n)
    img = _images(1, n, 5)
    dirs = np.array([[0.0, 0.0, 1.0]])
    dist = np.array([30e-10])
    vol = oracle.fourier_reconstruct(img, dirs, dist, geo, variant=variant)
    g, f = _filtered_plane(img[0], dist[0], geo)
    plane = np.fft.ifft2(f * g).real / (n * geo.voxel)
    want = np.broadcast_to(plane, (n, n, n))
    assert np.abs(plane).max() > 0
    np.testing.assert_allclose(vol, want, rtol=0, atol=1e-9 * np.abs(plane).max())


def test_view_along_x_maps_detector_columns_to_minus_z():
    """Eq. 9 rotation about y by 90 degrees: the beam runs along +x and the
    detector column axis along -z, so delta is constant along x and
    delta[iz, iy, ix] = plane[iy, N-1-iz]."""
    n = 15
    geo = _geo(n)
    img = _images(1, n, 6)
    dirs = np.array([[1.0, 0.0, 0.0]])
    dist = np.array([30e-10])
    vol = oracle.fourier_reconstruct(img, dirs, dist, geo)
    g, f = _filtered_plane(img[0], dist[0], geo)
    plane = np.fft.ifft2(f * g).real / (n * geo.voxel)
    want = np.broadcast_to(plane[:, ::-1].T[:, :, None], (n, n, n))
    np.testing.assert_allclose(vol, want, rtol=0, atol=1e-9 * np.abs(plane).max())


def test_nsr_threshold_scales_with_inverse_sqrt_of_sampling():
    """Section 3 noise filter: two identical views give S = 2 at every vertex and the
    threshold NSR M / sqrt(2) on the CTF-corrected coefficient |H G|."""
    n = 15
    geo = _geo(n)
    img = np.repeat(_images(1, n, 7), 2, axis=0)
    dirs = np.array([[0.0, 0.0, 1.0]] * 2)
    dist = np.full(2, 30e-10)
    g, f = _filtered_plane(img[0], dist[0], geo)
    hg = np.abs(f * g) * 4 * np.pi * np.sqrt(1 + geo.sigma ** 2) / geo.wavelength
    mags = np.sort(hg.ravel())
    gap = np.flatnonzero(np.diff(mags) > 1e-6 * mags[-1])   # +-k pairs share a magnitude
    i = gap[len(gap) // 2]
    nsr = 0.5 * (mags[i] + mags[i + 1]) * np.sqrt(2.0) / n   # between two distinct magnitudes
    vol = oracle.fourier_reconstruct(img, dirs, dist, geo, nsr=nsr)
    keep = hg >= nsr * n / np.sqrt(2.0)
    assert 0 < keep.sum() < keep.size
    plane = np.fft.ifft2(f * g * keep).real / (n * geo.voxel)
    np.testing.assert_allclose(vol, np.broadcast_to(plane, (n, n, n)), rtol=0,
                               atol=1e-9 * np.abs(plane).max())
    assert np.all(oracle.fourier_reconstruct(img, dirs, dist, geo, nsr=1e9) == 0)


def test_eq12_needs_one_distance():
    geo = _geo(15)
    img = _images(2, 15, 8)
    dirs = np.array([[0.0, 0.0, 1.0]] * 2)
    with pytest.raises(ValueError):
        oracle.fourier_reconstruct(img, dirs, np.array([1e-9, 2e-9]), geo, variant=12)


def _blob_case(lam, span, n_views, dist):
    n, dx = 32, 1e-10
    ph = phantoms.draw_blobs(7, n, dx, 0, 1.6e-10, 1e-5, sigma=-1.0, count=12, support=0.3)
    ref = forward.voxelize(ph, n, dx)
    dirs = scan.single_axis(n_views, span)
    r = np.full(n_views, dist)
    imgs = forward.born_images(ph, dirs, n, dx, lam, r, -1.0)
    c = (n - 1) / 2.0
    z, y, x = np.meshgrid(*(np.arange(n) - c,) * 3, indexing="ij")
    inside = (x * x + y * y + z * z) < (n / 2.0 - 1) ** 2
    return n, dx, ref, dirs, r, imgs, inside


def _rel(a, b, mask):
    return np.linalg.norm((a - b)[mask]) / np.linalg.norm(b[mask])


def test_ct_limit_recovers_phantom_and_agrees_with_real_space_form():
    """Eq. 11 by 3D gridding in the CT limit (lambda -> 0): the sampling matrix
    builds the ramp filter by itself (text after eq. 11) and the phantom returns;
    the real-space form of the same equation agrees to the interpolation error of
    the two discretisations.  Eq. 12 coincides here (flat paraboloids)."""
    n, dx, ref, dirs, dist, imgs, inside = _blob_case(1e-13, 180.0, 90, 1e-10)
    geo = oracle.Geometry(n, n, n, dx, 1e-13, -1.0, 1e-6, ewald=1, weight_mode="sampling")
    v11 = oracle.fourier_reconstruct(imgs, dirs, dist, geo)
    v12 = oracle.fourier_reconstruct(imgs, dirs, dist, geo, variant=12)
    real = oracle.reconstruct(imgs, dirs, dist, geo)
    assert _rel(v11, ref, inside) < 0.16
    assert _rel(v12, v11, inside) < 1e-3
    assert _rel(v11, real, inside) < 0.16


def test_fourier_form_needs_curvature_when_dof_is_small():
    """Section 3 (Ewald curvature on/off) for the Fourier-space form: DOF
    Delta^2/(2 lambda) = 0.25 A, 180 views over 360 degrees, defocus 30 A."""
    n, dx, ref, dirs, dist, imgs, inside = _blob_case(2e-10, 360.0, 180, 30e-10)
    errs = {}
    for ewald in (1, 0):
        geo = oracle.Geometry(n, n, n, dx, 2e-10, -1.0, 1e-6, ewald=ewald, weight_mode="sampling")
        errs[ewald] = _rel(oracle.fourier_reconstruct(imgs, dirs, dist, geo), ref, inside)
    assert errs[1] < 0.16, errs
    assert errs[0] > 1.5 * errs[1], errs
