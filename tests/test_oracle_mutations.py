"""Plausible mistakes planted in the oracle (on the CPU) must fail at least one pin.

Each case patches one oracle function with a typical slip -- a flipped sign, a
transposed operand, a dropped term, a wrong index -- and runs the pin that is
meant to catch it.
"""
import numpy as np
import pytest

import oracle
import oracle.utr as utr
import test_oracle_limits as limits
import test_oracle_pins as pins


def _flip_propagator(P, geo):
    if not geo.ewald:
        return np.fft.ifft2(P).real[None]
    m = geo.n_pix
    q = utr.signed_index(m) / (m * geo.voxel)
    q2 = q[:, None] ** 2 + q[None, :] ** 2
    z = utr.plane_depths(geo)
    prop = np.exp(+1j * np.pi * geo.wavelength * z[:, None, None] * q2[None])  # wrong sign
    return np.fft.ifft2(P[None] * prop, axes=(-2, -1)).real


def _transposed_spectrum(g):
    return np.swapaxes(np.fft.fft2(g, axes=(-2, -1)), -1, -2)


def _bracket_wrong_imag_sign(chi, eps, ewald):
    s, c = np.sin(chi), np.cos(chi)
    re = s / (s * s + eps)
    return re.astype(complex) if not ewald else re + 1j * c / (c * c + eps)


def _bracket_dropped_imag(chi, eps, ewald):
    s = np.sin(chi)
    return (s / (s * s + eps)).astype(complex)


_orig_frames = utr.frames


def _frames_left_handed(dirs, vaxes=None):
    u, v, d = _orig_frames(dirs, vaxes)
    return -u, v, d


_orig_depths = utr.plane_depths


def _depths_off_by_one(geo):
    return _orig_depths(geo) + geo.voxel


def _ramp_wrong_axis(u, v, d, geo):
    m = geo.n_pix
    q = utr.signed_index(m) / (m * geo.voxel)
    qy, _ = np.meshgrid(q, q, indexing="ij")
    return utr.axis_angle_weights(d)[:, None, None] * np.abs(qy)[None]


def _contrast_inverted(images, i_in=1.0):
    return np.log(i_in / np.asarray(images, dtype=np.float64))


def _contrast_without_flat_field(images, i_in=1.0):
    return np.log(np.asarray(images, dtype=np.float64))


def _lin_taps_swapped(f, size):
    i0 = np.floor(f).astype(np.int64)
    t = f - i0
    out = []
    for c in (0, 1):
        i = i0 + c
        w = (1.0 - t) if c else t                     # weights on the wrong neighbours
        ok = (i >= 0) & (i < size)
        out.append((np.clip(i, 0, size - 1), np.where(ok, w, 0.0)))
    return out


def _bracket_cos_for_sin(chi, eps, ewald):
    c = np.cos(chi)
    re = c / (c * c + eps)                            # the wrong CTF branch in the real part
    return re.astype(complex) if not ewald else re - 1j * c / (c * c + eps)


MUTATIONS = [
    ("contrast", _contrast_inverted, limits.test_contrast_is_log_of_intensity_over_flat_field),
    ("contrast", _contrast_without_flat_field, limits.test_flat_field_intensity_enters_as_a_divisor),
    ("_lin_taps", _lin_taps_swapped, lambda: limits.test_pct_limit_equals_textbook_filtered_backprojection(15, 16)),
    ("ctf_bracket", _bracket_cos_for_sin, lambda: limits.test_pct_limit_equals_textbook_filtered_backprojection(16, 16)),
    ("frames", _frames_left_handed, limits.test_central_sections_of_the_reconstruction_match_projected_delta),
    ("plane_depths", _depths_off_by_one, limits.test_curvature_terms_cancel_between_opposite_views),
    ("depth_planes", _flip_propagator, pins.test_ewald_curvature_matters_when_dof_is_small),
    ("spectrum", _transposed_spectrum, pins.test_ct_limit_recovers_phantom_from_fresnel_images),
    ("ctf_bracket", _bracket_wrong_imag_sign, pins.test_bracket_solves_opposite_pair_eq10),
    ("ctf_bracket", _bracket_dropped_imag, pins.test_ewald_curvature_matters_when_dof_is_small),
    ("frames", _frames_left_handed, pins.test_frames_rotation_about_y),
    ("frames", _frames_left_handed, pins.test_ct_limit_recovers_phantom_from_fresnel_images),
    ("plane_depths", _depths_off_by_one, pins.test_grid_aligned_reconstruction_equals_direct_backpropagation),
    ("density_weights", _ramp_wrong_axis, pins.test_ct_limit_recovers_phantom_from_fresnel_images),
]


@pytest.mark.parametrize("name,bad,pin", MUTATIONS, ids=[f"{m[0]}-{getattr(m[1], '__name__', '')}-{i}" for i, m in enumerate(MUTATIONS)])
def test_planted_mistake_is_caught(monkeypatch, name, bad, pin):
    monkeypatch.setattr(utr, name, bad)
    if hasattr(oracle, name):
        monkeypatch.setattr(oracle, name, bad)
    with pytest.raises(AssertionError):
        pin()


# ------------------------------------------------------------------ Fourier-space form
import oracle.fourier as fou  # noqa: E402
import test_oracle_fourier as fpins  # noqa: E402


def _spectra_no_centring(images, geo):
    return utr.spectrum(utr.contrast(images, geo.i_in))


def _grid_no_conjugate(values, u, v, d, geo):
    n = geo.n_vox
    pts = utr._paraboloid_points(u, v, d, geo).reshape(-1, 3)
    val = np.asarray(values).reshape(-1)
    F = np.zeros(n ** 3, dtype=complex)
    S = np.zeros(n ** 3)
    for sign in (1.0, -1.0):
        for flat, wgt, ok in utr._trilinear_taps(sign * pts, n):
            np.add.at(F, flat[ok], 0.5 * wgt[ok] * val[ok])        # reflection not conjugated
            np.add.at(S, flat[ok], 0.5 * wgt[ok])
    return F.reshape(n, n, n), S.reshape(n, n, n)


_orig_inverse = fou.inverse_dft3


def _inverse_xy_swapped(A, geo):
    return np.swapaxes(_orig_inverse(A, geo), 1, 2)


def _normalise_by_s_squared(F, S, geo, nsr=0.0):
    A = F / (S * S + geo.eps_sampling)
    if nsr > 0:
        thr = np.where(S > 0, nsr * geo.n_pix / np.sqrt(np.maximum(S, 1e-300)), np.inf)
        A = np.where(np.abs(A) >= thr, A, 0.0)
    return A


def _nsr_over_s(F, S, geo, nsr=0.0):
    A = F * S / (S * S + geo.eps_sampling)
    if nsr > 0:
        thr = np.where(S > 0, nsr * geo.n_pix / np.maximum(S, 1e-300), np.inf)   # S, not sqrt(S)
        A = np.where(np.abs(A) >= thr, A, 0.0)
    return A


def _paraboloid_flipped(u, v, d, geo):
    m = geo.n_pix
    q = utr.signed_index(m) / (m * geo.voxel)
    qy, qx = np.meshgrid(q, q, indexing="ij")
    qz = +geo.ewald * geo.wavelength * (qx ** 2 + qy ** 2) / 2.0                 # wrong sign
    p = (qx[None, :, :, None] * u[:, None, None, :] + qy[None, :, :, None] * v[:, None, None, :]
         + qz[None, :, :, None] * d[:, None, None, :])
    return p * (geo.n_vox * geo.voxel)


def _inverse_no_pixel_area(A, geo):
    return _orig_inverse(A, geo) / geo.voxel ** 2


def _single_view_even():
    fpins.test_single_view_on_grid_reduces_to_2d_inverse_dft(16, 11)


FOURIER_MUTATIONS = [
    ("centred_spectra", _spectra_no_centring, _single_view_even),
    ("fourier_grid", _grid_no_conjugate, _single_view_even),
    ("inverse_dft3", _inverse_xy_swapped, _single_view_even),
    ("inverse_dft3", _inverse_no_pixel_area, _single_view_even),
    ("fourier_normalise", _normalise_by_s_squared, fpins.test_nsr_threshold_scales_with_inverse_sqrt_of_sampling),
    ("fourier_normalise", _nsr_over_s, fpins.test_nsr_threshold_scales_with_inverse_sqrt_of_sampling),
    ("_paraboloid_points", _paraboloid_flipped, fpins.test_fourier_form_needs_curvature_when_dof_is_small),
]


@pytest.mark.parametrize("name,bad,pin", FOURIER_MUTATIONS,
                         ids=[f"{m[0]}-{m[1].__name__}" for m in FOURIER_MUTATIONS])
def test_planted_fourier_mistake_is_caught(monkeypatch, name, bad, pin):
    monkeypatch.setattr(fou, name, bad)
    with pytest.raises(AssertionError):
        pin()


# ------------------------------------------------------------------ network
import oracle.unet as un  # noqa: E402
import test_oracle_unet as upins  # noqa: E402

_orig_conv = un.conv3d
_orig_conv_bwd = un.conv3d_backward


def _conv_flipped(x, w, b):
    return _orig_conv(x, w[:, :, ::-1, ::-1, ::-1], b)          # convolution instead of correlation


def _conv_bwd_no_input_grad_transpose(x, w, g):
    gx, gw, gb = _orig_conv_bwd(x, w[:, :, ::-1, ::-1, ::-1], g)   # wrong tap orientation for dx
    return gx, _orig_conv_bwd(x, w, g)[1], gb


def _pool_bwd_unscaled(g):
    return un.up2(g)                                            # forgot the 1/8


UNET_MUTATIONS = [
    ("conv3d", _conv_flipped, upins.test_conv_is_scipy_correlation_with_zero_padding),
    ("conv3d_backward", _conv_bwd_no_input_grad_transpose, upins.test_network_gradient_matches_finite_differences),
    ("pool2_backward", _pool_bwd_unscaled, upins.test_resampling_operators_are_adjoint),
]


@pytest.mark.parametrize("name,bad,pin", UNET_MUTATIONS, ids=[f"{m[0]}-{m[1].__name__}" for m in UNET_MUTATIONS])
def test_planted_network_mistake_is_caught(monkeypatch, name, bad, pin):
    monkeypatch.setattr(un, name, bad)
    with pytest.raises(AssertionError):
        pin()
