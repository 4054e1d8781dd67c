"""Plausible mistakes planted in the oracle (on the CPU) must fail at least one pin.

Each case patches one oracle function with a typical slip -- a flipped sign, a
transposed operand, a dropped term, a wrong index -- and runs the pin that is
meant to catch it.
"""
import numpy as np
import pytest

import oracle
import oracle.utr as utr
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


MUTATIONS = [
    ("depth_planes", _flip_propagator, pins.test_ewald_curvature_matters_when_dof_is_small),
    ("spectrum", _transposed_spectrum, pins.test_ct_limit_recovers_phantom_from_fresnel_images),
    ("ctf_bracket", _bracket_wrong_imag_sign, pins.test_bracket_solves_opposite_pair_eq10),
    ("ctf_bracket", _bracket_dropped_imag, pins.test_ewald_curvature_matters_when_dof_is_small),
    ("frames", _frames_left_handed, pins.test_frames_rotation_about_y),
    ("frames", _frames_left_handed, pins.test_ct_limit_recovers_phantom_from_fresnel_images),
    ("plane_depths", _depths_off_by_one, pins.test_grid_aligned_reconstruction_equals_direct_backpropagation),
    ("density_weights", _ramp_wrong_axis, pins.test_ct_limit_recovers_phantom_from_fresnel_images),
]


@pytest.mark.parametrize("name,bad,pin", MUTATIONS, ids=[f"{m[0]}-{m[1].__name__}" for m in MUTATIONS])
def test_planted_mistake_is_caught(monkeypatch, name, bad, pin):
    monkeypatch.setattr(utr, name, bad)
    if hasattr(oracle, name):
        monkeypatch.setattr(oracle, name, bad)
    with pytest.raises(AssertionError):
        pin()
