"""FP64 CPU oracle of the paper's own Fourier-space UTR: eq. 11 (and its swapped
form, eq. 12) realised by 3D gridding of the filtered 2D spectra, division by the
regularised sampling matrix, the Fourier-space noise filter and one inverse 3D
Fourier transform.

TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this module; the product library
never does.  Plain numpy in float64; numpy.fft.fft2 is the only library
primitive (the 2D DFT of the images); the 3D inverse transform is written out
as three explicit sums over the signed frequency index.

Steps, each with the passage it follows:

  F1 samples     G_c = DFT2[ln(I_n/I_in)] with its phase origin moved to the
                 detector centre (m-1)/2, so a detector coordinate means the
                 same in both forms of the method   (F2 before eq. 3; eq. 11)
  F2 values      eq. 11: T_n = H_n G_c with the bracket H_n at the view's own
                 R_n; eq. 12: T_n = G_c (the bracket is applied after gridding)
  F3 gridding    every value goes to its paraboloid point
                 p = q_x u + q_y v - ewald (lambda q^2/2) d, and its complex
                 conjugate to -p (the object is real), each with half of its
                 eight trilinear weights on the N^3 grid of spacing 1/(N Delta);
                 the same weights summed give S   (text after eq. 11)
  F4 normalise   A = F S / (S^2 + eps_S): the regularised inverse S_eps^-1
                 replacing 1/n_q of eq. 11   (text after eq. 11)
  F5 noise       zero every A(k) with |A(k)| < NSR M / sqrt(S(k)): noise of
                 relative level NSR in an M x M image has DFT coefficients of
                 standard deviation NSR M (Parseval), averaged over S
                 uncorrelated contributions   (Section 3)
  F6 eq. 12      multiply by the bracket at the common R and the 3D
                 frequency magnitude |k| / (N Delta)   (eq. 12)
  F7 inverse     delta(r) = Re sum_k C Delta^2 A(k) exp(i 2 pi k.(r - c)/N) / (N Delta)^3
                 over the signed grid indices k in [-floor(N/2), ceil(N/2) - 1]^3,
                 voxel (iz, iy, ix), c = (N-1)/2: the continuous 3D inverse
                 Fourier integral sampled at the voxel centres; Delta^2 turns
                 DFT sums into 2D Fourier integrals   (eq. 11 left side)

Readings (where the paper leaves a choice):
  * the NSR threshold compares coefficients in the images' DFT units, i.e.
    CTF-corrected (eq. 11) or raw (eq. 12) averaged spectra, before the
    constant C Delta^2; S is counted with the Hermitian halves as in F3;
  * eq. 12 takes q^2 as the squared magnitude of the 3D grid frequency;
  * the Hermitian reflection -p of a sample on the lowest grid plane of an
    even N falls outside the grid and is dropped, as every tap outside it.
"""
from __future__ import annotations

import numpy as np

from .utr import (Geometry, _grid_lo_hi, _paraboloid_points, _trilinear_taps, contrast, ctf_bracket,
                  frames, signed_index, spectrum)

__all__ = ["centred_spectra", "fourier_values", "fourier_grid", "fourier_normalise",
           "eq12_bracket", "inverse_dft3", "fourier_reconstruct"]


def centred_spectra(images, geo: Geometry):
    """F1: DFT2 of the contrast with the phase origin at the detector centre, [n, M, M]."""
    m = geo.n_pix
    k = signed_index(m)
    shift = np.exp(1j * np.pi * (m - 1) / m * (k[:, None] + k[None, :]))
    return spectrum(contrast(images, geo.i_in)) * shift


def _chi(q2, dist, geo: Geometry):
    return np.pi * geo.wavelength * dist * q2 - np.arctan(geo.sigma)


def fourier_values(Gc, dist, geo: Geometry, variant=11):
    """F2: the values to be gridded, in DFT units."""
    if variant == 12:
        return Gc
    m = geo.n_pix
    q = signed_index(m) / (m * geo.voxel)
    q2 = q[:, None] ** 2 + q[None, :] ** 2
    chi = _chi(q2[None], np.asarray(dist, dtype=np.float64)[:, None, None], geo)
    return ctf_bracket(chi, geo.epsilon, geo.ewald) * Gc


def fourier_grid(values, u, v, d, geo: Geometry):
    """F3: complex accumulator F and sampling matrix S on the N^3 grid [kz, ky, kx]
    (signed index k stored at k - lo)."""
    n = geo.n_vox
    pts = _paraboloid_points(u, v, d, geo).reshape(-1, 3)
    val = np.asarray(values).reshape(-1)
    F = np.zeros(n ** 3, dtype=np.complex128)
    S = np.zeros(n ** 3)
    for sign, x in ((1.0, val), (-1.0, np.conj(val))):
        for flat, wgt, ok in _trilinear_taps(sign * pts, n):
            w = 0.5 * wgt[ok]
            F += np.bincount(flat[ok], weights=w * x[ok].real, minlength=n ** 3)
            F += 1j * np.bincount(flat[ok], weights=w * x[ok].imag, minlength=n ** 3)
            S += np.bincount(flat[ok], weights=w, minlength=n ** 3)
    return F.reshape(n, n, n), S.reshape(n, n, n)


def fourier_normalise(F, S, geo: Geometry, nsr=0.0):
    """F4 + F5: A = F S/(S^2 + eps_S), then the NSR threshold (nsr = 0 keeps all)."""
    A = F * S / (S * S + geo.eps_sampling)
    if nsr > 0:
        thr = np.full(S.shape, np.inf)
        pos = S > 0
        thr[pos] = nsr * geo.n_pix / np.sqrt(S[pos])
        A = np.where(np.abs(A) >= thr, A, 0.0)
    return A


def eq12_bracket(geo: Geometry, dist):
    """F6: the bracket of eq. 12 on the grid [kz, ky, kx] at the common distance R."""
    n = geo.n_vox
    lo, hi = _grid_lo_hi(n)
    k = np.arange(lo, hi + 1) / (n * geo.voxel)
    q2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    return ctf_bracket(_chi(q2, dist, geo), geo.epsilon, geo.ewald)


def inverse_dft3(A, geo: Geometry):
    """F7: delta[iz, iy, ix] from the grid coefficients A (DFT units)."""
    n = geo.n_vox
    lo, hi = _grid_lo_hi(n)
    k = np.arange(lo, hi + 1)
    c = (n - 1) / 2.0
    e = np.exp(2j * np.pi * np.outer(k, np.arange(n) - c) / n)     # [k, i]
    const = geo.wavelength / (4.0 * np.pi * np.sqrt(1.0 + geo.sigma ** 2))
    out = np.tensordot(A, e, axes=([2], [0]))                         # [kz, ky, ix]
    out = np.tensordot(out, e, axes=([1], [0]))                       # [kz, ix, iy]
    out = np.tensordot(out, e, axes=([0], [0]))                       # [ix, iy, iz]
    out = np.transpose(out, (2, 1, 0))
    return out.real * const * geo.voxel ** 2 / (n * geo.voxel) ** 3


def fourier_reconstruct(images, dirs, dist, geo: Geometry, vaxes=None, nsr=0.0, variant=11):
    """F1..F7: delta[z, y, x] by the Fourier-space UTR (variant 11 or 12)."""
    if variant not in (11, 12):
        raise ValueError("variant must be 11 or 12")
    dist = np.asarray(dist, dtype=np.float64)
    if variant == 12 and np.any(dist != dist[0]):
        raise ValueError("eq. 12 needs one common image-plane distance R")
    u, v, d = frames(dirs, vaxes)
    vals = fourier_values(centred_spectra(images, geo), dist, geo, variant)
    F, S = fourier_grid(vals, u, v, d, geo)
    A = fourier_normalise(F, S, geo, nsr)
    if variant == 12:
        A = A * eq12_bracket(geo, dist[0])
    return inverse_dft3(A, geo)
