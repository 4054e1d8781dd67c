"""Forward simulation of flat-field-normalised intensity images.

Two image models from the paper:

* `project_fresnel_images` -- projection approximation through the object
  (Section 2: a = (2pi/lambda) int beta dz, phi = (2pi/lambda) int delta dz,
  exit wave exp(-a + i phi) in the plane z'=0 through the rotation centre),
  then free-space Fresnel propagation over R_n to the detector (eq. 3),
  I = |U|^2.  Chord lengths through ellipsoids are exact (quadratic roots).
* `born_images` -- the first-Born / Ewald-sphere model of a monomorphous
  object, eq. (8): the 2D spectrum of ln(I/I_in) couples the object's 3D
  spectrum on the paraboloid (q, -lambda q^2/2) and its twin (q, +lambda q^2/2),
  with chi = pi lambda R q^2 - omega, omega = atan(sigma).  Object spectra are
  closed form (Gaussian atoms; uniform ellipsoids via the ball transform), so
  the images are exact samples of the band-limited model.

Pixel (row a, col b) of an M x M detector sits at x' = (b-(M-1)/2)*px,
y' = (a-(M-1)/2)*px in the view frame (u, v, d) of `scan.detector_frames`.
"""
from __future__ import annotations

import numpy as np
import torch

from .phantoms import BlobPhantom, EllipsoidPhantom
from .scan import detector_frames


def _signed_freq(m: int) -> np.ndarray:
    return np.fft.fftfreq(m) * m


def _chords(ph: EllipsoidPhantom, origins: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Chord length of the ray origins + t*d through each ellipsoid: [P, k]."""
    out = np.zeros((origins.shape[0], ph.centres.shape[0]))
    for e in range(ph.centres.shape[0]):
        rt = ph.rot[e].T
        w = ((origins - ph.centres[e]) @ rt.T) / ph.axes[e]
        s = (rt @ d) / ph.axes[e]
        a = s @ s
        b = w @ s
        c = np.sum(w * w, axis=1) - 1.0
        disc = b * b - a * c
        out[:, e] = np.where(disc > 0, 2.0 * np.sqrt(np.maximum(disc, 0.0)) / a, 0.0)
    return out


def _line_integrals(ph, origins: np.ndarray, d: np.ndarray):
    """(int delta dt, int beta dt) along origins + t*d for every ray: two [P] arrays."""
    if isinstance(ph, EllipsoidPhantom):
        L = _chords(ph, origins, d)
        return L @ ph.delta, L @ ph.beta
    if isinstance(ph, BlobPhantom):
        # a Gaussian of width s integrates to sqrt(2 pi) s exp(-rho^2 / (2 s^2)) along a
        # line at distance rho from its centre
        acc = np.zeros(origins.shape[0])
        for cc in ph.centres:
            w = origins - cc
            along = w @ d
            rho2 = np.sum(w * w, axis=1) - along ** 2
            acc += np.exp(-rho2 / (2.0 * ph.width ** 2))
        acc *= ph.delta0 * np.sqrt(2.0 * np.pi) * ph.width
        return acc, ph.sigma * acc
    raise TypeError("unsupported phantom")


def project_fresnel_images(ph, dirs: np.ndarray, n_pix: int, pixel: float,
                           wavelength: float, dist: np.ndarray, i_in: float = 1.0) -> np.ndarray:
    """Projection approximation + Fresnel propagation; returns I [n, M, M] (float64)."""
    u, v, d = detector_frames(dirs)
    n = d.shape[0]
    dist = np.broadcast_to(np.asarray(dist, dtype=np.float64), (n,))
    c = (n_pix - 1) / 2.0
    xs = (np.arange(n_pix) - c) * pixel
    yy, xx = np.meshgrid(xs, xs, indexing="ij")  # yy = row coordinate, xx = column coordinate
    k = _signed_freq(n_pix) / (n_pix * pixel)
    q2 = k[:, None] ** 2 + k[None, :] ** 2
    imgs = np.empty((n, n_pix, n_pix))
    kwave = 2.0 * np.pi / wavelength
    for i in range(n):
        origins = xx.reshape(-1, 1) * u[i] + yy.reshape(-1, 1) * v[i]
        int_delta, int_beta = _line_integrals(ph, origins, d[i])
        phi = kwave * int_delta
        att = kwave * int_beta
        u0 = np.sqrt(i_in) * np.exp(-att + 1j * phi).reshape(n_pix, n_pix)
        ur = np.fft.ifft2(np.fft.fft2(u0) * np.exp(-1j * np.pi * wavelength * dist[i] * q2))
        imgs[i] = np.abs(ur) ** 2
    return imgs


def _ball_ft(k: torch.Tensor) -> torch.Tensor:
    """3D Fourier transform of the unit-ball indicator at radial frequency k."""
    x = 2.0 * np.pi * k
    small = x < 1e-4
    xs = torch.where(small, torch.ones_like(x), x)
    val = 4.0 * np.pi * (torch.sin(xs) - xs * torch.cos(xs)) / xs ** 3
    return torch.where(small, torch.full_like(x, 4.0 * np.pi / 3.0), val)


def _object_spectrum(ph, u, v, d, qx, qy, qz, dev) -> torch.Tensor:
    """F3 delta at p = qx u + qy v + qz d for one view; qx, qy, qz are [M, M]."""
    p = qx[..., None] * u + qy[..., None] * v + qz[..., None] * d  # [M, M, 3]
    if isinstance(ph, EllipsoidPhantom):
        acc = torch.zeros(qx.shape, dtype=torch.complex128, device=dev)
        for e in range(ph.centres.shape[0]):
            rot = torch.as_tensor(ph.rot[e], device=dev)
            ax = torch.as_tensor(ph.axes[e], device=dev)
            s = (p @ rot) * ax  # principal-frame frequency scaled by the semi-axes
            amp = ph.delta[e] * float(np.prod(ph.axes[e])) * _ball_ft(torch.linalg.norm(s, dim=-1))
            ph_c = torch.as_tensor(ph.centres[e], device=dev)
            acc = acc + amp * torch.exp(-2j * np.pi * (p @ ph_c))
        return acc
    raise TypeError("unsupported phantom")


def _blob_spectrum_pair(ph: BlobPhantom, u, v, d, k1d, wavelength, dev):
    """F3 delta of the atoms on both paraboloids for one view: (A, B) [M, M].

    A = F3 delta(q, -lambda q^2/2), B = F3 delta(q, +lambda q^2/2).  The phase
    exp(-i 2 pi p.c) separates into an x factor and a y factor because
    q_z is proportional to qx^2 + qy^2, so the atom sum is a matrix product.
    """
    c = torch.as_tensor(ph.centres, device=dev)
    cu = c @ torch.as_tensor(u, device=dev)
    cv = c @ torch.as_tensor(v, device=dev)
    cd = c @ torch.as_tensor(d, device=dev)
    k = torch.as_tensor(k1d, device=dev)
    lin_x = torch.exp(-2j * np.pi * k[:, None] * cu[None, :])
    lin_y = torch.exp(-2j * np.pi * k[:, None] * cv[None, :])
    chirp_x = torch.exp(1j * np.pi * wavelength * (k[:, None] ** 2) * cd[None, :])
    chirp_y = torch.exp(1j * np.pi * wavelength * (k[:, None] ** 2) * cd[None, :])
    # A: q_z = -lambda q^2/2  ->  exp(-i2pi q_z (d.c)) = exp(+i pi lambda q^2 (d.c))
    sum_a = (lin_y * chirp_y) @ (lin_x * chirp_x).transpose(0, 1)
    sum_b = (lin_y * chirp_y.conj()) @ (lin_x * chirp_x.conj()).transpose(0, 1)
    q2 = k[:, None] ** 2 + k[None, :] ** 2
    p2 = q2 + (wavelength * q2 / 2.0) ** 2
    env = ph.delta0 * (2.0 * np.pi * ph.width ** 2) ** 1.5 * torch.exp(-2.0 * np.pi ** 2 * ph.width ** 2 * p2)
    return env * sum_a, env * sum_b


def born_images(ph, dirs: np.ndarray, n_pix: int, pixel: float, wavelength: float,
                dist: np.ndarray, sigma: float, i_in: float = 1.0,
                device: str | None = None) -> np.ndarray:
    """First-Born Ewald-sphere images of eq. (8); returns I [n, M, M] (float64)."""
    dev = torch.device(device or "cpu")
    u, v, d = detector_frames(dirs)
    n = d.shape[0]
    dist = np.broadcast_to(np.asarray(dist, dtype=np.float64), (n,))
    k1d = _signed_freq(n_pix) / (n_pix * pixel)
    k = torch.as_tensor(k1d, device=dev)
    qy, qx = torch.meshgrid(k, k, indexing="ij")
    q2 = qx ** 2 + qy ** 2
    omega = np.arctan(sigma)
    pref = 2j * np.pi * np.sqrt(1.0 + sigma ** 2) / wavelength
    # continuous FT of the pixel-centred samples -> DFT coefficients
    shift = torch.exp(-2j * np.pi * (qx + qy) * (n_pix - 1) * pixel / 2.0) / pixel ** 2
    out = np.empty((n, n_pix, n_pix))
    for i in range(n):
        if isinstance(ph, BlobPhantom):
            a, b = _blob_spectrum_pair(ph, u[i], v[i], d[i], k1d, wavelength, dev)
        else:
            ut, vt, dt = (torch.as_tensor(x, device=dev) for x in (u[i], v[i], d[i]))
            a = _object_spectrum(ph, ut, vt, dt, qx, qy, -wavelength * q2 / 2.0, dev)
            b = _object_spectrum(ph, ut, vt, dt, qx, qy, +wavelength * q2 / 2.0, dev)
        chi = np.pi * wavelength * dist[i] * q2 - omega
        g_spec = pref * (torch.exp(-1j * chi) * a - torch.exp(1j * chi) * b)
        g = torch.fft.ifft2(g_spec * shift).real
        out[i] = (i_in * torch.exp(g)).cpu().numpy()
    return out


def voxelize(ph, n_vox: int, voxel: float) -> np.ndarray:
    """Point samples of delta at voxel centres, volume [z, y, x] (float64)."""
    c = (n_vox - 1) / 2.0
    ax = (np.arange(n_vox) - c) * voxel
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    vol = np.zeros(pts.shape[0])
    if isinstance(ph, EllipsoidPhantom):
        for e in range(ph.centres.shape[0]):
            w = ((pts - ph.centres[e]) @ ph.rot[e]) / ph.axes[e]
            vol += np.where(np.sum(w * w, axis=1) <= 1.0, ph.delta[e], 0.0)
    elif isinstance(ph, BlobPhantom):
        s2 = 2.0 * ph.width ** 2
        cut = 6.0 * ph.width
        for cc in ph.centres:
            dd = pts - cc
            near = np.all(np.abs(dd) < cut, axis=1)
            vol[near] += ph.delta0 * np.exp(-np.sum(dd[near] ** 2, axis=1) / s2)
    return vol.reshape(n_vox, n_vox, n_vox)
