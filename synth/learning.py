"""Seeded phantoms and images for the artefact-correction network's training pairs.

The pairs live in the 128^3 diffraction-tomography regime of the dt_ewald_128 workload
(1 A voxels, lambda 0.0197 A, defocus 500 A, sigma = 0): every phantom is a set of
uniform ellipsoids, imaged by the first-Born model of eq. (8) once for a sparse view set
(30 views over [0, 180)) and once for a dense one (720 views).  Phantom k (k = 0 .. 2199;
0 .. 1999 train, 2000 .. 2199 held out) is drawn from numpy default_rng(220609151 +
4_000_000 + k): its ellipsoid count is 8 + k % 17, semi-axes U[0.03, 0.15] N voxel, delta
U[1e-5, 1e-4].

`born_images_batched` evaluates the same image model as forward.born_images (the
closed-form ellipsoid spectrum on both paraboloids, the CTF phase chi = pi lambda R q^2 -
omega, the pixel-centre phase origin) for a whole chunk of views at once on the GPU; it
holds no reconstruction arithmetic.
"""
from __future__ import annotations

import numpy as np
import torch

from .forward import _ball_ft, _signed_freq
from .phantoms import EllipsoidPhantom, draw_ellipsoids
from .scan import detector_frames
from .workloads import SEED_BASE

PAIR_SEED = SEED_BASE + 4_000_000
TRAIN, HELD_OUT = 2000, 200
SPARSE_VIEWS, DENSE_VIEWS = 30, 720


def pair_phantom(k: int, n_vox: int = 128, voxel: float = 1e-10) -> EllipsoidPhantom:
    """Phantom k of the training-pair set."""
    return draw_ellipsoids(PAIR_SEED + k, 8 + k % 17, n_vox, voxel, (1e-5, 1e-4), 0.0,
                           axis_range=(0.03, 0.15))


def born_images_batched(ph: EllipsoidPhantom, dirs: np.ndarray, n_pix: int, pixel: float, wavelength: float,
                        dist: np.ndarray, sigma: float, i_in: float = 1.0, device: str = "cuda",
                        chunk: int = 96) -> torch.Tensor:
    """First-Born images of eq. (8) for all views, float32 [n, M, M] on `device` (computed
    in FP64 and rounded once)."""
    dev = torch.device(device)
    u, v, d = detector_frames(dirs)
    n = d.shape[0]
    dist = np.broadcast_to(np.asarray(dist, dtype=np.float64), (n,))
    k = torch.as_tensor(_signed_freq(n_pix) / (n_pix * pixel), device=dev)
    qy, qx = torch.meshgrid(k, k, indexing="ij")
    q2 = qx ** 2 + qy ** 2
    omega = float(np.arctan(sigma))
    pref = 2j * np.pi * np.sqrt(1.0 + sigma ** 2) / wavelength
    shift = torch.exp(-2j * np.pi * (qx + qy) * (n_pix - 1) * pixel / 2.0) / pixel ** 2
    rot = torch.as_tensor(ph.rot, device=dev)                   # [E, 3, 3]
    axes = torch.as_tensor(ph.axes, device=dev)                 # [E, 3]
    cen = torch.as_tensor(ph.centres, device=dev)               # [E, 3]
    amp = torch.as_tensor(ph.delta * np.prod(ph.axes, axis=1), device=dev)   # [E]
    out = torch.empty((n, n_pix, n_pix), dtype=torch.float32, device=dev)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        U, V, D = (torch.as_tensor(x[c0:c1], device=dev) for x in (u, v, d))   # [C, 3]

        def spectrum(qz):
            # F3 delta at p = qx u + qy v + qz d for every view of the chunk: [C, M, M]
            p = (qx[None, ..., None] * U[:, None, None, :] + qy[None, ..., None] * V[:, None, None, :]
                 + qz[None, ..., None] * D[:, None, None, :])                    # [C, M, M, 3]
            s = torch.einsum("cyxa,eab->ecyxb", p, rot) * axes[:, None, None, None, :]
            ft = _ball_ft(torch.linalg.norm(s, dim=-1))                          # [E, C, M, M]
            ph_ = torch.exp(-2j * np.pi * torch.einsum("cyxa,ea->ecyx", p, cen))
            return torch.einsum("e,ecyx->cyx", amp.to(ph_.dtype), ft * ph_)

        a = spectrum(-wavelength * q2 / 2.0)
        b = spectrum(+wavelength * q2 / 2.0)
        chi = torch.as_tensor(np.pi * wavelength * dist[c0:c1], device=dev)[:, None, None] * q2[None] - omega
        g_spec = pref * (torch.exp(-1j * chi) * a - torch.exp(1j * chi) * b)
        g = torch.fft.ifft2(g_spec * shift[None]).real
        out[c0:c1] = (i_in * torch.exp(g)).to(torch.float32)
    return out
