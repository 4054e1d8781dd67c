"""FP64 CPU oracle: CTF-corrected Fresnel back-propagation onto depth planes and
real-space trilinear gridding, summed over all views.

TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this module; the product library
never does.  Plain numpy in float64; numpy.fft is the only library primitive
used (as the 2D DFT and its inverse).

Paper: Gureyev, Brown, Quiney, Allen, "Fast unified reconstruction algorithm
for conventional, phase-contrast and diffraction tomography" (arXiv
2206.09151).  Steps, each with the passage it follows:

  O1 frames      view frame (u, v, d) from the illumination direction
                 (Section 2: beam along z; eq. 9: rotation about y).
  O2 contrast    g = ln(I / I_in)                     (eq. 4 left side, eq. 11)
  O3 spectrum    G = DFT2(g), kernel exp(-i 2 pi ...)   (F2 definition before eq. 3)
  O4 weights     density compensation W_n(q) replacing 1/n_q of eq. 11:
                 ramp for a uniform single-axis scan, isotropic ramp for
                 directions uniform on the sphere, or the regularised inverse
                 of the trilinear sampling matrix S(q)   (text after eq. 11;
                 Section 4 on the automatically generated filter)
  O5 filter      P = C W H G,  C = lambda / (4 pi sqrt(1+sigma^2)),
                 H = sin chi/(sin^2 chi + eps) - i cos chi/(cos^2 chi + eps),
                 chi = pi lambda R_n q^2 - omega, omega = atan(sigma)   (eq. 11);
                 without Ewald curvature only the real part of H   (eq. 13)
  O6 planes      b_j = Re IDFT2[P exp(-i pi lambda z_j q^2)] at depths
                 z_j = (j - (K-1)/2) Delta: the view's paraboloid
                 (q, -lambda q^2/2) of eqs. 8/10 evaluated plane by plane with
                 the Fresnel propagator of eq. 3; one plane without curvature
  O7 gather      trilinear interpolation of the stack at each voxel's view-frame
                 position (text after eq. 11: eight neighbours, weights summing
                 to one, "3D linear interpolation"); taps outside the stack are 0
  O8 sum         V = sum over views                      (eq. 11 sum)

Conventions fixed here (readings of the paper):
  * voxel (iz, iy, ix) sits at ((ix, iy, iz) - (N-1)/2) * Delta; image pixel
    (row a, col b) at x' = (b - (M-1)/2) Delta, y' = (a - (M-1)/2) Delta;
  * signed frequency index k~ in numpy fftfreq order, q = k~ / (M Delta);
  * R_n is measured from the plane z' = 0 through the rotation centre;
  * the real part of the back-propagated field is kept, which pairs each
    view with the Hermitian conjugate of its opposite view (eq. 10).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "Geometry", "RAMP_AXIS", "RAMP_ISO", "SAMPLING",
    "frames", "contrast", "spectrum", "signed_index", "axis_angle_weights",
    "sampling_matrix", "density_weights", "ctf_bracket", "filtered_spectra",
    "plane_depths", "depth_planes", "gather", "reconstruct", "reconstruct_views",
    "reconstruct_at_voxels",
]

RAMP_AXIS = "ramp_axis"
RAMP_ISO = "ramp_iso"
SAMPLING = "sampling"


@dataclass(frozen=True)
class Geometry:
    """Problem constants as the paper states them (SI units)."""
    n_vox: int                 # N, volume edge in voxels
    n_pix: int                 # M, detector edge in pixels
    n_planes: int              # K, depth planes per view
    voxel: float               # Delta, voxel size = detector pixel size
    wavelength: float          # lambda
    sigma: float               # beta / delta (monomorphous object)
    epsilon: float             # Tikhonov epsilon of eq. 11
    ewald: int = 1             # 1: eq. 11 with depth planes; 0: eq. 13 (no curvature)
    weight_mode: str = RAMP_AXIS
    eps_sampling: float = 1e-3
    i_in: float = 1.0


# ----------------------------------------------------------------------------- O1
def frames(dirs, vaxes=None):
    """O1: detector frame (u, v, d) per view, each [n, 3].

    d is the unit illumination direction.  v is the lab y axis projected onto
    the detector plane (lab x when d is within 1e-6 of +-y), or the given
    vaxes after Gram-Schmidt against d.  u = v x d makes (u, v, d) right handed;
    rotation by theta about y gives u = (cos t, 0, -sin t), v = y.
    """
    d = np.asarray(dirs, dtype=np.float64)
    n = d.shape[0]
    if vaxes is None:
        ref = np.zeros((n, 3))
        ref[:, 1] = 1.0
        pole = np.linalg.norm(np.cross(ref, d), axis=1) < 1e-6
        ref[pole] = [1.0, 0.0, 0.0]
    else:
        ref = np.asarray(vaxes, dtype=np.float64)
    v = ref - np.sum(ref * d, axis=1)[:, None] * d
    v = v / np.linalg.norm(v, axis=1)[:, None]
    u = np.cross(v, d)
    return u, v, d


# ----------------------------------------------------------------------------- O2, O3
def contrast(images, i_in=1.0):
    """O2: g = ln(I / I_in), float64."""
    return np.log(np.asarray(images, dtype=np.float64) / i_in)


def spectrum(g):
    """O3: G[ky, kx] = sum_{a,b} g[a, b] exp(-i 2 pi (ky a + kx b) / M) over the last two axes."""
    return np.fft.fft2(g, axes=(-2, -1))


def signed_index(m):
    """Signed frequency index k~ in [-floor(m/2), ceil(m/2)-1], fftfreq order."""
    return np.fft.fftfreq(m) * m


# ----------------------------------------------------------------------------- O4
def axis_angle_weights(d):
    """Angular quadrature weight per view for a scan about the y axis.

    theta = atan2(d_x, d_z) folded into [0, pi); the weight is half the gap
    between the neighbouring folded angles on the circle of period pi (the
    trapezoid rule).  A uniform scan over [0, pi) or [0, 2 pi) with n views
    gives pi / n for every view: opposite views share one plane orientation.
    """
    d = np.asarray(d, dtype=np.float64)
    if np.max(np.abs(d[:, 1])) > 1e-9:
        raise ValueError("ramp_axis weights need directions perpendicular to the y axis")
    phi = np.mod(np.arctan2(d[:, 0], d[:, 2]), np.pi)
    order = np.lexsort((np.arange(len(phi)), phi))
    s = phi[order]
    nxt = np.roll(s, -1)
    prv = np.roll(s, 1)
    nxt[-1] += np.pi
    prv[0] -= np.pi
    w = np.empty_like(phi)
    w[order] = 0.5 * (nxt - prv)
    return w


def _paraboloid_points(u, v, d, geo: Geometry):
    """Sample positions p = qx u + qy v - ewald (lambda q^2/2) d of every view and
    detector frequency, in units of the 3D grid spacing 1/(N Delta): [n, M, M, 3]."""
    m = geo.n_pix
    q = signed_index(m) / (m * geo.voxel)
    qy, qx = np.meshgrid(q, q, indexing="ij")
    qz = -geo.ewald * geo.wavelength * (qx ** 2 + qy ** 2) / 2.0
    p = (qx[None, :, :, None] * u[:, None, None, :] + qy[None, :, :, None] * v[:, None, None, :]
         + qz[None, :, :, None] * d[:, None, None, :])
    return p * (geo.n_vox * geo.voxel)


def _grid_lo_hi(n):
    return -(n // 2), (n + 1) // 2 - 1


def _trilinear_taps(pts, n):
    """Yield (flat index, weight, valid) for the 8 trilinear taps of pts [P, 3]
    (lab x, y, z in grid units) on the N^3 grid indexed [z, y, x] from lo."""
    lo, hi = _grid_lo_hi(n)
    f = pts - lo
    i0 = np.floor(f).astype(np.int64)
    t = f - i0
    for cz in (0, 1):
        for cy in (0, 1):
            for cx in (0, 1):
                ix, iy, iz = i0[:, 0] + cx, i0[:, 1] + cy, i0[:, 2] + cz
                wgt = ((t[:, 0] if cx else 1 - t[:, 0]) * (t[:, 1] if cy else 1 - t[:, 1])
                       * (t[:, 2] if cz else 1 - t[:, 2]))
                ok = (ix >= 0) & (ix < n) & (iy >= 0) & (iy < n) & (iz >= 0) & (iz < n)
                flat = (np.clip(iz, 0, n - 1) * n + np.clip(iy, 0, n - 1)) * n + np.clip(ix, 0, n - 1)
                yield flat, wgt, ok


def sampling_matrix(u, v, d, geo: Geometry):
    """S(q) on the N^3 Fourier grid: every detector sample of every view and its
    point reflection (Hermitian counting) add half of their trilinear weights
    (text after eq. 11: fractional gridding weights summed per coefficient)."""
    n = geo.n_vox
    pts = _paraboloid_points(u, v, d, geo).reshape(-1, 3)
    s = np.zeros(n ** 3)
    for sign in (1.0, -1.0):
        for flat, wgt, ok in _trilinear_taps(sign * pts, n):
            s += np.bincount(flat[ok], weights=0.5 * wgt[ok], minlength=n ** 3)
    return s.reshape(n, n, n)


def density_weights(u, v, d, geo: Geometry):
    """O4: W_n[ky, kx] (1/m), replacing 1/n_q of eq. 11 so that the sum over views
    approximates the 3D inverse Fourier integral over the sampled surfaces."""
    n_views = d.shape[0]
    m = geo.n_pix
    q = signed_index(m) / (m * geo.voxel)
    qy, qx = np.meshgrid(q, q, indexing="ij")
    if geo.weight_mode == RAMP_AXIS:
        a = axis_angle_weights(d)
        return a[:, None, None] * np.abs(qx)[None]
    if geo.weight_mode == RAMP_ISO:
        return np.broadcast_to(2.0 * np.sqrt(qx ** 2 + qy ** 2) / n_views, (n_views, m, m)).copy()
    if geo.weight_mode == SAMPLING:
        n = geo.n_vox
        s = sampling_matrix(u, v, d, geo).reshape(-1)
        pts = _paraboloid_points(u, v, d, geo).reshape(-1, 3)
        shat = np.zeros(pts.shape[0])
        for flat, wgt, ok in _trilinear_taps(pts, n):
            shat += np.where(ok, wgt * s[flat], 0.0)
        lo, hi = _grid_lo_hi(n)
        inside = np.all((pts >= lo) & (pts <= hi), axis=1)
        w = (m * m) / (n ** 3 * geo.voxel) * shat / (shat ** 2 + geo.eps_sampling)
        return np.where(inside, w, 0.0).reshape(n_views, m, m)
    raise ValueError(geo.weight_mode)


# ----------------------------------------------------------------------------- O5
def ctf_bracket(chi, eps, ewald):
    """Bracket of eq. 11; its real part alone (eq. 13 limit) when ewald == 0."""
    s, c = np.sin(chi), np.cos(chi)
    re = s / (s * s + eps)
    if not ewald:
        return re.astype(np.complex128)
    return re - 1j * c / (c * c + eps)


def filtered_spectra(G, dist, W, geo: Geometry):
    """O5: P_n = C W_n H_n G_n  (complex [n, M, M])."""
    m = geo.n_pix
    q = signed_index(m) / (m * geo.voxel)
    q2 = q[:, None] ** 2 + q[None, :] ** 2
    omega = np.arctan(geo.sigma)
    const = geo.wavelength / (4.0 * np.pi * np.sqrt(1.0 + geo.sigma ** 2))
    chi = np.pi * geo.wavelength * np.asarray(dist, dtype=np.float64)[:, None, None] * q2[None] - omega
    return const * W * ctf_bracket(chi, geo.epsilon, geo.ewald) * G


# ----------------------------------------------------------------------------- O6
def plane_depths(geo: Geometry):
    """z_j = (j - (K-1)/2) Delta."""
    return (np.arange(geo.n_planes) - (geo.n_planes - 1) / 2.0) * geo.voxel


def depth_planes(P, geo: Geometry):
    """O6: real plane stack [K, M, M] of one view (a single plane without curvature)."""
    if not geo.ewald:
        return np.fft.ifft2(P).real[None]
    m = geo.n_pix
    q = signed_index(m) / (m * geo.voxel)
    q2 = q[:, None] ** 2 + q[None, :] ** 2
    z = plane_depths(geo)
    prop = np.exp(-1j * np.pi * geo.wavelength * z[:, None, None] * q2[None])
    return np.fft.ifft2(P[None] * prop, axes=(-2, -1)).real


# ----------------------------------------------------------------------------- O7
def _lin_taps(f, size):
    i0 = np.floor(f).astype(np.int64)
    t = f - i0
    out = []
    for c in (0, 1):
        i = i0 + c
        w = t if c else 1.0 - t
        ok = (i >= 0) & (i < size)
        out.append((np.clip(i, 0, size - 1), np.where(ok, w, 0.0)))
    return out


def gather(stack, u, v, d, geo: Geometry, voxels=None):
    """O7: trilinear value of one view's stack at each voxel.

    stack [K, M, M] (or [1, M, M] without curvature, then bilinear in the
    detector plane only).  voxels: None for the whole volume [N, N, N] (z, y, x),
    or an int array [P, 3] of (iz, iy, ix) indices.
    """
    n = geo.n_vox
    c = (n - 1) / 2.0
    if voxels is None:
        iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        shape = (n, n, n)
    else:
        vox = np.asarray(voxels)
        iz, iy, ix = vox[:, 0], vox[:, 1], vox[:, 2]
        shape = (vox.shape[0],)
    rx, ry, rz = ix - c, iy - c, iz - c
    m = geo.n_pix
    f_col = u[0] * rx + u[1] * ry + u[2] * rz + (m - 1) / 2.0
    f_row = v[0] * rx + v[1] * ry + v[2] * rz + (m - 1) / 2.0
    out = np.zeros(shape)
    cols, rows = _lin_taps(f_col, m), _lin_taps(f_row, m)
    if stack.shape[0] == 1 and not geo.ewald:
        for ir, wr in rows:
            for ic, wc in cols:
                out += wr * wc * stack[0][ir, ic]
        return out
    k = stack.shape[0]
    f_pl = d[0] * rx + d[1] * ry + d[2] * rz + (k - 1) / 2.0
    for ip, wp in _lin_taps(f_pl, k):
        for ir, wr in rows:
            for ic, wc in cols:
                out += wp * wr * wc * stack[ip, ir, ic]
    return out


# ----------------------------------------------------------------------------- O8
def reconstruct_views(images, dirs, dist, geo: Geometry, vaxes=None, views=None, voxels=None):
    """O1..O8 over the selected views (default all); returns V (float64).

    The density weights are always computed from the full direction set so a
    subset of views gives the corresponding partial sum of the full result.
    """
    u, v, d = frames(dirs, vaxes)
    W = density_weights(u, v, d, geo)
    sel = np.arange(d.shape[0]) if views is None else np.asarray(views)
    g = contrast(np.asarray(images)[sel], geo.i_in)
    P = filtered_spectra(spectrum(g), np.asarray(dist)[sel], W[sel], geo)
    out = None
    for i, nv in enumerate(sel):
        part = gather(depth_planes(P[i], geo), u[nv], v[nv], d[nv], geo, voxels)
        out = part if out is None else out + part
    return out


def reconstruct(images, dirs, dist, geo: Geometry, vaxes=None, voxels=None):
    """Full reconstruction V[z, y, x] (or V at the given voxel indices)."""
    return reconstruct_views(images, dirs, dist, geo, vaxes=vaxes, voxels=voxels)


def reconstruct_at_voxels(images, dirs, dist, geo: Geometry, voxels, vaxes=None):
    """V at the given voxels [P, 3] (iz, iy, ix) with O6 taken at the taps only.

    O1-O5 and the tap positions and weights of O7 are those of reconstruct; the plane
    value at a tap (plane j, row r, column c) is the inverse DFT of O6 written out at that
    one point,
        b_j[r, c] = Re (1/M^2) sum_{ky,kx} P[ky, kx] exp(-i pi lambda z_j (qy^2 + qx^2))
                                  exp(+i 2 pi (ky r + kx c) / M),
    summed over kx for every tap as one matrix product with P, then over ky.  No FFT: it
    costs M^2 per tap instead of K M^2 log M per view, for checks at a few voxels of large
    volumes (one plane at z = 0 without curvature)."""
    u, v, d = frames(dirs, vaxes)
    W = density_weights(u, v, d, geo)
    g = contrast(np.asarray(images), geo.i_in)
    P = filtered_spectra(spectrum(g), np.asarray(dist), W, geo)
    n, m = geo.n_vox, geo.n_pix
    c = (n - 1) / 2.0
    vox = np.asarray(voxels)
    rx, ry, rz = vox[:, 2] - c, vox[:, 1] - c, vox[:, 0] - c
    q2 = (signed_index(m) / (m * geo.voxel)) ** 2            # [M], by storage index
    kk = np.arange(m)
    depths = plane_depths(geo) if geo.ewald else np.zeros(1)
    out = np.zeros(vox.shape[0])
    for nv in range(d.shape[0]):
        f_col = u[nv, 0] * rx + u[nv, 1] * ry + u[nv, 2] * rz + (m - 1) / 2.0
        f_row = v[nv, 0] * rx + v[nv, 1] * ry + v[nv, 2] * rz + (m - 1) / 2.0
        if geo.ewald:
            k = geo.n_planes
            planes = _lin_taps(d[nv, 0] * rx + d[nv, 1] * ry + d[nv, 2] * rz + (k - 1) / 2.0, k)
        else:
            planes = [(np.zeros(vox.shape[0], dtype=np.int64), np.ones(vox.shape[0]))]
        tp, tr, tc, tw, owner = [], [], [], [], []
        for ip, wp in planes:
            for ir, wr in _lin_taps(f_row, m):
                for ic, wc in _lin_taps(f_col, m):
                    tp.append(ip), tr.append(ir), tc.append(ic), tw.append(wp * wr * wc)
                    owner.append(np.arange(vox.shape[0]))
        tp, tr, tc = np.concatenate(tp), np.concatenate(tr), np.concatenate(tc)
        tw, owner = np.concatenate(tw), np.concatenate(owner)
        z = depths[tp]
        bx = np.exp(-1j * np.pi * geo.wavelength * z[None, :] * q2[:, None] + 2j * np.pi * np.outer(kk, tc) / m)
        by = np.exp(-1j * np.pi * geo.wavelength * z[None, :] * q2[:, None] + 2j * np.pi * np.outer(kk, tr) / m)
        vals = np.sum(by * (P[nv] @ bx), axis=0).real / (m * m)
        out += np.bincount(owner, weights=tw * vals, minlength=vox.shape[0])
    return out
