"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test names the passage it checks.  None of them re-types an oracle
formula and compares it with itself: they use direct sums, the paper's own
forward equations (8)/(9), limits stated in the paper (eqs. 13-15), exactness
properties of linear interpolation, hand-derived index mappings, and recovery
of known phantoms from independently simulated images.
"""
import numpy as np
import pytest

import oracle
from synth import forward, phantoms, scan

RNG = np.random.default_rng(2206_09151)


def _inside(n, margin=1.0):
    c = (n - 1) / 2.0
    z, y, x = np.meshgrid(*(np.arange(n) - c,) * 3, indexing="ij")
    return (x * x + y * y + z * z) < (n / 2.0 - margin) ** 2


def _rel(a, b, mask):
    return np.linalg.norm((a - b)[mask]) / np.linalg.norm(b[mask])


def _slice_mean_removed(v):
    # The axis ramp |q_x| is zero on the q_x = 0 column of every view, i.e. on the
    # rotation-axis line of the 3D spectrum: each y slice loses its mean.
    return v - v.mean(axis=(0, 2), keepdims=True)


# ------------------------------------------------------------------ O3: DFT convention
@pytest.mark.parametrize("m", [8, 12, 15, 16, 20])
def test_spectrum_equals_direct_dft(m):
    """F2 of Section 2 uses exp(-i 2 pi r.q): compare with the O(M^4) direct sum."""
    g = RNG.standard_normal((m, m))
    a = np.arange(m)
    direct = np.empty((m, m), dtype=complex)
    for ky in range(m):
        for kx in range(m):
            direct[ky, kx] = np.sum(g * np.exp(-2j * np.pi * (ky * a[:, None] + kx * a[None, :]) / m))
    assert np.allclose(oracle.spectrum(g), direct, rtol=0, atol=1e-10 * np.abs(direct).max())


def test_signed_index_covers_nyquist():
    assert list(oracle.signed_index(6)) == [0, 1, 2, -3, -2, -1]
    assert list(oracle.signed_index(5)) == [0, 1, 2, -2, -1]


# ------------------------------------------------------------------ O1: frames
def test_frames_rotation_about_y():
    """Rotating the object about y (eq. 9) keeps v = y; u, v, d right handed."""
    th = np.deg2rad([0.0, 30.0, 90.0, 200.0])
    d = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    u, v, dd = oracle.frames(d)
    assert np.allclose(v, [[0, 1, 0]] * 4, atol=1e-15)
    assert np.allclose(u, np.stack([np.cos(th), 0 * th, -np.sin(th)], 1), atol=1e-15)
    assert np.allclose(np.cross(u, v), dd, atol=1e-15)


def test_frames_orthonormal_random_and_pole():
    d = scan.uniform_sphere(3, 50)
    d = np.vstack([d, [[0, 1, 0], [0, -1, 0]]])
    u, v, dd = oracle.frames(d)
    for a, b in ((u, v), (u, dd), (v, dd)):
        assert np.allclose(np.sum(a * b, 1), 0, atol=1e-14)
    for a in (u, v):
        assert np.allclose(np.linalg.norm(a, axis=1), 1, atol=1e-14)
    assert np.allclose(np.cross(u, v), dd, atol=1e-14)
    # given detector axes are honoured after Gram-Schmidt
    vax = np.tile([[0.3, 1.0, 0.1]], (d.shape[0], 1))
    u2, v2, _ = oracle.frames(d[:-2], vax[:-2])
    assert np.allclose(np.sum(v2 * d[:-2], 1), 0, atol=1e-14)


# ------------------------------------------------------------------ O4: weights
@pytest.mark.parametrize("span,n", [(180.0, 90), (360.0, 90), (180.0, 7)])
def test_axis_weights_uniform_scans(span, n):
    """Uniform scans over 180 or 360 degrees: each view gets pi/n (a plane through the
    rotation axis is covered once per half turn)."""
    w = oracle.axis_angle_weights(scan.single_axis(n, span))
    assert np.allclose(w, np.pi / n, rtol=1e-12)


def test_axis_weights_nonuniform_sum_to_half_turn():
    th = np.sort(RNG.uniform(0, np.pi, 40))
    d = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    w = oracle.axis_angle_weights(d)
    assert np.isclose(w.sum(), np.pi, rtol=1e-12)
    assert np.all(w > 0)


def test_sampling_matrix_gives_ramp_for_single_axis_scan():
    """Text after eq. 11 and Section 4: for a uniform 180-degree single-axis scan the
    sampling-matrix weights approximate the ramp filter |q_x|."""
    n_vox, dx = 32, 1e-6
    dirs = scan.single_axis(90)
    u, v, d = oracle.frames(dirs)
    geo_s = oracle.Geometry(n_vox, n_vox, n_vox, dx, 1e-10, 0.0, 1e-3, ewald=0, weight_mode="sampling")
    geo_r = oracle.Geometry(n_vox, n_vox, n_vox, dx, 1e-10, 0.0, 1e-3, ewald=0, weight_mode="ramp_axis")
    ws = oracle.density_weights(u, v, d, geo_s)
    wr = oracle.density_weights(u, v, d, geo_r)
    k = oracle.signed_index(n_vox)
    ky, kx = np.meshgrid(k, k, indexing="ij")
    sel = (np.abs(kx) >= 2) & (np.abs(kx) <= 12) & (np.abs(ky) <= 12)
    ratio = ws[:, sel] / wr[:, sel]
    assert abs(ratio.mean() - 1) < 0.02
    assert ratio.std() < 0.03
    assert np.all(np.abs(ratio - 1) < 0.1)


def test_sampling_matrix_hermitian_and_total_weight():
    """Every sample and its reflection add 1/2 each: S(-p) = S(p) and the total
    equals the number of samples whose taps all land inside the grid."""
    n_vox = 16
    dirs = scan.uniform_sphere(5, 12)
    u, v, d = oracle.frames(dirs)
    geo = oracle.Geometry(n_vox, n_vox, n_vox, 1e-10, 0.02e-10, 0.0, 1e-3, ewald=1,
                          weight_mode="sampling")
    s = oracle.sampling_matrix(u, v, d, geo)
    # reflection p -> -p on indices [-8, 7]: index i -> -i, valid for i in [-7, 7]
    core = s[1:, 1:, 1:]
    assert np.allclose(core, core[::-1, ::-1, ::-1], atol=1e-12)
    assert s.sum() <= 12 * 16 * 16 + 1e-9 and s.sum() > 0.5 * 12 * 16 * 16


# ------------------------------------------------------------------ O5: filter
def _eq8_pair(A, B, chi, sigma, lam):
    """Image spectra of a view and of its opposite view, eqs. (8) and (9)."""
    pref = 2j * np.pi * np.sqrt(1 + sigma ** 2) / lam
    g = pref * (np.exp(-1j * chi) * A - np.exp(1j * chi) * B)
    g_pi = pref * (np.exp(-1j * chi) * B - np.exp(1j * chi) * A)
    return g, g_pi


def test_bracket_solves_opposite_pair_eq10():
    """Eq. (10): with eps -> 0 the eq. 11 bracket H satisfies
    C/2 [H G(q) + conj(H) G_pi(q-)] = F3 delta(q, -lambda q^2/2) for any object."""
    lam, sigma = 0.025e-10, 0.37
    chi = RNG.uniform(0.1, 1.4, 200)
    A = RNG.standard_normal(200) + 1j * RNG.standard_normal(200)
    B = RNG.standard_normal(200) + 1j * RNG.standard_normal(200)
    g, g_pi = _eq8_pair(A, B, chi, sigma, lam)
    H = oracle.ctf_bracket(chi, 1e-15, 1)
    C = lam / (4 * np.pi * np.sqrt(1 + sigma ** 2))
    est = C / 2 * (H * g + np.conj(H) * g_pi)
    assert np.allclose(est, A, rtol=1e-9, atol=1e-9 * np.abs(A).max())


def test_bracket_real_part_is_eq13():
    """Eq. (13): with no curvature (A = B) the real part of the bracket inverts one image."""
    lam, sigma = 1e-10, -0.2
    omega = np.arctan(sigma)
    chi = RNG.uniform(0.05, 3.0, 100) - omega
    A = RNG.standard_normal(100) + 1j * RNG.standard_normal(100)
    g, _ = _eq8_pair(A, A, chi, sigma, lam)
    H = oracle.ctf_bracket(chi, 1e-15, 0)
    assert np.allclose(H.imag, 0)
    C = lam / (4 * np.pi * np.sqrt(1 + sigma ** 2))
    assert np.allclose(C * H * g, A, rtol=1e-9)


def _filter_only(geo, dist, q_index_max=6):
    m = geo.n_pix
    G = np.ones((1, m, m), dtype=complex)
    W = np.ones((1, m, m))
    return oracle.filtered_spectra(G, np.array([dist]), W, geo)[0]


def test_filter_absorption_ct_limit_eq15():
    """Eq. (15): R -> 0 and pure absorption (|sigma| -> inf): mu-spectrum = -F2 ln(I/I_in),
    with mu = (4 pi / lambda) sigma delta."""
    lam, sigma = 1e-10, 1e7
    geo = oracle.Geometry(16, 16, 16, 1e-6, lam, sigma, 1e-14, ewald=0)
    P = _filter_only(geo, 0.0)
    mu = 4 * np.pi / lam * sigma * P
    assert np.allclose(mu, -1.0, rtol=1e-6)


def test_filter_tie_hom_limit_eq14():
    """Eq. (14): small lambda R q^2 turns the filter into -1/(1 - (pi lambda R/sigma) q^2)
    for mu = (4 pi/lambda) sigma delta (homogeneous TIE)."""
    lam, sigma, dx, m = 1e-10, -0.05, 1e-6, 16
    R = 1e-6  # pi lambda R q^2 <= 1.6e-4: the sin/cos expansion errors are O(1e-8)
    geo = oracle.Geometry(m, m, m, dx, lam, sigma, 1e-16, ewald=0)
    P = _filter_only(geo, R)
    mu = 4 * np.pi / lam * sigma * P
    q = oracle.signed_index(m) / (m * dx)
    q2 = q[:, None] ** 2 + q[None, :] ** 2
    expect = -1.0 / (1.0 - np.pi * lam * R / sigma * q2)
    assert np.max(np.abs(expect + 1)) > 2e-3        # the q^2 term is resolved
    assert np.allclose(mu, expect, rtol=2e-7, atol=0)


# ------------------------------------------------------------------ O6: depth planes
def test_planes_propagate_a_plane_wave_eq3():
    """Eq. (3): a single spatial frequency acquires exp(-i pi lambda z q^2) at depth z;
    the real part of the inverse DFT is a cosine with that phase."""
    m, k, dx, lam = 16, 16, 1e-6, 5e-9
    geo = oracle.Geometry(m, m, k, dx, lam, 0.0, 1e-3, ewald=1)
    P = np.zeros((m, m), dtype=complex)
    ky, kx = 3, 14  # signed (3, -2)
    P[ky, kx] = m * m * (0.7 - 0.2j)
    st = oracle.depth_planes(P, geo)
    q2 = (3.0 ** 2 + 2.0 ** 2) / (m * dx) ** 2
    a = np.arange(m)
    for j in (0, 5, k - 1):
        z = (j - (k - 1) / 2) * dx
        field = (0.7 - 0.2j) * np.exp(-1j * np.pi * lam * z * q2) \
            * np.exp(2j * np.pi * (3 * a[:, None] - 2 * a[None, :]) / m)
        assert np.allclose(st[j], field.real, atol=1e-12)


# ------------------------------------------------------------------ O7: gather
def test_gather_grid_aligned_mapping_by_hand():
    """Hand-derived voxel -> (plane, row, col) for rotations by 0/90/180/270 deg about y
    with N = M = K: a delta planted in the stack lights exactly one voxel."""
    n = 6
    geo = oracle.Geometry(n, n, n, 1e-6, 1e-10, 0.0, 1e-3, ewald=1)
    # (theta, voxel (iz, iy, ix)) -> stack (plane, row, col)
    cases = {
        0: ((1, 2, 4), (1, 2, 4)),         # u = x, d = z: col = ix, plane = iz
        90: ((1, 2, 4), (4, 2, 4)),        # u = -z, d = x: col = N-1-iz, plane = ix
        180: ((1, 2, 4), (4, 2, 1)),       # u = -x, d = -z: col = N-1-ix, plane = N-1-iz
        270: ((1, 2, 4), (1, 2, 1)),       # u = z, d = -x: col = iz, plane = N-1-ix
    }
    for deg, (vox, tap) in cases.items():
        th = np.deg2rad(deg)
        d = np.array([[np.sin(th), 0.0, np.cos(th)]])
        u, v, dd = oracle.frames(d)
        st = np.zeros((n, n, n))
        st[tap] = 1.0
        vol = oracle.gather(st, u[0], v[0], dd[0], geo)
        hits = np.argwhere(np.abs(vol) > 1e-9)
        assert hits.tolist() == [list(vox)], (deg, hits)
        assert np.isclose(vol[vox], 1.0)


def test_gather_reproduces_affine_functions():
    """Trilinear interpolation is exact on affine functions (weights sum to one and are
    linear in the offset), for any oblique view, wherever all eight taps exist."""
    n, k = 10, 12
    geo = oracle.Geometry(n, n, k, 1e-6, 1e-10, 0.0, 1e-3, ewald=1)
    d = scan.uniform_sphere(11, 3)
    u, v, dd = oracle.frames(d)
    pl, rw, cl = np.meshgrid(np.arange(k), np.arange(n), np.arange(n), indexing="ij")
    st = 0.3 * pl - 1.1 * rw + 0.7 * cl + 2.0
    c = (n - 1) / 2
    iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    r = np.stack([ix - c, iy - c, iz - c], -1)
    for i in range(3):
        vol = oracle.gather(st, u[i], v[i], dd[i], geo)
        fc = r @ u[i] + (n - 1) / 2
        fr = r @ v[i] + (n - 1) / 2
        fp = r @ dd[i] + (k - 1) / 2
        ok = (fc >= 0) & (fc <= n - 1) & (fr >= 0) & (fr <= n - 1) & (fp >= 0) & (fp <= k - 1)
        assert ok.sum() > 100
        assert np.allclose(vol[ok], (0.3 * fp - 1.1 * fr + 0.7 * fc + 2.0)[ok], atol=1e-12)
        # taps outside the stack contribute nothing: far outside the value is 0
        far = (fc < -1) | (fc > n) | (fr < -1) | (fr > n) | (fp < -1) | (fp > k)
        assert np.all(vol[far] == 0)


def test_gather_is_adjoint_of_trilinear_splat():
    """<G b, w> = <b, G^T w> with G^T the trilinear splat written independently."""
    n, k = 7, 9
    geo = oracle.Geometry(n, n, k, 1e-6, 1e-10, 0.0, 1e-3, ewald=1)
    u, v, d = oracle.frames(scan.uniform_sphere(2, 1))
    b = RNG.standard_normal((k, n, n))
    w = RNG.standard_normal((n, n, n))
    gb = oracle.gather(b, u[0], v[0], d[0], geo)
    gtw = np.zeros_like(b)
    c = (n - 1) / 2
    for iz in range(n):
        for iy in range(n):
            for ix in range(n):
                r = np.array([ix - c, iy - c, iz - c])
                f = np.array([r @ d[0] + (k - 1) / 2, r @ v[0] + (n - 1) / 2, r @ u[0] + (n - 1) / 2])
                lim = (k, n, n)
                i0 = np.floor(f).astype(int)
                t = f - i0
                for corner in np.ndindex(2, 2, 2):
                    idx = i0 + np.array(corner)
                    if np.any(idx < 0) or np.any(idx >= lim):
                        continue
                    wt = np.prod(np.where(np.array(corner) == 1, t, 1 - t))
                    gtw[tuple(idx)] += wt * w[iz, iy, ix]
    assert np.isclose(np.sum(gb * w), np.sum(b * gtw), rtol=1e-12)


# ------------------------------------------------------------------ O1..O8 end to end
def test_grid_aligned_reconstruction_equals_direct_backpropagation():
    """Views at 0/90/180/270 deg about y with N = M = K put every voxel on a stack node,
    so the result must equal the interpolation-free sum over views of
    Re (1/M^2) sum_k P(k) exp(i 2 pi q.r') exp(-i pi lambda z' q^2) evaluated directly."""
    n, dx, lam = 8, 1e-6, 3e-8
    geo = oracle.Geometry(n, n, n, dx, lam, 0.1, 1e-3, ewald=1)
    th = np.deg2rad([0.0, 90.0, 180.0, 270.0])
    dirs = np.stack([np.sin(th), 0 * th, np.cos(th)], 1)
    dist = np.array([0.1, 0.12, 0.09, 0.11])
    imgs = np.exp(0.01 * RNG.standard_normal((4, n, n)))
    vol = oracle.reconstruct(imgs, dirs, dist, geo)
    u, v, d = oracle.frames(dirs)
    W = oracle.density_weights(u, v, d, geo)
    P = oracle.filtered_spectra(oracle.spectrum(oracle.contrast(imgs)), dist, W, geo)
    kk = oracle.signed_index(n)
    c = (n - 1) / 2
    rng = np.random.default_rng(1)
    for _ in range(25):
        iz, iy, ix = rng.integers(0, n, 3)
        r = np.array([ix - c, iy - c, iz - c])
        tot = 0.0
        for i in range(4):
            xcol = r @ u[i] + (n - 1) / 2     # pixel index along columns
            yrow = r @ v[i] + (n - 1) / 2
            z = (r @ d[i]) * dx
            ph = np.exp(2j * np.pi * (kk[:, None] * yrow + kk[None, :] * xcol) / n)
            q2 = (kk[:, None] ** 2 + kk[None, :] ** 2) / (n * dx) ** 2
            tot += np.real(np.sum(P[i] * ph * np.exp(-1j * np.pi * lam * z * q2))) / n ** 2
        assert np.isclose(vol[iz, iy, ix], tot, rtol=1e-10, atol=1e-12 * np.abs(vol).max())


def test_linearity_in_log_contrast():
    """Eq. (11) is linear in F2 ln(I/I_in): R(a g1 + b g2) = a R(g1) + b R(g2)."""
    n = 10
    geo = oracle.Geometry(n, n, n, 1e-6, 1e-9, 0.05, 1e-3, ewald=1, weight_mode="ramp_iso")
    dirs = scan.uniform_sphere(8, 5)
    dist = np.full(5, 0.05)
    g1 = 0.01 * RNG.standard_normal((5, n, n))
    g2 = 0.01 * RNG.standard_normal((5, n, n))
    r1 = oracle.reconstruct(np.exp(g1), dirs, dist, geo)
    r2 = oracle.reconstruct(np.exp(g2), dirs, dist, geo)
    r12 = oracle.reconstruct(np.exp(2.5 * g1 - 0.5 * g2), dirs, dist, geo)
    assert np.allclose(r12, 2.5 * r1 - 0.5 * r2, rtol=1e-10, atol=1e-13 * np.abs(r12).max())


def test_ct_limit_recovers_phantom_from_fresnel_images():
    """Eq. (13) / Fourier slice theorem of phase CT: large DOF, weak monomorphous object,
    images from the projection approximation + Fresnel propagation (an independent
    forward model): the reconstruction returns delta inside the object."""
    n, dx, lam = 32, 1e-6, 1e-10
    ph = phantoms.draw_blobs(7, n, dx, 0, 1.6e-6, -1e-10, sigma=-1.0, count=12, support=0.3)
    ref = forward.voxelize(ph, n, dx)
    dirs = scan.single_axis(90)
    dist = np.full(90, 0.2)
    imgs = forward.project_fresnel_images(ph, dirs, n, dx, lam, dist)
    inside = _inside(n)
    for ewald in (0, 1):
        geo = oracle.Geometry(n, n, n, dx, lam, -1.0, 1e-6, ewald=ewald)
        vol = oracle.reconstruct(imgs, dirs, dist, geo)
        err = _rel(_slice_mean_removed(vol), _slice_mean_removed(ref), inside)
        assert err < 0.065, (ewald, err)


def test_ewald_curvature_matters_when_dof_is_small():
    """Section 3 (Ewald sphere correction on/off): first-Born images of eq. (8) with
    DOF = Delta^2/(2 lambda) = 0.5 A << object thickness, 180 views over 360 deg.
    With the curvature the phantom is recovered; dropping it (eq. 13 used beyond its
    validity) is markedly worse."""
    n, dx, lam = 32, 1e-10, 1e-10
    ph = phantoms.draw_blobs(7, n, dx, 0, 1.6e-10, 1e-5, sigma=-1.0, count=12, support=0.3)
    ref = forward.voxelize(ph, n, dx)
    dirs = scan.single_axis(180, 360.0)
    dist = np.full(180, 1e-10)
    imgs = forward.born_images(ph, dirs, n, dx, lam, dist, -1.0)
    inside = _inside(n)
    errs = {}
    for ewald in (1, 0):
        geo = oracle.Geometry(n, n, n, dx, lam, -1.0, 1e-6, ewald=ewald)
        vol = oracle.reconstruct(imgs, dirs, dist, geo)
        errs[ewald] = _rel(_slice_mean_removed(vol), _slice_mean_removed(ref), inside)
    assert errs[1] < 0.065, errs
    assert errs[0] > 1.5 * errs[1], errs


def test_isotropic_ramp_recovers_phantom_from_sphere_scan():
    """Directions uniform on the sphere (the paper's Fe-Pt scan geometry) with the
    isotropic density weight 2|q|/n: weak phantom recovered in the CT limit."""
    n, dx, lam = 24, 1e-6, 1e-10
    ph = phantoms.draw_blobs(9, n, dx, 0, 1.5e-6, -1e-10, sigma=-1.0, count=8, support=0.3)
    ref = forward.voxelize(ph, n, dx)
    dirs = scan.uniform_sphere(4, 400)
    dist = np.full(400, 0.05)
    imgs = forward.project_fresnel_images(ph, dirs, n, dx, lam, dist)
    geo = oracle.Geometry(n, n, n, dx, lam, -1.0, 1e-6, ewald=0, weight_mode="ramp_iso")
    vol = oracle.reconstruct(imgs, dirs, dist, geo)
    err = _rel(vol - vol.mean(), ref - ref.mean(), _inside(n))
    assert err < 0.12, err


def test_opposite_views_mirror_in_flat_limit():
    """Text before eq. (13): without curvature I_pi(r-) = I(r) (generator property).

    The condition is lambda z q^2 << 1 *and* a CTF phase chi of order one
    (sigma = -1 here); for chi -> 0 the z/R variation of the defocus survives."""
    n, dx = 15, 1e-10
    ph = phantoms.draw_blobs(3, n, dx, 0, 1.2e-10, 1e-5, sigma=-1.0, count=6, support=0.3)
    dirs = scan.single_axis(2, 360.0, offset_deg=20.0)   # 20 and 200 degrees
    imgs = forward.born_images(ph, dirs, n, dx, 1e-16, np.full(2, 50e-10), -1.0)
    g0, g1 = np.log(imgs[0]), np.log(imgs[1])
    assert np.abs(g0).max() > 1e-4
    assert np.allclose(g1[:, ::-1], g0, rtol=0, atol=1e-6 * np.abs(g0).max())
    imgs = forward.born_images(ph, dirs, n, dx, 2e-11, np.full(2, 50e-10), -1.0)
    g0, g1 = np.log(imgs[0]), np.log(imgs[1])
    assert not np.allclose(g1[:, ::-1], g0, rtol=0, atol=1e-3 * np.abs(g0).max())
