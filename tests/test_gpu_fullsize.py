"""Parity at the benchmarked sizes, run the way bench.py runs them (automatic angle
batch, plan-time gridding autotune, steps enqueued with tomo_reconstruct_async and
closed with tomo_sync), against the oracle over the whole volume:

* the 128^3, 180-view diffraction-tomography workload (1 A voxels, lambda 0.0197 A,
  128 depth planes, Gaussian atoms at 40 per 1000 A^3, first-Born images);
* the 64^3, 90-view CT-limit workload as stated (Ewald curvature on, 64 depth planes,
  projection approximation + Fresnel images);
* the 256^3, 360-view tilted X-ray workload: the whole scan at 64 seeded voxels (the
  oracle's planes evaluated at the taps only), and one 8-view launch batch at 3000 voxels
  in each plane storage type.

The oracle's view sum is split over the host's threads (tests/_oracle_par.py).  Bar:
rel-L2 <= 1e-5 and max|got - ref| <= 1e-5 max|ref|."""
import numpy as np
import pytest

import oracle
import _oracle_par

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _assert_close(got, ref, tol, what):
    got = np.asarray(got, dtype=np.float64)
    rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    worst = float(np.abs(got - ref).max() / np.abs(ref).max())
    print(f"{what}: rel-L2 {rel:.3e}, max|d|/max|ref| {worst:.3e}", flush=True)
    assert rel < tol and worst < tol, (what, rel, worst)


def _bench_like_run(w, imgs, dirs, dist):
    from paper_2206_09151_amd import tomo
    params = tomo.Params(n_vox=w.n_vox, n_angles=w.n_views, voxel_size=w.voxel, wavelength=w.wavelength,
                         sigma=w.sigma, epsilon=w.epsilon, n_pix=w.M, n_planes=w.K, ewald=w.ewald,
                         weight_mode=w.weight_mode, eps_sampling=w.eps_sampling, i_in=w.i_in, tune=1)
    stream = torch.cuda.current_stream()
    plan = tomo.Plan(params, dirs, dist, stream=stream)
    d_img = torch.from_numpy(imgs).to("cuda:0")
    vol = torch.full((w.n_vox,) * 3, float("nan"), dtype=torch.float32, device="cuda:0")
    for _ in range(2):                       # two enqueued steps, as the bench's loop does
        plan.reconstruct_async(d_img, vol, stream=stream)
    plan.sync(stream)
    out = vol.cpu().numpy()
    assert np.isfinite(out).all()
    return plan, out


@pytest.mark.parametrize("workload", ["dt_ewald_128", "ct_pct_64"])
def test_benchmarked_workload_whole_volume_matches_oracle(workload):
    from synth import workloads
    w = workloads.WORKLOADS[workload]
    ph, dirs, dist, imgs64 = workloads.make_workload(w, device="cuda")
    imgs = imgs64.astype(np.float32)
    plan, got = _bench_like_run(w, imgs, dirs, dist)
    print(f"{workload}: batch {plan.batch}, grid rows {plan.grid_rows}", flush=True)
    geo = oracle.Geometry(w.n_vox, w.M, w.K if w.ewald else 1, w.voxel, w.wavelength, w.sigma, w.epsilon,
                          ewald=w.ewald, weight_mode=w.weight_mode, eps_sampling=w.eps_sampling, i_in=w.i_in)
    ref = _oracle_par.reconstruct_views(imgs.astype(np.float64), dirs, dist, geo)
    _assert_close(got, ref, 1e-5, workload)


def test_xray_jitter_256_whole_scan_matches_oracle_at_sampled_voxels(xray_case):
    """All 360 views through tomo_reconstruct_async as bench.py runs them (automatic
    batch, autotuned near-axis gridding), at 64 seeded voxels against the FP64 oracle."""
    w, dirs, dist, imgs, *_ = xray_case
    plan, got = _bench_like_run(w, imgs, dirs, dist)
    print(f"xray_jitter_256: batch {plan.batch}, grid rows {plan.grid_rows}", flush=True)
    vox = np.random.default_rng(12).integers(0, w.n_vox, size=(64, 3))
    geo = oracle.Geometry(w.n_vox, w.M, w.K, w.voxel, w.wavelength, w.sigma, w.epsilon, ewald=w.ewald,
                          weight_mode=w.weight_mode, eps_sampling=w.eps_sampling, i_in=w.i_in)
    ref = oracle.reconstruct_at_voxels(imgs.astype(np.float64), dirs, dist, geo, vox)
    _assert_close(got[vox[:, 0], vox[:, 1], vox[:, 2]], ref, 1e-5, "xray_jitter_256 whole scan")
    plan.destroy()


@pytest.fixture(scope="module")
def xray_case():
    """The 256^3, 360-view X-ray workload and the oracle's partial sum over one launch
    batch of 8 views (first = 100) at 3000 seeded voxels, computed once."""
    from synth import workloads
    w = workloads.WORKLOADS["xray_jitter_256"]
    ph, dirs, dist, imgs64 = workloads.make_workload(w, device="cuda")
    imgs = imgs64.astype(np.float32)
    first, nb = 100, 8
    vox = np.random.default_rng(11).integers(0, w.n_vox, size=(3000, 3))
    geo = oracle.Geometry(w.n_vox, w.M, w.K, w.voxel, w.wavelength, w.sigma, w.epsilon, ewald=w.ewald,
                          weight_mode=w.weight_mode)
    ref = _oracle_par.reconstruct_views(imgs.astype(np.float64), dirs, dist, geo,
                                        views=np.arange(first, first + nb), voxels=vox)
    return w, dirs, dist, imgs, first, nb, vox, ref


@pytest.mark.parametrize("storage,bound", [(0, 1e-5), (1, 3 * 2.0 ** -9), (2, 3 * 2.0 ** -11)],
                         ids=["f32", "bf16", "fp16"])
def test_xray_jitter_256_view_batch_matches_oracle(xray_case, storage, bound):
    """Full size, +-5 deg tilt jitter, sampling-matrix weights from all 360 directions on
    both sides: one launch batch of 8 views through the stage entry points (the kernels
    and launch shapes tomo_reconstruct uses), compared at 3000 seeded voxels."""
    from paper_2206_09151_amd import tomo
    w, dirs, dist, imgs, first, nb, vox, ref = xray_case
    params = tomo.Params(n_vox=w.n_vox, n_angles=w.n_views, voxel_size=w.voxel, wavelength=w.wavelength,
                         sigma=w.sigma, epsilon=w.epsilon, n_pix=w.M, n_planes=w.K, ewald=w.ewald,
                         weight_mode=w.weight_mode, plane_dtype=storage)
    plan = tomo.Plan(params, dirs, dist)
    assert plan.batch == nb
    d_img = torch.from_numpy(imgs[first:first + nb]).to("cuda:0")
    st = torch.empty(plan.stack_shape(nb), dtype=plan.stack_dtype, device="cuda:0")
    vol = torch.zeros((w.n_vox,) * 3, dtype=torch.float32, device="cuda:0")
    plan.backpropagate(d_img, first, nb, st)
    plan.grid(st, first, nb, vol)
    got = vol.cpu().numpy()
    g = got[vox[:, 0], vox[:, 1], vox[:, 2]].astype(np.float64)
    _assert_close(g, ref, bound, f"xray_jitter_256 storage={storage}")


@pytest.fixture(scope="module")
def dt128_fourier_case():
    """The 128^3, 180-view workload and the Fourier-space oracle over all voxels, computed once."""
    from synth import workloads
    w = workloads.WORKLOADS["dt_ewald_128"]
    ph, dirs, dist, imgs64 = workloads.make_workload(w, device="cuda")
    imgs = imgs64.astype(np.float32)
    geo = oracle.Geometry(w.n_vox, w.M, w.K, w.voxel, w.wavelength, w.sigma, w.epsilon, ewald=w.ewald,
                          weight_mode=w.weight_mode, eps_sampling=w.eps_sampling)
    ref = oracle.fourier_reconstruct(imgs.astype(np.float64), dirs, dist, geo)
    return w, dirs, dist, imgs, ref


@pytest.mark.parametrize("mode", [1, 2], ids=["operator", "splat"])
def test_dt_ewald_128_fourier_form_matches_oracle(dt128_fourier_case, mode):
    """The Fourier-space form (eq. 11 by 3D gridding) on the same full workload,
    compared over all 128^3 voxels, with the gridding operator and with the splat."""
    from paper_2206_09151_amd import tomo
    w, dirs, dist, imgs, ref = dt128_fourier_case
    params = tomo.Params(n_vox=w.n_vox, n_angles=w.n_views, voxel_size=w.voxel, wavelength=w.wavelength,
                         sigma=w.sigma, epsilon=w.epsilon, n_pix=w.M, n_planes=w.K, ewald=w.ewald,
                         weight_mode=w.weight_mode, eps_sampling=w.eps_sampling, fourier=mode)
    plan = tomo.Plan(params, dirs, dist)
    vol = torch.empty((w.n_vox,) * 3, dtype=torch.float32, device="cuda:0")
    plan.fourier_reconstruct(torch.from_numpy(imgs).to("cuda:0"), vol)
    got = vol.cpu().numpy().astype(np.float64)
    _assert_close(got, ref, 1e-5, f"dt_ewald_128 Fourier-space form (mode {mode}, {plan.fourier_entries} entries)")
