"""Parity at the benchmarked size: the 128^3, 180-view diffraction-tomography
workload (1 A voxels, lambda 0.0197 A, 128 depth planes, Gaussian atoms at 40 per
1000 A^3, first-Born images), run exactly as bench.py runs it (automatic angle
batch).  The oracle evaluates a seeded sample of voxels one by one (all 180
views, full plane stacks per view)."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_dt_ewald_128_sampled_voxels_match_oracle():
    from paper_2206_09151_amd import tomo
    from synth import workloads
    w = workloads.WORKLOADS["dt_ewald_128"]
    ph, dirs, dist, imgs64 = workloads.make_workload(w, device="cuda")
    imgs = imgs64.astype(np.float32)
    params = tomo.Params(n_vox=w.n_vox, n_angles=w.n_views, voxel_size=w.voxel, wavelength=w.wavelength,
                         sigma=w.sigma, epsilon=w.epsilon, n_pix=w.M, n_planes=w.K, ewald=w.ewald,
                         weight_mode=w.weight_mode)
    plan = tomo.Plan(params, dirs, dist)
    vol = torch.empty((w.n_vox,) * 3, dtype=torch.float32, device="cuda:0")
    plan.reconstruct(torch.from_numpy(imgs).to("cuda:0"), vol)
    got = vol.cpu().numpy()
    rng = np.random.default_rng(7)
    vox = rng.integers(0, w.n_vox, size=(48, 3))
    vox = np.vstack([vox, [[0, 0, 0], [127, 127, 127], [64, 64, 64], [0, 127, 5]]])   # corners and centre
    geo = oracle.Geometry(w.n_vox, w.M, w.K, w.voxel, w.wavelength, w.sigma, w.epsilon, ewald=w.ewald,
                          weight_mode=w.weight_mode)
    ref = oracle.reconstruct(imgs.astype(np.float64), dirs, dist, geo, voxels=vox)
    g = got[vox[:, 0], vox[:, 1], vox[:, 2]].astype(np.float64)
    rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    assert rel < 1e-5, rel
    assert np.isfinite(got).all()
