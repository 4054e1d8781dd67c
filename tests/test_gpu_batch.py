"""Batched uneven jobs through one recorded HIP graph (tomo_batch_*).

Every replay of the graph must reproduce, bit for bit, what tomo_reconstruct gives
each job on its own (the kernels and their order per job are the same), with eager
work and synchronisations between replays; the jobs themselves are checked against
the FP64 oracle (whole volume for the small problems, sampled voxels for the
batched-workload jobs with 160/192-pixel detectors, and for all 64 jobs of the
benchmarked batch at their full size)."""
import numpy as np
import pytest

import oracle
import _problems

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
tomo = pytest.importorskip("paper_2206_09151_amd.tomo")

MIXED = ["axis32", "sphere45", "ragged44", "pct64", "sampling32", "m160", "vaxes32"]


def _eager(plan, imgs, n_vox):
    vol = torch.empty((n_vox,) * 3, dtype=torch.float32, device="cuda:0")
    plan.reconstruct(imgs, vol)
    torch.cuda.synchronize()
    return vol.cpu().numpy()


def test_batch_replays_match_eager_jobs():
    probs = [_problems.make(nm) for nm in MIXED]
    plans = [tomo.Plan(p.params(), p.dirs, p.dist, vaxes=p.vaxes) for p in probs]
    imgs = [torch.from_numpy(p.images).to("cuda:0") for p in probs]
    eager = [_eager(pl, im, p.n_vox) for pl, im, p in zip(plans, imgs, probs)]
    vols = [torch.full((p.n_vox,) * 3, float("nan"), dtype=torch.float32, device="cuda:0") for p in probs]
    batch = tomo.Batch(plans, imgs, vols, lanes=3)
    for rep in range(3):
        for v in vols:
            v.fill_(float("nan"))
        batch.launch()
        batch.sync()
        for j, (v, e) in enumerate(zip(vols, eager)):
            got = v.cpu().numpy()
            assert np.array_equal(got, e), (rep, MIXED[j])
        # eager work between replays
        again = _eager(plans[rep], imgs[rep], probs[rep].n_vox)
        assert np.array_equal(again, eager[rep])
    # the eager results are the oracle's (spot check of two jobs over all voxels)
    for j in (0, 5):
        p = probs[j]
        want = oracle.reconstruct(p.images.astype(np.float64), p.dirs, p.dist, p.oracle_geometry(), vaxes=p.vaxes)
        rel = np.linalg.norm(eager[j] - want) / np.linalg.norm(want)
        assert rel <= 1e-5, (MIXED[j], rel)
    batch.destroy()


def test_batch_reports_the_job_with_a_bad_image():
    probs = [_problems.make(nm) for nm in ("axis32", "oddk16", "sampling32")]
    plans = [tomo.Plan(p.params(), p.dirs, p.dist) for p in probs]
    imgs = [torch.from_numpy(p.images).to("cuda:0") for p in probs]
    imgs[1][2, 3, 4] = 0.0
    vols = [torch.empty((p.n_vox,) * 3, dtype=torch.float32, device="cuda:0") for p in probs]
    batch = tomo.Batch(plans, imgs, vols)
    batch.launch()
    with pytest.raises(tomo.TomoError) as ei:
        batch.sync()
    assert ei.value.status == tomo.EDOMAIN and "job 1" in str(ei.value)
    imgs[1][2, 3, 4] = 1.0
    batch.launch()
    batch.sync()
    batch.destroy()


def test_batch_argument_errors():
    p = _problems.make("axis32")
    plan = tomo.Plan(p.params(), p.dirs, p.dist)
    im = torch.from_numpy(p.images).to("cuda:0")
    v = torch.empty((p.n_vox,) * 3, dtype=torch.float32, device="cuda:0")
    with pytest.raises(tomo.TomoError) as ei:
        tomo.Batch([plan, plan], [im, im], [v, v])
    assert ei.value.status == tomo.EINVAL


def test_batched_workload_jobs_match_oracle_at_sampled_voxels():
    """Six jobs of the batched-workload generator (sizes 64-192, single-axis and sphere
    scans, axis-ramp and sampling-matrix weights), fewer views, one graph."""
    from synth import workloads
    jobs = workloads.batch_jobs(count=6, seed=workloads.SEED_BASE + 33, views=(12, 24))
    jobs = [w.scaled(n_vox=nv) for w, nv in zip(jobs, (64, 160, 96, 192, 160, 96))]
    data = [workloads.make_workload(w) for w in jobs]
    plans, imgs, vols = [], [], []
    for w, (ph, dirs, dist, im) in zip(jobs, data):
        params = tomo.Params(n_vox=w.n_vox, n_angles=w.n_views, voxel_size=w.voxel, wavelength=w.wavelength,
                             sigma=w.sigma, epsilon=w.epsilon, ewald=w.ewald, weight_mode=w.weight_mode)
        plans.append(tomo.Plan(params, dirs, dist))
        imgs.append(torch.from_numpy(im.astype(np.float32)).to("cuda:0"))
        vols.append(torch.empty((w.n_vox,) * 3, dtype=torch.float32, device="cuda:0"))
    batch = tomo.Batch(plans, imgs, vols)
    batch.launch()
    batch.sync()
    rng = np.random.default_rng(5)
    for w, (ph, dirs, dist, im), v in zip(jobs, data, vols):
        print(f"batch job N={w.n_vox} n={w.n_views} {w.geometry}", flush=True)
        vox = rng.integers(0, w.n_vox, size=(200, 3))
        geo = oracle.Geometry(w.n_vox, w.M, w.K, w.voxel, w.wavelength, w.sigma, w.epsilon, ewald=w.ewald,
                              weight_mode=w.weight_mode)
        want = oracle.reconstruct(im.astype(np.float32).astype(np.float64), dirs, dist, geo, voxels=vox)
        got = v.cpu().numpy()[vox[:, 0], vox[:, 1], vox[:, 2]].astype(np.float64)
        rel = np.linalg.norm(got - want) / np.linalg.norm(want)
        print(f"  rel-L2 {rel:.3g}", flush=True)
        assert rel <= 1e-5
    batch.destroy()


def test_full_batched_workload_matches_oracle_at_sampled_voxels():
    """All 64 jobs of the benchmarked batch (N 64-192, 60-240 views, 9807 views in all),
    launched as one graph exactly as bench.py builds it, against the FP64 oracle at 16
    seeded voxels per job (rel-L2 and max error <= 1e-5 per job).  The oracle runs in a
    spawn pool while the GPU works, each worker rebuilding its job's seeded inputs and
    evaluating the planes at the taps only."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor, ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    import _oracle_par
    from synth import workloads
    jobs = workloads.batch_jobs()
    rng = np.random.default_rng(64)
    vox = [rng.integers(0, w.n_vox, size=(16, 3)) for w in jobs]
    workers = _oracle_par.host_threads()
    with ProcessPoolExecutor(workers, mp_context=multiprocessing.get_context("spawn")) as pool:
        # largest jobs first, so that the pool drains evenly
        order = sorted(range(len(jobs)), key=lambda j: -jobs[j].n_vox ** 3 * jobs[j].n_views)
        futs = {j: pool.submit(_oracle_par.batch_job_at_voxels, j, vox[j]) for j in order}

        def make(w):
            _, dirs, dist, imgs = workloads.make_workload(w)
            return dirs, dist, imgs.astype(np.float32)

        with threadpool_limits(1), ThreadPoolExecutor(workers) as ex:
            data = list(ex.map(make, jobs))
        plans, imgs, vols = [], [], []
        for w, (dirs, dist, im) in zip(jobs, data):
            params = tomo.Params(n_vox=w.n_vox, n_angles=w.n_views, voxel_size=w.voxel, wavelength=w.wavelength,
                                 sigma=w.sigma, epsilon=w.epsilon, ewald=w.ewald, weight_mode=w.weight_mode,
                                 eps_sampling=w.eps_sampling, i_in=w.i_in, tune=1)
            plans.append(tomo.Plan(params, dirs, dist))
            imgs.append(torch.from_numpy(im).to("cuda:0"))
            vols.append(torch.full((w.n_vox,) * 3, float("nan"), dtype=torch.float32, device="cuda:0"))
        batch = tomo.Batch(plans, imgs, vols)
        batch.launch()
        batch.sync()
        got = [v.cpu().numpy()[x[:, 0], x[:, 1], x[:, 2]].astype(np.float64) for v, x in zip(vols, vox)]
        batch.destroy()
        for p in plans:
            p.destroy()
        for j, w in enumerate(jobs):
            want = futs[j].result()
            rel = float(np.linalg.norm(got[j] - want) / np.linalg.norm(want))
            worst = float(np.abs(got[j] - want).max() / np.abs(want).max())
            assert rel <= 1e-5 and worst <= 1e-5, (j, w.n_vox, w.n_views, w.geometry, rel, worst)
