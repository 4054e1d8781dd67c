"""The oracle's sum over views, split over host threads (test infrastructure).

oracle.reconstruct_views computes the partial sum over any subset of views with the
density weights of the full direction set, so the views are cut into contiguous
chunks, each chunk runs in its own thread (numpy releases the interpreter lock in its
array work; BLAS is held to one thread per worker), and the partial volumes are added
in chunk order.  The oracle's arithmetic is unchanged.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle


def host_threads() -> int:
    """Threads to use: the CPUs this process may run on, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:   # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def reconstruct_views(images, dirs, dist, geo, vaxes=None, views=None, voxels=None, threads=None):
    from threadpoolctl import threadpool_limits
    sel = np.arange(np.asarray(dirs).shape[0]) if views is None else np.asarray(views)
    t = min(threads or host_threads(), len(sel))
    chunks = [c for c in np.array_split(sel, t) if len(c)]

    def part(c):
        return oracle.reconstruct_views(images, dirs, dist, geo, vaxes=vaxes, views=c, voxels=voxels)

    with threadpool_limits(1):
        with ThreadPoolExecutor(len(chunks)) as ex:
            parts = list(ex.map(part, chunks))
    out = parts[0]
    for p in parts[1:]:
        out = out + p
    return out


def batch_job_at_voxels(job: int, voxels):
    """Oracle values of job `job` of the batched workload at the given voxels: the job's
    seeded inputs are generated again here (the generator is deterministic), the images
    rounded to FP32 as the GPU receives them, and the view sum taken at the voxels' taps
    (oracle.reconstruct_at_voxels).  Runs in a worker process of a spawn pool."""
    from threadpoolctl import threadpool_limits
    from synth import workloads
    w = workloads.batch_jobs()[job]
    with threadpool_limits(1):
        _, dirs, dist, imgs = workloads.make_workload(w)
        geo = oracle.Geometry(w.n_vox, w.M, w.K, w.voxel, w.wavelength, w.sigma, w.epsilon, ewald=w.ewald,
                              weight_mode=w.weight_mode, eps_sampling=w.eps_sampling, i_in=w.i_in)
        return oracle.reconstruct_at_voxels(imgs.astype(np.float32).astype(np.float64), dirs, dist, geo, voxels)
