"""The training-pair generator: its batched first-Born images equal the per-view image
model (synth.forward.born_images) for the same phantom and views, and its phantoms are
reproducible from their index."""
import numpy as np

from synth import forward, learning, scan


def test_batched_images_equal_per_view_model():
    ph = learning.pair_phantom(3, n_vox=24)
    dirs = scan.single_axis(5, 180.0)
    dist = np.full(5, 500e-10)
    a = learning.born_images_batched(ph, dirs, 24, 1e-10, 0.0197e-10, dist, 0.0, device="cpu", chunk=2).numpy()
    b = forward.born_images(ph, dirs, 24, 1e-10, 0.0197e-10, dist, 0.0).astype(np.float32)
    assert np.array_equal(a, b)


def test_pair_phantoms_are_seeded_by_index():
    a, b = learning.pair_phantom(17), learning.pair_phantom(17)
    assert np.array_equal(a.centres, b.centres) and np.array_equal(a.delta, b.delta)
    assert len(learning.pair_phantom(0).delta) == 8 and len(learning.pair_phantom(16).delta) == 24
    assert not np.array_equal(learning.pair_phantom(18).centres[:8], a.centres[:8])
    assert learning.DENSE_VIEWS % learning.SPARSE_VIEWS == 0     # the sparse views are every 24th dense view
