"""The oracle's tap-point form of the depth planes (oracle.reconstruct_at_voxels) against
its FFT form (oracle.reconstruct): the plane values at a voxel's taps written out as the
inverse DFT of the propagated spectrum at those points must give the same view sums as
inverse FFTs of whole planes followed by the trilinear gather (the inverse DFT of the
F2 definition before eq. (3), evaluated two ways)."""
import numpy as np
import pytest

import oracle
import _problems


@pytest.mark.parametrize("name", ["axis32", "sphere45", "pct64", "oddk16", "vaxes32", "narrow48", "iin32",
                                  "pole24"])
def test_tap_evaluation_equals_fft_planes(name):
    pb = _problems.make(name)
    geo = pb.oracle_geometry()
    rng = np.random.default_rng(17)
    vox = np.concatenate([rng.integers(0, pb.n_vox, size=(40, 3)),
                          [[0, 0, 0], [pb.n_vox - 1] * 3, [pb.n_vox // 2] * 3]])
    imgs = pb.images.astype(np.float64)
    want = oracle.reconstruct(imgs, pb.dirs, pb.dist, geo, vaxes=pb.vaxes, voxels=vox)
    got = oracle.reconstruct_at_voxels(imgs, pb.dirs, pb.dist, geo, vox, vaxes=pb.vaxes)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
