"""Every supported detector size M (all 2,3,5-smooth M in [16, 256]): the plane stacks and
the whole reconstruction against the oracle, including the sizes whose transform is split
into 2 x 2 or 3 x 3 blocks (162, 180, 200, 216, 225, 240, 243, 250, 256), odd sizes (whose
stack rows cannot be fetched as 16-byte chunks, so general-frame gridding serves them), and
16-bit plane storage on a few of them.  Bar: rel-L2 and max|d| / max|ref| <= 1e-5 (FP32)."""
import numpy as np
import pytest

import oracle
import _problems
from test_gpu_parity import assert_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIZES = _problems.smooth_sizes()


def _oracle_stacks(pb):
    geo = pb.oracle_geometry()
    u, v, d = oracle.frames(pb.dirs, pb.vaxes)
    W = oracle.density_weights(u, v, d, geo)
    P = oracle.filtered_spectra(oracle.spectrum(oracle.contrast(pb.images.astype(np.float64), pb.i_in)),
                                pb.dist, W, geo)
    return P, [np.transpose(oracle.depth_planes(P[i], geo), (1, 0, 2)) for i in range(pb.n)]


@pytest.mark.parametrize("m", SIZES)
def test_size_plane_stacks_and_reconstruction_match_oracle(m):
    from paper_2206_09151_amd import tomo
    pb = _problems.size_problem(m)
    print(f"size {m}: N={pb.n_vox} K={pb.n_planes} views={pb.n} {pb.weight_mode}", flush=True)
    plan = tomo.Plan(pb.params(angle_batch=2), pb.dirs, pb.dist)
    dev = torch.device("cuda:0")
    img = torch.from_numpy(pb.images).to(dev)
    st = torch.full(plan.stack_shape(pb.n), float("nan"), dtype=torch.float32, device=dev)
    plan.backpropagate(img, 0, pb.n, st)
    vol = torch.full((pb.n_vox,) * 3, float("nan"), dtype=torch.float32, device=dev)
    plan.reconstruct(img, vol)
    got_st = st.cpu().numpy()
    P, ref_st = _oracle_stacks(pb)
    for i in range(pb.n):
        assert_close(got_st[i], ref_st[i], 1e-5, (m, "planes", i))
    ref = oracle.reconstruct(pb.images.astype(np.float64), pb.dirs, pb.dist, pb.oracle_geometry())
    assert_close(vol.cpu().numpy(), ref, 1e-5, (m, "volume"))
    plan.destroy()


@pytest.mark.parametrize("m", [160, 192, 256])
@pytest.mark.parametrize("per_launch", [1, 3, 4, 9])
def test_row_split_planes_for_every_view_mapping(m, per_launch):
    """The row-split plane kernels (160, 192, 256) deal a launch's (view, pair, block) units over
    the XCDs one way for 1, 2 or 4 views and another for more: nine views through launches of
    1, 3, 4 or 9 views (ragged last launches included), every stack against the oracle."""
    from paper_2206_09151_amd import tomo
    pb = _problems.size_problem(m, n=9)
    plan = tomo.Plan(pb.params(angle_batch=per_launch), pb.dirs, pb.dist)
    dev = torch.device("cuda:0")
    img = torch.from_numpy(pb.images).to(dev)
    st = torch.full(plan.stack_shape(per_launch), float("nan"), dtype=torch.float32, device=dev)
    _, ref_st = _oracle_stacks(pb)
    for first in range(0, pb.n, per_launch):
        nb = min(per_launch, pb.n - first)
        plan.backpropagate(img[first:first + nb].contiguous(), first, nb, st)
        got = st.cpu().numpy()
        for i in range(nb):
            assert_close(got[i], ref_st[first + i], 1e-5, (m, per_launch, first + i))
    plan.destroy()


@pytest.mark.parametrize("m", [25, 27, 162, 200, 225, 243, 250])
def test_size_filtered_spectra_match_oracle(m):
    from paper_2206_09151_amd import tomo
    pb = _problems.size_problem(m)
    plan = tomo.Plan(pb.params(), pb.dirs, pb.dist)
    out = torch.empty((pb.n, m, m, 2), dtype=torch.float32, device="cuda:0")
    plan.filtered_spectra(torch.from_numpy(pb.images).to("cuda:0"), 0, pb.n, out)
    got = out.cpu().numpy().astype(np.float64)
    P, _ = _oracle_stacks(pb)
    assert_close(got[..., 0] + 1j * got[..., 1], P, 2e-6, m)
    plan.destroy()


@pytest.mark.parametrize("m,dtype,bound", [(27, 1, 3 * 2.0 ** -9), (45, 2, 3 * 2.0 ** -11),
                                           (225, 2, 3 * 2.0 ** -11), (250, 1, 3 * 2.0 ** -9),
                                           (180, 2, 3 * 2.0 ** -11)])
def test_size_16bit_planes_within_rounding_bound(m, dtype, bound):
    """16-bit plane storage: one rounding of each stored value (3 u in rel-L2)."""
    from paper_2206_09151_amd import tomo
    pb = _problems.size_problem(m)
    plan = tomo.Plan(pb.params(plane_dtype=dtype), pb.dirs, pb.dist)
    vol = torch.empty((pb.n_vox,) * 3, dtype=torch.float32, device="cuda:0")
    plan.reconstruct(torch.from_numpy(pb.images).to("cuda:0"), vol)
    got = vol.cpu().numpy().astype(np.float64)
    ref = oracle.reconstruct(pb.images.astype(np.float64), pb.dirs, pb.dist, pb.oracle_geometry())
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"size {m} dtype {dtype}: rel-L2 {rel:.3e}", flush=True)
    assert rel < bound
    plan.destroy()


@pytest.mark.parametrize("m", [32, 45, 128, 256])
def test_single_view_plan_matches_oracle(m):
    """A scan of one view (the degenerate quadrature: the axis ramp gives it the whole half
    turn, pi; the isotropic ramp 2|q|): every launch holds one view, so the plane kernels take
    their one-view XCD mapping and the gridding launches one view; stack and volume against
    the oracle."""
    from paper_2206_09151_amd import tomo
    pb = _problems.size_problem(m, n=1)
    print(f"size {m}: one view, N={pb.n_vox} K={pb.n_planes} {pb.weight_mode}", flush=True)
    plan = tomo.Plan(pb.params(), pb.dirs, pb.dist)
    dev = torch.device("cuda:0")
    img = torch.from_numpy(pb.images).to(dev)
    st = torch.full(plan.stack_shape(1), float("nan"), dtype=torch.float32, device=dev)
    plan.backpropagate(img, 0, 1, st)
    vol = torch.full((pb.n_vox,) * 3, float("nan"), dtype=torch.float32, device=dev)
    plan.reconstruct(img, vol)
    _, ref_st = _oracle_stacks(pb)
    assert_close(st.cpu().numpy()[0], ref_st[0], 1e-5, (m, "planes"))
    ref = oracle.reconstruct(pb.images.astype(np.float64), pb.dirs, pb.dist, pb.oracle_geometry())
    assert_close(vol.cpu().numpy(), ref, 1e-5, (m, "volume"))
    plan.destroy()
