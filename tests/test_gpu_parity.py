"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerance: relative L2 <= 1e-5 for FP32 results against FP64 (the stated bar
for FP32), and beside it an element-wise bound max|got - ref| <= 1e-5 max|ref|, so
that a few wrong voxels (a mis-mapped tile, a ragged edge) cannot hide under the
volume norm; per-stage checks are tighter where the arithmetic allows.
"""
import numpy as np
import pytest

import oracle
import _oracle_par
import _problems

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def _tomo():
    from paper_2206_09151_amd import tomo
    return tomo


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def assert_close(got, ref, tol, what=""):
    """rel-L2 <= tol and max|got - ref| <= tol * max|ref|."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rel = _rel(got, ref)
    worst = float(np.abs(got - ref).max() / np.abs(ref).max())
    assert rel < tol and worst < tol, (what, rel, worst)


def _oracle_inputs(pb):
    return pb.images.astype(np.float64)


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def _plan(pb, **kw):
    tomo = _tomo()
    return tomo.Plan(pb.params(**kw), pb.dirs, pb.dist, vaxes=pb.vaxes)


@pytest.mark.parametrize("name", ["axis32", "sphere45", "sampling32", "m96", "m256", "m160", "m192", "iin32",
                                  "m256iin", "pole24", "m128"])
def test_filtered_spectra_match_oracle(dev, name):
    pb = _problems.make(name)
    plan = _plan(pb, angle_batch=pb.n)
    img = torch.from_numpy(pb.images).to(dev)
    out = torch.empty((pb.n, pb.n_pix, pb.n_pix, 2), dtype=torch.float32, device=dev)
    plan.filtered_spectra(img, 0, pb.n, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    got = got[..., 0] + 1j * got[..., 1]
    geo = pb.oracle_geometry()
    u, v, d = oracle.frames(pb.dirs, pb.vaxes)
    W = oracle.density_weights(u, v, d, geo)
    P = oracle.filtered_spectra(oracle.spectrum(oracle.contrast(_oracle_inputs(pb), pb.i_in)), pb.dist, W, geo)
    assert_close(got, P, 2e-6, name)


@pytest.mark.parametrize("name", ["axis32", "ragged44", "sphere45", "pct64", "oddk16", "m80", "m256", "m256sph", "m160",
                                  "m192", "m128", "iin32", "m256iin"])
def test_plane_stacks_match_oracle(dev, name):
    pb = _problems.make(name)
    plan = _plan(pb, angle_batch=pb.n)
    img = torch.from_numpy(pb.images).to(dev)
    st = torch.empty(plan.stack_shape(pb.n), dtype=torch.float32, device=dev)
    plan.backpropagate(img, 0, pb.n, st)
    torch.cuda.synchronize()
    got = st.cpu().numpy()
    geo = pb.oracle_geometry()
    u, v, d = oracle.frames(pb.dirs, pb.vaxes)
    W = oracle.density_weights(u, v, d, geo)
    P = oracle.filtered_spectra(oracle.spectrum(oracle.contrast(_oracle_inputs(pb), pb.i_in)), pb.dist, W, geo)
    for i in range(pb.n):
        ref = np.transpose(oracle.depth_planes(P[i], geo), (1, 0, 2))  # -> [row][plane][col]
        assert_close(got[i], ref, TOL, (name, i))


@pytest.mark.parametrize("name", ["axis32", "ragged44", "sphere45", "pct64", "sampling32", "oddk16", "narrow48",
                                  "pole24"])
def test_grid_of_oracle_planes_matches_oracle_gather(dev, name):
    """Gridding alone: the oracle's FP64 planes, rounded to FP32, gridded by both sides."""
    pb = _problems.make(name)
    plan = _plan(pb, angle_batch=pb.n)
    geo = pb.oracle_geometry()
    u, v, d = oracle.frames(pb.dirs, pb.vaxes)
    W = oracle.density_weights(u, v, d, geo)
    P = oracle.filtered_spectra(oracle.spectrum(oracle.contrast(_oracle_inputs(pb), pb.i_in)), pb.dist, W, geo)
    stacks = np.stack([oracle.depth_planes(P[i], geo) for i in range(pb.n)]).astype(np.float32)
    ref = np.zeros((pb.n_vox,) * 3)
    for i in range(pb.n):
        ref += oracle.gather(stacks[i].astype(np.float64), u[i], v[i], d[i], geo)
    dev_st = torch.from_numpy(np.ascontiguousarray(np.transpose(stacks, (0, 2, 1, 3)))).to(dev)
    vol = torch.zeros((pb.n_vox,) * 3, dtype=torch.float32, device=dev)
    plan.grid(dev_st, 0, pb.n, vol)
    torch.cuda.synchronize()
    assert_close(vol.cpu().numpy(), ref, 2e-6, name)


@pytest.mark.parametrize("name", _problems.SMALL)
def test_reconstruct_matches_oracle(dev, name):
    pb = _problems.make(name)
    plan = _plan(pb, angle_batch=7)
    img = torch.from_numpy(pb.images).to(dev)
    vol = torch.full((pb.n_vox,) * 3, float("nan"), dtype=torch.float32, device=dev)
    plan.reconstruct(img, vol)
    got = vol.cpu().numpy()
    ref = _oracle_par.reconstruct_views(_oracle_inputs(pb), pb.dirs, pb.dist, pb.oracle_geometry(), vaxes=pb.vaxes)
    assert np.isfinite(got).all()
    assert_close(got, ref, TOL, name)


def test_reconstruct_is_bitwise_deterministic(dev):
    pb = _problems.make("sphere45")
    plan = _plan(pb, angle_batch=4)
    img = torch.from_numpy(pb.images).to(dev)
    a = torch.empty((pb.n_vox,) * 3, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    plan.reconstruct(img, a)
    plan.reconstruct(img, b)
    assert torch.equal(a, b)


def test_angle_batch_does_not_change_result(dev):
    pb = _problems.make("axis32")
    img = torch.from_numpy(pb.images).to(dev)
    outs = []
    for ab in (1, 7, pb.n):
        plan = _plan(pb, angle_batch=ab)
        v = torch.empty((pb.n_vox,) * 3, dtype=torch.float32, device=dev)
        plan.reconstruct(img, v)
        outs.append(v.cpu().numpy().astype(np.float64))
    for o in outs[1:]:
        assert _rel(o, outs[0]) < 1e-6


def test_backpropagate_then_grid_equals_reconstruct(dev):
    pb = _problems.make("ragged44")
    plan = _plan(pb, angle_batch=5)
    img = torch.from_numpy(pb.images).to(dev)
    full = torch.empty((pb.n_vox,) * 3, dtype=torch.float32, device=dev)
    plan.reconstruct(img, full)
    acc = torch.zeros_like(full)
    st = torch.empty(plan.stack_shape(5), dtype=torch.float32, device=dev)
    for first in range(0, pb.n, 5):
        nb = min(5, pb.n - first)
        plan.backpropagate(img[first:first + nb].contiguous(), first, nb, st)
        plan.grid(st, first, nb, acc)
    torch.cuda.synchronize()
    assert torch.equal(acc, full)


def test_domain_error_reported_and_cleared(dev):
    tomo = _tomo()
    pb = _problems.make("oddk16")
    plan = _plan(pb)
    bad = pb.images.copy()
    bad[2, 3, 4] = 0.0
    bad[1, 0, 0] = np.nan
    vol = torch.empty((pb.n_vox,) * 3, dtype=torch.float32, device=dev)
    with pytest.raises(tomo.TomoError) as e:
        plan.reconstruct(torch.from_numpy(bad).to(dev), vol)
    assert e.value.status == tomo.EDOMAIN
    plan.reconstruct(torch.from_numpy(pb.images).to(dev), vol)   # flag was cleared


@pytest.mark.parametrize("name", ["axis32", "sphere45"])
def test_async_reconstruct_equals_reconstruct(dev, name):
    """Enqueued reconstructions (no per-call synchronisation) give the synchronous result bit
    for bit, also when several are in flight on the stream before one sync."""
    pb = _problems.make(name)
    plan = _plan(pb, angle_batch=5)
    img = torch.from_numpy(pb.images).to(dev)
    ref = torch.empty((pb.n_vox,) * 3, dtype=torch.float32, device=dev)
    plan.reconstruct(img, ref)
    out = torch.full_like(ref, float("nan"))
    for _ in range(3):
        plan.reconstruct_async(img, out)
    plan.sync()
    assert torch.equal(out, ref)


def test_async_reconstruct_reports_domain_error_at_sync(dev):
    tomo = _tomo()
    pb = _problems.make("oddk16")
    plan = _plan(pb)
    bad = pb.images.copy()
    bad[0, 5, 5] = -1.0
    vol = torch.empty((pb.n_vox,) * 3, dtype=torch.float32, device=dev)
    plan.reconstruct_async(torch.from_numpy(bad).to(dev), vol)   # returns without waiting
    with pytest.raises(tomo.TomoError) as e:
        plan.sync()
    assert e.value.status == tomo.EDOMAIN
    plan.reconstruct_async(torch.from_numpy(pb.images).to(dev), vol)
    plan.sync()                                                   # flag was cleared


def test_range_errors(dev):
    tomo = _tomo()
    pb = _problems.make("oddk16")
    plan = _plan(pb, angle_batch=2)
    img = torch.from_numpy(pb.images).to(dev)
    st = torch.empty(plan.stack_shape(3), dtype=torch.float32, device=dev)
    with pytest.raises(tomo.TomoError) as e:
        plan.backpropagate(img, 4, 2, st)       # past the last view
    assert e.value.status == tomo.EINVAL
    with pytest.raises(tomo.TomoError):
        plan.grid(st, -1, 1, torch.zeros((pb.n_vox,) * 3, device=dev))


def test_empty_view_range_is_a_no_op(dev):
    """nb = 0 (also at first = n_angles, the end of the range) launches nothing: outputs keep
    their contents, even when the buffers passed are empty tensors."""
    tomo = _tomo()
    pb = _problems.make("oddk16")
    plan = _plan(pb, angle_batch=2)
    img = torch.from_numpy(pb.images).to(dev)
    st = torch.full(plan.stack_shape(2), 7.0, dtype=torch.float32, device=dev)
    vol = torch.full((pb.n_vox,) * 3, -3.0, dtype=torch.float32, device=dev)
    spec = torch.full((2, pb.n_pix, pb.n_pix, 2), 5.0, dtype=torch.float32, device=dev)
    empty_st = torch.empty(plan.stack_shape(0), dtype=torch.float32, device=dev)
    for first in (0, 3, pb.n):
        plan.backpropagate(img, first, 0, st)
        plan.backpropagate_noalloc(img, first, 0, st)
        plan.backpropagate(img, first, 0, empty_st)
        plan.filtered_spectra(img, first, 0, spec)
        plan.grid(st, first, 0, vol)
        plan.grid(empty_st, first, 0, vol)
    torch.cuda.synchronize()
    assert bool((st == 7.0).all()) and bool((vol == -3.0).all()) and bool((spec == 5.0).all())
    # a negative count is a range error, not an empty range
    with pytest.raises(tomo.TomoError) as e:
        plan.backpropagate(img, 0, -1, st)
    assert e.value.status == tomo.EINVAL


@pytest.mark.parametrize("name", ["axis32", "ragged44", "pct64", "oddk16", "m160", "sphere45"])
def test_autotuned_gridding_gives_identical_volumes(name):
    """Plan-time autotuning only picks the voxel rows per gridding thread.  On the
    single-axis path the per-voxel arithmetic is the same, so the volumes are bitwise
    equal (ragged tiles, odd view counts, the flat CT limit and odd K included); on the
    general path the staged box (and so the FP32 box-local coordinates) follows the tile's
    height, which moves only the rounding."""
    tomo = _tomo()
    prob = _problems.make(name)
    imgs = torch.from_numpy(prob.images).to("cuda:0")
    axis = name != "sphere45"
    out = []
    for tune in (0, 1):
        plan = tomo.Plan(prob.params(tune=tune), prob.dirs, prob.dist, vaxes=prob.vaxes)
        assert plan.grid_rows in (0, 2, 4, 8, -8, -4, -2)
        if plan.grid_rows == 2:
            assert axis
        vol = torch.empty((prob.n_vox,) * 3, dtype=torch.float32, device="cuda:0")
        plan.reconstruct(imgs, vol)
        out.append(vol.cpu().numpy())
        plan.destroy()
    if axis:
        assert np.array_equal(out[0], out[1])
    else:
        assert np.linalg.norm(out[0] - out[1]) <= 1e-6 * np.linalg.norm(out[0])


@pytest.mark.parametrize("name", ["axis32", "ragged44", "pct64", "oddk16", "m128"])
def test_two_row_single_axis_gridding_is_bitwise_equal(name):
    """tune = 5 puts single-axis plans on the 2-row gridding tiles; the per-voxel
    arithmetic is that of the 8-row tiles (tune = 0), so the volumes are bitwise equal."""
    tomo = _tomo()
    prob = _problems.make(name)
    imgs = torch.from_numpy(prob.images).to("cuda:0")
    out = []
    for tune, rows in ((0, 8), (5, 2)):
        plan = tomo.Plan(prob.params(tune=tune), prob.dirs, prob.dist, vaxes=prob.vaxes)
        assert plan.grid_rows == rows
        vol = torch.empty((prob.n_vox,) * 3, dtype=torch.float32, device="cuda:0")
        plan.reconstruct(imgs, vol)
        out.append(vol.cpu().numpy())
        plan.destroy()
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("name", ["sphere45", "vaxes32", "m256sph", "m192", "sampling32", "pole24"])
def test_cubic_tile_gridding_matches_oracle(name):
    """The cubic-tile gridding kernel (tune = 2) over general frames, whole volume."""
    tomo = _tomo()
    prob = _problems.make(name)
    plan = tomo.Plan(prob.params(tune=2), prob.dirs, prob.dist, vaxes=prob.vaxes)
    assert plan.grid_rows == 0
    vol = torch.empty((prob.n_vox,) * 3, dtype=torch.float32, device="cuda:0")
    plan.reconstruct(torch.from_numpy(prob.images).to("cuda:0"), vol)
    got = vol.cpu().numpy().astype(np.float64)
    want = oracle.reconstruct(prob.images.astype(np.float64), prob.dirs, prob.dist, prob.oracle_geometry(),
                              vaxes=prob.vaxes)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"cubic tiles {name}: rel-L2 {err:.3g}", flush=True)
    assert_close(got, want, 1e-5, name)


def test_cubic_tile_gridding_over_more_than_64_views_in_one_launch():
    """The FP32 cubic-tile kernel forms the box origins of 64 views at a time; 70 views in one
    launch take a second round of them."""
    tomo = _tomo()
    prob = _problems.make("sphere70")
    plan = tomo.Plan(prob.params(tune=2, angle_batch=70), prob.dirs, prob.dist, vaxes=prob.vaxes)
    assert plan.grid_rows == 0 and plan.batch == 70
    vol = torch.empty((prob.n_vox,) * 3, dtype=torch.float32, device="cuda:0")
    plan.reconstruct(torch.from_numpy(prob.images).to("cuda:0"), vol)
    want = oracle.reconstruct(prob.images.astype(np.float64), prob.dirs, prob.dist, prob.oracle_geometry(),
                              vaxes=prob.vaxes)
    assert_close(vol.cpu().numpy().astype(np.float64), want, 1e-5, "sphere70")
    plan.destroy()


def test_binding_refuses_short_or_mistyped_buffers(dev):
    """The binding checks element type and size against the plan before the call, so a
    buffer the kernels would overrun never reaches a launch."""
    tomo = _tomo()
    pb = _problems.make("axis32")
    plan = _plan(pb, angle_batch=4)
    img = torch.from_numpy(pb.images).to(dev)
    vol = torch.zeros((pb.n_vox,) * 3, dtype=torch.float32, device=dev)
    st = torch.empty(plan.stack_shape(4), dtype=torch.float32, device=dev)
    cases = [
        lambda: plan.backpropagate(img, 0, 4, st.to(torch.bfloat16)),                  # planes of another type
        lambda: plan.backpropagate(img, 0, 4, st[:3]),                                 # 3 stacks for 4 views
        lambda: plan.backpropagate(img[:2].contiguous(), 0, 4, st),                    # 2 images for 4 views
        lambda: plan.grid(st, 0, 4, vol[:-1]),                                         # volume one slab short
        lambda: plan.grid(st, 0, 4, vol.double()),                                     # volume of doubles
        lambda: plan.reconstruct(img[:-1].contiguous(), vol),                          # one image short
        lambda: plan.reconstruct(img.half(), vol),                                     # images of halves
        lambda: plan.filtered_spectra(img, 0, 4, torch.empty((4, 32, 32), device=dev)),  # no imaginary parts
    ]
    for bad in cases:
        with pytest.raises(ValueError):
            bad()
    assert torch.count_nonzero(vol) == 0                                              # nothing ran


@pytest.mark.parametrize("name", ["sampling32", "iin32", "sphere45", "vaxes32", "m256sph", "m192", "pole24",
                                  "m256iin"])
@pytest.mark.parametrize("tune,rows", [(3, -4), (4, -8), (5, -2)])
def test_near_axis_box_gridding_matches_oracle(name, tune, rows):
    """The near-axis LDS-fetch box kernel (tune = 3, 4, 5: 4, 8, 2 voxel rows per thread) over
    general frames: tilted single-axis scans (every footprint fits the box), and directions on
    the sphere and at the poles (many do not: those views take its global-gather path), whole
    volume."""
    tomo = _tomo()
    prob = _problems.make(name)
    plan = tomo.Plan(prob.params(tune=tune, angle_batch=5), prob.dirs, prob.dist, vaxes=prob.vaxes)
    assert plan.grid_rows == rows
    vol = torch.empty((prob.n_vox,) * 3, dtype=torch.float32, device="cuda:0")
    plan.reconstruct(torch.from_numpy(prob.images).to("cuda:0"), vol)
    want = _oracle_par.reconstruct_views(prob.images.astype(np.float64), prob.dirs, prob.dist,
                                         prob.oracle_geometry(), vaxes=prob.vaxes)
    assert_close(vol.cpu().numpy(), want, 1e-5, name)
