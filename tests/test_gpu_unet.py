"""GPU parity of the artefact-correction network's kernels against the FP64 oracle
(forward, loss, every layer's gradient, Adam), determinism, and a training run that
shows what the trained network gains over the plain sparse-view reconstruction.

Tolerances: the GPU convolves with BF16-rounded weights (the oracle rounds the same
FP32 parameters the same way); on the matrix cores each FP32 activation or gradient is
split into BF16 hi + lo (relative remainder <= 2^-18) and the products are summed in FP32:
forward rel-L2 <= 1e-5 on the network's correction y - x, gradients rel-L2 <= 1e-4 per
layer (sums over every voxel) wherever the gradient is unique: a ReLU unit whose
pre-activation lies within the GPU path's rounding of zero (found by the oracle, see
AMBIGUOUS_REL) may switch either way, and the gradients of its layer and of the layers before
it are then checked to 1e-2 only.  n = 20 leaves ragged tiles in every kernel (levels of 20,
10 and 5 voxels, the last two not multiples of 4); one of its cases has such a unit in e1b, the
other none, so that at this size too every layer is held to 1e-4."""
import numpy as np
import pytest

import oracle.unet as ou
from synth import netinit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
tomo = pytest.importorskip("paper_2206_09151_amd.tomo")
unet = pytest.importorskip("paper_2206_09151_amd.unet")


def _dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", dtype)


def _case(n, seed):
    rng = np.random.default_rng(seed)
    theta = netinit.init_params(seed, out_scale=0.2)
    # non-zero biases so every bias path is exercised
    theta = theta + (rng.standard_normal(theta.size) * 0.02).astype(np.float32) * (np.abs(theta) == 0)
    x = rng.standard_normal((n, n, n)).astype(np.float32)
    t = rng.standard_normal((n, n, n)).astype(np.float32)
    return theta, x, t


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# input (oracle cache key) of every ReLU layer, in forward order
_RELU_INPUT = {"e1a": "x", "e1b": "e1a", "e2a": "p1", "e2b": "e2a", "b_a": "p2", "b_b": "b_a", "d2a": "c2",
               "d2b": "d2a", "d1a": "c1", "d1b": "d1a"}
# A ReLU decision is taken in floating point: a pre-activation within the GPU path's rounding
# of zero may land on either side (the matrix-core products carry a relative error of up to
# 2^-18 each, about 4e-6 of a layer's mean |pre-activation| after a 27 * cin sum).  Units
# closer to zero than AMBIGUOUS_REL * mean|z| make the gradients of their layer and of every
# earlier layer (all of them its ancestors) non-unique.
AMBIGUOUS_REL = 5e-6


def _last_ambiguous_layer(theta64, cache):
    """Index (in LAYERS order) of the last layer with a near-zero pre-activation, or -1."""
    p = ou.unpack(theta64, True)
    last = -1
    for i, (name, _, _, _) in enumerate(ou.LAYERS):
        if name not in _RELU_INPUT:
            continue
        z = np.abs(ou.conv3d(cache[_RELU_INPUT[name]], *p[name]))
        if z.min() < AMBIGUOUS_REL * z.mean():
            last = i
    return last


@pytest.mark.parametrize("n", [8, 16, 20, 24])
def test_forward_matches_oracle(n):
    theta, x, _ = _case(n, 11 + n)
    net = unet.Net(n)
    y = torch.empty((n, n, n), device="cuda:0")
    net.forward(_dev(theta), _dev(x), y)
    torch.cuda.synchronize()
    want, _ = ou.forward(theta.astype(np.float64), x.astype(np.float64), bf16=True)
    got = y.cpu().numpy().astype(np.float64)
    err = _rel(got - x, want - x)
    print(f"unet forward n={n}: rel-L2 of the correction {err:.3g}", flush=True)
    assert err <= 1e-5
    net.destroy()


# (size, seed): seeds 21 + n as before; at n = 20 seed 41 has a near-zero unit in e1b, and
# seed 45 none, so that every layer of the ragged size also meets the 1e-4 bar
@pytest.mark.parametrize("n,seed,unique", [(8, 29, False), (16, 37, False), (20, 41, False), (20, 45, True)])
def test_gradient_matches_oracle(n, seed, unique):
    theta, x, t = _case(n, seed)
    net = unet.Net(n)
    g = torch.empty(theta.size, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float64, device="cuda:0")
    net.gradient(_dev(theta), _dev(x), _dev(t), g, loss)
    torch.cuda.synchronize()
    th64 = theta.astype(np.float64)
    y, cache = ou.forward(th64, x.astype(np.float64), bf16=True)
    want_loss, gy = ou.mse(y, t.astype(np.float64))
    want, _ = ou.backward(th64, cache, gy, bf16=True)
    assert abs(loss.item() - want_loss) <= 1e-5 * want_loss
    got = g.cpu().numpy().astype(np.float64)
    last = _last_ambiguous_layer(th64, cache)
    if unique:
        assert last == -1, "this case has no near-zero ReLU unit: every gradient is unique"
    off = 0
    bad = []
    for i, (name, ci, co, k) in enumerate(ou.LAYERS):
        nw = co * ci * k ** 3
        # unique result: the FP32 bar; behind a near-zero ReLU unit: still the same gradient
        # up to that unit's flip (a few voxels' contributions)
        tol = 1e-4 if i > last else 1e-2
        for part, sl in (("w", slice(off, off + nw)), ("b", slice(off + nw, off + nw + co))):
            err = _rel(got[sl], want[sl])
            print(f"unet grad n={n} {name}.{part}: rel-L2 {err:.3g} (bar {tol:g})", flush=True)
            if not err <= tol:
                bad.append((name, part, err))
        off += nw + co
    net.destroy()
    assert not bad, bad
    assert last < len(ou.LAYERS) - 3, "the case leaves too few layers with a unique gradient"


def test_adam_matches_oracle():
    rng = np.random.default_rng(5)
    p = ou.param_count()
    # parameters small against the step, so FP32 storage of theta keeps the update's digits
    th, gr = (rng.standard_normal(p) * 1e-4).astype(np.float32), rng.standard_normal(p).astype(np.float32)
    m, v = (rng.standard_normal(p) * 0.1).astype(np.float32), (rng.random(p) * 0.1).astype(np.float32)
    net = unet.Net(8)
    dt, dm, dv = _dev(th), _dev(m), _dev(v)
    net.adam(dt, _dev(gr), dm, dv, step=3, lr=1e-3)
    torch.cuda.synchronize()
    want, wm, wv = ou.adam_step(th.astype(np.float64), gr.astype(np.float64), m.astype(np.float64),
                                v.astype(np.float64), 3, 1e-3)
    assert _rel(dt.cpu().numpy() - th, want - th) <= 1e-5
    assert _rel(dm.cpu().numpy(), wm) <= 1e-6 and _rel(dv.cpu().numpy(), wv) <= 1e-6
    net.destroy()


def test_gradient_is_bitwise_reproducible():
    theta, x, t = _case(16, 3)
    net = unet.Net(16)
    outs = []
    for _ in range(2):
        g = torch.empty(theta.size, device="cuda:0")
        loss = torch.empty(1, dtype=torch.float64, device="cuda:0")
        net.gradient(_dev(theta), _dev(x), _dev(t), g, loss)
        torch.cuda.synchronize()
        outs.append((g.cpu().numpy(), loss.item()))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]
    net.destroy()


def test_trained_network_beats_the_sparse_reconstruction():
    """Pairs (10-view -> 90-view reconstruction, 32^3 DT, blob phantoms) made by the
    library's own reconstruction; 24 for training, 4 held out.  After 150 Adam steps the
    held-out error against the dense reconstruction is at most half the error of the
    sparse reconstruction itself (the untrained network is the identity)."""
    from synth import forward, phantoms, scan
    n, dx, lam, R = 32, 1e-10, 0.05e-10, 60e-10

    def recon(ph, nviews):
        dirs = scan.single_axis(nviews, 180.0)
        dist = np.full(nviews, R)
        im = forward.born_images(ph, dirs, n, dx, lam, dist, 0.0, device="cuda").astype(np.float32)
        plan = tomo.Plan(tomo.Params(n_vox=n, n_angles=nviews, voxel_size=dx, wavelength=lam, sigma=0.0,
                                     epsilon=1e-3), dirs, dist)
        v = torch.empty((n, n, n), device="cuda:0")
        plan.reconstruct(_dev(im), v)
        plan.destroy()
        return v

    pairs = []
    for s in range(28):
        ph = phantoms.draw_blobs(700 + s, n, dx, 0.0, 1.2e-10, 2e-5, sigma=0.0, count=40, support=0.4)
        pairs.append((recon(ph, 10), recon(ph, 90)))
    scale = float(torch.sqrt(torch.stack([(d * d).mean() for _, d in pairs]).mean()))
    pairs = [(a / scale, b / scale) for a, b in pairs]
    train, held = pairs[:24], pairs[24:]
    net = unet.Net(n)
    theta = _dev(netinit.init_params(9))
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    g = torch.empty_like(theta)
    loss = torch.empty(1, dtype=torch.float64, device="cuda:0")
    for step in range(1, 151):
        a, b = train[(step - 1) % len(train)]
        net.gradient(theta, a, b, g, loss)
        net.adam(theta, g, m, v, step, 1e-3)
    y = torch.empty((n, n, n), device="cuda:0")
    base = corr = 0.0
    for a, b in held:
        net.forward(theta, a, y)
        torch.cuda.synchronize()
        base += float(((a - b) ** 2).mean())
        corr += float(((y - b) ** 2).mean())
    print(f"held-out MSE: sparse {base / 4:.4g}, corrected {corr / 4:.4g} (ratio {corr / base:.3f})", flush=True)
    assert corr <= 0.5 * base
    net.destroy()
