"""GPU parity of the artefact-correction network's kernels against the FP64 oracle
(forward, loss, every layer's gradient, Adam), determinism, and a training run that
shows what the trained network gains over the plain sparse-view reconstruction.

Tolerances: the GPU convolves with BF16-rounded weights (the oracle rounds the same
FP32 parameters the same way) and sums in FP32: forward rel-L2 <= 1e-5 on the network's
correction y - x, gradients rel-L2 <= 1e-4 per layer (sums over every voxel)."""
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


@pytest.mark.parametrize("n", [8, 16, 24])
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


@pytest.mark.parametrize("n", [8, 16])
def test_gradient_matches_oracle(n):
    theta, x, t = _case(n, 21 + n)
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
    off = 0
    for name, ci, co, k in ou.LAYERS:
        nw = co * ci * k ** 3
        for part, sl in (("w", slice(off, off + nw)), ("b", slice(off + nw, off + nw + co))):
            err = _rel(got[sl], want[sl])
            print(f"unet grad n={n} {name}.{part}: rel-L2 {err:.3g}", flush=True)
            assert err <= 1e-4, (name, part, err)
        off += nw + co
    net.destroy()


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
