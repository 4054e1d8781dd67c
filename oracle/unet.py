"""FP64 CPU oracle of the learned artefact-correction network (a small 3D U-Net) and
its training step.  This part is not in the paper: it corrects the sparse-angle
artefacts of the reconstruction, trained on pairs (sparse-view reconstruction ->
dense-view reconstruction) that the method itself produces.

TEST INFRASTRUCTURE.  Only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import this module.  Plain numpy in float64; numpy.einsum
(a channel contraction) is the only library primitive.

Architecture (volumes [C][D][H][W], D = H = W = n, n a multiple of 4; every conv is
3x3x3 with zero padding 1 and a bias; ReLU after every conv except the last):

  e1 = relu(conv(relu(conv(x, 1->16)), 16->16))             level 1, n^3
  e2 = relu(conv(relu(conv(pool(e1), 16->32)), 32->32))     level 2, (n/2)^3
  b  = relu(conv(relu(conv(pool(e2), 32->64)), 64->64))     level 3, (n/4)^3
  d2 = relu(conv(relu(conv([up(b), e2], 96->32)), 32->32))  level 2
  d1 = relu(conv(relu(conv([up(d2), e1], 48->16)), 16->16)) level 1
  y  = x + conv1x1(d1, 16->1)                               residual output

pool = 2x2x2 average, up = 2x nearest-neighbour repeat, [a, b] = channel concatenation
(upsampled features first).  Loss: mean squared error over the voxels.  Optimiser:
Adam (Kingma & Ba 2015, Algorithm 1) with bias correction.

Parameter vector (float32 on the device, float64 here): for each layer in the order
above, its weights [Cout][Cin][3][3][3] ([1][16] for the last) then its bias [Cout].
"""
from __future__ import annotations

import numpy as np

__all__ = ["LAYERS", "param_count", "unpack", "bf16_round", "conv3d", "conv3d_backward", "pool2",
           "pool2_backward", "up2", "up2_backward", "forward", "backward", "mse", "adam_step"]

# (name, Cin, Cout, kernel edge)
LAYERS = [("e1a", 1, 16, 3), ("e1b", 16, 16, 3), ("e2a", 16, 32, 3), ("e2b", 32, 32, 3),
          ("b_a", 32, 64, 3), ("b_b", 64, 64, 3), ("d2a", 96, 32, 3), ("d2b", 32, 32, 3),
          ("d1a", 48, 16, 3), ("d1b", 16, 16, 3), ("out", 16, 1, 1)]


def param_count():
    return sum(co * ci * k ** 3 + co for _, ci, co, k in LAYERS)


def bf16_round(a):
    """Nearest bfloat16 (8 significant bits, ties to the even significand) of float32 values."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta, bf16=False):
    """{name: (w [Cout][Cin][k][k][k], b [Cout])} of the flat parameter vector; with bf16
    the weights are their BF16 roundings (the precision the network's convolutions use)."""
    out, off = {}, 0
    for name, ci, co, k in LAYERS:
        nw = co * ci * k ** 3
        w = theta[off:off + nw].reshape(co, ci, k, k, k)
        if bf16:
            w = bf16_round(w)
        off += nw
        out[name] = (w, theta[off:off + co])
        off += co
    return out


# ----------------------------------------------------------------------------- building blocks
def conv3d(x, w, b):
    """out[o] = b[o] + sum_c sum_t w[o, c, t] x[c, r + t - h] (cross-correlation, zero padding h = k//2)."""
    k = w.shape[-1]
    h = k // 2
    c, d, hh, ww = x.shape
    xp = np.pad(x, ((0, 0), (h, h), (h, h), (h, h)))
    out = np.broadcast_to(b[:, None, None, None], (w.shape[0], d, hh, ww)).copy()
    for dz in range(k):
        for dy in range(k):
            for dx in range(k):
                out += np.einsum("oc,czyx->ozyx", w[:, :, dz, dy, dx], xp[:, dz:dz + d, dy:dy + hh, dx:dx + ww])
    return out


def conv3d_backward(x, w, g):
    """Gradients of sum(g * conv3d(x, w, b)) with respect to x, w and b."""
    k = w.shape[-1]
    h = k // 2
    c, d, hh, ww = x.shape
    xp = np.pad(x, ((0, 0), (h, h), (h, h), (h, h)))
    gx = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dz in range(k):
        for dy in range(k):
            for dx in range(k):
                sl = (slice(None), slice(dz, dz + d), slice(dy, dy + hh), slice(dx, dx + ww))
                gw[:, :, dz, dy, dx] = np.einsum("ozyx,czyx->oc", g, xp[sl])
                gx[sl] += np.einsum("oc,ozyx->czyx", w[:, :, dz, dy, dx], g)
    return gx[:, h:h + d, h:h + hh, h:h + ww], gw, g.sum(axis=(1, 2, 3))


def pool2(x):
    c, d, h, w = x.shape
    return x.reshape(c, d // 2, 2, h // 2, 2, w // 2, 2).mean(axis=(2, 4, 6))


def pool2_backward(g):
    return up2(g) / 8.0


def up2(x):
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def up2_backward(g):
    c, d, h, w = g.shape
    return g.reshape(c, d // 2, 2, h // 2, 2, w // 2, 2).sum(axis=(2, 4, 6))


def _relu(z):
    return np.maximum(z, 0.0)


# ----------------------------------------------------------------------------- network
def forward(theta, x, bf16=False):
    """y = x + f(x) for one volume x [n][n][n]; returns (y, cache)."""
    p = unpack(theta, bf16)
    a = {}
    a["x"] = x[None]
    a["e1a"] = _relu(conv3d(a["x"], *p["e1a"]))
    a["e1b"] = _relu(conv3d(a["e1a"], *p["e1b"]))
    a["p1"] = pool2(a["e1b"])
    a["e2a"] = _relu(conv3d(a["p1"], *p["e2a"]))
    a["e2b"] = _relu(conv3d(a["e2a"], *p["e2b"]))
    a["p2"] = pool2(a["e2b"])
    a["b_a"] = _relu(conv3d(a["p2"], *p["b_a"]))
    a["b_b"] = _relu(conv3d(a["b_a"], *p["b_b"]))
    a["c2"] = np.concatenate([up2(a["b_b"]), a["e2b"]], axis=0)
    a["d2a"] = _relu(conv3d(a["c2"], *p["d2a"]))
    a["d2b"] = _relu(conv3d(a["d2a"], *p["d2b"]))
    a["c1"] = np.concatenate([up2(a["d2b"]), a["e1b"]], axis=0)
    a["d1a"] = _relu(conv3d(a["c1"], *p["d1a"]))
    a["d1b"] = _relu(conv3d(a["d1a"], *p["d1b"]))
    y = x + conv3d(a["d1b"], *p["out"])[0]
    return y, a


def backward(theta, cache, gy, bf16=False):
    """Gradient of sum(gy * y) with respect to the parameter vector (and to x); with bf16
    the weights are rounded as in forward (gradients are taken at the rounded weights)."""
    p = unpack(theta, bf16)
    a = cache
    grads = {}

    def step(name, inp, gout, relu_out=None):
        if relu_out is not None:
            gout = gout * (relu_out > 0)
        gx, gw, gb = conv3d_backward(inp, p[name][0], gout)
        grads[name] = (gw, gb)
        return gx

    g = step("out", a["d1b"], gy[None])
    g = step("d1b", a["d1a"], g, a["d1b"])
    g = step("d1a", a["c1"], g, a["d1a"])
    g_up1, g_e1b = g[:32], g[32:]
    g = step("d2b", a["d2a"], up2_backward(g_up1), a["d2b"])
    g = step("d2a", a["c2"], g, a["d2a"])
    g_upb, g_e2b = g[:64], g[64:]
    g = step("b_b", a["b_a"], up2_backward(g_upb), a["b_b"])
    g = step("b_a", a["p2"], g, a["b_a"])
    g = step("e2b", a["e2a"], pool2_backward(g) + g_e2b, a["e2b"])
    g = step("e2a", a["p1"], g, a["e2a"])
    g = step("e1b", a["e1a"], pool2_backward(g) + g_e1b, a["e1b"])
    g = step("e1a", a["x"], g, a["e1a"])
    gtheta = np.concatenate([np.concatenate([grads[n][0].ravel(), grads[n][1]]) for n, _, _, _ in LAYERS])
    return gtheta, gy + g[0]


def mse(y, t):
    """Mean squared error and its gradient with respect to y."""
    r = y - t
    return float(np.mean(r * r)), 2.0 * r / r.size


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step t >= 1); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
