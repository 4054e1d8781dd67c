"""Seeded initial parameters of the artefact-correction network (He-normal weights,
zero biases, zero output layer so the untrained network is the identity), in the
parameter layout of the network: per layer weights [Cout][Cin][k][k][k] then bias.
Holds only random draws and the layer shapes, no network arithmetic."""
from __future__ import annotations

import numpy as np

# (Cin, Cout, kernel edge) per layer, in order
LAYERS = [(1, 16, 3), (16, 16, 3), (16, 32, 3), (32, 32, 3), (32, 64, 3), (64, 64, 3), (96, 32, 3), (32, 32, 3),
          (48, 16, 3), (16, 16, 3), (16, 1, 1)]


def init_params(seed: int, out_scale: float = 0.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = []
    for i, (ci, co, k) in enumerate(LAYERS):
        fan_in = ci * k ** 3
        last = i == len(LAYERS) - 1
        scale = out_scale if last else np.sqrt(2.0 / fan_in)
        parts.append(rng.standard_normal(co * ci * k ** 3) * scale)
        parts.append(np.zeros(co) if not last or out_scale == 0.0 else rng.standard_normal(co) * 0.01)
    return np.concatenate(parts).astype(np.float32)
