"""Reference 3x3x3 convolutional network for the learned preconditioner stage
(oracle side, float64 NumPy).

The paper has no learned component; the network is the library's own: six 3x3x3
convolutions with zero padding, channels 3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 2,
bias on every layer, ReLU after the first five.  Volumes are channels-last,
shape (nz, ny, nx, C) with x fastest, matching the grid ordering of the solver.
Weights have shape (Cout, Cin, 3, 3, 3) indexed [co, ci, dz, dy, dx]; the
layer computes the cross-correlation

    y[z, y, x, co] = b[co] + sum_{ci, dz, dy, dx} w[co, ci, dz, dy, dx]
                              * xpad[z + dz, y + dy, x + dx, ci]

with xpad the input padded by one zero voxel on every face.  Training uses
the mean squared error and Adam (Kingma and Ba, 2015).

Parity: pinned by scipy.signal.correlate (a library routine for the same
sum, channel pair by channel pair), by the identity kernel, by the adjoint
identity <conv(x), g> = <x, conv_data_backward(g)>, by central finite
differences of the whole network's loss, and by Adam's closed-form first step.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

CHANNELS = (3, 32, 32, 32, 32, 32, 2)


def conv3d(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Forward 3x3x3 correlation with zero padding (module docstring)."""
    nz, ny, nx, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((nz, ny, nx, w.shape[0]))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                win = xp[dz:dz + nz, dy:dy + ny, dx:dx + nx, :]
                y += win @ w[:, :, dz, dy, dx].T
    return y + b


def conv3d_backward(x: np.ndarray, w: np.ndarray, gy: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Gradients of sum(gy * conv3d(x, w, b)) with respect to x, w and b."""
    nz, ny, nx, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                win = xp[dz:dz + nz, dy:dy + ny, dx:dx + nx, :]
                # d/dw[co, ci, dz, dy, dx] = sum_voxels gy[..., co] * win[..., ci]
                gw[:, :, dz, dy, dx] = np.einsum("zyxo,zyxi->oi", gy, win)
                # each input voxel feeds the outputs it was a window of
                gxp[dz:dz + nz, dy:dy + ny, dx:dx + nx, :] += gy @ w[:, :, dz, dy, dx]
    gb = gy.sum(axis=(0, 1, 2))
    return gxp[1:-1, 1:-1, 1:-1, :], gw, gb


def init_params(seed: int, channels=CHANNELS) -> List[Dict[str, np.ndarray]]:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        std = np.sqrt(2.0 / (cin * 27))
        params.append({"w": rng.standard_normal((cout, cin, 3, 3, 3)) * std, "b": np.zeros(cout)})
    return params


def forward(params, x: np.ndarray):
    """Network output and the activations the backward pass needs."""
    acts = [x]
    h = x
    for l, p in enumerate(params):
        h = conv3d(h, p["w"], p["b"])
        if l < len(params) - 1:
            h = np.maximum(h, 0.0)
        acts.append(h)
    return h, acts


def backward(params, acts, gy: np.ndarray):
    """Parameter gradients of sum(gy * forward(x)) by the chain rule, layer by
    layer from the last; ReLU passes the gradient where its output is > 0."""
    grads = [None] * len(params)
    g = gy
    for l in range(len(params) - 1, -1, -1):
        if l < len(params) - 1:
            g = g * (acts[l + 1] > 0)
        gx, gw, gb = conv3d_backward(acts[l], params[l]["w"], g)
        grads[l] = {"w": gw, "b": gb}
        g = gx
    return grads


def mse_loss_and_grad(params, x: np.ndarray, target: np.ndarray):
    """Mean squared error over every output value and its parameter gradients."""
    y, acts = forward(params, x)
    diff = y - target
    loss = float(np.mean(diff * diff))
    gy = 2.0 * diff / diff.size
    return loss, backward(params, acts, gy)


def adam_step(params, grads, state, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1), in place.  state holds
    the step count and the first and second moment estimates."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    if "m" not in state:
        state["m"] = [{k: np.zeros_like(v) for k, v in p.items()} for p in params]
        state["v"] = [{k: np.zeros_like(v) for k, v in p.items()} for p in params]
    for p, g, m, v in zip(params, grads, state["m"], state["v"]):
        for k in p:
            m[k] = beta1 * m[k] + (1 - beta1) * g[k]
            v[k] = beta2 * v[k] + (1 - beta2) * g[k] * g[k]
            mhat = m[k] / (1 - beta1 ** t)
            vhat = v[k] / (1 - beta2 ** t)
            p[k] = p[k] - lr * mhat / (np.sqrt(vhat) + eps)


def to_bf16(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 value (ties to even), returned as float64.
    Used to hand the oracle exactly the values the mixed-precision kernels see."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)
