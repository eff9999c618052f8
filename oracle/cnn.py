"""Plain FP64 reference of the learned warm start (test infrastructure only).

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this module.
It exists so the GPU network kernels can be checked against a version simple
enough to read by eye, and it shares no code with them.

The network exists for 2D fields (3x3 taps) and 3D fields (3x3x3 taps, the
same construction with one more axis).

The paper has no learned component: it starts every deconvolution from the
filtered field, u0 = ubar (Algorithms 1-4).  The warm start replaces that
u0 with a residual correction predicted by a small convolutional network:

    s   = RMS of ubar over the sample
    x0  = ubar / s                                   (1 channel)
    a_l = relu(conv_l(a_{l-1}))       l = 1 .. L-1   (C channels)
    z   = conv_L(a_{L-1})                            (1 channel, no activation)
    y   = G^m z                                      (the deconvolution filter, m >= 1 times)
    u0  = ubar + s * y

conv_l is a periodic 3x3 cross-correlation with bias (the fields are periodic,
like the filter G).  The final G keeps the correction in the range of G, as
the paper's own start u0 = ubar is: without it, the correction carries
content where G's transfer function nearly vanishes (next to the Nyquist
planes), the one place where the Krylov solvers converge slowly.  Applied m
times (`smooth`), it damps the network's rounding noise outside the band of
the fields by G_hat^m while the network learns G^-m of the correction on the
band, where G_hat is bounded below.  Training
minimises the mean over all points of (y - t)^2 with t = (u - ubar) / s, the
per-sample normalised correction, with Adam.

Layouts: activations (B, ny, nx, C) or (B, nz, ny, nx, C) (channels
fastest); the weights of layer l are W[cout][tap][cin] with
tap = 3 (dy + 1) + (dx + 1) in 2D and 9 (dz + 1) + 3 (dy + 1) + (dx + 1) in 3D,
offsets in {-1, 0, 1}, followed by the bias[cout]; all layers are packed in
order into one flat parameter vector.

`emulate_bf16=True` rounds the weights and every stored activation and
activation gradient to bfloat16 (round to nearest even) where the GPU
network stores them in bfloat16; everything else stays FP64.
"""
from __future__ import annotations

import numpy as np

from . import filter as g_filter

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
TAPS3 = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def taps(ndim: int):
    return TAPS if ndim == 2 else TAPS3


def layer_dims(channels: int = 32, layers: int = 6):
    """(cin, cout) per layer: 1 -> C, C -> C (layers - 2 times), C -> 1."""
    dims = [(1, channels)]
    dims += [(channels, channels)] * (layers - 2)
    dims += [(channels, 1)]
    return dims


def param_count(channels: int = 32, layers: int = 6, ndim: int = 2) -> int:
    nt = len(taps(ndim))
    return sum(co * nt * ci + co for ci, co in layer_dims(channels, layers))


def unpack(params: np.ndarray, channels: int = 32, layers: int = 6, ndim: int = 2):
    """Views (W, b) per layer into the flat parameter vector."""
    nt = len(taps(ndim))
    out, off = [], 0
    for ci, co in layer_dims(channels, layers):
        W = params[off:off + co * nt * ci].reshape(co, nt, ci)
        off += co * nt * ci
        b = params[off:off + co]
        off += co
        out.append((W, b))
    assert off == params.size
    return out


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (via float32, both steps round to nearest even)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = f.view(np.uint32).astype(np.uint64)
    bits = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16) << 16
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def shifted(x: np.ndarray, off) -> np.ndarray:
    """x at the point offset by `off` (per spatial axis, periodic):
    x[:, (y + dy) mod ny, (x + dx) mod nx, :] in 2D, likewise in 3D."""
    nd = len(off)
    return np.roll(x, shift=tuple(-o for o in off), axis=tuple(range(1, nd + 1)))


def conv(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Periodic 3x3 (3x3x3) cross-correlation: out[., p, o] = b[o] +
    sum_tap sum_c W[o, tap, c] * x[., p + off(tap), c]."""
    nd = x.ndim - 2
    out = np.zeros(x.shape[:-1] + (W.shape[0],))
    for t, off in enumerate(taps(nd)):
        out += shifted(x, off) @ W[:, t, :].T
    return out + b


def conv_grad_input(g: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Adjoint of conv in its input: dx[., p, c] =
    sum_tap sum_o W[o, tap, c] * g[., p - off(tap), o]."""
    nd = g.ndim - 2
    out = np.zeros(g.shape[:-1] + (W.shape[2],))
    for t, off in enumerate(taps(nd)):
        out += shifted(g, tuple(-o for o in off)) @ W[:, t, :]
    return out


def conv_grad_weight(x: np.ndarray, g: np.ndarray):
    """dW[o, tap, c] = sum_points g[., p, o] * x[., p + off(tap), c];
    db[o] = sum_points g[., p, o]."""
    nd = x.ndim - 2
    co, ci = g.shape[-1], x.shape[-1]
    tp = taps(nd)
    dW = np.zeros((co, len(tp), ci))
    gf = g.reshape(-1, co)
    for t, off in enumerate(tp):
        dW[:, t, :] = gf.T @ shifted(x, off).reshape(-1, ci)
    return dW, gf.sum(axis=0)


def rms(ubar: np.ndarray) -> np.ndarray:
    """Per-sample RMS (1 where the sample is identically zero)."""
    s = np.sqrt(np.mean(ubar.reshape(ubar.shape[0], -1) ** 2, axis=1))
    return np.where(s > 0, s, 1.0)


def g_power(x: np.ndarray, ndim: int, m: int) -> np.ndarray:
    """G^m x: the trapezoidal filter applied m times."""
    for _ in range(m):
        x = g_filter(x, ndim)
    return x


def forward(params, ubar, channels=32, layers=6, emulate_bf16=False, ndim=2, smooth=1):
    """Network forward on ubar (B, ny, nx) or (B, nz, ny, nx).  Returns a dict
    with the input scale s, the input x0, the stored activations a_1 ..
    a_{L-1}, the output y = G^smooth z and the warm start u0."""
    ubar = np.asarray(ubar, dtype=np.float64)
    P = unpack(np.asarray(params, dtype=np.float64), channels, layers, ndim)
    if emulate_bf16:
        P = [(bf16(W), b) for W, b in P]
    s = rms(ubar)
    sb = s.reshape((-1,) + (1,) * ndim)
    x0 = (ubar / sb)[..., None]
    acts = []
    a = x0
    for li, (W, b) in enumerate(P):
        z = conv(a, W, b)
        if li == len(P) - 1:
            y = g_power(z[..., 0], ndim, smooth)
            break
        a = np.maximum(z, 0.0)
        if emulate_bf16:
            a = bf16(a)
        acts.append(a)
    u0 = ubar + sb * y
    return {"s": s, "x0": x0, "acts": acts, "y": y, "u0": u0, "P": P}


def loss_and_grad(params, ubar, u, channels=32, layers=6, emulate_bf16=False, ndim=2, smooth=1):
    """Training loss mean((y - t)^2), t = (u - ubar) / s, and its gradient
    with respect to the flat parameter vector (backpropagation)."""
    f = forward(params, ubar, channels, layers, emulate_bf16, ndim, smooth)
    s = f["s"].reshape((-1,) + (1,) * ndim)
    t = (np.asarray(u, dtype=np.float64) - ubar) / s
    r = f["y"] - t
    n = r.size
    loss = float(np.sum(r * r) / n)
    g = g_power((2.0 / n) * r, ndim, smooth)[..., None]   # dL/dz = G^m dL/dy (G is symmetric)
    grads = [None] * len(f["P"])
    ins = [f["x0"]] + f["acts"]
    for li in range(len(f["P"]) - 1, -1, -1):
        W, _ = f["P"][li]
        grads[li] = conv_grad_weight(ins[li], g)
        if li == 0:
            break
        g = conv_grad_input(g, W) * (ins[li] > 0)   # through the ReLU of layer li
        if emulate_bf16:
            g = bf16(g)
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss, flat


def adam_step(params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); `step` counts from 1.  Returns new
    (params, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
