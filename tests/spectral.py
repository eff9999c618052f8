"""Independent constructions used to pin the oracle (tests only).

Nothing here calls the oracle.  The filter appears in two forms derived from
its definition (weights 1/4, 1/2, 1/4 per axis, periodic):
  * its Fourier transfer function G_hat(k) = prod_d cos^2(pi k_d / n_d)
    (the DFT of the 1D stencil is 1/2 + cos(2 pi k / n)/2);
  * its dense matrix, a Kronecker product of 1D circulants (separability).
"""
from __future__ import annotations

import math

import numpy as np


def ghat(shape) -> np.ndarray:
    """Transfer function on the full FFT grid of an array of this shape."""
    out = np.ones(shape)
    for d, n in enumerate(shape):
        k = np.arange(n)
        g1 = np.cos(np.pi * k / n) ** 2
        sl = [None] * len(shape)
        sl[d] = slice(None)
        out = out * g1[tuple(sl)]
    return out


def apply_fft(x: np.ndarray, mult: np.ndarray) -> np.ndarray:
    """Real field times a Fourier multiplier over the last len(mult.shape) axes."""
    axes = tuple(range(x.ndim - mult.ndim, x.ndim))
    return np.real(np.fft.ifftn(np.fft.fftn(x, axes=axes) * mult, axes=axes))


def circulant_1d(n: int) -> np.ndarray:
    eye = np.eye(n)
    return 0.5 * eye + 0.25 * (np.roll(eye, 1, axis=1) + np.roll(eye, -1, axis=1))


def dense_g(shape) -> np.ndarray:
    """Dense matrix of G for C-order fields of this shape (last axis fastest)."""
    m = np.ones((1, 1))
    for n in shape:
        m = np.kron(m, circulant_1d(n))
    return m


def spacing_weight(shape) -> float:
    w = 1.0
    for n in shape:
        w *= 2 * math.pi / n
    return w


def distinct_values(vals: np.ndarray, rtol=1e-12) -> np.ndarray:
    v = np.sort(vals.ravel())
    keep = [v[0]]
    for x in v[1:]:
        if abs(x - keep[-1]) > rtol * max(1.0, abs(x)):
            keep.append(x)
    return np.array(keep)


def cg_krylov_iterate(gm: np.ndarray, ubar: np.ndarray, u0: np.ndarray, n: int) -> np.ndarray:
    """Minimiser of the G-norm error over u0 + K_n(G, r0), by brute force.

    Builds an orthonormal basis of the Krylov space and solves the projected
    normal equations (V^T G V) y = V^T r0 (exact solution u* drops out since
    G (u* - u0) = r0).
    """
    r0 = ubar - gm @ u0
    cols = [r0]
    for _ in range(n - 1):
        cols.append(gm @ cols[-1])
    k = np.stack(cols, axis=1)
    q, _ = np.linalg.qr(k)
    a = q.T @ gm @ q
    y = np.linalg.solve(a, q.T @ r0)
    return u0 + q @ y
