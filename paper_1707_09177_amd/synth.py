"""Seeded synthetic turbulence fields: the inputs of the deconvolution solve.

This module only draws fields. It holds none of the deconvolution arithmetic:
no filter, no inner product, no solver step. Both the CPU oracle tests and the
GPU path take their inputs from here, so they see the same numbers.

The paper runs its a-priori study on DNS snapshots: decaying 2D Kraichnan
turbulence at Re=32000 with a k^-3 inertial range (Section 4.1) and the 3D
Taylor-Green vortex at Re=1600 with a k^-5/3 range (Section 4.2). Those
snapshots are not available, so fields with the same spectral shapes and
random phases stand in for them.

Recipe (all grids periodic on [0, 2*pi]^d, C-contiguous, x fastest):
  * RNG: numpy PCG64 seeded by SeedSequence([1707, 9177, cfg, inst]).
  * Integer wavenumbers k_d = fftfreq(n_d) * n_d and |k| = sqrt(sum k_d^2).
  * 2D vorticity: |w_hat(k)| = sqrt(|k| E(|k|)), since in 2D the energy
    spectrum and the vorticity spectrum differ by a factor k / pi.
  * 3D velocity: |u_hat(k)| = sqrt(E(|k|)) / |k|, a complex random 3-vector
    projected onto the plane normal to k (divergence-free), then rescaled.
  * Amplitude zero outside [kmin, kmax], at k = 0 and on Nyquist planes of
    even grid sizes.
  * Phases uniform on [0, 2*pi); Hermitian symmetry is enforced exactly, so
    every retained mode has exactly the prescribed amplitude.
  * The real field is normalised to unit RMS (over all components in 3D).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng_for", "field_2d", "velocity_3d", "scalar_3d",
    "spectrum_kraichnan", "spectrum_kolmogorov", "spectrum_c1",
    "config_fields", "batch_instances", "training_fields",
]


def rng_for(cfg: int, inst: int) -> np.random.Generator:
    """Generator for config ``cfg`` and instance ``inst``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([1707, 9177, int(cfg), int(inst)])))


def spectrum_kraichnan(k):
    """E(k) ~ k^-3 (2D enstrophy-cascade range)."""
    return k ** -3.0


def spectrum_kolmogorov(k):
    """E(k) ~ k^-5/3 (3D inertial range)."""
    return k ** (-5.0 / 3.0)


def spectrum_c1(k):
    """E(k) ~ k^4 exp(-(k/10)^2): the small smooth 64x64 test spectrum."""
    return k ** 4 * np.exp(-(k / 10.0) ** 2)


def _hermitian_fix_last_axis_zero(c: np.ndarray) -> None:
    """Make the kx=0 (and only) plane of a half spectrum Hermitian in place.

    For a real field the coefficient at (-k_rest, 0) must equal the conjugate
    of the one at (k_rest, 0). We keep one of each pair (the lexicographically
    positive index) and overwrite the other.
    """
    plane = c[..., 0]
    shape = plane.shape
    idx = np.indices(shape).reshape(len(shape), -1)
    neg = np.stack([(-idx[d]) % shape[d] for d in range(len(shape))])
    flat_i = np.ravel_multi_index(tuple(idx), shape)
    flat_n = np.ravel_multi_index(tuple(neg), shape)
    keep = flat_i < flat_n           # one representative of each (k, -k) pair
    selfconj = flat_i == flat_n      # k == -k (zero and Nyquist indices)
    p = plane.reshape(-1)
    p[flat_n[keep]] = np.conj(p[flat_i[keep]])
    p[flat_i[selfconj]] = p[flat_i[selfconj]].real
    c[..., 0] = p.reshape(shape)


def _wavenumber_grids(shape):
    """Full-spectrum integer wavenumbers for all axes but x, half for x."""
    axes = []
    for d, n in enumerate(shape):
        if d == len(shape) - 1:
            axes.append(np.fft.rfftfreq(n) * n)
        else:
            axes.append(np.fft.fftfreq(n) * n)
    return np.meshgrid(*axes, indexing="ij")


def _nyquist_mask(shape, grids):
    m = np.zeros(grids[0].shape, dtype=bool)
    for n, kd in zip(shape, grids):
        if n % 2 == 0:
            m |= np.abs(kd) == n // 2
    return m


def field_2d(n, spectrum, kmin, kmax, rng, dtype=np.float64):
    """One 2D scalar (vorticity) field of shape (ny, nx), unit RMS."""
    ny, nx = (n, n) if np.isscalar(n) else tuple(n)
    ky, kx = _wavenumber_grids((ny, nx))
    K = np.sqrt(kx ** 2 + ky ** 2)
    band = (K >= kmin) & (K <= kmax) & (K > 0) & ~_nyquist_mask((ny, nx), (ky, kx))
    amp = np.zeros_like(K)
    amp[band] = np.sqrt(K[band] * spectrum(K[band]))
    theta = rng.uniform(0.0, 2.0 * np.pi, size=K.shape)
    c = amp * np.exp(1j * theta)
    _hermitian_fix_last_axis_zero(c)
    u = np.fft.irfft2(c, s=(ny, nx))
    rms = np.sqrt(np.mean(u * u))
    if rms > 0:
        u /= rms
    return np.ascontiguousarray(u, dtype=dtype)


def velocity_3d(n, spectrum, kmin, kmax, rng, dtype=np.float64):
    """Divergence-free 3D velocity, shape (3, nz, ny, nx), unit RMS overall."""
    nz, ny, nx = (n, n, n) if np.isscalar(n) else tuple(n)
    kz, ky, kx = _wavenumber_grids((nz, ny, nx))
    K = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    band = (K >= kmin) & (K <= kmax) & (K > 0) & ~_nyquist_mask((nz, ny, nx), (kz, ky, kx))
    amp = np.zeros_like(K)
    amp[band] = np.sqrt(spectrum(K[band])) / K[band]
    theta = rng.uniform(0.0, 2.0 * np.pi, size=(3,) + K.shape)
    v = np.exp(1j * theta)
    Ks = np.where(K > 0, K, 1.0)
    kh = (kx / Ks, ky / Ks, kz / Ks)  # unit wave vector, components (x, y, z)
    kdotv = kh[0] * v[0] + kh[1] * v[1] + kh[2] * v[2]
    vp = np.stack([v[d] - kh[d] * kdotv for d in range(3)])
    mag = np.sqrt(np.sum(np.abs(vp) ** 2, axis=0))
    safe = mag > 1e-12
    coef = np.where(safe & band, amp / np.where(safe, mag, 1.0), 0.0)
    out = np.empty((3, nz, ny, nx), dtype=np.float64)
    for d in range(3):
        c = vp[d] * coef
        _hermitian_fix_last_axis_zero(c)
        out[d] = np.fft.irfftn(c, s=(nz, ny, nx), axes=(0, 1, 2))
    rms = np.sqrt(np.mean(out * out))
    if rms > 0:
        out /= rms
    return np.ascontiguousarray(out, dtype=dtype)


def scalar_3d(n, spectrum, kmin, kmax, rng, dtype=np.float64):
    """3D scalar field with the amplitude law of one velocity component."""
    nz, ny, nx = (n, n, n) if np.isscalar(n) else tuple(n)
    kz, ky, kx = _wavenumber_grids((nz, ny, nx))
    K = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    band = (K >= kmin) & (K <= kmax) & (K > 0) & ~_nyquist_mask((nz, ny, nx), (kz, ky, kx))
    amp = np.zeros_like(K)
    amp[band] = np.sqrt(spectrum(K[band])) / K[band]
    theta = rng.uniform(0.0, 2.0 * np.pi, size=K.shape)
    c = amp * np.exp(1j * theta)
    _hermitian_fix_last_axis_zero(c)
    u = np.fft.irfftn(c, s=(nz, ny, nx), axes=(0, 1, 2))
    rms = np.sqrt(np.mean(u * u))
    if rms > 0:
        u /= rms
    return np.ascontiguousarray(u, dtype=dtype)


def config_fields(cfg: int, n=None, count=None, dtype=np.float64):
    """Fields u (the unfiltered truth) for the paper-shaped workloads.

    cfg 1: 64^2, E ~ k^4 exp(-(k/10)^2), all k >= 1, one field.
    cfg 2: 2048^2, E ~ k^-3 on 4 <= k <= 512, 16 fields.
    cfg 3: 256^3 divergence-free velocity, E ~ k^-5/3 on 2 <= k <= 80;
           returned as 3 scalar instances (one per component).
    ``n`` and ``count`` shrink the grid / batch while keeping the spectral
    shape (band edges scale with n).  Returns an array (count, *grid).
    """
    if cfg == 1:
        n = 64 if n is None else n
        count = 1 if count is None else count
        return np.stack([field_2d(n, spectrum_c1, 1.0, np.inf, rng_for(1, i), dtype) for i in range(count)])
    if cfg == 2:
        n = 2048 if n is None else n
        count = 16 if count is None else count
        return np.stack([field_2d(n, spectrum_kraichnan, 4.0, n / 4.0, rng_for(2, i), dtype) for i in range(count)])
    if cfg == 3:
        n = 256 if n is None else n
        count = 3 if count is None else count
        comps = []
        i = 0
        while len(comps) < count:
            v = velocity_3d(n, spectrum_kolmogorov, 2.0, n * 80.0 / 256.0, rng_for(3, i), dtype)
            comps.extend(list(v))
            i += 1
        return np.stack(comps[:count])
    raise ValueError(f"no generator for cfg {cfg}")


def batch_instances(count=200, seed_cfg=4, min2d=4, max2d=32, min3d=4, max3d=12):
    """Sizes for the uneven batch: 2D n = 64*U{4..32}, 3D n = 16*U{4..12}.

    Returns a list of (ndim, n) drawn from seed; 3D with probability 1/2.
    """
    rng = rng_for(seed_cfg, 10**6)
    out = []
    for _ in range(count):
        if rng.uniform() < 0.5:
            out.append((3, int(16 * rng.integers(min3d, max3d + 1))))
        else:
            out.append((2, int(64 * rng.integers(min2d, max2d + 1))))
    return out


def batch_field(ndim: int, n: int, inst: int, seed_cfg=4, dtype=np.float64):
    """Field for one uneven-batch instance: spectra as for the large configs."""
    rng = rng_for(seed_cfg, inst)
    if ndim == 2:
        return field_2d(n, spectrum_kraichnan, 4.0, n / 4.0, rng, dtype)
    return scalar_3d(n, spectrum_kolmogorov, 2.0, 0.3125 * n, rng, dtype)


def cnn_init_params(seed: int, channels: int = 32, layers: int = 6, ndim: int = 2) -> np.ndarray:
    """Initial weights of the warm-start network, flat FP64, in the layer
    order 1 -> C, C -> C (layers - 2 times), C -> 1, each layer W[cout][taps][cin]
    (9 taps in 2D, 27 in 3D)
    followed by bias[cout]: He-normal weights (fan-in 9*cin), zero biases, the
    last layer scaled by 0.1 so the untrained network starts near u0 = ubar."""
    rng = np.random.default_rng(np.random.SeedSequence([1707, 9177, 5 if ndim == 2 else 6, seed]))
    nt = 9 if ndim == 2 else 27
    dims = [(1, channels)] + [(channels, channels)] * (layers - 2) + [(channels, 1)]
    parts = []
    for li, (ci, co) in enumerate(dims):
        W = rng.standard_normal((co, nt, ci)) * np.sqrt(2.0 / (nt * ci))
        if li == len(dims) - 1:
            W *= 0.1
        parts += [W.ravel(), np.zeros(co)]
    return np.concatenate(parts)


def training_pairs(count: int, n: int = 512, crop: int = 128, seed0: int = 0, dtype=np.float32):
    """Random crops of 2D k^-3 fields (4 <= k <= n/4) for the warm-start
    network: `count` arrays (crop, crop).  The filtered inputs are made by the
    caller (ubar = G u).  Crops of periodic fields are not periodic; the
    network treats every sample as periodic anyway."""
    out = []
    per = max(1, (n // crop) ** 2)
    for i in range((count + per - 1) // per):
        f = field_2d(n, spectrum_kraichnan, 4.0, n / 4.0, rng_for(5, 1000 + seed0 + i), np.float64)
        for cy in range(n // crop):
            for cx in range(n // crop):
                if len(out) < count:
                    out.append(f[cy * crop:(cy + 1) * crop, cx * crop:(cx + 1) * crop].astype(dtype))
    return out


def training_fields(count: int = 4096, n: int = 512, seed0: int = 0, dtype=np.float32, workers: int = 0):
    """The warm-start network's training set: `count` whole periodic 2D
    fields (n, n) with a k^-3 spectrum on 4 <= k <= n/4, returned stacked
    (count, n, n); the filtered inputs are made by the caller (ubar = G u).
    Field i is seeded by (5, 100000 + seed0 + i) and does not depend on
    `workers` (threads that draw fields in parallel; 0 = one per CPU, at
    most 16)."""
    from concurrent.futures import ThreadPoolExecutor
    import os
    out = np.empty((count, n, n), dtype=dtype)

    def one(i):
        out[i] = field_2d(n, spectrum_kraichnan, 4.0, n / 4.0, rng_for(5, 100000 + seed0 + i), dtype)
    nw = workers if workers > 0 else max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(nw) as ex:
        list(ex.map(one, range(count)))
    return out


def training_pairs_3d(count: int, n: int = 64, seed0: int = 0, dtype=np.float32):
    """3D scalar fields for the 3D warm-start network: `count` arrays (n, n, n)
    with a k^-5/3 spectrum on 2 <= k <= 0.3125 n (the uneven-batch 3D law)."""
    return [scalar_3d(n, spectrum_kolmogorov, 2.0, 0.3125 * n, rng_for(6, 2000 + seed0 + i), dtype)
            for i in range(count)]
