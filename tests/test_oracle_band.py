"""Pins of the oracle's band projection (oracle.band_project), CPU only.

The projection keeps a start's correction u0 - ubar on the wavenumbers where
ubar has content.  Its threshold is relative to the mean mode power of ubar;
the closed forms below fix that normalisation: for
ubar = A cos(k1.x) + B cos(k2.x) on N points the unnormalized DFT has
|ubar_hat(+-k1)|^2 = (A N / 2)^2, |ubar_hat(+-k2)|^2 = (B N / 2)^2 and mean
power E = N (A^2 + B^2) / 2, so k1 survives exactly when
tau < A^2 N / (2 (A^2 + B^2)).
"""
import numpy as np
import pytest

import oracle
from paper_1707_09177_amd import synth


def wave(shape, k):
    """cos(k . x) on the 2 pi periodic grid of `shape` (last axis x)."""
    grids = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in shape], indexing="ij")
    return np.cos(sum(kk * g for kk, g in zip(k, grids)))


@pytest.mark.parametrize("shape", [(32, 48), (8, 16, 12)])
def test_two_mode_threshold_closed_form(shape):
    nd = len(shape)
    n = float(np.prod(shape))
    k1 = (1,) * nd
    k2 = (2,) + (0,) * (nd - 1)
    k3 = (0,) * (nd - 1) + (5,)            # absent from ubar
    a, b = 1.0, 0.5
    ubar = a * wave(shape, k1) + b * wave(shape, k2)
    extra = wave(shape, k1) + wave(shape, k2) + wave(shape, k3)
    u0 = ubar + extra
    # thresholds: k2 survives below tau = 0.1 N, k1 below 0.4 N
    got = oracle.band_project(ubar, u0, nd, 0.05 * n)
    np.testing.assert_allclose(got, ubar + wave(shape, k1) + wave(shape, k2), atol=1e-12)
    got = oracle.band_project(ubar, u0, nd, 0.2 * n)
    np.testing.assert_allclose(got, ubar + wave(shape, k1), atol=1e-12)
    got = oracle.band_project(ubar, u0, nd, 0.5 * n)
    np.testing.assert_allclose(got, ubar, atol=1e-12)


def test_band_limited_truth_is_kept_and_outside_content_removed():
    """u band-limited (k <= n/4), ubar = G u: the exact correction u - ubar
    lies in ubar's support and survives; a mode outside the band, or any
    white noise projected, ends inside it."""
    n = 64
    u = synth.field_2d(n, synth.spectrum_kraichnan, 4.0, n / 4.0, synth.rng_for(5, 123), np.float64)
    ubar = oracle.filter(u, 2)
    tau = 1e-10
    np.testing.assert_allclose(oracle.band_project(ubar, u, 2, tau), u, rtol=0, atol=1e-12 * np.abs(u).max())
    out_of_band = wave((n, n), (0, 30))     # |k| = 30 > n/4 = 16
    got = oracle.band_project(ubar, u + 0.1 * out_of_band, 2, tau)
    np.testing.assert_allclose(got, u, rtol=0, atol=1e-12 * np.abs(u).max())
    noise = np.random.default_rng(1).standard_normal((n, n))
    p = oracle.band_project(ubar, ubar + noise, 2, tau) - ubar
    ph = np.fft.fft2(p)
    k = np.fft.fftfreq(n, 1.0 / n)
    kr = np.hypot(k[:, None], k[None, :])
    assert np.abs(ph[kr > n / 4 + 1]).max() < 1e-9 * np.abs(ph).max()
    # idempotent
    q = oracle.band_project(ubar, ubar + p, 2, tau) - ubar
    np.testing.assert_allclose(q, p, atol=1e-12 * np.abs(p).max())


def test_full_support_and_zero_tau_keep_everything():
    r = np.random.default_rng(2)
    ubar = r.standard_normal((2, 16, 24))       # white noise: content at every mode
    u0 = r.standard_normal((2, 16, 24))
    np.testing.assert_allclose(oracle.band_project(ubar, u0, 2, 0.0), u0, atol=1e-12)


def test_thresholds_are_per_field():
    """A field scaled by 1e3 keeps the same modes as the unscaled one."""
    shape = (16, 16)
    ubar1 = wave(shape, (1, 1)) + 0.01 * wave(shape, (3, 0))
    ubar = np.stack([ubar1, 1e3 * ubar1])
    extra = wave(shape, (1, 1)) + wave(shape, (3, 0)) + wave(shape, (0, 5))
    u0 = ubar + extra
    tau = 1e-3 * 256        # keeps (1,1), drops (3,0): (0.01 N/2)^2 / E ~ 5e-5 N < tau < 0.5 N
    got = oracle.band_project(ubar, u0, 2, tau)
    for b in range(2):
        np.testing.assert_allclose(got[b], ubar[b] + wave(shape, (1, 1)), atol=1e-9 * np.abs(ubar[b]).max())
