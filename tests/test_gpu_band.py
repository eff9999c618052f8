"""band_project on the GPU against the oracle's (oracle.band_project).

The two share nothing: the library transforms the half spectrum with its own
FFTs in the field's precision and sums mode powers in FP64; the oracle takes
full complex DFTs in FP64.  Inputs keep every mode far from the threshold (a
band-limited ubar, whose in-band modes sit orders of magnitude above tau times
the mean power and whose other modes at its rounding level, far below), so
both keep the same modes.  Tolerances: the result's error is the FFT
round-trip error of the correction plus that of ubar's spectrum, relative L2
<= 2e-6 of the result in FP32 (a few units in the last place of log2(N)
butterfly stages), <= 1e-12 in FP64.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import rel_l2, to_dev
from paper_1707_09177_amd import gdecon, synth

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 2e-6, torch.float64: 1e-12}


def band_limited(shape, seed):
    """ubar = G u for u with content at |k| <= n_min / 4 only, and u."""
    nd = len(shape)
    n = min(shape)
    if nd == 2:
        u = synth.field_2d(shape, synth.spectrum_kraichnan, 2.0, n / 4.0, synth.rng_for(7, seed), np.float64)
    else:
        u = synth.scalar_3d(shape, synth.spectrum_kolmogorov, 2.0, n / 4.0, synth.rng_for(7, seed), np.float64)
    return oracle.filter(u, nd), u


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("shape", [(64, 64), (32, 128), (256, 256), (16, 16, 16), (16, 32, 64), (64, 64, 64)])
def test_band_project_matches_oracle(shape, dtype):
    nd = len(shape)
    fields = [band_limited(shape, 10 + b) for b in range(3)]
    ubar = np.stack([f[0] for f in fields])
    ubar[1] *= 1e3                                    # per-field thresholds
    r = np.random.default_rng(3)
    u0 = ubar + 0.05 * np.abs(ubar).max(axis=tuple(range(1, nd + 1)), keepdims=True) * r.standard_normal(ubar.shape)
    ub_t, u0_t = to_dev(ubar, dtype), to_dev(u0, dtype)
    ubar_r = ub_t.double().cpu().numpy()              # what the GPU sees
    u0_r = u0_t.double().cpu().numpy()
    got = gdecon.band_project(ub_t, u0_t, ndim=nd).double().cpu().numpy()
    want = oracle.band_project(ubar_r, u0_r, nd, gdecon.BAND_TAU)
    for b in range(3):
        e = rel_l2(got[b], want[b])
        assert e <= TOL[dtype], (b, e)
    # the projected start holds no content outside the band
    k = [np.fft.fftfreq(n, 1.0 / n) for n in shape]
    kk = np.sqrt(sum(g ** 2 for g in np.meshgrid(*k, indexing="ij")))
    spec = np.abs(np.fft.fftn(got[0] - ubar_r[0]))
    assert spec[kk > min(shape) / 4 + 1].max() <= 1e-4 * spec.max()


def test_band_project_keeps_an_exact_correction():
    """u0 = u, the exact solution, comes back unchanged (to rounding)."""
    ubar, u = band_limited((128, 128), 40)
    ub_t, u_t = to_dev(ubar[None], torch.float64), to_dev(u[None], torch.float64)
    got = gdecon.band_project(ub_t, u_t.clone(), ndim=2).cpu().numpy()[0]
    assert rel_l2(got, u) <= 1e-13


def test_band_project_zero_tau_keeps_full_support():
    r = np.random.default_rng(5)
    ubar = r.standard_normal((2, 32, 64))
    u0 = r.standard_normal((2, 32, 64))
    got = gdecon.band_project(to_dev(ubar, torch.float64), to_dev(u0, torch.float64), ndim=2, tau=0.0)
    assert rel_l2(got.cpu().numpy(), u0) <= 1e-13


def test_band_project_errors():
    lib = gdecon.load()
    x = torch.zeros((3, 48, 64), device="cuda")
    with pytest.raises(gdecon.GdError):
        gdecon.band_project(x, x.clone(), ndim=2)          # 48 is not a power of two
    y = torch.zeros((2, 32, 32), device="cuda")
    with pytest.raises(gdecon.GdError):
        gdecon.band_project(y, y.clone(), ndim=2, tau=-1.0)
    with pytest.raises(gdecon.GdError):
        gdecon.band_project(y, y, ndim=2)                  # u0 overlaps ubar
    g = gdecon.make_grid(y.shape, 2, y.dtype)
    assert lib.band_project_workspace_bytes(g) > 0


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_differential_filter_warm_start_is_band_projected(dtype):
    """deconvolve_germano band-projects a warm start on the Fourier
    coefficients it holds.  A start that is the exact solution plus content
    outside ubar's band becomes the exact solution: its residual is at the
    rounding level, the start is taken, and the result matches the oracle's
    (which projects the same start the same way)."""
    n, gamma = 64, 0.1
    u = synth.field_2d(n, synth.spectrum_kraichnan, 2.0, n / 4.0, synth.rng_for(7, 77), np.float64)
    ubar = oracle.germano_filter(u, 2, gamma)[None]
    mode = np.cos(2 * np.pi * 27 * np.arange(n) / n)[None, :] * np.ones((n, 1))   # |k| = 27 > n / 4
    u0 = (u + 0.05 * mode)[None]
    ub_t, u0_t = to_dev(ubar, dtype), to_dev(u0, dtype)
    got, infos, _ = gdecon.deconvolve_germano("bicgstab", ub_t, 50, gamma, tol=1e-6, init="warm", u0=u0_t)
    assert infos[0]["start"] == "given"
    assert infos[0]["r0"] <= (1e-6 if dtype == torch.float32 else 1e-12) * infos[0]["r_ref"] * 100
    want, winfo, _ = oracle.solve("bicgstab", ub_t.double().cpu().numpy(), 2, 50, tol=1e-6, init="warm",
                                  u0=u0_t.double().cpu().numpy(), gamma=gamma)
    assert winfo[0]["start"] == "given" and winfo[0]["iters"] == infos[0]["iters"]
    assert rel_l2(got.double().cpu().numpy(), want) <= TOL[dtype] * 10
    # without the projection the out-of-band mode costs passes
    _, plain, _ = gdecon.deconvolve_germano("bicgstab", ub_t, 50, gamma, tol=1e-6, init="given", u0=u0_t)
    assert plain[0]["iters"] > infos[0]["iters"]
