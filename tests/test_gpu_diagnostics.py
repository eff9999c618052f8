"""A-priori diagnostics on the GPU (energy_spectrum, pdf_counts) against the
oracle (oracle/diagnostics.py).

- PDF counts are integers decided in FP64 on both sides from the same stored
  values: bit-exact.
- Spectra: each shell sum adds FFT-computed |f_hat|^2 values; the FFT's
  relative error (order u log2 N) bounds the error of every term, so each
  shell agrees to 1e-12 (FP64) or 2e-5 (FP32) relative to the total
  mean(f^2)/2, the largest a shell can be.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import to_dev
from oracle import diagnostics as dg
from paper_1707_09177_amd import gdecon, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", [(8, 8), (2, 2), (16, 64), (256, 128), (4, 4, 4), (8, 16, 32), (2, 2, 2)])
@pytest.mark.parametrize("kpow", [0.0, -2.0, 2.0, -4.0, -5.0 / 3.0, 1.0])
def test_spectrum_matches_oracle(shape, dtype, kpow):
    nd = len(shape)
    x = np.random.default_rng(5 + len(shape)).standard_normal((3,) + shape)
    if dtype == torch.float32:
        x = x.astype(np.float32).astype(np.float64)
    want = dg.spectrum(x, nd, kpow)
    got = gdecon.energy_spectrum(to_dev(x, dtype), nd, kpow).cpu().numpy()
    assert got.shape == want.shape
    tot = dg.spectrum(x, nd, kpow).sum(-1, keepdims=True)
    tol = 1e-12 if dtype == torch.float64 else 2e-5
    assert np.all(np.abs(got - want) <= tol * tot)


def test_spectrum_full_size_and_parseval():
    """2048^2 x 4 k^-3 fields (FP32): shells against the oracle, and the sum
    against mean(f^2) / 2 computed directly."""
    u = synth.config_fields(2, count=4, dtype=np.float32)
    got = gdecon.energy_spectrum(torch.from_numpy(u).cuda(), 2).cpu().numpy()
    u64 = u.astype(np.float64)
    want = dg.spectrum(u64, 2)
    tot = 0.5 * np.mean(u64 * u64, axis=(1, 2))
    assert np.all(np.abs(got - want) <= 2e-5 * tot[:, None])
    np.testing.assert_allclose(got.sum(-1), tot, rtol=1e-5)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", [(9, 7), (1, 1), (130, 300), (5, 3, 7), (64, 64, 64)])
@pytest.mark.parametrize("nbins", [1, 17, 256, 8192])
def test_pdf_counts_bit_exact(shape, dtype, nbins):
    nd = len(shape)
    x = np.random.default_rng(9).standard_normal((2,) + shape) * 1.3
    x.flat[0], x.flat[1] = -3.0, 3.0             # both edges
    if x.size > 2:
        x.flat[2] = np.nan
    if dtype == torch.float32:
        x = x.astype(np.float32).astype(np.float64)
    want = dg.pdf_counts(x, nd, -3.0, 3.0, nbins)
    got = gdecon.pdf_counts(to_dev(x, dtype), -3.0, 3.0, nbins, ndim=nd).cpu().numpy()
    np.testing.assert_array_equal(got, want)


def test_pdf_full_size_twice():
    """2048^2 x 16 FP32 fields: exact counts, and a second call on the same
    buffer clears the previous counts first."""
    u = synth.config_fields(2, dtype=np.float32)
    t = torch.from_numpy(u).cuda()
    a = gdecon.pdf_counts(t, -5.0, 5.0, 200)
    want = dg.pdf_counts(u.astype(np.float64), 2, -5.0, 5.0, 200)
    np.testing.assert_array_equal(a.cpu().numpy(), want)
    lib = gdecon.load()
    g = gdecon.make_grid(t.shape, 2, t.dtype)
    assert lib.pdf_counts(gdecon.ctypes.byref(g), -5.0, 5.0, 200, t.data_ptr(), a.data_ptr(), None) == 0
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a.cpu().numpy(), want)


@pytest.mark.parametrize("shape", [(1024, 2048), (64, 64, 64), (4096, 4096)])
def test_spectrum_bitwise_repeatable(shape):
    """Each shell is summed in a fixed order (per-wave bins, then waves, then
    chunks in order), so repeated calls, with unrelated work in between to
    change the timing, give the same bits."""
    nd = len(shape)
    x = torch.randn((2,) + shape, dtype=torch.float32, device="cuda:0",
                    generator=torch.Generator("cuda:0").manual_seed(3))
    first = gdecon.energy_spectrum(x, nd, -2.0)
    torch.cuda.synchronize()
    for rep in range(4):
        (torch.randn(1 << 22, device="cuda:0") * 3).sum().item()
        again = gdecon.energy_spectrum(x, nd, -2.0)
        torch.cuda.synchronize()
        assert torch.equal(again, first), rep
