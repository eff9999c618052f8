"""Pins of the diagnostics oracle (energy spectra and PDFs of recovered
fields; readings in oracle/diagnostics.py)."""
import itertools

import numpy as np
import pytest

from oracle import diagnostics as dg


def test_shell_index_is_nearest_integer():
    k2 = np.arange(0, 200000)
    want = np.array([int(np.floor(np.sqrt(v) + 0.5)) for v in k2])
    np.testing.assert_array_equal(dg.shell_index(k2), want)
    assert dg.num_shells((2048, 2048)) == 1449 and dg.num_shells((256, 256, 256)) == 223


@pytest.mark.parametrize("shape", [(16, 16), (12, 20), (8, 8, 8), (6, 10, 4)])
def test_parseval(shape):
    x = np.random.default_rng(1).standard_normal((3,) + shape)
    s = dg.spectrum(x, len(shape))
    np.testing.assert_allclose(s.sum(-1), 0.5 * np.mean(x * x, axis=tuple(range(1, x.ndim))), rtol=1e-12)


@pytest.mark.parametrize("shape", [(16, 16), (10, 14), (8, 12, 6)])
def test_single_mode(shape):
    """a cos(k.x) puts a^2 / 4 (mean square a^2 / 2, halved) in the shell of |k|;
    with p = -2 that becomes a^2 / (4 |k|^2)."""
    nd = len(shape)
    coords = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in shape], indexing="ij")
    k = [1, 3] + ([2] if nd == 3 else [])
    x = 1.7 * np.cos(sum(kd * c for kd, c in zip(k, coords)) + 0.3)
    s = dg.spectrum(x, nd)
    k2 = sum(kd * kd for kd in k)
    sh = int(np.floor(np.sqrt(k2) + 0.5))
    want = np.zeros_like(s)
    want[sh] = 1.7 ** 2 / 4
    np.testing.assert_allclose(s, want, atol=1e-13)
    np.testing.assert_allclose(dg.spectrum(x, nd, kpow=-2.0)[sh], 1.7 ** 2 / (4 * k2), rtol=1e-12)


def test_brute_force_dft():
    shape = (4, 6)
    x = np.random.default_rng(2).standard_normal(shape)
    ns = dg.num_shells(shape)
    want = np.zeros(ns)
    for kx, ky in itertools.product(range(shape[0]), range(shape[1])):
        a = kx if kx <= shape[0] // 2 else kx - shape[0]
        b = ky if ky <= shape[1] // 2 else ky - shape[1]
        f = sum(x[i, j] * np.exp(-2j * np.pi * (kx * i / shape[0] + ky * j / shape[1]))
                for i in range(shape[0]) for j in range(shape[1])) / x.size
        want[int(np.floor(np.sqrt(a * a + b * b) + 0.5))] += 0.5 * (a * a + b * b) * abs(f) ** 2
    np.testing.assert_allclose(dg.spectrum(x, 2, kpow=2.0), want, atol=1e-14)


def test_pdf_brute_force_and_edges():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 7, 9))
    x[0, 0, 0], x[0, 0, 1], x[0, 0, 2], x[0, 0, 3] = -2.0, 2.0, 2.5, np.nan  # lo, hi, outside, NaN
    c = dg.pdf_counts(x, 2, -2.0, 2.0, 16)
    for b in range(2):
        want = np.zeros(16, dtype=np.int64)
        for v in x[b].ravel():
            if v >= -2.0 and v <= 2.0:
                want[min(int(np.floor((v + 2.0) * 4.0)), 15)] += 1
        np.testing.assert_array_equal(c[b], want)
    assert c[0, 0] >= 1 and c[0, 15] >= 1
    # away from bin edges the counts are numpy's histogram
    y = rng.uniform(-3, 3, 5000)
    np.testing.assert_array_equal(dg.pdf_counts(y[None], 1, -3.0, 3.0, 12)[0], np.histogram(y, 12, (-3, 3))[0])
