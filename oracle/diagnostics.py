"""A-priori diagnostics of recovered fields -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use this module; the GPU library shares no code with it.

The paper judges the recovered fields by their energy spectra and by the
probability density functions of the fields (Sec. 4, the spectra and PDF
figures of the 2D and 3D cases) without writing either out.  Readings:

- spectrum: f_hat(k) = (1/N) sum_x f(x) exp(-i k.x) on the 2 pi periodic
  grid (integer wavenumbers, FFT order), and
      S(s) = 1/2 sum_{k in shell s} |k|^p |f_hat(k)|^2,
  shell s holding the wavenumbers whose |k| rounds to s (|k|^2 is an integer,
  so no |k| lies half way between two integers).  p = 0 gives the spectrum of
  f itself (sum_s S(s) = mean(f^2) / 2); p = -2 turns a 2D vorticity field
  into the kinetic energy spectrum (|u_hat| = |w_hat| / |k|), the k = 0 mode
  then contributing nothing.  For a 3D velocity the spectra of the
  components add.
- PDF: counts of the field's values in nbins equal bins over [lo, hi]; the
  bin of v is floor((v - lo) * (nbins / (hi - lo))) evaluated in FP64, v = hi
  falls in the last bin, values outside [lo, hi] and NaN are not counted.
  Dividing by the count times the bin width gives the density.
"""
from __future__ import annotations

import numpy as np


def shell_index(k2: np.ndarray) -> np.ndarray:
    """Nearest integer to sqrt(k2) for integer k2 >= 0, in integer arithmetic:
    the s with (2s - 1)^2 <= 4 k2 < (2s + 1)^2."""
    k2 = np.asarray(k2, dtype=np.int64)
    s = np.floor(np.sqrt(k2.astype(np.float64))).astype(np.int64)
    s = np.where((2 * s + 1) ** 2 <= 4 * k2, s + 1, s)
    s = np.where((s > 0) & ((2 * s - 1) ** 2 > 4 * k2), s - 1, s)
    return s


def num_shells(shape) -> int:
    """Shells 0 .. s_max, s_max the shell of the corner wavenumber (n_d / 2 per axis)."""
    return int(shell_index(np.array(sum((n // 2) ** 2 for n in shape)))) + 1


def spectrum(x: np.ndarray, ndim: int, kpow: float = 0.0) -> np.ndarray:
    """S(s) for every field in the leading dimensions of x: shape (..., nshells)."""
    x = np.asarray(x, dtype=np.float64)
    shape = x.shape[-ndim:]
    npts = int(np.prod(shape))
    axes = tuple(range(x.ndim - ndim, x.ndim))
    fh = np.fft.fftn(x, axes=axes) / npts            # full spectrum: no half-plane weights to get wrong
    ks = np.meshgrid(*[np.fft.fftfreq(n, 1.0 / n).astype(np.int64) for n in shape], indexing="ij")
    k2 = sum(k * k for k in ks)
    shells = shell_index(k2).ravel()
    if kpow == 0:
        w = np.ones(k2.shape)
    else:
        w = np.where(k2 > 0, np.power(np.maximum(k2, 1).astype(np.float64), kpow / 2.0), 0.0)
    ns = num_shells(shape)
    lead = x.shape[:-ndim]
    p = (0.5 * w * np.abs(fh) ** 2).reshape(lead + (-1,))
    flat = p.reshape(-1, npts)
    out = np.stack([np.bincount(shells, weights=f, minlength=ns) for f in flat])
    return out.reshape(lead + (ns,))


def pdf_counts(x: np.ndarray, ndim: int, lo: float, hi: float, nbins: int) -> np.ndarray:
    """Counts per bin for every field in the leading dimensions: shape (..., nbins)."""
    x = np.asarray(x, dtype=np.float64)
    lead = x.shape[:-ndim]
    flat = x.reshape(-1, int(np.prod(x.shape[-ndim:])))
    scale = float(nbins) / (float(hi) - float(lo))
    out = np.zeros((flat.shape[0], nbins), dtype=np.int64)
    for b, v in enumerate(flat):
        ok = (v >= lo) & (v <= hi)
        idx = np.floor((v[ok] - lo) * scale).astype(np.int64)
        idx = np.minimum(idx, nbins - 1)
        out[b] = np.bincount(idx, minlength=nbins)
    return out.reshape(lead + (nbins,))
