"""The seeded input generator: spectra, phases, symmetry, divergence."""
import numpy as np

from paper_1707_09177_amd import synth


def test_2d_exact_amplitudes_and_band():
    n = 64
    u = synth.field_2d(n, synth.spectrum_kraichnan, 4.0, 16.0, synth.rng_for(2, 0))
    assert u.shape == (n, n) and u.dtype == np.float64
    assert abs(np.sqrt(np.mean(u * u)) - 1) < 1e-12
    uh = np.fft.fft2(u)
    k = np.fft.fftfreq(n) * n
    K = np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)
    band = (K >= 4) & (K <= 16) & (np.abs(k)[:, None] != n // 2) & (np.abs(k)[None, :] != n // 2)
    assert np.max(np.abs(uh[~band])) < 1e-9
    # |w_hat|^2 / (k E(k)) is one constant on the band (exact amplitudes)
    ratio = np.abs(uh[band]) ** 2 / (K[band] * K[band] ** -3.0)
    assert np.std(ratio) / np.mean(ratio) < 1e-9


def test_3d_divergence_free_and_amplitude():
    n = 24
    v = synth.velocity_3d(n, synth.spectrum_kolmogorov, 2.0, 7.5, synth.rng_for(3, 0))
    assert v.shape == (3, n, n, n)
    vh = np.stack([np.fft.fftn(v[d]) for d in range(3)])
    kz, ky, kx = np.meshgrid(*[np.fft.fftfreq(n) * n] * 3, indexing="ij")
    div = kx * vh[0] + ky * vh[1] + kz * vh[2]
    assert np.max(np.abs(div)) < 1e-8 * np.max(np.abs(vh))
    K = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
    band = np.sum(np.abs(vh) ** 2, axis=0) > 1e-20
    assert K[band].min() >= 2 and K[band].max() <= 7.5
    ratio = np.sum(np.abs(vh[:, band]) ** 2, axis=0) * K[band] ** 2 / K[band] ** (-5.0 / 3.0)
    assert np.std(ratio) / np.mean(ratio) < 1e-9


def test_seeded_and_distinct():
    a = synth.config_fields(2, n=64, count=2)
    b = synth.config_fields(2, n=64, count=2)
    assert np.array_equal(a, b)
    assert not np.allclose(a[0], a[1])


def test_batch_sizes_recipe():
    inst = synth.batch_instances()
    assert len(inst) == 200
    for nd, n in inst:
        if nd == 2:
            assert n % 64 == 0 and 256 <= n <= 2048
        else:
            assert nd == 3 and n % 16 == 0 and 64 <= n <= 192
    assert 60 < sum(1 for nd, _ in inst if nd == 3) < 140
