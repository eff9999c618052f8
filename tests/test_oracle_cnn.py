"""Pins of the FP64 warm-start network reference (oracle/cnn.py), CPU only.

Each pin comes from outside the reference's own code: circular correlation
through the FFT, central finite differences of the loss, the closed form of
Adam's first step, exact invariances of the construction, and bfloat16
rounding checked against hand-made bit patterns.
"""
import numpy as np
import pytest

import oracle
from oracle import cnn
from paper_1707_09177_amd import synth


def rng(seed):
    return np.random.default_rng(seed)


def fft_correlate(x, w):
    """Periodic cross-correlation of one channel plane with a 3x3 kernel,
    computed in Fourier space: sum_{dy,dx} w[dy,dx] x[y+dy, x+dx]."""
    ny, nx = x.shape
    k = np.zeros((ny, nx))
    for t, (dy, dx) in enumerate(cnn.TAPS):
        k[(-dy) % ny, (-dx) % nx] += w[t]
    return np.real(np.fft.ifft2(np.fft.fft2(x) * np.fft.fft2(k)))


@pytest.mark.parametrize("shape", [(7, 9), (8, 8), (3, 2), (1, 5)])
def test_conv_is_fft_circular_correlation(shape):
    B, ci, co = 2, 3, 4
    x = rng(1).standard_normal((B,) + shape + (ci,))
    W = rng(2).standard_normal((co, 9, ci))
    b = rng(3).standard_normal(co)
    out = cnn.conv(x, W, b)
    for bb in range(B):
        for o in range(co):
            want = b[o] + sum(fft_correlate(x[bb, :, :, c], W[o, :, c]) for c in range(ci))
            np.testing.assert_allclose(out[bb, :, :, o], want, rtol=0, atol=1e-12)


def test_conv_adjoint_identity():
    """<conv(x) - b, g> == <x, conv_grad_input(g)> and the weight gradient is
    the derivative of <conv(x), g> in W (both linear identities)."""
    x = rng(4).standard_normal((2, 6, 5, 3))
    g = rng(5).standard_normal((2, 6, 5, 4))
    W = rng(6).standard_normal((4, 9, 3))
    b = np.zeros(4)
    lhs = np.sum((cnn.conv(x, W, b)) * g)
    rhs = np.sum(x * cnn.conv_grad_input(g, W))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    dW, db = cnn.conv_grad_weight(x, g)
    assert abs(np.sum(dW * W) - lhs) <= 1e-11 * abs(lhs)
    np.testing.assert_allclose(db, g.reshape(-1, 4).sum(0), rtol=1e-13)


@pytest.mark.parametrize("channels,shape", [(4, (6, 7)), (32, (5, 4))])
def test_backprop_matches_central_differences(channels, shape):
    params = synth.cnn_init_params(3, channels=channels)
    params[-1] = 0.05                                  # exercise the output bias too
    ub = rng(7).standard_normal((2,) + shape)
    u = ub + 0.3 * rng(8).standard_normal((2,) + shape)
    loss, g = cnn.loss_and_grad(params, ub, u, channels=channels)
    pick = rng(9).choice(params.size, size=min(60, params.size), replace=False)
    eps = 1e-6
    for i in pick:
        p1, p2 = params.copy(), params.copy()
        p1[i] += eps
        p2[i] -= eps
        l1, _ = cnn.loss_and_grad(p1, ub, u, channels=channels)
        l2, _ = cnn.loss_and_grad(p2, ub, u, channels=channels)
        fd = (l1 - l2) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_param_count_and_layout():
    assert cnn.param_count() == (288 + 32) + 4 * (9216 + 32) + (288 + 1) == 37601
    p = np.arange(cnn.param_count(), dtype=np.float64)
    layers = cnn.unpack(p)
    assert [W.shape for W, _ in layers] == [(32, 9, 1)] + [(32, 9, 32)] * 4 + [(1, 9, 32)]
    assert layers[1][0][0, 0, 0] == 320 and layers[1][1][0] == 320 + 9216


def test_zero_network_returns_ubar_and_loss_is_target_energy():
    p = np.zeros(cnn.param_count())
    ub = rng(10).standard_normal((3, 8, 6))
    u = rng(11).standard_normal((3, 8, 6))
    f = cnn.forward(p, ub)
    np.testing.assert_array_equal(f["u0"], ub)
    loss, _ = cnn.loss_and_grad(p, ub, u)
    t = (u - ub) / cnn.rms(ub)[:, None, None]
    assert abs(loss - np.mean(t * t)) <= 1e-14 * loss


def test_scale_equivariance():
    """The input normalisation makes u0(c * ubar) = c * u0(ubar) for c > 0."""
    p = synth.cnn_init_params(4)
    p[cnn.param_count() - 1] = 0.1
    ub = rng(12).standard_normal((2, 9, 8))
    a = cnn.forward(p, ub)["u0"]
    b = cnn.forward(p, 7.5 * ub)["u0"]
    np.testing.assert_allclose(b, 7.5 * a, rtol=1e-12, atol=1e-12)


def test_identity_path_network():
    """Delta kernels and positive pre-activations carry x0 straight through:
    with every layer passing channel 0's centre tap, z = x0, so
    u0 = ubar + G ubar."""
    p = np.zeros(cnn.param_count())
    layers = cnn.unpack(p)
    ub = np.abs(rng(13).standard_normal((1, 5, 6))) + 0.1   # positive, so the ReLUs pass it
    for W, b in layers:
        W[0, 4, 0] = 1.0
    f = cnn.forward(p, ub)
    np.testing.assert_allclose(f["u0"], ub + oracle.filter(ub, 2), rtol=1e-14)


def test_correction_lies_in_the_range_of_g():
    """On an even grid the stencil's transfer function vanishes on the Nyquist
    lines, so the correction u0 - ubar has no content there (checked by FFT)."""
    p = synth.cnn_init_params(6)
    p[cnn.param_count() - 1] = 0.2
    ub = rng(14).standard_normal((2, 8, 6))
    corr = cnn.forward(p, ub)["u0"] - ub
    F = np.fft.fft2(corr)
    assert np.max(np.abs(F[:, 4, :])) <= 1e-12 * np.max(np.abs(F))
    assert np.max(np.abs(F[:, :, 3])) <= 1e-12 * np.max(np.abs(F))


def test_adam_first_step_closed_form():
    """After one step from zero moments, the bias-corrected update is
    lr * g / (|g| + eps) (a signed step of nearly lr)."""
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p = np.ones(4)
    p1, m, v = cnn.adam_step(p, np.zeros(4), np.zeros(4), g, 1, lr=0.01)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_bf16_rounding_bit_patterns():
    # exact, halfway cases (ties to even) and plain rounding
    one = 1.0
    ulp = 2.0 ** -7                         # bf16 spacing just above 1
    x = np.array([one, one + ulp / 2, one + 1.5 * ulp, one + 0.3 * ulp, -2.0 - 0.7 * ulp * 2, 0.0])
    want = np.array([one, one, one + 2 * ulp, one, -2.0 - 2 * ulp, 0.0])
    np.testing.assert_array_equal(cnn.bf16(x), want)


# ------------------------------------------------------------------ 3D network
def fft_correlate3(x, w):
    """3D periodic cross-correlation with a 3x3x3 kernel through the FFT."""
    k = np.zeros(x.shape)
    for t, (dz, dy, dx) in enumerate(cnn.TAPS3):
        k[(-dz) % x.shape[0], (-dy) % x.shape[1], (-dx) % x.shape[2]] += w[t]
    return np.real(np.fft.ifftn(np.fft.fftn(x) * np.fft.fftn(k)))


@pytest.mark.parametrize("shape", [(4, 5, 6), (3, 3, 3), (1, 2, 5)])
def test_conv3d_is_fft_circular_correlation(shape):
    x = rng(21).standard_normal((2,) + shape + (3,))
    W = rng(22).standard_normal((2, 27, 3))
    b = rng(23).standard_normal(2)
    out = cnn.conv(x, W, b)
    for bb in range(2):
        for o in range(2):
            want = b[o] + sum(fft_correlate3(x[bb, ..., c], W[o, :, c]) for c in range(3))
            np.testing.assert_allclose(out[bb, ..., o], want, rtol=0, atol=1e-12)


def test_conv3d_adjoints():
    x = rng(24).standard_normal((1, 3, 4, 5, 2))
    g = rng(25).standard_normal((1, 3, 4, 5, 3))
    W = rng(26).standard_normal((3, 27, 2))
    lhs = np.sum(cnn.conv(x, W, np.zeros(3)) * g)
    assert abs(lhs - np.sum(x * cnn.conv_grad_input(g, W))) <= 1e-11 * abs(lhs)
    dW, _ = cnn.conv_grad_weight(x, g)
    assert abs(np.sum(dW * W) - lhs) <= 1e-11 * abs(lhs)


def test_param_count_3d():
    assert cnn.param_count(ndim=3) == (864 + 32) + 4 * (27648 + 32) + (864 + 1) == 112481
    assert synth.cnn_init_params(0, ndim=3).size == 112481


def test_backprop_3d_matches_central_differences():
    params = synth.cnn_init_params(3, channels=4, ndim=3)
    params[-1] = 0.05
    ub = rng(27).standard_normal((2, 3, 4, 5))
    u = ub + 0.3 * rng(28).standard_normal((2, 3, 4, 5))
    loss, g = cnn.loss_and_grad(params, ub, u, channels=4, ndim=3)
    pick = rng(29).choice(params.size, size=60, replace=False)
    eps = 1e-6
    for i in pick:
        p1, p2 = params.copy(), params.copy()
        p1[i] += eps
        p2[i] -= eps
        fd = (cnn.loss_and_grad(p1, ub, u, channels=4, ndim=3)[0] - cnn.loss_and_grad(p2, ub, u, channels=4, ndim=3)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_3d_correction_in_range_of_g_and_scale_equivariant():
    p = synth.cnn_init_params(7, ndim=3)
    p[cnn.param_count(ndim=3) - 1] = 0.2
    ub = rng(30).standard_normal((1, 4, 6, 8))
    f = cnn.forward(p, ub, ndim=3)
    F = np.fft.fftn(f["u0"][0] - ub[0])
    for ax, n in enumerate((4, 6, 8)):
        sl = [slice(None)] * 3
        sl[ax] = n // 2
        assert np.max(np.abs(F[tuple(sl)])) <= 1e-12 * np.max(np.abs(F))
    np.testing.assert_allclose(cnn.forward(p, 3.0 * ub, ndim=3)["u0"], 3.0 * f["u0"], rtol=1e-12, atol=1e-12)


def test_smoothed_output_transfer_function():
    """smooth = m: the correction is G^m z, whose Fourier coefficients are
    those of z times the closed-form transfer function to the m-th power,
    prod_d cos^(2m)(pi k_d / n_d); checked by FFT against a run with smooth=1
    (whose correction is G z) on the same network."""
    p = synth.cnn_init_params(11)
    p[cnn.param_count() - 1] = 0.1
    ub = rng(15).standard_normal((2, 10, 12))
    c1 = cnn.forward(p, ub, smooth=1)["u0"] - ub
    c3 = cnn.forward(p, ub, smooth=3)["u0"] - ub
    ky = np.arange(10)[:, None]
    kx = np.arange(12)[None, :]
    gh = np.cos(np.pi * ky / 10) ** 2 * np.cos(np.pi * kx / 12) ** 2
    np.testing.assert_allclose(np.fft.fft2(c3), np.fft.fft2(c1) * gh ** 2, atol=1e-12 * np.abs(np.fft.fft2(c1)).max())


@pytest.mark.parametrize("ndim,shape", [(2, (5, 6)), (3, (3, 4, 5))])
def test_backprop_with_smoothing_matches_central_differences(ndim, shape):
    params = synth.cnn_init_params(4, channels=4, ndim=ndim)
    params[-1] = 0.05
    ub = rng(17).standard_normal((2,) + shape)
    u = ub + 0.3 * rng(18).standard_normal((2,) + shape)
    loss, g = cnn.loss_and_grad(params, ub, u, channels=4, ndim=ndim, smooth=3)
    pick = rng(19).choice(params.size, size=40, replace=False)
    eps = 1e-6
    for i in pick:
        p1, p2 = params.copy(), params.copy()
        p1[i] += eps
        p2[i] -= eps
        l1, _ = cnn.loss_and_grad(p1, ub, u, channels=4, ndim=ndim, smooth=3)
        l2, _ = cnn.loss_and_grad(p2, ub, u, channels=4, ndim=ndim, smooth=3)
        fd = (l1 - l2) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])
