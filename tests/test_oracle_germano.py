"""Pins of the oracle with the paper's own filter: the differential filter
G = (I - delta^2 lap)^-1 applied through the FFT (Sec. 4, Eqs. df, df2).

Independent constructions: single Fourier modes written with np.cos, and the
dense matrix of G built from complex exponentials (np.exp, no FFT), on which
the solver pins (Krylov optimality, BiCGSTAB residual polynomials, exact
inverse) are checked.
"""
import numpy as np
import pytest

import oracle
import spectral as sp
from test_oracle_pins import bicgstab_from_cg_polynomials


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def signed(k, n):
    return k if k <= n // 2 else k - n


def ghat_closed(k, shape, gamma):
    """1 / (1 + |k|^2 / k_c^2), k_c = gamma * min(n) / 2, k the aliased integer wavenumber."""
    kc = gamma * min(shape) / 2.0
    k2 = sum(signed(kd, n) ** 2 for kd, n in zip(k, shape))
    return 1.0 / (1.0 + k2 / kc ** 2)


def dense_germano(shape, gamma):
    """G = (1/N) F^H diag(G_hat) F with F[k, x] = exp(-2 pi i k.x / n)."""
    pts = np.array(np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")).reshape(len(shape), -1)
    ks = pts.copy()
    phase = sum(np.outer(ks[d], pts[d]) / shape[d] for d in range(len(shape)))
    F = np.exp(-2j * np.pi * phase)
    g = np.array([ghat_closed(tuple(ks[:, j]), shape, gamma) for j in range(ks.shape[1])])
    return np.real(F.conj().T @ (g[:, None] * F)) / F.shape[0]


SHAPES = [(8, 8), (6, 10), (9, 7), (4, 6, 8), (5, 3, 7)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("gamma", [0.1, 0.5, 1.0])
def test_single_modes_closed_form(shape, gamma):
    nd = len(shape)
    rng = np.random.default_rng(1)
    coords = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in shape], indexing="ij")
    modes = [tuple(n // 2 for n in shape)] + [tuple(int(rng.integers(0, n)) for n in shape) for _ in range(5)]
    for k in modes:
        phi = rng.uniform(0, 2 * np.pi)
        x = np.cos(sum(kd * c for kd, c in zip(k, coords)) + phi)
        y = oracle.germano_filter(x, nd, gamma)
        assert np.max(np.abs(y - ghat_closed(k, shape, gamma) * x)) < 1e-14, k


@pytest.mark.parametrize("shape", SHAPES)
def test_matches_dense_matrix_spd_and_contraction(shape):
    nd = len(shape)
    gm = dense_germano(shape, 0.3)
    x = np.random.default_rng(2).standard_normal((3,) + shape)
    y = oracle.germano_filter(x, nd, 0.3)
    for b in range(3):
        np.testing.assert_allclose(y[b].ravel(), gm @ x[b].ravel(), atol=1e-13)
    assert np.max(np.abs(gm - gm.T)) < 1e-14
    ev = np.linalg.eigvalsh(gm)
    assert ev.min() > 0 and ev.max() <= 1 + 1e-13        # SPD, stable (|1 - G_hat| <= 1)
    assert abs(np.sum(y) - np.sum(x)) < 1e-10              # the mean is kept (G_hat(0) = 1)


@pytest.mark.parametrize("shape", [(8, 8), (4, 6, 8)])
@pytest.mark.parametrize("N", [1, 3, 6])
def test_vancittert_transfer_closed_form(shape, N):
    """u_N on one mode = sum_{n=0..N} (1 - G_hat)^n G_hat times the mode."""
    nd = len(shape)
    coords = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in shape], indexing="ij")
    k = tuple(min(3, n // 2) for n in shape)
    mode = np.cos(sum(kd * c for kd, c in zip(k, coords)))
    g = ghat_closed(k, shape, 0.2)
    u, _, _ = oracle.solve("vc", g * mode, nd, N, gamma=0.2)
    want = sum((1 - g) ** n for n in range(N + 1)) * g * mode
    assert np.max(np.abs(u - want)) < 1e-13


@pytest.mark.parametrize("shape", [(8, 8), (9, 7), (4, 6, 8)])
def test_cg_is_krylov_optimal(shape):
    nd = len(shape)
    gm = dense_germano(shape, 0.2)
    ub = (gm @ np.random.default_rng(3).standard_normal(int(np.prod(shape)))).reshape(shape)
    for n in range(1, 6):
        u, _, _ = oracle.solve("cg", ub, nd, n, gamma=0.2)
        want = sp.cg_krylov_iterate(gm, ub.ravel(), ub.ravel().copy(), n)
        assert rel(u.ravel(), want) < 1e-9, n


@pytest.mark.parametrize("shape", [(8, 8), (5, 3, 7)])
def test_bicgstab_matches_stabilised_cg_polynomials(shape):
    """(gamma 0.6: the brute-force Krylov basis loses digits on stiffer filters)"""
    nd = len(shape)
    gm = dense_germano(shape, 0.6)
    ub = (gm @ np.random.default_rng(4).standard_normal(int(np.prod(shape)))).reshape(shape)
    want = bicgstab_from_cg_polynomials(gm, ub.ravel(), ub.ravel().copy(), 4)
    for n in range(1, 5):
        u, _, _ = oracle.solve("bicgstab", ub, nd, n, gamma=0.6)
        r = ub.ravel() - gm @ u.ravel()
        assert rel(r, want[n - 1]) < 1e-8, n


@pytest.mark.parametrize("solver", ["cg", "bicgstab", "sd", "vc"])
def test_converges_to_exact_inverse(solver):
    """u_hat = (1 + (k / k_c)^2) ubar_hat, the inverse of Eq. df2, applied with the dense matrix."""
    shape = (8, 10)
    gamma = 0.6 if solver in ("sd", "vc") else 0.2
    gm = dense_germano(shape, gamma)
    u_true = np.random.default_rng(5).standard_normal(int(np.prod(shape)))
    ub = (gm @ u_true).reshape(shape)
    u, info, _ = oracle.solve(solver, ub, 2, 5000, tol=1e-12, gamma=gamma)
    assert info[0]["status_name"] == "CONVERGED"
    assert rel(u.ravel(), u_true) < 1e-9
    assert rel(np.linalg.solve(gm, ub.ravel()), u_true) < 1e-12


def test_sd_successive_residuals_orthogonal():
    shape = (8, 8)
    gm = dense_germano(shape, 0.2)
    ub = (gm @ np.random.default_rng(6).standard_normal(64)).reshape(shape)
    rs = []
    for n in range(0, 4):
        u, _, _ = oracle.solve("sd", ub, 2, n, gamma=0.2)
        rs.append(ub.ravel() - gm @ u.ravel())
    for a, b in zip(rs, rs[1:]):
        assert abs(np.dot(a, b)) < 1e-10 * np.linalg.norm(a) * np.linalg.norm(b)


def test_conditioning_of_the_papers_settings():
    """kappa = 1 + (k_max / k_c)^2 with k_max = sqrt(d) n / 2: about 2e4 at
    gamma = 0.01 and about 200 at gamma = 0.1 (2D)."""
    for gamma, want in [(0.01, 2.0e4), (0.1, 2.0e2)]:
        g = oracle.germano_hat((256, 256), 2, gamma)
        kappa = g.max() / g.min()
        assert abs(kappa - (1 + 2 / gamma ** 2)) < 1e-6 * kappa
        assert 0.9 * want < kappa < 1.1 * want
