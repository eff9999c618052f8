"""Pins of the oracle's closure stress tau_ij = ubar_i ubar_j - G(u*_i u*_j)
(Sec. 2, Eq. fge3, with the deconvolved velocity of Sec. 3).

Each pin is fixed by something other than the oracle's own formula:
- single Fourier modes, where the filter's transfer function gives tau in
  closed form (catches a dropped term, a wrong pair or a transposed operand);
- a brute-force loop over the 3x3 / 3x3x3 trapezoidal weights on tiny grids;
- the exact identity for a uniform velocity shift, whose extra terms are the
  deconvolution residual r = ubar - G u*;
- u* = ubar (Eq. tau2) and u* after two van Cittert terms (Eq. tau3).
"""
import itertools

import numpy as np
import pytest

import oracle


def ghat(k, shape):
    """Transfer function of the trapezoidal filter: prod cos^2(pi k_d / n_d)."""
    return float(np.prod([np.cos(np.pi * kd / n) ** 2 for kd, n in zip(k, shape)]))


def mode(k, phi, shape):
    coords = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in shape], indexing="ij")
    return np.cos(sum(kd * c for kd, c in zip(k, coords)) + phi)


@pytest.mark.parametrize("shape", [(12, 16), (9, 14), (8, 10, 12), (7, 6, 9)])
def test_single_modes_closed_form(shape):
    """u_i = cos(a_i.x + p_i) and ubar = G u: then
    ubar_i ubar_j = Ghat(a_i) Ghat(a_j) u_i u_j and
    G(u_i u_j) = (Ghat(a_i + a_j) cos((a_i + a_j).x + p_i + p_j)
                 + Ghat(a_i - a_j) cos((a_i - a_j).x + p_i - p_j)) / 2."""
    nd = len(shape)
    rng = np.random.default_rng(3)
    a = [[int(rng.integers(0, n)) for n in shape] for _ in range(nd)]
    p = rng.uniform(0, 2 * np.pi, nd)
    u = np.stack([mode(a[i], p[i], shape) for i in range(nd)])
    ub = np.stack([ghat(a[i], shape) * u[i] for i in range(nd)])
    tau = oracle.closure_stress(ub, u, nd)
    for q, (i, j) in enumerate(oracle.stress_pairs(nd)):
        s = [ai + aj for ai, aj in zip(a[i], a[j])]
        d = [ai - aj for ai, aj in zip(a[i], a[j])]
        want = ghat(a[i], shape) * ghat(a[j], shape) * u[i] * u[j] - 0.5 * (
            ghat(s, shape) * mode(s, p[i] + p[j], shape) + ghat(d, shape) * mode(d, p[i] - p[j], shape))
        assert np.max(np.abs(tau[q] - want)) < 1e-13, (i, j)


def brute(ub, us, nd):
    """Pure-Python loops: weights 1/2 (centre) and 1/4 (each neighbour) per
    axis, periodic wrap, pairs in the order 11, 12, (13,) 22, ..."""
    shape = ub.shape[1:]
    w = {-1: 0.25, 0: 0.5, 1: 0.25}
    pairs = [(i, j) for i in range(nd) for j in range(nd) if i <= j]
    out = np.zeros((len(pairs),) + shape)
    for q, (i, j) in enumerate(pairs):
        for pt in itertools.product(*[range(n) for n in shape]):
            acc = 0.0
            for off in itertools.product((-1, 0, 1), repeat=nd):
                nb = tuple((c + o) % n for c, o, n in zip(pt, off, shape))
                acc += np.prod([w[o] for o in off]) * us[i][nb] * us[j][nb]
            out[(q,) + pt] = ub[i][pt] * ub[j][pt] - acc
    return out


@pytest.mark.parametrize("shape", [(3, 4), (1, 5), (2, 3, 4), (3, 1, 2)])
def test_matches_brute_force(shape):
    nd = len(shape)
    rng = np.random.default_rng(4)
    ub = rng.standard_normal((nd,) + shape)
    us = rng.standard_normal((nd,) + shape)
    np.testing.assert_allclose(oracle.closure_stress(ub, us, nd), brute(ub, us, nd), rtol=0, atol=1e-14)


@pytest.mark.parametrize("shape", [(10, 14), (6, 5, 8)])
def test_uniform_shift_adds_residual_terms(shape):
    """tau(ubar + U, u* + U) - tau(ubar, u*) = U_i r_j + U_j r_i with
    r = ubar - G u* (G keeps constants): zero when u* solves G u* = ubar."""
    nd = len(shape)
    rng = np.random.default_rng(5)
    u = rng.standard_normal((nd,) + shape)
    ub = oracle.filter(u, nd)
    us = u + 0.1 * rng.standard_normal(u.shape)           # an inexact deconvolution
    U = rng.standard_normal(nd)
    Ub = U.reshape((nd,) + (1,) * nd)
    r = ub - oracle.filter(us, nd)
    d = oracle.closure_stress(ub + Ub, us + Ub, nd) - oracle.closure_stress(ub, us, nd)
    for q, (i, j) in enumerate(oracle.stress_pairs(nd)):
        np.testing.assert_allclose(d[q], U[i] * r[j] + U[j] * r[i], atol=1e-12)
    # the exact deconvolution: the stress is unchanged by the shift
    d0 = oracle.closure_stress(ub + Ub, u + Ub, nd) - oracle.closure_stress(ub, u, nd)
    assert np.max(np.abs(d0)) < 1e-12


def test_constant_and_symmetry():
    rng = np.random.default_rng(6)
    c = rng.standard_normal(3).reshape(3, 1, 1, 1) * np.ones((3, 4, 5, 6))
    assert np.max(np.abs(oracle.closure_stress(c, c, 3))) < 1e-14
    # swapping components 1 and 3 of both fields permutes the pairs
    ub = rng.standard_normal((3, 4, 5, 6))
    us = rng.standard_normal((3, 4, 5, 6))
    t = oracle.closure_stress(ub, us, 3)
    ts = oracle.closure_stress(ub[[2, 1, 0]], us[[2, 1, 0]], 3)
    pairs = oracle.stress_pairs(3)
    swap = {0: 2, 1: 1, 2: 0}
    for q, (i, j) in enumerate(pairs):
        a, b = sorted((swap[i], swap[j]))
        np.testing.assert_array_equal(ts[pairs.index((a, b))], t[q])


@pytest.mark.parametrize("nd", [2, 3])
def test_layton_and_second_order_ad(nd):
    """u* = ubar gives Eq. tau2; u* = 2 ubar - G ubar (one van Cittert update
    from u0 = ubar, Eq. adm1) gives the second-order model of Eq. tau3."""
    shape = (9, 12) if nd == 2 else (5, 6, 7)
    rng = np.random.default_rng(7)
    ub = oracle.filter(rng.standard_normal((nd,) + shape), nd)
    t2 = oracle.closure_stress(ub, ub, nd)
    u1 = np.stack([oracle.solve("vc", ub[c], nd, 1)[0] for c in range(nd)])
    np.testing.assert_allclose(u1, 2 * ub - oracle.filter(ub, nd), atol=1e-14)
    t3 = oracle.closure_stress(ub, u1, nd)
    ubb = oracle.filter(ub, nd)
    for q, (i, j) in enumerate(oracle.stress_pairs(nd)):
        np.testing.assert_allclose(t2[q], ub[i] * ub[j] - oracle.filter(ub[i] * ub[j], nd), atol=1e-14)
        want = ub[i] * ub[j] - oracle.filter((2 * ub[i] - ubb[i]) * (2 * ub[j] - ubb[j]), nd)
        np.testing.assert_allclose(t3[q], want, atol=1e-13)


def test_batch_leading_dims():
    rng = np.random.default_rng(8)
    ub = rng.standard_normal((2, 3, 2, 6, 7))
    us = rng.standard_normal(ub.shape)
    t = oracle.closure_stress(ub, us, 2)
    assert t.shape == (2, 3, 3, 6, 7)
    np.testing.assert_array_equal(t[1, 2], oracle.closure_stress(ub[1, 2], us[1, 2], 2))
