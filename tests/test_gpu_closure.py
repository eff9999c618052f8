"""Closure stress on the GPU (closure_stress) against the oracle's
tau_ij = ubar_i ubar_j - G(u*_i u*_j) (Sec. 2, Eq. fge3; Sec. 3).

Tolerance, from the arithmetic: each output is one product minus a sum of
9 (2D) or 27 (3D) weighted products with power-of-two weights; with unit
roundoff u every rounding error is at most u times a partial sum bounded by
S_ij = max|ubar_i ubar_j| + max|u*_i u*_j|, and there are fewer than 60 of
them, so |tau_gpu - tau_oracle| <= 60 u S_ij: 4e-6 S_ij in FP32 (u = 2^-24;
the inputs are FP32 values, so the oracle sees exactly what the GPU sees) and
1.5e-14 S_ij in FP64 (the oracle's own rounding included).
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import to_dev
from paper_1707_09177_amd import gdecon, synth

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 4e-6, torch.float64: 1.5e-14}


def velocity(shape, nd, batch, seed, dtype):
    """(batch, nd, *shape) velocities u, ubar = G u and an inexact u*."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((batch, nd) + shape)
    ub = oracle.filter(u, nd)
    us = u + 0.05 * rng.standard_normal(u.shape)
    if dtype == torch.float32:
        ub = ub.astype(np.float32).astype(np.float64)
        us = us.astype(np.float32).astype(np.float64)
    return ub, us


def check(got, want, ub, us, nd, dtype):
    ax = -nd - 1
    for q, (i, j) in enumerate(oracle.stress_pairs(nd)):
        s = (np.max(np.abs(np.take(ub, i, axis=ax) * np.take(ub, j, axis=ax)))
             + np.max(np.abs(np.take(us, i, axis=ax) * np.take(us, j, axis=ax))))
        err = np.max(np.abs(np.take(got, q, axis=ax) - np.take(want, q, axis=ax)))
        assert err <= TOL[dtype] * s, ((i, j), err, s)


SHAPES = [(9, 7), (1, 1), (1, 5), (8, 32), (64, 64), (130, 300), (33, 1000),
          (5, 3, 7), (1, 1, 1), (2, 3, 4), (40, 17, 70), (65, 9, 33), (33, 8, 32), (3, 64, 8)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("batch", [1, 2])
def test_closure_matches_oracle(shape, dtype, batch):
    nd = len(shape)
    ub, us = velocity(shape, nd, batch, 10 + len(shape) + batch, dtype)
    want = oracle.closure_stress(ub, us, nd)
    tau = gdecon.closure_stress(to_dev(ub, dtype), to_dev(us, dtype), nd)
    torch.cuda.synchronize()
    assert tuple(tau.shape) == want.shape
    check(tau.double().cpu().numpy(), want, ub, us, nd, dtype)


def test_closure_deterministic_and_fields_independent():
    ub, us = velocity((40, 17, 70), 3, 3, 1, torch.float32)
    a, b = to_dev(ub, torch.float32), to_dev(us, torch.float32)
    t = gdecon.closure_stress(a, b, 3)
    t2 = gdecon.closure_stress(a, b, 3)
    t1 = gdecon.closure_stress(a[1:2].contiguous(), b[1:2].contiguous(), 3)
    torch.cuda.synchronize()
    assert torch.equal(t, t2)
    assert torch.equal(t[1:2], t1)


@pytest.mark.parametrize("nd", [2, 3])
def test_second_order_ad_end_to_end(nd):
    """The deconvolution and the closure chained on the GPU: one van Cittert
    update from u0 = ubar (u* = 2 ubar - G ubar) gives the second-order model
    (Eq. tau3); the oracle runs its own solve for u*."""
    shape = (72, 96) if nd == 2 else (20, 24, 36)
    u = np.random.default_rng(30 + nd).standard_normal((nd,) + shape)
    ub = oracle.filter(u, nd)
    ust, _, _ = gdecon.deconvolve("vc", to_dev(ub, torch.float64), 1, ndim=nd)
    tau = gdecon.closure_stress(to_dev(ub, torch.float64)[None], ust[None], nd)
    torch.cuda.synchronize()
    us_ref = oracle.solve("vc", ub, nd, 1)[0]
    want = oracle.closure_stress(ub[None], us_ref[None], nd)
    np.testing.assert_allclose(tau.cpu().numpy(), want, rtol=0, atol=1e-13)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("case", ["2048sq_x8", "256cube"])
def test_closure_full_size(case):
    """The bench's closure workloads at full size, FP32, compared at every point:
    eight 2D velocities of 2048^2 with the k^-3 spectrum, and one 3D
    divergence-free 256^3 velocity with the k^-5/3 spectrum."""
    if case == "2048sq_x8":
        nd = 2
        u = synth.config_fields(2, dtype=np.float32).reshape(8, 2, 2048, 2048).astype(np.float64)
    else:
        nd = 3
        u = synth.config_fields(3, dtype=np.float32).reshape(1, 3, 256, 256, 256).astype(np.float64)
    ub = oracle.filter(u, nd).astype(np.float32).astype(np.float64)
    us = (u + 0.01 * np.random.default_rng(40).standard_normal(u.shape)).astype(np.float32).astype(np.float64)
    want = oracle.closure_stress(ub, us, nd)
    tau = gdecon.closure_stress(to_dev(ub, torch.float32), to_dev(us, torch.float32), nd)
    torch.cuda.synchronize()
    check(tau.double().cpu().numpy(), want, ub, us, nd, torch.float32)


def test_closure_rejects_mismatch():
    x = torch.zeros((2, 8, 8), device="cuda")
    with pytest.raises(ValueError):
        gdecon.closure_stress(x, x, 3)
    with pytest.raises(ValueError):
        gdecon.closure_stress(x, x.double(), 2)


@pytest.mark.parametrize("nd", [2, 3])
def test_bardina_and_layton_forms(nd):
    """The scale-similarity models are closure_stress calls with particular
    inputs: u* = ubar gives Eq. tau2; ubar := G ubar, u* = ubar gives the
    Bardina model of Eq. tau1."""
    shape = (40, 56) if nd == 2 else (12, 20, 24)
    ub = oracle.filter(np.random.default_rng(50 + nd).standard_normal((1, nd) + shape), nd)
    ubb = oracle.filter(ub, nd)
    d_ub, d_ubb = to_dev(ub, torch.float64), to_dev(ubb, torch.float64)
    lay = gdecon.closure_stress(d_ub, d_ub, nd)
    bar = gdecon.closure_stress(d_ubb, d_ub, nd)
    torch.cuda.synchronize()
    for q, (i, j) in enumerate(oracle.stress_pairs(nd)):
        prod = ub[0, i] * ub[0, j]
        want_l = prod - oracle.filter(prod, nd)
        want_b = ubb[0, i] * ubb[0, j] - oracle.filter(prod, nd)
        np.testing.assert_allclose(lay[0, q].cpu().numpy(), want_l, rtol=0, atol=1e-14)
        np.testing.assert_allclose(bar[0, q].cpu().numpy(), want_b, rtol=0, atol=1e-14)
