"""Van Cittert with several passes per sweep (deconvolve_vancittert_blocked)
against the oracle's Algorithm 1 and against the one-pass-per-sweep GPU solve.

The blocked solve evaluates the same stencil in LDS instead of in registers,
so it differs from both by rounding only: relative L2 <= 1e-12 (FP64) and
<= 1e-5 (FP32) on u, exact pass counts and statuses, and histories to the
same tolerances.  Fixed pass counts straddle the sweep boundaries (K = 8 in
2D, 2 in 3D); tolerance runs stop inside a sweep, which exercises the
recomputation of that sweep.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import rel_l2_per_field, to_dev
from paper_1707_09177_amd import gdecon

pytestmark = pytest.mark.gpu

SHAPES = [(9, 7), (1, 1), (2, 3), (130, 300), (33, 1000), (64, 64), (5, 3, 7), (1, 1, 1), (20, 24, 36), (17, 33, 9),
          (8, 13, 70)]


def rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def run(ub, nd, N, dtype, tol=0.0, init="ubar", u0=None, norm_ref="r0ubar"):
    t = to_dev(ub, dtype)
    d = gdecon.BlockedVanCittert(t.shape, nd, dtype)
    out = to_dev(u0, dtype) if u0 is not None else None
    hist = torch.full((d.batch, N + 1), float("nan"), dtype=torch.float64, device="cuda")
    res = d.solve(t, N, tol, init=init, out=out, norm_ref=norm_ref, history=hist)
    torch.cuda.synchronize()
    return res.u.double().cpu().numpy(), res.info(), hist.cpu().numpy()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("N", [1, 3, 8, 13])
def test_fixed_passes_match_oracle(shape, dtype, N):
    nd = len(shape)
    ub = oracle.filter(rand((2,) + shape, 3 + len(shape)), nd)
    if dtype == torch.float32:
        ub = ub.astype(np.float32).astype(np.float64)
    want, winf, whist = oracle.solve("vc", ub, nd, N)
    got, ginf, ghist = run(ub, nd, N, dtype)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    for e in rel_l2_per_field(got, want, nd):
        assert e <= tol, e
    for b, (gi, wi) in enumerate(zip(ginf, winf)):
        if wi["r_ref"] <= 1e-13 * np.linalg.norm(ub[b]):
            # G is the identity up to rounding (a 1-point grid): r_ref is 0 or
            # rounding noise depending on the summation order, so ZERO_REF
            # against a few passes on noise is a rounding decision
            assert gi["status_name"] in ("ZERO_REF", wi["status_name"])
            continue
        assert gi["iters"] == wi["iters"] and gi["status_name"] == wi["status_name"]
        for k in ("r_ref", "r0", "r_final", "r_true"):
            assert abs(gi[k] - wi[k]) <= tol * max(wi["r_ref"], 1e-300), k
        np.testing.assert_allclose(ghist[b], whist[b], rtol=tol, atol=1e-300)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", [(130, 300), (64, 64), (20, 24, 36), (17, 33, 9)])
def test_tolerance_stops_inside_a_sweep(shape, dtype):
    """Fields of different smoothness stop at different passes, most of them
    inside a sweep; pass counts, statuses and u match the oracle."""
    nd = len(shape)
    u = np.stack([oracle.filter(rand(shape, 40 + i), nd) for i in range(4)])
    u[1::2] = oracle.filter(u[1::2], nd)                  # smoother fields stop sooner
    ub = oracle.filter(u, nd)
    if dtype == torch.float32:
        ub = ub.astype(np.float32).astype(np.float64)
    want, winf, _ = oracle.solve("vc", ub, nd, 300, tol=3e-3)
    got, ginf, _ = run(ub, nd, 300, dtype, tol=3e-3)
    iters = [w["iters"] for w in winf]
    assert len(set(iters)) > 1, iters                     # the fields really stop apart
    for gi, wi in zip(ginf, winf):
        assert gi["status_name"] == wi["status_name"] == "CONVERGED"
        assert abs(gi["iters"] - wi["iters"]) <= (0 if dtype == torch.float64 else 1)
    if dtype == torch.float64:
        for e in rel_l2_per_field(got, want, nd):
            assert e <= 1e-11, e


@pytest.mark.parametrize("init", ["zero", "given"])
@pytest.mark.parametrize("norm_ref", ["r0ubar", "ubar"])
@pytest.mark.parametrize("shape", [(40, 72), (6, 10, 12)])
def test_starts_and_norms(init, norm_ref, shape):
    nd = len(shape)
    ub = oracle.filter(rand((2,) + shape, 60), nd)
    u0 = 0.3 * ub + 0.1 * rand(ub.shape, 61) if init == "given" else None
    want, winf, _ = oracle.solve("vc", ub, nd, 11, init=init, u0=u0, norm_ref=norm_ref)
    got, ginf, _ = run(ub, nd, 11, torch.float64, init=init, u0=u0, norm_ref=norm_ref)
    for e in rel_l2_per_field(got, want, nd):
        assert e <= 1e-12, e
    for gi, wi in zip(ginf, winf):
        assert abs(gi["r_ref"] - wi["r_ref"]) <= 1e-12 * wi["r_ref"]
        assert abs(gi["r0"] - wi["r0"]) <= 1e-12 * wi["r_ref"]


def test_matches_one_pass_solver_and_zero_ref():
    ub = oracle.filter(rand((3, 96, 160), 70), 2)
    ub[1] = 0.0                                           # ZERO_REF field
    got, ginf, _ = run(ub, 2, 20, torch.float32, tol=1e-5)
    one, oinf, _ = gdecon.deconvolve("vc", to_dev(ub, torch.float32), 20, tol=1e-5)
    assert ginf[1]["status_name"] == oinf[1]["status_name"] == "ZERO_REF"
    for gi, oi in zip(ginf, oinf):
        assert gi["iters"] == oi["iters"] and gi["status_name"] == oi["status_name"]
    assert np.max(np.abs(got[1])) == 0.0
    for b in (0, 2):
        assert np.linalg.norm(got[b] - one[b].double().cpu().numpy()) <= 1e-5 * np.linalg.norm(got[b])


def test_bench_size_converges_like_the_oracle():
    """2048^2 x 16 FP32 to 1e-6 (the bench's Van Cittert comparison): the
    same pass counts as the one-pass GPU solve (within one, plus one for each
    residual replacement the one-pass solve made), true residuals within
    twice the tolerance (the blocked solve stops on its recursive residual)."""
    from paper_1707_09177_amd import synth
    u = torch.from_numpy(synth.config_fields(2, dtype=np.float32)).cuda()
    ub = gdecon.filter_apply(u, ndim=2)
    d = gdecon.BlockedVanCittert(ub.shape, 2, ub.dtype)
    res = d.solve(ub, 500, 1e-6)
    info = res.info()
    _, oinf, _ = gdecon.deconvolve("vc", ub, 500, tol=1e-6)
    for gi, oi in zip(info, oinf):
        assert gi["status_name"] == "CONVERGED" and abs(gi["iters"] - oi["iters"]) <= 1 + oi["replaced"]
        assert gi["r_true"] <= 2e-6 * gi["r_ref"]


@pytest.mark.parametrize("max_iter", [9, 10, 12, 17, 300])
@pytest.mark.parametrize("shape", [(130, 300), (20, 24, 36)])
def test_predicted_sweep_lengths_match_oracle(shape, max_iter):
    """A sweep is shortened to the passes the residual's last decay rate
    predicts to the tolerance.  On random fields the decay slows down, so
    predictions fall short and a field takes short sweeps, or runs into
    max_iter within one: pass counts, statuses, histories and u match the
    oracle."""
    nd = len(shape)
    ub = oracle.filter(rand((3,) + shape, 80), nd)
    tol = 2e-2
    want, winf, whist = oracle.solve("vc", ub, nd, max_iter, tol=tol)
    got, ginf, ghist = run(ub, nd, max_iter, torch.float64, tol=tol)
    for gi, wi in zip(ginf, winf):
        assert gi["iters"] == wi["iters"] and gi["status_name"] == wi["status_name"], (gi, wi)
    for e in rel_l2_per_field(got, want, nd):
        assert e <= 1e-11, e
    for b in range(ub.shape[0]):
        n = winf[b]["iters"]
        np.testing.assert_allclose(ghist[b][:n + 1], whist[b][:n + 1], rtol=1e-11, atol=1e-300)
