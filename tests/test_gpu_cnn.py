"""Learned warm start on the GPU (warmstart_forward / warmstart_train_step)
against the FP64 network reference in oracle/cnn.py.

Tolerances: the GPU stores weights, activations and activation gradients in
bfloat16 and accumulates in FP32.  The reference run with `emulate_bf16`
rounds the same quantities the same way, so the two differ only by FP32
accumulation order, which flips an occasional bfloat16 rounding (one unit in
the 8th bit): relative L2 <= 3e-3 on the network output and the loss, <= 2e-2
on each layer's weight gradient (sums of many such products).  Against the
unrounded FP64 reference the output must agree to bfloat16 precision (2e-2).
The benefit of training is empirical (parity unpinned): only convergence of
the warm-started solve is asserted.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import rel_l2, to_dev
from oracle import cnn
from paper_1707_09177_amd import gdecon, synth

pytestmark = pytest.mark.gpu


def params_with_bias(seed):
    p = synth.cnn_init_params(seed)
    r = np.random.default_rng(seed + 100)
    for W, b in cnn.unpack(p):
        b[:] = 0.05 * r.standard_normal(b.shape)
    return p


def fields(shape, B, seed, dtype=np.float32):
    u = np.stack([np.random.default_rng(seed + i).standard_normal(shape) for i in range(B)])
    u = np.stack([oracle.filter(x, 2) for x in u])      # smooth-ish truth
    ub = np.stack([oracle.filter(x, 2) for x in u])
    return ub.astype(dtype).astype(np.float64), u.astype(dtype).astype(np.float64)


@pytest.mark.parametrize("shape", [(40, 72), (1, 1), (3, 5), (64, 64), (33, 100)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("smooth", [1, 2, 3])
def test_forward_matches_reference(shape, dtype, smooth):
    p = params_with_bias(1)
    ub, _ = fields(shape, 2, 10)
    ws = gdecon.WarmStart(p, smooth=smooth, band=None)
    u0 = ws.forward(to_dev(ub, dtype))
    torch.cuda.synchronize()
    got = u0.double().cpu().numpy()
    ref = cnn.forward(p, ub, emulate_bf16=True, smooth=smooth)
    s = ref["s"][:, None, None]
    y_got, y_ref = (got - ub) / s, ref["y"]
    assert rel_l2(y_got, y_ref) <= 3e-3, rel_l2(y_got, y_ref)
    exact = cnn.forward(p, ub, smooth=smooth)["y"]
    assert rel_l2(y_got, exact) <= 2e-2
    # deterministic
    u1 = ws.forward(to_dev(ub, dtype))
    torch.cuda.synchronize()
    assert torch.equal(u0, u1)


@pytest.mark.parametrize("smooth", [1, 2])
def test_gradients_loss_and_adam_match_reference(smooth):
    p = params_with_bias(2)
    ub, u = fields((48, 80), 3, 20)
    ws = gdecon.WarmStart(p, lr=1e-3, smooth=smooth)
    loss = ws.train_step(to_dev(ub, torch.float32), to_dev(u, torch.float32))
    torch.cuda.synchronize()
    g_gpu = ws.grad.double().cpu().numpy()
    l_ref, g_ref = cnn.loss_and_grad(p, ub, u, emulate_bf16=True, smooth=smooth)
    assert abs(loss.item() - l_ref) <= 3e-3 * l_ref
    off = 0
    for li, (W, b) in enumerate(cnn.unpack(p)):
        n = W.size + b.size
        e = rel_l2(g_gpu[off:off + n], g_ref[off:off + n])
        assert e <= 2e-2, (li, e)
        off += n
    # the Adam update is applied to the GPU's own gradient
    p32 = p.astype(np.float32).astype(np.float64)
    want, _, _ = cnn.adam_step(p32, np.zeros_like(p32), np.zeros_like(p32), g_gpu, 1, lr=1e-3)
    got = ws.params.double().cpu().numpy()
    np.testing.assert_allclose(got, want, rtol=1e-5, atol=1e-7)
    assert int(ws.step.item()) == 1
    # second step: bias corrections use step 2, moments carried over
    m = 0.1 * g_gpu
    v = 0.001 * g_gpu * g_gpu
    ws.train_step(to_dev(ub, torch.float32), to_dev(u, torch.float32))
    torch.cuda.synchronize()
    g2 = ws.grad.double().cpu().numpy()
    want2, _, _ = cnn.adam_step(got, m, v, g2, 2, lr=1e-3)
    np.testing.assert_allclose(ws.params.double().cpu().numpy(), want2, rtol=1e-5, atol=1e-7)
    assert int(ws.step.item()) == 2


def test_train_step_deterministic():
    p = params_with_bias(3)
    ub, u = fields((32, 64), 2, 30)
    a, b = gdecon.WarmStart(p), gdecon.WarmStart(p)
    for _ in range(3):
        la = a.train_step(to_dev(ub, torch.float32), to_dev(u, torch.float32)).clone()
        lb = b.train_step(to_dev(ub, torch.float32), to_dev(u, torch.float32)).clone()
    torch.cuda.synchronize()
    assert torch.equal(a.params, b.params) and torch.equal(la, lb)


def test_training_lowers_loss_and_warm_start_solves():
    """Empirical: a short training run on k^-3 crops lowers the loss; the
    trained network's u0 then starts BiCGSTAB, which still converges with a
    true residual within the stopping tolerance."""
    crops = synth.training_pairs(16, n=256, crop=64)
    u = torch.from_numpy(np.stack(crops)).cuda()
    ub = gdecon.filter_apply(u, ndim=2)
    ws = gdecon.WarmStart(synth.cnn_init_params(0), lr=2e-3)
    first = ws.train_step(ub, u).item()
    for _ in range(150):
        ws.train_step(ub, u)
    last = ws.train_step(ub, u).item()
    assert last < 0.7 * first, (first, last)
    test = torch.from_numpy(synth.field_2d(128, synth.spectrum_kraichnan, 4.0, 32.0, synth.rng_for(5, 99),
                                           np.float32)).cuda()[None]
    tub = gdecon.filter_apply(test, ndim=2)
    u0 = ws.forward(tub)
    uw, infos_w, _ = gdecon.deconvolve("bicgstab", tub, 100, tol=1e-6, init="warm", u0=u0)
    _, infos_b, _ = gdecon.deconvolve("bicgstab", tub, 100, tol=1e-6)
    print("iterations: warm start", infos_w[0]["iters"], "ubar start", infos_b[0]["iters"])
    assert infos_w[0]["status_name"] == "CONVERGED"
    assert infos_w[0]["r_true"] <= 1e-6 * infos_w[0]["r_ref"]


def test_rejects_mismatched_dimensions():
    ws = gdecon.WarmStart(synth.cnn_init_params(0))
    g = gdecon.make_grid((4, 8, 8), 3, torch.float32)     # 3D fields for the 2D network
    lib = gdecon.load()
    assert lib.warmstart_workspace_bytes(ws.net, g, 0) == 0
    x = torch.zeros((4, 8, 8), device="cuda")
    assert lib.warmstart_forward(ws.net, g, x.data_ptr(), torch.zeros_like(x).data_ptr(), x.data_ptr(), 1 << 20,
                                 None) == -1
    assert "2D" in lib.gd_last_error().decode()
    assert lib.warmstart_param_count(gdecon.WarmStart(synth.cnn_init_params(0, ndim=3), ndim=3).net) == 112481


# ------------------------------------------------------------------ 3D network
def fields3(shape, B, seed):
    u = np.stack([oracle.filter(np.random.default_rng(seed + i).standard_normal(shape), 3) for i in range(B)])
    ub = np.stack([oracle.filter(x, 3) for x in u])
    return ub.astype(np.float32).astype(np.float64), u.astype(np.float32).astype(np.float64)


def params3_with_bias(seed):
    p = synth.cnn_init_params(seed, ndim=3)
    r = np.random.default_rng(seed + 200)
    for W, b in cnn.unpack(p, ndim=3):
        b[:] = 0.05 * r.standard_normal(b.shape)
    return p


@pytest.mark.parametrize("shape", [(6, 10, 40), (1, 3, 5), (3, 9, 33), (16, 16, 16)])
@pytest.mark.parametrize("smooth", [1, 2])
def test_forward_3d_matches_reference(shape, smooth):
    p = params3_with_bias(1)
    ub, _ = fields3(shape, 2, 60)
    ws = gdecon.WarmStart(p, ndim=3, smooth=smooth, band=None)
    u0 = ws.forward(to_dev(ub, torch.float32))
    torch.cuda.synchronize()
    got = u0.double().cpu().numpy()
    ref = cnn.forward(p, ub, emulate_bf16=True, ndim=3, smooth=smooth)
    s = ref["s"][:, None, None, None]
    y_got = (got - ub) / s
    assert rel_l2(y_got, ref["y"]) <= 3e-3, rel_l2(y_got, ref["y"])
    assert rel_l2(y_got, cnn.forward(p, ub, ndim=3, smooth=smooth)["y"]) <= 2e-2
    u1 = ws.forward(to_dev(ub, torch.float32))
    torch.cuda.synchronize()
    assert torch.equal(u0, u1)


def test_gradients_and_adam_3d_match_reference():
    p = params3_with_bias(2)
    ub, u = fields3((6, 12, 36), 2, 70)
    ws = gdecon.WarmStart(p, lr=1e-3, ndim=3)
    loss = ws.train_step(to_dev(ub, torch.float32), to_dev(u, torch.float32))
    torch.cuda.synchronize()
    g_gpu = ws.grad.double().cpu().numpy()
    l_ref, g_ref = cnn.loss_and_grad(p, ub, u, emulate_bf16=True, ndim=3)
    assert abs(loss.item() - l_ref) <= 3e-3 * l_ref
    off = 0
    for li, (W, b) in enumerate(cnn.unpack(p, ndim=3)):
        n = W.size + b.size
        e = rel_l2(g_gpu[off:off + n], g_ref[off:off + n])
        assert e <= 2e-2, (li, e)
        off += n
    p32 = p.astype(np.float32).astype(np.float64)
    want, _, _ = cnn.adam_step(p32, np.zeros_like(p32), np.zeros_like(p32), g_gpu, 1, lr=1e-3)
    np.testing.assert_allclose(ws.params.double().cpu().numpy(), want, rtol=1e-5, atol=1e-7)


def test_training_3d_lowers_loss_and_warm_start_solves():
    """Empirical: a short 3D training run lowers the loss, and the trained
    network's u0 starts a 3D BiCGSTAB solve that converges."""
    fields = synth.training_pairs_3d(4, n=32)
    u = torch.from_numpy(np.stack(fields)).cuda()
    ub = gdecon.filter_apply(u, ndim=3)
    ws = gdecon.WarmStart(synth.cnn_init_params(0, ndim=3), lr=2e-3, ndim=3)
    first = ws.train_step(ub, u).item()
    for _ in range(80):
        ws.train_step(ub, u)
    last = ws.train_step(ub, u).item()
    assert last < 0.7 * first, (first, last)
    test = torch.from_numpy(synth.training_pairs_3d(1, n=32, seed0=50)[0]).cuda()[None]
    tub = gdecon.filter_apply(test, ndim=3)
    u0 = ws.forward(tub)
    _, infos, _ = gdecon.deconvolve("bicgstab", tub, 100, tol=1e-6, ndim=3, init="given", u0=u0)
    assert infos[0]["status_name"] == "CONVERGED"
    assert infos[0]["r_true"] <= 1e-6 * infos[0]["r_ref"]


# ------------------------------------------------------- the start in a solve
def train(ws, ub, u, steps, batch, seed=0):
    """Adam on shuffled minibatches of the pairs; the rate drops 10x for the last third."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm, pos = torch.randperm(ub.shape[0], generator=g), 0
    lr = ws.net.lr
    for k in range(steps):
        if pos + batch > ub.shape[0]:
            perm, pos = torch.randperm(ub.shape[0], generator=g), 0
        idx = perm[pos:pos + batch].cuda()
        pos += batch
        ws.train_step(ub.index_select(0, idx), u.index_select(0, idx))
        if k == (2 * steps) // 3:
            ws.set_lr(lr / 10)
    torch.cuda.synchronize()


def test_trained_start_needs_fewer_passes_on_held_out_1024sq_fields():
    """Empirical gain of the learned start (parity unpinned: a property of
    the trained network, not of a formula).  A network trained on the GPU on
    256 seeded k^-3 fields of 256^2 (4 <= k <= n/4) starts BiCGSTAB on four
    held-out 1024^2 fields (4 <= k <= 256) after the band projection.  Every
    solve must converge with its true residual within the tolerance, reach
    the ubar start's solution, and take fewer passes on average than from
    ubar (5 here) -- or from zero (6)."""
    U = torch.from_numpy(synth.training_fields(256, n=256, seed0=7000)).cuda()
    UB = gdecon.filter_apply(U, ndim=2)
    ws = gdecon.WarmStart(synth.cnn_init_params(0), lr=1e-3)
    train(ws, UB, U, 900, 8)
    ev = np.stack([synth.field_2d(1024, synth.spectrum_kraichnan, 4.0, 256.0, synth.rng_for(5, 90000 + i), np.float32)
                   for i in range(4)])
    ub = gdecon.filter_apply(torch.from_numpy(ev).cuda(), ndim=2)
    u_ubar, inf_ubar, _ = gdecon.deconvolve("bicgstab", ub, 100, tol=1e-6)
    _, inf_zero, _ = gdecon.deconvolve("bicgstab", ub, 100, tol=1e-6, init="zero")
    u0 = ws.forward(ub)
    u_cnn, inf_cnn, _ = gdecon.deconvolve("bicgstab", ub, 100, tol=1e-6, init="warm", u0=u0)
    p_ubar = [i["iters"] for i in inf_ubar]
    p_zero = [i["iters"] for i in inf_zero]
    p_cnn = [i["iters"] for i in inf_cnn]
    print("passes: ubar", p_ubar, "zero", p_zero, "cnn", p_cnn, "starts", [i["start"] for i in inf_cnn],
          "r0/r_ref", [round(i["r0"] / i["r_ref"], 4) for i in inf_cnn])
    for i in inf_cnn:
        assert i["status_name"] == "CONVERGED" and i["start"] == "given"
        assert i["r_true"] <= 1e-6 * i["r_ref"]
    assert np.mean(p_cnn) < np.mean(p_ubar) and np.mean(p_cnn) < np.mean(p_zero)
    for b in range(4):
        assert rel_l2(u_cnn[b].double().cpu().numpy(), u_ubar[b].double().cpu().numpy()) <= 2e-5


def test_a_bad_network_start_falls_back_to_the_plain_solve():
    """An untrained network whose output is scaled up 1000x, and a start
    holding a NaN: the library judges both worse than ubar (their residual
    is not below ||ubar - G ubar||) and runs the plain ubar-start solve
    instead, bit for bit."""
    p = synth.cnn_init_params(3)
    W6, _ = cnn.unpack(p)[-1]
    W6 *= 1e3
    ws = gdecon.WarmStart(p)
    ev = np.stack([synth.field_2d(256, synth.spectrum_kraichnan, 4.0, 64.0, synth.rng_for(5, 91000 + i), np.float32)
                   for i in range(3)])
    ub = gdecon.filter_apply(torch.from_numpy(ev).cuda(), ndim=2)
    u0 = ws.forward(ub)
    u0[2, 5, 7] = float("nan")
    u_plain, inf_plain, _ = gdecon.deconvolve("bicgstab", ub, 100, tol=1e-6)
    u_warm, inf_warm, _ = gdecon.deconvolve("bicgstab", ub, 100, tol=1e-6, init="warm", u0=u0)
    assert [i["start"] for i in inf_warm] == ["ubar"] * 3
    assert torch.equal(u_plain, u_warm)
    for a, b in zip(inf_plain, inf_warm):
        assert {k: v for k, v in a.items() if k != "start"} == {k: v for k, v in b.items() if k != "start"}


def test_fused_forward_spans_strips_and_row_chunks():
    """The 2D inference kernel cuts a field into strips of 54 columns and
    chunks of 256 rows: a field of 300 x 130 spans three strips (the last
    ragged) and two chunks (the second ragged); it must match the reference
    like any other."""
    p = params_with_bias(4)
    ub, _ = fields((300, 130), 1, 80)
    ws = gdecon.WarmStart(p, band=None)
    got = ws.forward(to_dev(ub, torch.float32)).double().cpu().numpy()
    ref = cnn.forward(p, ub, emulate_bf16=True)
    y_got = (got - ub) / ref["s"][:, None, None]
    assert rel_l2(y_got, ref["y"]) <= 3e-3, rel_l2(y_got, ref["y"])
