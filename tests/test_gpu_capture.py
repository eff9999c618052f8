"""Graph capture of the stream-ordered entry points added beside the solve:
the differential-filter solve (FFTs + persistent solve), the blocked Van
Cittert (its launch sequence, including the recomputation of a stopped
sweep), the closure stress, the PDF counts (cleared by a kernel), the
energy spectrum, and the warm start's forward pass and Adam step.  Every replay, with unrelated eager work between replays,
must reproduce the eager result bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import DEV, to_dev
from paper_1707_09177_amd import gdecon

pytestmark = pytest.mark.gpu


def replays(g, outs, fill=float("nan")):
    for rep in range(3):
        for o in outs:
            o.fill_(fill)
        junk = torch.randn(1 << 20, device=DEV)          # unrelated eager work between replays
        (junk * 2).sum().item()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        yield rep


def test_germano_solve_capture():
    ub = to_dev(oracle.germano_filter(np.random.default_rng(1).standard_normal((3, 64, 128)), 2, 0.1),
                torch.float32)
    d = gdecon.GermanoDeconvolver(ub.shape, 2, ub.dtype, "bicgstab", 0.1)
    out = torch.empty_like(ub)
    res = d.solve(ub, 100, 1e-4, out=out)
    torch.cuda.synchronize()
    eager, eager_info = out.clone(), res.info()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        d.solve(ub, 100, 1e-4, out=out)
    for rep in replays(g, [out]):
        assert torch.equal(out, eager), rep
        assert res.info() == eager_info, rep


def test_blocked_vancittert_capture():
    """Fields that stop at different passes, one inside a sweep."""
    u = np.random.default_rng(2).standard_normal((3, 96, 160))
    u[1] = oracle.filter(u[1], 2)
    ub = to_dev(oracle.filter(u, 2), torch.float64)
    d = gdecon.BlockedVanCittert(ub.shape, 2, ub.dtype)
    out = torch.empty_like(ub)
    res = d.solve(ub, 100, 3e-3, out=out)
    torch.cuda.synchronize()
    eager, eager_info = out.clone(), res.info()
    assert len({i["iters"] for i in eager_info}) > 1
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        d.solve(ub, 100, 3e-3, out=out)
    for rep in replays(g, [out]):
        assert torch.equal(out, eager), rep
        assert res.info() == eager_info, rep


def test_closure_pdf_spectrum_capture():
    rng = np.random.default_rng(3)
    vb = to_dev(rng.standard_normal((2, 3, 16, 24, 32)), torch.float32)
    vs = to_dev(rng.standard_normal((2, 3, 16, 24, 32)), torch.float32)
    f = to_dev(rng.standard_normal((4, 128, 256)), torch.float32)
    tau = gdecon.closure_stress(vb, vs, 3)
    counts = gdecon.pdf_counts(f, -3.0, 3.0, 100)
    spec = gdecon.energy_spectrum(f, 2, -2.0)
    torch.cuda.synchronize()
    e_tau, e_counts, e_spec = tau.clone(), counts.clone(), spec.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gdecon.closure_stress(vb, vs, 3, out=tau)
        c2 = gdecon.pdf_counts(f, -3.0, 3.0, 100)
        s2 = gdecon.energy_spectrum(f, 2, -2.0)
    for rep in range(3):
        tau.fill_(float("nan"))
        c2.fill_(-7)                                       # the captured clear must reset them
        s2.fill_(float("nan"))
        (torch.randn(1 << 20, device=DEV) * 2).sum().item()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(tau, e_tau), rep
        assert torch.equal(c2, e_counts), rep
        assert torch.equal(s2, e_spec), rep


def test_warm_start_capture():
    """The warm start's forward pass and one Adam step captured together: every
    replay matches the same calls made eagerly on a twin network (same
    parameters and step count), bit for bit: outputs, loss and parameters."""
    from paper_1707_09177_amd import synth
    p = synth.cnn_init_params(0)
    g0 = torch.Generator(DEV).manual_seed(11)
    x = torch.randn(2, 64, 128, device=DEV, generator=g0)   # power-of-two sizes: the band projection is captured too
    u = torch.randn(2, 64, 128, device=DEV, generator=g0)
    eager, cap = gdecon.WarmStart(p, lr=1e-3), gdecon.WarmStart(p, lr=1e-3)
    out_e, out_c = torch.empty_like(x), torch.empty_like(x)
    for ws, out in ((eager, out_e), (cap, out_c)):     # workspaces are allocated here, outside the capture
        ws.forward(x, out=out)
        ws.train_step(x, u)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cap.forward(x, out=out_c)
        cap.train_step(x, u)
    for rep in range(3):
        out_c.fill_(float("nan"))
        (torch.randn(1 << 20, device=DEV) * 2).sum().item()
        g.replay()
        eager.forward(x, out=out_e)
        eager.train_step(x, u)
        torch.cuda.synchronize()
        assert torch.equal(out_c, out_e), rep
        assert torch.equal(cap.loss, eager.loss), rep
        assert torch.equal(cap.params, eager.params), rep
        assert torch.equal(cap.step, eager.step), rep
