"""Graph capture of the stream-ordered entry points added beside the solve:
the differential-filter solve (FFTs + persistent solve), the blocked Van
Cittert (its launch sequence, including the recomputation of a stopped
sweep), the closure stress, the PDF counts (cleared by a kernel) and the
energy spectrum.  Every replay, with unrelated eager work between replays,
must reproduce the eager result: bit for bit, except the spectrum, whose
per-workgroup shell sums are added by unordered LDS atomics (within 1e-12).
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
        assert torch.allclose(s2, e_spec, rtol=1e-12, atol=0), rep
