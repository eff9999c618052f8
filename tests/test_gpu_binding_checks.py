"""The Python binding refuses caller buffers that do not match what the
library writes (shape, dtype, device) before it launches anything: the C
entry points see bare pointers, so a short output would be overrun."""
import pytest
import torch

from gpu_helpers import DEV
from paper_1707_09177_amd import gdecon, synth

pytestmark = pytest.mark.gpu


def bad_out(x, which):
    if which == 0:                                     # one column short
        return torch.full(x.shape[:-1] + (x.shape[-1] - 1,), 7.0, dtype=x.dtype, device=DEV)
    if which == 1:                                     # wrong dtype
        return torch.full(x.shape, 7.0, dtype=torch.float64, device=DEV)
    return torch.full(x.shape, 7.0, dtype=x.dtype)     # host memory


@pytest.mark.parametrize("which", range(3))
def test_every_out_argument_is_checked(which):
    x = torch.randn(2, 16, 32, device=DEV)
    out = bad_out(x, which)
    keep = out.clone()
    calls = [
        lambda: gdecon.filter_apply(x, 2, out=out),
        lambda: gdecon.germano_filter(x, 0.1, 2, out=out),
        lambda: gdecon.Deconvolver(x.shape, 2, x.dtype, "cg").solve(x, 3, out=out),
        lambda: gdecon.autotune("cg", x, 2, out=out),
        lambda: gdecon.GermanoDeconvolver(x.shape, 2, x.dtype, "cg", 0.1).autotune(x, out=out),
        lambda: gdecon.WarmStart(synth.cnn_init_params(0)).forward(x, out=out),
    ]
    for i, c in enumerate(calls):
        with pytest.raises(ValueError):
            c()
    torch.cuda.synchronize()
    assert torch.equal(out, keep)


def test_inputs_on_another_device_are_refused():
    x = torch.randn(2, 16, 32, device=DEV)
    d = gdecon.Deconvolver(x.shape, 2, x.dtype, "bicgstab")
    with pytest.raises(ValueError):
        d.solve(x.cpu(), 3)
    with pytest.raises(ValueError):
        d.solve(x, 3, history=torch.zeros(2 * 4, dtype=torch.float64))
    v = torch.randn(3, 8, 8, 16, device=DEV)
    with pytest.raises(ValueError):
        gdecon.closure_stress(v, v.cpu(), 3)
    with pytest.raises(ValueError):                    # 3 pairs where 3D needs 6
        gdecon.closure_stress(v, v, 3, out=torch.empty(3, 8, 8, 16, device=DEV))
    b = gdecon.BatchDeconvolver([(16, 32), (8, 8, 8)], torch.float32, "cg")
    with pytest.raises(ValueError):
        b.solve([torch.randn(16, 32, device=DEV), torch.randn(8, 8, 8)], 3)
    ubs = [torch.randn(16, 32, device=DEV), torch.randn(8, 8, 8, device=DEV)]
    with pytest.raises(ValueError):
        b.solve(ubs, 3, histories=[torch.zeros(4, dtype=torch.float64, device=DEV)])
    with pytest.raises(ValueError):
        b.solve(ubs, 3, histories=[torch.zeros(4, dtype=torch.float64, device=DEV), torch.zeros(4, dtype=torch.float64)])


def test_warm_start_keeps_one_workspace_per_3d_size():
    """Fields that differ only in n_z get workspaces of their own, and the
    results do not depend on what ran before."""
    p = synth.cnn_init_params(0, ndim=3)
    ws = gdecon.WarmStart(p, ndim=3, band=None)   # n_z = 12: no band projection (power-of-two sizes only)
    ubs = {nz: torch.randn(nz, 8, 16, device=DEV, generator=torch.Generator(DEV).manual_seed(nz)) for nz in (4, 12)}
    got = {nz: ws.forward(ubs[nz]).clone() for nz in (4, 12, 4)}
    torch.cuda.synchronize()
    assert len(ws._work) == 2
    fresh = gdecon.WarmStart(p, ndim=3, band=None).forward(ubs[12])
    torch.cuda.synchronize()
    assert torch.equal(got[12], fresh)
