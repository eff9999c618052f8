"""deconvolve_noalloc: the solve with the library's fixed device workspace,
called through the C ABI, against the solver's own entry point with a
caller-owned workspace.  Two calls in a row on one GPU share the fixed
array, the second on a smaller batch: each must equal the workspace call bit
for bit (the same kernels, launch shape and reduction order), u and info
alike.  Sizes whose workspace exceeds the array are refused before any
launch."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import DEV, to_dev
from paper_1707_09177_amd import gdecon

pytestmark = pytest.mark.gpu


def reference(solver, ub, nd, max_iter, tol):
    d = gdecon.Deconvolver(ub.shape, nd, ub.dtype, solver)
    out = torch.empty_like(ub)
    res = d.solve(ub, max_iter, tol, out=out)
    torch.cuda.synchronize()
    return out.clone(), res.info()


def noalloc(solver, ub, nd, max_iter, tol):
    info = torch.zeros(int(np.prod(ub.shape[:-nd]) if ub.dim() > nd else 1) * gdecon.INFO_BYTES,
                       dtype=torch.uint8, device=ub.device)
    u = gdecon.deconvolve_noalloc(solver, ub, max_iter, info, tol=tol, ndim=nd)
    torch.cuda.synchronize()
    return u, gdecon.decode_info(info.cpu().numpy())


@pytest.mark.parametrize("solver,dtype", [("bicgstab", torch.float32), ("cg", torch.float64), ("vc", torch.float32)])
def test_noalloc_matches_the_workspace_call_twice(solver, dtype):
    rng = np.random.default_rng(17)
    calls = [((3, 256, 320), 2), ((2, 40, 56, 48), 3), ((1, 96, 72), 2)]   # later calls smaller than the first
    for shape, nd in calls:
        ub = to_dev(oracle.filter(rng.standard_normal(shape), nd), dtype)
        got, ginfo = noalloc(solver, ub, nd, 60, 1e-6)
        want, winfo = reference(solver, ub, nd, 60, 1e-6)
        assert torch.equal(got, want), (shape, solver)
        assert ginfo == winfo, (shape, ginfo, winfo)


def test_noalloc_refuses_oversized_solves():
    lib = gdecon.load()
    cap = int(lib.deconvolve_noalloc_max_bytes())
    assert cap == 32 << 20
    ub = torch.zeros((4, 1024, 1024), dtype=torch.float32, device=DEV)   # BiCGSTAB needs ~112 MiB here
    info = torch.zeros(4 * gdecon.INFO_BYTES, dtype=torch.uint8, device=DEV)
    with pytest.raises(gdecon.GdError) as e:
        gdecon.deconvolve_noalloc("bicgstab", ub, 5, info, ndim=2)
    assert e.value.code == -2
