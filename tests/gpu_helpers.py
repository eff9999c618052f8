"""Helpers shared by the GPU tests: run the HIP library, compare with the oracle."""
import numpy as np
import torch

import oracle
from paper_1707_09177_amd import gdecon

DEV = "cuda:0"


def to_dev(a: np.ndarray, dtype) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def gpu_solve(solver, ubar_np, ndim, max_iter, tol=0.0, dtype=torch.float64, init="ubar", u0=None,
              norm_ref="r0ubar", history=True):
    ub = to_dev(ubar_np, dtype)
    u0t = to_dev(u0, dtype) if u0 is not None else None
    u, infos, hist = gdecon.deconvolve(solver, ub, max_iter, tol=tol, ndim=ndim, init=init, u0=u0t,
                                       norm_ref=norm_ref, history=history)
    return (u.double().cpu().numpy(), infos,
            hist.cpu().numpy() if hist is not None else None)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rel_l2_per_field(a, b, ndim):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    fa = a.reshape(-1, int(np.prod(a.shape[-ndim:])))
    fb = b.reshape(-1, int(np.prod(b.shape[-ndim:])))
    return [rel_l2(x, y) for x, y in zip(fa, fb)]


def filtered_input(u_np, ndim, dtype):
    """ubar = G u by the oracle (FP64), rounded to the storage type once."""
    ub = oracle.filter(u_np, ndim)
    if dtype == torch.float32:
        ub = ub.astype(np.float32).astype(np.float64)
    return ub
