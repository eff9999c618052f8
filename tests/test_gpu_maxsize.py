"""Fields of 2^31 points (8 GiB per FP32 vector), past any 32-bit index.

G is shift-invariant on the periodic grid, so a field made of a base field
repeated k times along each axis is deconvolved into the same repetition of
the base field's solution.  Its inner products carry the weight h^d with
h = 2 pi / n, so they equal the base field's: every scalar of Algorithm 4
(alpha, beta, omega, rho) and every norm agrees up to summation order.  The
oracle solves the base field; sampled copies of it in the GPU's solution of
the large field (corners, centre, last) must match within the FP32
tolerance of the small-size tests (1e-5 relative L2), and the reported norms
must be the base field's.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import DEV, filtered_input, rel_l2, to_dev
from paper_1707_09177_amd import gdecon, synth

pytestmark = pytest.mark.gpu

F32_TOL = 1e-5
PASSES = 5

# ndim: (base shape (slow axis first), repetitions per axis); 2^31 points each
CASES = {2: ((1024, 2048), (32, 32)), 3: ((128, 128, 128), (16, 8, 8))}


@pytest.mark.timeout(300)
@pytest.mark.parametrize("nd", [2, 3])
def test_two_to_the_31_points(nd):
    base, reps = CASES[nd]
    big = tuple(b * r for b, r in zip(base, reps))
    assert int(np.prod(big)) == 1 << 31
    u = synth.config_fields(nd, n=base[-1], count=1)[0] if nd == 3 else synth.config_fields(2, n=2048, count=1)[0][:1024]
    ub = filtered_input(u, nd, torch.float32)
    want, winf, _ = oracle.solve("bicgstab", ub, nd, PASSES)
    dub = to_dev(ub, torch.float32).repeat(*reps).contiguous()
    assert tuple(dub.shape) == big
    d = gdecon.Deconvolver(big, nd, torch.float32, "bicgstab")
    out = torch.empty_like(dub)
    info = d.solve(dub, PASSES, out=out).info()[0]
    del dub
    assert info["iters"] == PASSES and info["status_name"] == winf[0]["status_name"]
    for k in ("r_ref", "r0", "r_final"):
        assert abs(info[k] - winf[0][k]) <= F32_TOL * winf[0]["r_ref"], (k, info[k], winf[0][k])
    last = tuple(r - 1 for r in reps)
    for t in [(0,) * nd, last, tuple(r // 2 for r in reps), (0,) * (nd - 1) + (reps[-1] - 1,)]:
        sl = tuple(slice(i * b, (i + 1) * b) for i, b in zip(t, base))
        got = out[sl].double().cpu().numpy()
        e = rel_l2(got, want)
        print(nd, "tile", t, "rel L2 vs oracle %.2e" % e)
        assert e <= F32_TOL, (t, e)
