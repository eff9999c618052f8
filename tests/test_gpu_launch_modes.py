"""Every launch configuration the autotuner can choose gives the same answer.

Each case pins one configuration (gd_tune_set / gd_tune_set_batch): tile
granularity, short tail tiles, interleaved pools, per-wave claims,
workgroups per CU (one, two, or as many as fit), and in 3D a fixed number
of long tiles per column (whatever the wave count).  It then
checks the solve against the CPU FP64 oracle: relative L2 <= 1e-10 in FP64
and equal pass counts.  Configurations only change which wave handles which
tile and how the partial sums are split, never what is computed.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import rel_l2, to_dev
from paper_1707_09177_amd import gdecon

pytestmark = pytest.mark.gpu

MODES = [dict(tiles_per_wave=tpw, tail_pct=tail, interleave=ilv, wave_claims=wc, blocks_per_cu=0 if ilv == wc else 2)
         for tpw in (1, 3) for tail in (0, 25) for ilv in (0, 1) for wc in (0, 1)]


@pytest.fixture(autouse=True)
def _forget_choices():
    yield
    gdecon.tune_reset()


def mode_id(m):
    return (f"tpw{m['tiles_per_wave']}-tail{m['tail_pct']}-ilv{m['interleave']}-wc{m['wave_claims']}"
            f"-bpc{m['blocks_per_cu']}")


@pytest.mark.parametrize("mode", MODES, ids=mode_id)
@pytest.mark.parametrize("solver,shape", [("bicgstab", (3, 96, 160)), ("cg", (2, 20, 24, 36)), ("vc", (130, 300))])
def test_uniform_modes_match_oracle(mode, solver, shape):
    nd = 3 if len(shape) == 4 else 2
    u = np.random.default_rng(len(shape) + 3).standard_normal(shape)
    ub = oracle.filter(u, nd)
    N = 4
    want, winfo, _ = oracle.solve(solver, ub, nd, N)
    ubt = to_dev(ub, torch.float64)
    out = torch.empty_like(ubt)
    gdecon.tune_set(solver, ubt, out, ndim=nd, **mode)
    d = gdecon.Deconvolver(ubt.shape, nd, ubt.dtype, solver)
    res = d.solve(ubt, N, 0.0, out=out)
    infos = res.info()
    got = out.cpu().numpy()
    for b, (gi, wi) in enumerate(zip(infos, winfo)):
        assert gi["iters"] == wi["iters"]
    assert rel_l2(got, want) <= 1e-10


@pytest.mark.parametrize("mode", MODES, ids=mode_id)
def test_batch_modes_match_oracle(mode):
    shapes = [(64, 64), (9, 7), (3, 5, 7), (40, 130), (17, 33, 9), (20, 24, 36)]
    ubs = [oracle.filter(np.random.default_rng(40 + i).standard_normal(sh), len(sh)) for i, sh in enumerate(shapes)]
    ubt = [to_dev(x, torch.float64) for x in ubs]
    outs = [torch.empty_like(x) for x in ubt]
    bd = gdecon.BatchDeconvolver(shapes, torch.float64, "bicgstab")
    bd.tune_set(ubt, outs, **mode)
    res = bd.solve(ubt, 5, 0.0, outs=outs)
    infos = res.info()
    for i, ub in enumerate(ubs):
        want, winfo, _ = oracle.solve("bicgstab", ub, ub.ndim, 5)
        assert infos[i]["iters"] == winfo[0]["iters"]
        assert rel_l2(outs[i].cpu().numpy(), want) <= 1e-10, (i, shapes[i])


@pytest.mark.parametrize("segments", [1, 2, 3, 5])
@pytest.mark.parametrize("rows", [0, 1, 2, 4])
@pytest.mark.parametrize("shape", [(2, 20, 24, 36), (3, 9, 8, 132), (1, 41, 13, 260)],
                         ids=lambda s: "x".join(map(str, s)))
def test_tiles_per_column_match_oracle(segments, rows, shape):
    """3D columns cut into a fixed number of long tiles (the last one
    ragged, or below the minimum tile length) with one or two workgroups
    per CU."""
    u = np.random.default_rng(segments + 7 * rows + sum(shape)).standard_normal(shape)
    ub = oracle.filter(u, 3)
    N = 4
    want, winfo, _ = oracle.solve("bicgstab", ub, 3, N)
    ubt = to_dev(ub, torch.float64)
    out = torch.empty_like(ubt)
    gdecon.tune_set("bicgstab", ubt, out, ndim=3, tiles_per_wave=1, rows=rows, tail_pct=0,
                    blocks_per_cu=1 + segments % 2, segments=segments)
    res = gdecon.Deconvolver(ubt.shape, 3, ubt.dtype, "bicgstab").solve(ubt, N, 0.0, out=out)
    nz = shape[1]
    assert gdecon.last_launch()["L"] == max(8, -(-nz // segments))
    for gi, wi in zip(res.info(), winfo):
        assert gi["iters"] == wi["iters"]
    assert rel_l2(out.cpu().numpy(), want) <= 1e-10
