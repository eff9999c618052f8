"""3D tile shapes pinned one by one (rows per tile 1, 2 and 4) against the
CPU FP64 oracle.

Rows = 4 with 16-byte lanes is the two-lane-row tile: two half-waves of 32
lanes stacked in y, two rows per lane, the rows between the halves passed
across lanes.  The shapes are ragged on purpose: row counts that are not a
multiple of the tile's rows, x extents that leave a partial half-wave span
(132, 260) or a one-lane span (4), and extents below one tile.  FP64: relative
L2 <= 1e-10 at equal pass counts; FP32: <= 1e-5 against the oracle run on the
FP32-rounded input.  The zero start with the ||ubar|| reference norm also
runs the pointwise sweeps over the same tiles.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import rel_l2, to_dev
from paper_1707_09177_amd import gdecon

pytestmark = pytest.mark.gpu

SHAPES = [(6, 5, 132), (9, 8, 256), (4, 13, 8), (7, 4, 260), (5, 6, 384), (3, 9, 4), (2, 7, 136)]


@pytest.fixture(autouse=True)
def _forget_choices():
    yield
    gdecon.tune_reset()


def _ubar(shape, seed, dtype):
    u = np.random.default_rng(seed).standard_normal(shape)
    ub = oracle.filter(u, 3)
    if dtype == torch.float32:
        ub = ub.astype(np.float32).astype(np.float64)
    return ub


@pytest.mark.parametrize("rows", [1, 2, 4])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("solver", ["bicgstab", "cg", "vc"])
def test_rows_fp64_match_oracle(rows, shape, solver):
    ub = _ubar(shape, 7 + sum(shape), torch.float64)
    N = 4
    want, winfo, _ = oracle.solve(solver, ub, 3, N)
    ubt = to_dev(ub, torch.float64)
    out = torch.empty_like(ubt)
    gdecon.tune_set(solver, ubt, out, ndim=3, rows=rows)
    d = gdecon.Deconvolver(ubt.shape, 3, ubt.dtype, solver)
    res = d.solve(ubt, N, 0.0, out=out)
    assert gdecon.last_launch()["R"] == rows
    info = res.info()[0]
    assert info["iters"] == winfo[0]["iters"]
    assert rel_l2(out.cpu().numpy(), want) <= 1e-10, (shape, rows)


@pytest.mark.parametrize("rows", [2, 4])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_rows_fp32_zero_start_match_oracle(rows, shape):
    ub = _ubar(shape, 11 + sum(shape), torch.float32)
    N = 3
    want, winfo, _ = oracle.solve("bicgstab", ub, 3, N, init="zero", norm_ref="ubar")
    ubt = to_dev(ub, torch.float32)
    out = torch.empty_like(ubt)
    gdecon.tune_set("bicgstab", ubt, out, ndim=3, rows=rows)
    d = gdecon.Deconvolver(ubt.shape, 3, ubt.dtype, "bicgstab")
    res = d.solve(ubt, N, 0.0, init="zero", norm_ref="ubar", out=out)
    assert gdecon.last_launch()["R"] == rows
    assert res.info()[0]["iters"] == winfo[0]["iters"]
    assert rel_l2(out.cpu().numpy().astype(np.float64), want) <= 1e-5, (shape, rows)


def test_row_shapes_agree():
    """The three tile shapes give the same FP64 solve to rounding."""
    ub = _ubar((5, 11, 132), 99, torch.float64)
    ubt = to_dev(ub, torch.float64)
    outs = []
    for rows in (1, 2, 4):
        out = torch.empty_like(ubt)
        gdecon.tune_set("bicgstab", ubt, out, ndim=3, rows=rows)
        gdecon.Deconvolver(ubt.shape, 3, ubt.dtype, "bicgstab").solve(ubt, 5, 0.0, out=out)
        outs.append(out.cpu().numpy())
        gdecon.tune_reset()
    for o in outs[1:]:
        assert rel_l2(o, outs[0]) <= 1e-12
