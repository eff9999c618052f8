"""The solve's control paths beyond Algorithms 1-4 themselves.

Guarded warm start (init='warm'): per field, the solve starts from the
caller's guess only where its residual ||ubar - G u0|| is finite and below
that of the paper's start u0 = ubar, and from ubar otherwise; the oracle's
``warm_choice`` states the same rule, and both sides then run the algorithm
from the start they chose.

Exit on the true residual: with tol > 0 a field stops CONVERGED only once
||ubar - G u||, evaluated in FP64 arithmetic, meets tol * r_ref.  Where the
recursive residual met tol but the true one does not (the FP32 rounding
floor), r is replaced by the true residual and CG / BiCGSTAB restart from
the current iterate; after max_replace replacements the field stops
GD_STAGNATED.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import filtered_input, rel_l2, rel_l2_per_field, to_dev
from paper_1707_09177_amd import gdecon, synth

pytestmark = pytest.mark.gpu

F64_TOL = 1e-10


def kraichnan(n, count, seed):
    """count k^-3 vorticity fields on 4 <= k <= n/4 (the benchmark's band
    scaled to n: G_hat >= 1/2 on it), FP64 copies of the FP32 fields."""
    return np.stack([synth.field_2d(n, synth.spectrum_kraichnan, 4.0, n / 4.0, synth.rng_for(2, seed + i),
                                    np.float32) for i in range(count)]).astype(np.float64)


def guesses(ub, nd, seed):
    """Per field of ub: a good guess (ubar plus most of the missing
    correction), a bad one (noise far above the residual), and a non-finite
    one."""
    rng = np.random.default_rng(seed)
    good = ub + 0.9 * (ub - oracle.filter(ub, nd))
    bad = ub + rng.standard_normal(ub.shape)
    nan = ub.copy()
    nan.reshape(-1)[7] = np.nan
    return good, bad, nan


@pytest.mark.parametrize("solver", ["bicgstab", "cg", "vc", "sd"])
@pytest.mark.parametrize("nd,shape", [(2, (48, 72)), (3, (12, 10, 20))])
def test_warm_start_choice_and_parity(solver, nd, shape):
    u = np.random.default_rng(5).standard_normal((3,) + shape)
    ub = oracle.filter(u, nd)
    good, bad, nan = guesses(ub[0], nd, 6)
    u0 = np.stack([good, bad, nan])
    want_start = oracle.warm_choice(ub, u0, nd)
    assert want_start == ["given", "ubar", "ubar"]
    for N in (1, 6):
        want, winfo, _ = oracle.solve(solver, ub, nd, N, init="warm", u0=u0)
        got, ginfo, _ = gdecon.deconvolve(solver, to_dev(ub, torch.float64), N, ndim=nd, init="warm",
                                          u0=to_dev(u0, torch.float64))
        got = got.cpu().numpy()
        for b in range(3):
            assert ginfo[b]["start"] == winfo[b]["start"] == want_start[b], (b, ginfo[b])
            assert ginfo[b]["iters"] == winfo[b]["iters"] and ginfo[b]["status"] == winfo[b]["status"]
            assert rel_l2(got[b], want[b]) <= F64_TOL, (b, rel_l2(got[b], want[b]))
            for key in ("r_ref", "r0", "r_true"):
                assert abs(ginfo[b][key] - winfo[b][key]) <= 1e-10 * winfo[b]["r_ref"], key
    # a rejected guess gives exactly the ubar start's solve
    u_ubar, info_ubar, _ = gdecon.deconvolve(solver, to_dev(ub, torch.float64), 6, ndim=nd)
    u_warm, info_warm, _ = gdecon.deconvolve(solver, to_dev(ub, torch.float64), 6, ndim=nd, init="warm",
                                             u0=to_dev(u0, torch.float64))
    assert torch.equal(u_ubar[1:], u_warm[1:])
    for a, b in zip(info_ubar[1:], info_warm[1:]):
        assert b["start"] == "ubar" and {k: v for k, v in a.items() if k != "start"} == \
            {k: v for k, v in b.items() if k != "start"}


def test_warm_start_reference_norms():
    """With norm_ref='ubar' the warm start still judges the guess against
    ||ubar - G ubar|| while the relative residual uses ||ubar||."""
    u = np.random.default_rng(7).standard_normal((2, 40, 56))
    ub = oracle.filter(u, 2)
    good, bad, _ = guesses(ub[0], 2, 8)
    u0 = np.stack([good, bad])
    # 8 passes: BiCGSTAB on white noise turns chaotic (rounding-level
    # differences grow) well beyond that
    want, winfo, _ = oracle.solve("bicgstab", ub, 2, 8, init="warm", u0=u0, norm_ref="ubar")
    got, ginfo, _ = gdecon.deconvolve("bicgstab", to_dev(ub, torch.float64), 8, ndim=2, init="warm",
                                      u0=to_dev(u0, torch.float64), norm_ref="ubar")
    assert [i["start"] for i in ginfo] == [i["start"] for i in winfo] == ["given", "ubar"]
    for b in range(2):
        assert ginfo[b]["iters"] == winfo[b]["iters"] and ginfo[b]["status_name"] == winfo[b]["status_name"]
        assert abs(ginfo[b]["r_ref"] - np.sqrt(oracle.dot(ub[b], ub[b], oracle.spacing_weight(ub.shape, 2)))) \
            <= 1e-12 * ginfo[b]["r_ref"]
        assert rel_l2(got[b].cpu().numpy(), want[b]) <= F64_TOL


def test_warm_start_uneven_batch_and_differential_filter():
    rng = np.random.default_rng(9)
    shapes = [(40, 64), (9, 7), (6, 10, 12), (32, 32)]
    ubs = [oracle.filter(rng.standard_normal(sh), len(sh)) for sh in shapes]
    u0s = [guesses(ub, ub.ndim, 10 + i)[i % 2] for i, ub in enumerate(ubs)]   # good, bad, good, bad
    us, infos, _ = gdecon.deconvolve_batch("cg", [to_dev(x, torch.float64) for x in ubs], 8, init="warm",
                                           u0s=[to_dev(x, torch.float64) for x in u0s])
    for i, ub in enumerate(ubs):
        want, winfo, _ = oracle.solve("cg", ub, ub.ndim, 8, init="warm", u0=u0s[i])
        assert infos[i]["start"] == winfo[0]["start"] == ("given" if i % 2 == 0 else "ubar")
        assert rel_l2(us[i].cpu().numpy(), want) <= F64_TOL
    # the paper's differential filter: the guess is judged on the Fourier coefficients
    ug = rng.standard_normal((2, 32, 64))
    ubg = oracle.germano_filter(ug, 2, 0.2)
    u0g = np.stack([ug[0] * 0.9 + 0.1 * ubg[0], ubg[1] + rng.standard_normal((32, 64))])
    got, ginfo, _ = gdecon.deconvolve_germano("bicgstab", to_dev(ubg, torch.float64), 6, 0.2, init="warm",
                                              u0=to_dev(u0g, torch.float64))
    want, winfo, _ = oracle.solve("bicgstab", ubg, 2, 6, init="warm", u0=u0g, gamma=0.2)
    assert [i["start"] for i in ginfo] == [i["start"] for i in winfo] == ["given", "ubar"]
    assert max(rel_l2_per_field(got.cpu().numpy(), want, 2)) <= F64_TOL


@pytest.mark.parametrize("solver", ["bicgstab", "cg", "vc", "sd"])
def test_converged_means_true_residual_within_tol(solver):
    """FP32 solves of k^-3 fields: whenever a field stops CONVERGED, the
    true residual it reports, and the one the oracle recomputes in FP64 from
    its u, meet tol."""
    u = synth.config_fields(2, n=256, count=6, dtype=np.float32).astype(np.float64)
    ub = filtered_input(u, 2, torch.float32)
    for tol in (1e-6, 6e-7):
        got, infos, _ = gdecon.deconvolve(solver, to_dev(ub, torch.float32), 400, tol=tol, ndim=2)
        got = got.double().cpu().numpy()
        for b, inf in enumerate(infos):
            assert inf["status_name"] in ("CONVERGED", "STAGNATED"), (b, inf)
            r_ref = np.linalg.norm(ub[b] - oracle.filter(ub[b], 2))
            r = np.linalg.norm(ub[b] - oracle.filter(got[b], 2))
            if inf["status_name"] == "CONVERGED":
                assert inf["r_true"] <= tol * inf["r_ref"], (b, inf)
                assert r <= tol * r_ref * (1 + 1e-9), (b, r / r_ref)
            else:
                assert inf["replaced"] == 2 and inf["r_true"] > tol * inf["r_ref"], (b, inf)
            assert abs(r / r_ref - inf["r_true"] / inf["r_ref"]) <= 1e-9


# tolerances from the FP32 rounding floor of the true residual upwards
FLOOR_TOLS = (1e-6, 5e-7, 3e-7, 2e-7, 1.5e-7, 1.2e-7)


def check_outcome(inf, tol, max_iter, max_replace):
    """The invariants of the exit rule for one field."""
    rt, rf, ref = inf["r_true"], inf["r_final"], inf["r_ref"]
    if inf["status_name"] == "CONVERGED":
        assert rt <= tol * ref, inf
    elif inf["status_name"] == "STAGNATED":
        assert inf["replaced"] == max_replace and rt > tol * ref and rf <= tol * ref, inf
    else:
        assert inf["status_name"] == "MAXITER" and inf["iters"] == max_iter, inf
    assert inf["replaced"] <= max_replace


def test_replacement_near_the_fp32_floor():
    """FP32 solves at tolerances approaching the rounding floor of the true
    residual: every outcome obeys the exit rule (CONVERGED only with the
    true residual within tol; GD_STAGNATED only after every allowed
    replacement, with the recursive residual within tol and the true one
    not), with the default two replacements and with none; the sweep must
    reach the floor (some field needs a replacement).  In FP64 the same
    fields converge with no replacement and with the oracle's pass count."""
    ub = filtered_input(kraichnan(256, 4, 400), 2, torch.float32)
    dub = to_dev(ub, torch.float32)
    replaced = stagnated = 0
    for tol in FLOOR_TOLS:
        _, infos, _ = gdecon.deconvolve("bicgstab", dub, 200, tol=tol, ndim=2)
        _, infos0, _ = gdecon.deconvolve("bicgstab", dub, 200, tol=tol, ndim=2, max_replace=-1)
        for inf, inf0 in zip(infos, infos0):
            check_outcome(inf, tol, 200, 2)
            check_outcome(inf0, tol, 200, 0)
            replaced += inf["replaced"]
            stagnated += inf0["status_name"] == "STAGNATED"
            # without replacements a field stops at its first check, which
            # the default run passes through at the same pass
            assert inf0["iters"] <= inf["iters"]
    print("replacements", replaced, "stagnated without", stagnated)
    assert replaced >= 1 and stagnated >= 1
    ub64 = oracle.filter(kraichnan(256, 4, 400), 2)
    _, infos64, _ = gdecon.deconvolve("bicgstab", to_dev(ub64, torch.float64), 200, tol=1e-9, ndim=2)
    _, winfo, _ = oracle.solve("bicgstab", ub64, 2, 200, tol=1e-9)
    for g, w in zip(infos64, winfo):
        assert g["status_name"] == "CONVERGED" and g["replaced"] == 0 and g["iters"] == w["iters"]


def test_replacement_restarts_from_the_current_iterate():
    """After a replacement the solve continues as a solve started from the
    iterate at the failed check would.  At a tolerance where some field's
    first check fails, the batch is solved twice in FP32: without
    replacements (such a field stops at its failed check, pass n1, with
    iterate u1) and with one (it restarts at n1 and stops at its next check,
    pass n2).  The first n1 passes are the same arithmetic in both runs.  The
    oracle, started from u1 and run n2 - n1 passes, must land on the second
    run's u: FP32 against FP64 arithmetic from one start, within 1e-6."""
    ub = filtered_input(kraichnan(256, 4, 400), 2, torch.float32)
    dub = to_dev(ub, torch.float32)
    checked = 0
    for tol in FLOOR_TOLS:
        u1, i1, _ = gdecon.deconvolve("bicgstab", dub, 200, tol=tol, ndim=2, max_replace=-1)
        fields = [b for b, inf in enumerate(i1) if inf["status_name"] == "STAGNATED"]
        if not fields:
            continue
        u2, i2, _ = gdecon.deconvolve("bicgstab", dub, 200, tol=tol, ndim=2, max_replace=1)
        for b in fields:
            assert i2[b]["replaced"] == 1, i2[b]
            n1, n2 = i1[b]["iters"], i2[b]["iters"]
            assert n2 > n1, (n1, n2)
            want, _, _ = oracle.solve("bicgstab", ub[b], 2, n2 - n1, tol=0.0, init="given",
                                      u0=u1[b].double().cpu().numpy())
            e = rel_l2(u2[b].double().cpu().numpy(), want)
            print("tol", tol, "field", b, "passes", n1, n2, "rel L2 %.2e" % e)
            assert e <= 1e-6
            checked += 1
        break
    assert checked >= 1
