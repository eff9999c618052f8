"""Pins of the CPU oracle against facts it does not compute itself.

Every test here runs on the CPU.  Each one compares the oracle with a closed
form, an invariant, a brute-force construction or a textbook property, so that
a dropped term, a wrong sign, a wrong index or a transposed operand anywhere in
the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
import spectral as sp
from paper_1707_09177_amd import synth

GRIDS_2D = [(8, 8), (9, 7), (1, 5), (2, 3), (16, 12)]
GRIDS_3D = [(4, 6, 8), (5, 3, 7), (1, 2, 3), (8, 8, 8)]


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


# ---------------------------------------------------------------- the filter
@pytest.mark.parametrize("shape", GRIDS_2D + GRIDS_3D)
def test_filter_single_modes_closed_form(shape):
    """G cos(k.x + phi) = G_hat(k) cos(k.x + phi), G_hat = prod cos^2(pi k/n)."""
    nd = len(shape)
    rng = np.random.default_rng(1)
    coords = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in shape], indexing="ij")
    for _ in range(6):
        k = [int(rng.integers(0, n)) for n in shape]
        phi = rng.uniform(0, 2 * np.pi)
        x = np.cos(sum(kd * c for kd, c in zip(k, coords)) + phi)
        g = np.prod([np.cos(np.pi * kd / n) ** 2 for kd, n in zip(k, shape)])
        y = oracle.filter(x, nd)
        assert np.max(np.abs(y - g * x)) < 1e-14


@pytest.mark.parametrize("shape", GRIDS_2D + GRIDS_3D)
def test_filter_matches_kronecker_of_circulants(shape):
    nd = len(shape)
    x = np.random.default_rng(2).standard_normal(shape)
    y = oracle.filter(x, nd)
    gm = sp.dense_g(shape)
    assert np.max(np.abs(y.ravel() - gm @ x.ravel())) < 1e-14


@pytest.mark.parametrize("shape", [(9, 7), (8, 8), (5, 3, 7)])
def test_filter_mean_symmetry_psd_contraction(shape):
    nd = len(shape)
    rng = np.random.default_rng(3)
    x, z = rng.standard_normal(shape), rng.standard_normal(shape)
    gx, gz = oracle.filter(x, nd), oracle.filter(z, nd)
    assert abs(gx.sum() - x.sum()) < 1e-12                 # G_hat(0) = 1
    assert abs(np.vdot(x, gz) - np.vdot(gx, z)) < 1e-12    # symmetric
    assert np.vdot(x, gx) >= 0                             # 0 <= G_hat <= 1
    assert np.linalg.norm(gx) <= np.linalg.norm(x) + 1e-12
    # the stability condition |1 - G_hat| <= 1 of Eq. (radius)
    g = sp.ghat(shape)
    assert np.all(np.abs(1 - g) <= 1 + 1e-15)


def test_filter_batch_leading_dims():
    x = np.random.default_rng(4).standard_normal((3, 6, 5))
    y = oracle.filter(x, 2)
    for b in range(3):
        assert np.array_equal(y[b], oracle.filter(x[b], 2))


# ----------------------------------------------------------- inner product
def test_dot_is_weighted_exact_sum():
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal(10007) * 1e3, rng.standard_normal(10007)
    hw = 0.37
    exact = math.fsum((a * b).tolist())
    for mode in (0, 1, 2):
        assert abs(oracle.dot(a, b, hw, mode) - hw * exact) <= 1e-9 * abs(hw * exact) + 1e-12
    # compensated sum is within a couple of ulps of the correctly rounded sum
    assert abs(oracle.dot(a, b, 1.0, 0) - exact) <= 4 * np.spacing(abs(exact))


# --------------------------------------------------------- Van Cittert
@pytest.mark.parametrize("shape", [(8, 8), (9, 7), (16, 12), (4, 6, 8), (5, 3, 7)])
@pytest.mark.parametrize("N", [0, 1, 2, 5, 13])
def test_vancittert_transfer_closed_form(shape, N):
    """u_N = sum_{n=0..N} (I-G)^n ubar from u0 = ubar (Algorithm 1, N passes)."""
    nd = len(shape)
    rng = np.random.default_rng(6)
    ubar = oracle.filter(rng.standard_normal(shape), nd)
    g = sp.ghat(shape)
    mult = sum((1 - g) ** n for n in range(N + 1))
    want = sp.apply_fft(ubar, mult)
    u, info, hist = oracle.solve("vc", ubar, nd, N)
    assert rel(u[...], want) < 1e-12
    assert info[0]["iters"] == N
    # residual history: r_n = (I-G)^{n+1} ubar, norms via Parseval
    hw = sp.spacing_weight(shape)
    for n in range(N + 1):
        rn = sp.apply_fft(ubar, (1 - g) ** (n + 1))
        assert abs(hist[0, n] - math.sqrt(hw * np.sum(rn * rn))) <= 1e-11 * max(hist[0, 0], 1e-300)
    # monotone non-increasing since |1 - G_hat| <= 1
    assert np.all(np.diff(hist[0, : N + 1]) <= 1e-13 * hist[0, 0])


@pytest.mark.parametrize("N", [1, 3, 6])
def test_vancittert_zero_start_is_neumann_partial_sum(N):
    """From u0 = 0, N passes give sum_{n=0..N-1} (I-G)^n ubar (the Neumann series)."""
    shape = (9, 7)
    ubar = oracle.filter(np.random.default_rng(7).standard_normal(shape), 2)
    g = sp.ghat(shape)
    want = sp.apply_fft(ubar, sum((1 - g) ** n for n in range(N)))
    u, info, _ = oracle.solve("vc", ubar, 2, N, init="zero")
    assert rel(u, want) < 1e-12


# ---------------------------------------------------------- CG
@pytest.mark.parametrize("shape", [(9, 7), (5, 3, 7)])
@pytest.mark.parametrize("init", ["ubar", "zero"])
def test_cg_is_krylov_optimal(shape, init):
    """u_n minimises the G-norm error over u0 + K_n(G, r0) (brute force)."""
    nd = len(shape)
    ubar = oracle.filter(np.random.default_rng(8).standard_normal(shape), nd)
    gm = sp.dense_g(shape)
    u0 = ubar.ravel() if init == "ubar" else np.zeros(ubar.size)
    for n in range(1, 6):
        u, info, _ = oracle.solve("cg", ubar, nd, n, init=init)
        want = sp.cg_krylov_iterate(gm, ubar.ravel(), u0, n)
        assert rel(u.ravel(), want) < 1e-9, n


def band_limited(shape, kmax, seed):
    """Random real field keeping only modes with |k_d| <= kmax on every axis."""
    x = np.random.default_rng(seed).standard_normal(shape)
    xh = np.fft.fftn(x)
    keep = np.ones(shape, dtype=bool)
    for d, n in enumerate(shape):
        k = np.abs(np.fft.fftfreq(n) * n)
        sl = [None] * len(shape)
        sl[d] = slice(None)
        keep &= (k <= kmax)[tuple(sl)]
    return np.real(np.fft.ifftn(xh * keep)), keep


@pytest.mark.parametrize("shape,kmax", [((9, 7), 2), ((7, 9), 2), ((11, 13), 2), ((5, 3, 7), 1), ((7, 5, 9), 1)])
def test_cg_finite_termination_exact_inverse(shape, kmax):
    """On odd grids G is invertible; CG is exact after m = #distinct G_hat passes
    over the support of r0 (the k = 0 mode, G_hat = 1, drops out of r0)."""
    nd = len(shape)
    u_true, keep = band_limited(shape, kmax, 9)
    ubar = oracle.filter(u_true, nd)
    g = sp.ghat(shape)
    assert g.min() > 0
    m = len(sp.distinct_values(g[keep & (g < 1 - 1e-12)]))
    u, info, hist = oracle.solve("cg", ubar, nd, m)
    assert hist[0, m] / hist[0, 0] < 1e-11
    if m > 1:
        assert hist[0, m - 1] / hist[0, 0] > 1e-9   # and not one pass earlier
    exact = sp.apply_fft(ubar, 1.0 / g)
    assert rel(u, exact) < 1e-10
    assert rel(u, u_true) < 1e-10


def test_cg_residuals_mutually_orthogonal():
    """(r_n, r_m) = 0 for n != m, Eq. (cg5) and its consequences."""
    shape = (9, 7)
    ubar = oracle.filter(np.random.default_rng(10).standard_normal(shape), 2)
    rs = []
    for n in range(0, 6):
        u, _, _ = oracle.solve("cg", ubar, 2, n)
        rs.append((ubar - oracle.filter(u, 2)).ravel())
    for i in range(len(rs)):
        for j in range(i + 1, len(rs)):
            c = np.dot(rs[i], rs[j]) / (np.linalg.norm(rs[i]) * np.linalg.norm(rs[j]))
            assert abs(c) < 1e-9


def test_cg_single_mode_exact_in_one_pass():
    shape = (8, 8)
    x = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in shape], indexing="ij")
    u_true = np.sin(3 * x[1] + 0.3) + 0 * x[0]
    ubar = oracle.filter(u_true, 2)
    u, info, hist = oracle.solve("cg", ubar, 2, 1)
    assert rel(u, u_true) < 1e-13


# ---------------------------------------------------------- BiCGSTAB
def bicgstab_from_cg_polynomials(gm, ubar, u0, nmax):
    """BiCGSTAB residuals built from CG residuals alone.

    For symmetric G and shadow residual f0 = r0, BiCG residual polynomials are
    the CG ones, and BiCGSTAB's residual is r_n = Q_n(G) r_n^CG with
    Q_n(x) = prod_j (1 - w_j x); each w_n minimises ||(I - w G) v|| for
    v = Q_{n-1}(G) r_n^CG.  The CG residuals come from the Krylov brute force.
    """
    q_apply = []  # list of omegas
    out = []
    for n in range(1, nmax + 1):
        rcg = ubar - gm @ sp.cg_krylov_iterate(gm, ubar, u0, n)
        v = rcg
        for w in q_apply:
            v = v - w * (gm @ v)
        gv = gm @ v
        w = np.dot(v, gv) / np.dot(gv, gv)
        q_apply.append(w)
        out.append(v - w * gv)
    return out


@pytest.mark.parametrize("shape", [(9, 7), (5, 3, 7)])
def test_bicgstab_matches_stabilised_cg_polynomials(shape):
    nd = len(shape)
    ubar = oracle.filter(np.random.default_rng(11).standard_normal(shape), nd)
    gm = sp.dense_g(shape)
    want = bicgstab_from_cg_polynomials(gm, ubar.ravel(), ubar.ravel().copy(), 5)
    for n in range(1, 6):
        u, info, _ = oracle.solve("bicgstab", ubar, nd, n)
        r = ubar.ravel() - gm @ u.ravel()
        assert rel(r, want[n - 1]) < 1e-8, n


def test_bicgstab_first_pass_closed_form():
    """p1 = r0, alpha = (r0,r0)/(r0,Gr0), s = r0 - alpha G r0, omega = (s,Gs)/(Gs,Gs)."""
    shape = (8, 8)
    ubar = oracle.filter(np.random.default_rng(12).standard_normal(shape), 2)
    g = sp.ghat(shape)
    G = lambda v: sp.apply_fft(v, g)
    r0 = ubar - G(ubar)
    a = np.sum(r0 * r0) / np.sum(r0 * G(r0))
    s = r0 - a * G(r0)
    w = np.sum(s * G(s)) / np.sum(G(s) * G(s))
    want = ubar + a * r0 + w * s
    u, info, _ = oracle.solve("bicgstab", ubar, 2, 1)
    assert rel(u, want) < 1e-12


@pytest.mark.parametrize("shape", [(9, 7), (5, 3, 7)])
def test_bicgstab_converges_to_exact_inverse(shape):
    nd = len(shape)
    u_true = np.random.default_rng(13).standard_normal(shape)
    ubar = oracle.filter(u_true, nd)
    u, info, _ = oracle.solve("bicgstab", ubar, nd, 200, tol=1e-13)
    assert info[0]["status_name"] == "CONVERGED"
    assert rel(u, u_true) < 1e-10


def test_bicgstab_single_mode_half_step():
    """A single Fourier mode makes s vanish: the half-step guard stops at pass 1."""
    shape = (8, 8)
    x = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in shape], indexing="ij")
    u_true = np.cos(2 * x[0] + 3 * x[1])
    ubar = oracle.filter(u_true, 2)
    u, info, _ = oracle.solve("bicgstab", ubar, 2, 10, tol=1e-8)
    assert info[0]["status_name"] == "CONVERGED" and info[0]["iters"] == 1
    assert rel(u, u_true) < 1e-13


# ---------------------------------------------------------- steepest descent
def test_sd_successive_residuals_orthogonal():
    """(r_n, r_{n+1}) = 0, Eq. (inner2)."""
    shape = (9, 7)
    ubar = oracle.filter(np.random.default_rng(14).standard_normal(shape), 2)
    prev = None
    for n in range(0, 6):
        u, _, _ = oracle.solve("sd", ubar, 2, n)
        r = (ubar - oracle.filter(u, 2)).ravel()
        if prev is not None:
            assert abs(np.dot(prev, r)) < 1e-10 * np.dot(prev, prev)
        prev = r


def test_sd_step_minimises_g_norm_error_along_residual():
    shape = (9, 7)
    u_true = np.random.default_rng(15).standard_normal(shape)
    ubar = oracle.filter(u_true, 2)
    gm = sp.dense_g(shape)
    u1, _, _ = oracle.solve("sd", ubar, 2, 1)
    r0 = (ubar - oracle.filter(ubar, 2)).ravel()
    err = lambda a: (u_true.ravel() - ubar.ravel() - a * r0) @ gm @ (u_true.ravel() - ubar.ravel() - a * r0)
    a_star = (r0 @ r0) / (r0 @ gm @ r0)
    assert rel(u1.ravel(), ubar.ravel() + a_star * r0) < 1e-12
    assert err(a_star) <= min(err(a_star * 0.99), err(a_star * 1.01))


# ---------------------------------------------------------- all solvers
@pytest.mark.parametrize("solver", ["vc", "cg", "bicgstab", "sd"])
def test_residual_history_independent_of_phases(solver):
    """G is diagonal in Fourier space, so scalars depend only on |u_hat|."""
    n = 32
    f1 = synth.field_2d(n, synth.spectrum_c1, 1.0, np.inf, synth.rng_for(99, 1))
    f2 = synth.field_2d(n, synth.spectrum_c1, 1.0, np.inf, synth.rng_for(99, 2))
    assert np.allclose(np.abs(np.fft.fft2(f1)), np.abs(np.fft.fft2(f2)), atol=1e-9)
    assert not np.allclose(f1, f2)
    h = []
    for f in (f1, f2):
        ub = oracle.filter(f, 2)
        _, info, hist = oracle.solve(solver, ub, 2, 8)
        h.append(hist[0])
    assert np.allclose(h[0], h[1], rtol=1e-9, atol=0)


@pytest.mark.parametrize("solver", ["vc", "cg", "bicgstab", "sd"])
def test_mean_is_preserved(solver):
    """G_hat(0) = 1: the residual has zero mean, so every iterate keeps ubar's mean."""
    shape = (9, 7)
    ubar = oracle.filter(np.random.default_rng(16).standard_normal(shape) + 0.7, 2)
    u, _, _ = oracle.solve(solver, ubar, 2, 4)
    assert abs(u.mean() - ubar.mean()) < 1e-12


@pytest.mark.parametrize("solver", ["vc", "cg", "bicgstab", "sd"])
def test_given_exact_start_converges_at_once(solver):
    shape = (9, 7)
    u_true = np.random.default_rng(17).standard_normal(shape)
    ubar = oracle.filter(u_true, 2)
    u, info, _ = oracle.solve(solver, ubar, 2, 5, tol=1e-8, init="given", u0=u_true)
    assert info[0]["status_name"] == "CONVERGED" and info[0]["iters"] == 0
    assert np.array_equal(u, u_true)


@pytest.mark.parametrize("solver", ["vc", "cg", "bicgstab", "sd"])
def test_guards(solver):
    shape = (8, 6)
    z = np.zeros(shape)
    _, info, _ = oracle.solve(solver, z, 2, 5)
    assert info[0]["status_name"] == "ZERO_REF" and info[0]["iters"] == 0
    c = np.full(shape, 2.5)                                  # G c = c: r_ref = 0
    u, info, _ = oracle.solve(solver, c, 2, 5)
    assert info[0]["status_name"] == "ZERO_REF" and np.array_equal(u, c)
    bad = oracle.filter(np.random.default_rng(18).standard_normal(shape), 2)
    bad[2, 3] = np.nan
    _, info, _ = oracle.solve(solver, bad, 2, 5)
    assert info[0]["status_name"] == "NONFINITE"
    ub = oracle.filter(np.random.default_rng(19).standard_normal(shape), 2)
    u, info, _ = oracle.solve(solver, ub, 2, 0)
    assert info[0]["status_name"] == "MAXITER" and np.array_equal(u, ub)
    # ||ubar|| as the reference norm
    _, info, _ = oracle.solve(solver, ub, 2, 3, norm_ref="ubar")
    assert abs(info[0]["r_ref"] - math.sqrt(sp.spacing_weight(shape) * np.sum(ub * ub))) < 1e-12


def test_true_residual_and_reference_norm():
    shape = (16, 12)
    ubar = oracle.filter(np.random.default_rng(20).standard_normal(shape), 2)
    gm = sp.dense_g(shape)
    hw = sp.spacing_weight(shape)
    u, info, _ = oracle.solve("cg", ubar, 2, 3)
    rt = ubar.ravel() - gm @ u.ravel()
    assert abs(info[0]["r_true"] - math.sqrt(hw * rt @ rt)) < 1e-12
    r0 = ubar.ravel() - gm @ ubar.ravel()
    assert abs(info[0]["r_ref"] - math.sqrt(hw * r0 @ r0)) < 1e-12


def test_even_grid_nyquist_null_space():
    """On even grids G_hat = 0 on Nyquist planes; from u0 = ubar iterates stay in range(G)."""
    shape = (8, 8)
    g = sp.ghat(shape)
    assert np.isclose(g[4, :], 0).all() and np.isclose(g[:, 4], 0).all()
    ubar = oracle.filter(np.random.default_rng(21).standard_normal(shape), 2)
    u, _, _ = oracle.solve("cg", ubar, 2, 6)
    uh = np.fft.fft2(u)
    assert np.max(np.abs(uh[4, :])) < 1e-12 and np.max(np.abs(uh[:, 4])) < 1e-12


def test_threaded_timing_mode_is_thread_count_independent():
    """The oracle's multi-core timing mode (fixed-chunk compensated sums,
    loops split over points) gives bitwise the same result on one thread and
    on every core, and agrees with the serial compensated sums to rounding."""
    rng = np.random.default_rng(31)
    ub = oracle.filter(rng.standard_normal((2, 96, 80)), 2)
    one = oracle.solve("bicgstab", ub, 2, 12, sum_mode=oracle.SUM_CHUNKED)
    used = oracle.set_threads(max(2, oracle.host_procs()))
    try:
        assert used >= 2
        many = oracle.solve("bicgstab", ub, 2, 12, sum_mode=oracle.SUM_CHUNKED)
        with pytest.raises(ValueError):            # only the chunked sums may run threaded
            oracle.solve("bicgstab", ub, 2, 12)
    finally:
        oracle.set_threads(1)
    assert np.array_equal(one[0], many[0]) and one[1] == many[1]
    assert np.array_equal(one[2], many[2], equal_nan=True)
    serial = oracle.solve("bicgstab", ub, 2, 12)
    assert np.max(np.abs(serial[0] - one[0])) <= 1e-13 * np.max(np.abs(serial[0]))
    # the chunked sum itself: exact on integer-valued data
    a = rng.integers(-1000, 1000, 100003).astype(np.float64)
    assert oracle.dot(a, a, 1.0, oracle.SUM_CHUNKED) == float(np.sum(a.astype(np.int64) ** 2))


def test_warm_choice_rule():
    """The guarded warm start keeps a guess only when its residual is finite
    and strictly below that of the paper's start u0 = ubar."""
    rng = np.random.default_rng(32)
    u = rng.standard_normal((9, 11))                 # odd sizes: G is invertible
    ub = oracle.filter(u, 2)
    near = ub + 0.5 * (u - ub)                       # residual (1 - G/2 ... ) smaller than ubar's
    nan = u.copy()
    nan[3, 4] = np.nan
    inf = u.copy()
    inf[0, 0] = np.inf
    picks = oracle.warm_choice(np.stack([ub] * 6), np.stack([u, near, ub, ub + 1.0, nan, inf]), 2)
    assert picks == ["given", "given", "ubar", "ubar", "ubar", "ubar"]
    # the solve from the accepted exact guess converges at once; the rejected
    # ones run exactly the ubar start
    x, infos, _ = oracle.solve("cg", np.stack([ub] * 3), 2, 5, tol=1e-12, init="warm",
                               u0=np.stack([u, ub + 1.0, nan]))
    assert [i["start"] for i in infos] == ["given", "ubar", "ubar"]
    assert infos[0]["iters"] == 0 and infos[0]["status_name"] == "CONVERGED"
    y, jinfos, _ = oracle.solve("cg", np.stack([ub] * 2), 2, 5, tol=1e-12)
    assert np.array_equal(x[1:], y) and [i["iters"] for i in infos[1:]] == [i["iters"] for i in jinfos]
