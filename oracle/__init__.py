"""CPU FP64 oracle for the deconvolution solve -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.

``gd_oracle.c`` holds the filter and the four solvers (Algorithms 1-4 of the
paper) as plain scalar loops; this module loads it with ctypes and marshals
numpy arrays, and writes the closure stress out from its definition.  ``cnn.py`` holds the FP64 reference for the warm-start network.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SOLVERS = {"vc": 0, "cg": 1, "bicgstab": 2, "sd": 3}
INITS = {"ubar": 0, "zero": 1, "given": 2}
NORM_REFS = {"r0ubar": 0, "ubar": 1}
STATUS = {0: "CONVERGED", 1: "MAXITER", 2: "BREAKDOWN_RHO", 3: "BREAKDOWN_OMEGA", 4: "NONFINITE", 5: "ZERO_REF"}


_APPLY = ctypes.CFUNCTYPE(None, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction; OpenMP for the
    timed multi-core mode only, see ``set_threads``)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                               "-std=c11", "-fopenmp", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("r_ref", ctypes.c_double),
                ("r0", ctypes.c_double), ("r_final", ctypes.c_double), ("r_true", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        lib.or_filter.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, dp, dp]
        lib.or_filter.restype = None
        lib.or_dot.argtypes = [dp, dp, ctypes.c_int64, ctypes.c_double, ctypes.c_int]
        lib.or_dot.restype = ctypes.c_double
        lib.or_solve.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_double, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, dp, ctypes.POINTER(_Info)]
        lib.or_solve.restype = ctypes.c_int
        lib.or_solve_with.argtypes = lib.or_solve.argtypes + [_APPLY]
        lib.or_solve_with.restype = ctypes.c_int
        lib.or_set_threads.argtypes = [ctypes.c_int]
        lib.or_set_threads.restype = ctypes.c_int
        lib.or_host_procs.argtypes = []
        lib.or_host_procs.restype = ctypes.c_int
        _lib = lib
    return _lib


# the summation mode whose result does not depend on the thread count
SUM_CHUNKED = 3


def set_threads(n: int) -> int:
    """Threads of the oracle's loops (1 = serial, the default).  For timing on
    the host's cores only: with n > 1, solve() needs sum_mode=SUM_CHUNKED
    (fixed chunks summed in order), whose result is bitwise the same for any
    n.  Returns the count in effect."""
    return int(_load().or_set_threads(int(n)))


def host_procs() -> int:
    """Logical processors the host offers to the oracle's threads."""
    return int(_load().or_host_procs())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _grid(shape, ndim):
    g = tuple(shape[-ndim:])
    if ndim == 2:
        ny, nx = g
        return nx, ny, 1
    nz, ny, nx = g
    return nx, ny, nz


def spacing_weight(shape, ndim, h=None):
    """h^d for the inner product; h_d = 2*pi/n_d by default (domain [0,2pi]^d)."""
    nx, ny, nz = _grid(shape, ndim)
    if h is None:
        hs = [2 * math.pi / nx, 2 * math.pi / ny] + ([2 * math.pi / nz] if ndim == 3 else [])
    else:
        hs = list(h)[:ndim]
    w = 1.0
    for v in hs:
        w *= v
    return w


def filter(x: np.ndarray, ndim: int) -> np.ndarray:
    """y = G x for every field in the leading (batch) dimensions of x."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    nx, ny, nz = _grid(x.shape, ndim)
    npts = nx * ny * nz
    flat = x.reshape(-1, npts)
    out = np.empty_like(flat)
    for b in range(flat.shape[0]):
        xb = np.ascontiguousarray(flat[b])
        yb = np.empty_like(xb)
        lib.or_filter(ndim, nx, ny, nz, _ptr(xb), _ptr(yb))
        out[b] = yb
    return out.reshape(x.shape)


def germano_hat(shape, ndim: int, gamma: float) -> np.ndarray:
    """Transfer function of the differential filter G = (I - delta^2 lap)^-1
    on the half spectrum of numpy's rfftn over the last ndim axes (Sec. 4,
    Eqs. df and df2): G_hat(k) = 1 / (1 + (|k| / k_c)^2), delta = 1 / k_c,
    k_c = gamma k_m.  The domain is 2 pi periodic, so wavenumbers are
    integers; k_m, the highest wavenumber the grid resolves, is min_d n_d / 2."""
    shape = tuple(shape[-ndim:])
    ks = [np.fft.fftfreq(n, 1.0 / n) for n in shape[:-1]] + [np.fft.rfftfreq(shape[-1], 1.0 / shape[-1])]
    grids = np.meshgrid(*ks, indexing="ij")
    k2 = sum(g * g for g in grids)
    kc = gamma * min(shape) / 2.0
    return 1.0 / (1.0 + k2 / (kc * kc))


def germano_filter(x: np.ndarray, ndim: int, gamma: float) -> np.ndarray:
    """y = G x with the differential filter, applied through the FFT (Sec. 4)."""
    x = np.asarray(x, dtype=np.float64)
    axes = tuple(range(x.ndim - ndim, x.ndim))
    gh = germano_hat(x.shape, ndim, gamma)
    return np.fft.irfftn(np.fft.rfftn(x, axes=axes) * gh, s=x.shape[-ndim:], axes=axes)


def stress_pairs(ndim: int):
    """The independent pairs (i, j), i <= j, in output order."""
    return [(i, j) for i in range(ndim) for j in range(i, ndim)]


def closure_stress(ubar: np.ndarray, ustar: np.ndarray, ndim: int) -> np.ndarray:
    """tau_ij = ubar_i ubar_j - G(u*_i u*_j) for i <= j.

    The sub-filter stress of the filtered momentum equation (Sec. 2,
    Eq. fge3) with the unfiltered velocity replaced by its deconvolved
    approximation u* (Sec. 3: u* = ubar gives Eq. tau2, two van Cittert
    steps give the second-order Eq. tau3).  ubar and ustar are
    (..., ndim, [nz,] ny, nx); the result is (..., npairs, [nz,] ny, nx)
    with the pairs of `stress_pairs`.
    """
    ubar = np.asarray(ubar, dtype=np.float64)
    ustar = np.asarray(ustar, dtype=np.float64)
    assert ubar.shape == ustar.shape and ubar.shape[-ndim - 1] == ndim
    ax = -ndim - 1                       # the component axis
    out = []
    for i, j in stress_pairs(ndim):
        resolved = np.take(ubar, i, axis=ax) * np.take(ubar, j, axis=ax)
        out.append(resolved - filter(np.take(ustar, i, axis=ax) * np.take(ustar, j, axis=ax), ndim))
    return np.stack(out, axis=-ndim - 1)


WARM_BAND_TAU = 1e-10   # the differential-filter solve's band projection of a warm start


def band_project(ubar: np.ndarray, u0: np.ndarray, ndim: int, tau: float) -> np.ndarray:
    """u0 restricted to the Fourier support of ubar around ubar:
    ubar + P (u0 - ubar), P keeping the modes k of each field with
    |ubar_hat(k)|^2 > tau * E, E the mean of |ubar_hat(k)|^2 over all N
    wavenumbers (ubar_hat the unnormalized DFT; by Parseval E = sum_x ubar^2).
    The filters are diagonal in Fourier space, so G^-1 ubar has no content
    outside that support.  Full complex DFTs over the last ndim axes."""
    ubar = np.asarray(ubar, dtype=np.float64)
    u0 = np.asarray(u0, dtype=np.float64)
    fshape = ubar.shape[-ndim:]
    ub = ubar.reshape((-1,) + fshape)
    g0 = u0.reshape(ub.shape)
    out = np.empty_like(ub)
    for b in range(ub.shape[0]):
        UB = np.fft.fftn(ub[b])
        U0 = np.fft.fftn(g0[b])
        power = np.abs(UB) ** 2
        keep = power > tau * power.mean()
        out[b] = ub[b] + np.real(np.fft.ifftn(np.where(keep, U0 - UB, 0.0)))
    return out.reshape(ubar.shape)


def dot(a: np.ndarray, b: np.ndarray, hw: float, sum_mode: int = 0) -> float:
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
    return float(lib.or_dot(_ptr(a), _ptr(b), a.size, hw, sum_mode))


def warm_choice(ubar: np.ndarray, u0: np.ndarray, ndim: int, gamma=None, h=None, sum_mode: int = 0) -> list[str]:
    """The start a guarded warm start takes per field: the guess u0 where its
    residual ||ubar - G u0|| is finite and below that of the paper's start
    u0 = ubar (Algorithms 1-4), ||ubar - G ubar||; ubar otherwise."""
    ubar = np.asarray(ubar, dtype=np.float64)
    nx, ny, nz = _grid(ubar.shape, ndim)
    npts = nx * ny * nz
    fshape = ubar.shape[-ndim:]
    hw = spacing_weight(ubar.shape, ndim, h)
    ub = ubar.reshape(-1, npts)
    g0 = np.asarray(u0, dtype=np.float64).reshape(ub.shape)

    def gf(x):
        x = x.reshape(fshape)
        return (filter(x, ndim) if gamma is None else germano_filter(x, ndim, gamma)).ravel()
    out = []
    for b in range(ub.shape[0]):
        r_given = ub[b] - gf(g0[b])
        r_ubar = ub[b] - gf(ub[b])
        a = math.sqrt(dot(r_given, r_given, hw, sum_mode))
        c = math.sqrt(dot(r_ubar, r_ubar, hw, sum_mode))
        out.append("given" if math.isfinite(a) and a < c else "ubar")
    return out


def solve(solver: str, ubar: np.ndarray, ndim: int, max_iter: int, tol: float = 0.0, init: str = "ubar",
          u0: np.ndarray | None = None, norm_ref: str = "r0ubar", h=None, sum_mode: int = 0, gamma=None):
    """Run one of Algorithms 1-4 on every field of ``ubar`` (leading dims = batch).

    G is the trapezoidal stencil, or with ``gamma`` set the differential
    filter of Sec. 4 (``germano_filter``).  init: 'ubar' (the paper's),
    'zero', 'given' (u0), or 'warm' (u0 where ``warm_choice`` accepts it,
    else ubar).  With ``gamma`` a warm u0 is first band-projected
    (``band_project`` with WARM_BAND_TAU): with the differential filter the
    solve works on Fourier coefficients, where the projection costs nothing.
    Returns (u, infos, hist): u like ubar; infos a list of dicts (with the
    start used); hist an array (batch, max_iter+1) of ||r_k|| with NaN past
    the last pass.
    """
    lib = _load()
    ubar = np.ascontiguousarray(ubar, dtype=np.float64)
    nx, ny, nz = _grid(ubar.shape, ndim)
    npts = nx * ny * nz
    hw = spacing_weight(ubar.shape, ndim, h)
    flat = ubar.reshape(-1, npts)
    B = flat.shape[0]
    u = np.zeros_like(flat)
    starts = [init] * B
    if init in ("given", "warm"):
        if u0 is None:
            raise ValueError(f"init='{init}' needs u0")
        if init == "warm" and gamma is not None:
            u0 = band_project(ubar, u0, ndim, WARM_BAND_TAU)
        u[:] = np.asarray(u0, dtype=np.float64).reshape(B, npts)
        if init == "warm":
            starts = warm_choice(ubar, u0, ndim, gamma=gamma, h=h, sum_mode=sum_mode)
    hist = np.full((B, max_iter + 1), np.nan)
    infos = []
    for b in range(B):
        ub = np.ascontiguousarray(flat[b])
        uo = np.ascontiguousarray(u[b])
        hb = np.full(max_iter + 1, np.nan)
        info = _Info()
        args = (SOLVERS[solver], ndim, nx, ny, nz, hw, _ptr(ub), _ptr(uo), int(max_iter), float(tol),
                INITS[starts[b]], NORM_REFS[norm_ref], int(sum_mode), _ptr(hb), ctypes.byref(info))
        if gamma is None:
            rc = lib.or_solve(*args)
        else:
            fshape = ubar.shape[-ndim:]

            def apply(xp, yp):
                xv = np.ctypeslib.as_array(xp, shape=(npts,))
                np.ctypeslib.as_array(yp, shape=(npts,))[:] = germano_filter(xv.reshape(fshape), ndim,
                                                                              gamma).ravel()
            cb = _APPLY(apply)
            rc = lib.or_solve_with(*args, cb)
        if rc != 0:
            raise ValueError("oracle rejected the arguments")
        u[b] = uo
        hist[b] = hb
        infos.append({"iters": info.iters, "status": info.status, "status_name": STATUS[info.status],
                      "r_ref": info.r_ref, "r0": info.r0, "r_final": info.r_final, "r_true": info.r_true,
                      "start": starts[b]})
    return u.reshape(ubar.shape), infos, hist
