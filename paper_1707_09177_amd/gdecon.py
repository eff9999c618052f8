"""ctypes binding of libgdecon.so (the HIP deconvolution library).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch provides device memory and the stream.  If the shared
library is missing the import fails; there is no CPU fallback.

Fields are torch tensors on a ROCm device, C-contiguous with x fastest:
shape (..., ny, nx) for ndim=2 or (..., nz, ny, nx) for ndim=3; the leading
dimensions form the batch of independent fields.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgdecon.so")

F64, F32 = 0, 1
SOLVERS = {"vc": 0, "cg": 1, "bicgstab": 2, "sd": 3}
INITS = {"ubar": 0, "zero": 1, "given": 2, "warm": 3}
START_NAMES = {0: "ubar", 1: "zero", 2: "given"}
NORM_REFS = {"r0ubar": 0, "ubar": 1}
STATUS = {0: "CONVERGED", 1: "MAXITER", 2: "BREAKDOWN_RHO", 3: "BREAKDOWN_OMEGA", 4: "NONFINITE", 5: "ZERO_REF",
          6: "TIMEOUT", 7: "STAGNATED"}
ERRORS = {-1: "GD_EINVAL", -2: "GD_EWORKSPACE", -3: "GD_EHIP", -4: "GD_EALIGN"}


class GdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("dtype", ctypes.c_int32), ("n", ctypes.c_int64 * 3),
                ("h", ctypes.c_double * 3), ("batch", ctypes.c_int64)]


class Opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("init", ctypes.c_int32), ("norm_ref", ctypes.c_int32),
                ("max_replace", ctypes.c_int32), ("tol", ctypes.c_double), ("history", ctypes.c_void_p),
                ("wait_limit_us", ctypes.c_int64)]


class LaunchInfo(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("vw", ctypes.c_int32), ("R", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("L", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("blocks", ctypes.c_int64), ("waves", ctypes.c_int64)]


class Instance(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("reserved", ctypes.c_int32), ("n", ctypes.c_int64 * 3),
                ("h", ctypes.c_double * 3), ("ubar", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("history", ctypes.c_void_p)]


class TuneInfo(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int32), ("best", ctypes.c_int32), ("tiles_per_wave", ctypes.c_int32),
                ("rows", ctypes.c_int32), ("tail_pct", ctypes.c_int32), ("interleave", ctypes.c_int32),
                ("wave_claims", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("segments", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]


class Cnn(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("channels", ctypes.c_int32), ("layers", ctypes.c_int32),
                ("smooth", ctypes.c_int32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("params", ctypes.c_void_p),
                ("grad", ctypes.c_void_p), ("adam_m", ctypes.c_void_p), ("adam_v", ctypes.c_void_p),
                ("step", ctypes.c_void_p)]


INFO_BYTES = 48  # gd_info: int32 iters, int32 status, 4 doubles, int32 start, int32 replaced

EXPORTS = ["filter_apply", "deconvolve_workspace_bytes", "deconvolve_vancittert", "deconvolve_cg",
           "deconvolve_bicgstab", "deconvolve_steepest_descent", "gd_status_string", "gd_last_error",
           "gd_last_launch", "gd_set_trace", "deconvolve_batch_workspace_bytes", "deconvolve_batch",
           "deconvolve_autotune", "deconvolve_batch_autotune", "gd_tune_reset", "gd_tune_set", "gd_tune_set_batch", "warmstart_param_count",
           "warmstart_workspace_bytes", "warmstart_forward", "warmstart_train_step", "closure_stress",
           "germano_filter", "GermanoDeconvolver", "deconvolve_germano", "energy_spectrum", "pdf_counts", "BlockedVanCittert",
           "deconvolve_noalloc"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libgdecon.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(paper_1707_09177_amd/csrc/build.py); there is no fallback")
    lib = ctypes.CDLL(path)
    vp, gp, op = ctypes.c_void_p, ctypes.POINTER(Grid), ctypes.POINTER(Opts)
    lib.filter_apply.argtypes = [gp, vp, vp, vp]
    lib.filter_apply.restype = ctypes.c_int
    lib.deconvolve_workspace_bytes.argtypes = [gp, ctypes.c_int32]
    lib.deconvolve_workspace_bytes.restype = ctypes.c_size_t
    for name in ("deconvolve_vancittert", "deconvolve_cg", "deconvolve_bicgstab", "deconvolve_steepest_descent"):
        f = getattr(lib, name)
        f.argtypes = [gp, vp, vp, op, vp, ctypes.c_size_t, vp, vp]
        f.restype = ctypes.c_int
    lib.gd_status_string.argtypes = [ctypes.c_int32]
    lib.gd_status_string.restype = ctypes.c_char_p
    lib.gd_last_error.argtypes = []
    lib.gd_last_error.restype = ctypes.c_char_p
    lib.gd_last_launch.argtypes = [ctypes.POINTER(LaunchInfo)]
    lib.gd_last_launch.restype = ctypes.c_int
    lib.gd_set_trace.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    lib.gd_set_trace.restype = ctypes.c_int
    ip, i32, tp = ctypes.POINTER(Instance), ctypes.c_int32, ctypes.POINTER(TuneInfo)
    lib.deconvolve_noalloc_max_bytes.argtypes = []
    lib.deconvolve_noalloc_max_bytes.restype = ctypes.c_size_t
    lib.deconvolve_noalloc.argtypes = [i32, gp, vp, vp, op, vp, vp]
    lib.deconvolve_noalloc.restype = ctypes.c_int
    lib.deconvolve_batch_workspace_bytes.argtypes = [i32, i32, ip, i32]
    lib.deconvolve_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.deconvolve_batch.argtypes = [i32, i32, ip, i32, op, vp, ctypes.c_size_t, vp, vp]
    lib.deconvolve_batch.restype = ctypes.c_int
    lib.deconvolve_autotune.argtypes = [i32, gp, vp, vp, vp, ctypes.c_size_t, vp, vp, tp]
    lib.deconvolve_autotune.restype = ctypes.c_int
    lib.deconvolve_batch_autotune.argtypes = [i32, i32, ip, i32, vp, ctypes.c_size_t, vp, vp, tp]
    lib.deconvolve_batch_autotune.restype = ctypes.c_int
    lib.gd_tune_reset.argtypes = []
    lib.gd_tune_reset.restype = None
    lib.gd_tune_set.argtypes = [i32, gp, vp, vp, tp]
    lib.gd_tune_set.restype = ctypes.c_int
    lib.gd_tune_set_batch.argtypes = [i32, i32, ip, i32, tp]
    lib.gd_tune_set_batch.restype = ctypes.c_int
    lib.vancittert_blocked_workspace_bytes.argtypes = [gp]
    lib.vancittert_blocked_workspace_bytes.restype = ctypes.c_size_t
    lib.vancittert_blocked_passes.argtypes = [gp]
    lib.vancittert_blocked_passes.restype = ctypes.c_int32
    lib.deconvolve_vancittert_blocked.argtypes = [gp, vp, vp, op, vp, ctypes.c_size_t, vp, vp]
    lib.deconvolve_vancittert_blocked.restype = ctypes.c_int
    lib.germano_workspace_bytes.argtypes = [gp, ctypes.c_int32]
    lib.germano_workspace_bytes.restype = ctypes.c_size_t
    lib.germano_filter_apply.argtypes = [gp, ctypes.c_double, vp, vp, vp, ctypes.c_size_t, vp]
    lib.germano_filter_apply.restype = ctypes.c_int
    lib.deconvolve_germano.argtypes = [ctypes.c_int32, gp, ctypes.c_double, vp, vp, op, vp, ctypes.c_size_t, vp, vp]
    lib.deconvolve_germano.restype = ctypes.c_int
    lib.deconvolve_germano_autotune.argtypes = [ctypes.c_int32, gp, ctypes.c_double, vp, vp, vp, ctypes.c_size_t, vp,
                                                vp, ctypes.POINTER(TuneInfo)]
    lib.deconvolve_germano_autotune.restype = ctypes.c_int
    lib.spectrum_shells.argtypes = [gp]
    lib.spectrum_shells.restype = ctypes.c_int32
    lib.spectrum_workspace_bytes.argtypes = [gp]
    lib.spectrum_workspace_bytes.restype = ctypes.c_size_t
    lib.energy_spectrum.argtypes = [gp, ctypes.c_double, vp, vp, vp, ctypes.c_size_t, vp]
    lib.energy_spectrum.restype = ctypes.c_int
    lib.pdf_counts.argtypes = [gp, ctypes.c_double, ctypes.c_double, ctypes.c_int32, vp, vp, vp]
    lib.pdf_counts.restype = ctypes.c_int
    lib.band_project_workspace_bytes.argtypes = [gp]
    lib.band_project_workspace_bytes.restype = ctypes.c_size_t
    lib.band_project.argtypes = [gp, ctypes.c_double, vp, vp, vp, ctypes.c_size_t, vp]
    lib.band_project.restype = ctypes.c_int
    lib.closure_stress.argtypes = [gp, vp, vp, vp, vp]
    lib.closure_stress.restype = ctypes.c_int
    cp = ctypes.POINTER(Cnn)
    lib.warmstart_param_count.argtypes = [cp]
    lib.warmstart_param_count.restype = ctypes.c_int64
    lib.warmstart_workspace_bytes.argtypes = [cp, gp, i32]
    lib.warmstart_workspace_bytes.restype = ctypes.c_size_t
    lib.warmstart_forward.argtypes = [cp, gp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.warmstart_forward.restype = ctypes.c_int
    lib.warmstart_train_step.argtypes = [cp, gp, vp, vp, vp, ctypes.c_size_t, vp, vp]
    lib.warmstart_train_step.restype = ctypes.c_int
    _lib = lib
    return lib


def last_launch() -> dict:
    """Tile shape and persistent grid of the last solve launched from this thread."""
    li = LaunchInfo()
    load().gd_last_launch(ctypes.byref(li))
    return {k: int(getattr(li, k)) for k, _ in LaunchInfo._fields_ if k != "reserved"}


def set_trace(buf: torch.Tensor | None):
    """Record grid-barrier timestamps of later solves into ``buf`` (int64, on
    the device; see gd_set_trace).  ``None`` switches recording off."""
    if buf is None:
        load().gd_set_trace(None, 0)
    else:
        load().gd_set_trace(_dev_ptr(buf), buf.numel())


def _check(rc: int):
    if rc != 0:
        raise GdError(rc, load().gd_last_error().decode())


def _stream_handle(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def make_grid(field_shape, ndim: int, dtype: torch.dtype, h=None) -> Grid:
    if ndim not in (2, 3):
        raise ValueError("ndim must be 2 or 3")
    if len(field_shape) < ndim:
        raise ValueError(f"a {ndim}D field needs at least {ndim} dimensions")
    g = Grid()
    g.ndim = ndim
    g.dtype = F32 if dtype == torch.float32 else F64 if dtype == torch.float64 else -1
    if g.dtype < 0:
        raise ValueError("fields must be float32 or float64")
    sp = tuple(field_shape[-ndim:])[::-1]  # (nx, ny[, nz])
    for d in range(3):
        g.n[d] = sp[d] if d < ndim else 1
        g.h[d] = (h[d] if h is not None else 0.0) if d < ndim else 0.0
    g.batch = int(math.prod(field_shape[:-ndim])) if len(field_shape) > ndim else 1
    return g


def _dev_ptr(t: torch.Tensor) -> int:
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return t.data_ptr()


def _out(out: torch.Tensor | None, shape, like: torch.Tensor, name: str = "out") -> torch.Tensor:
    """A new output tensor shaped `shape` with like's dtype and device, or the
    caller's, which must match exactly: the library writes through a bare
    pointer, so a short or differently typed buffer would be overrun."""
    shape = tuple(int(v) for v in shape)
    if out is None:
        return torch.empty(shape, dtype=like.dtype, device=like.device)
    if tuple(out.shape) != shape or out.dtype != like.dtype or out.device != like.device:
        raise ValueError(f"{name} must have shape {shape} and dtype {like.dtype} on {like.device}, "
                         f"got {tuple(out.shape)} {out.dtype} on {out.device}")
    return out


def filter_apply(x: torch.Tensor, ndim: int = 2, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """y = G x with the periodic trapezoidal stencil (per field of the batch)."""
    lib = load()
    g = make_grid(x.shape, ndim, x.dtype)
    y = _out(out, x.shape, x)
    _check(lib.filter_apply(ctypes.byref(g), _dev_ptr(x), _dev_ptr(y), _stream_handle(stream)))
    return y


def workspace_bytes(field_shape, ndim: int, dtype: torch.dtype, solver: str) -> int:
    g = make_grid(field_shape, ndim, dtype)
    n = load().deconvolve_workspace_bytes(ctypes.byref(g), SOLVERS[solver])
    if n == 0:
        raise GdError(-1, "bad grid or solver")
    return int(n)


def decode_info(raw: np.ndarray) -> list[dict]:
    """raw: uint8 array of batch*48 bytes copied from the device info buffer."""
    out = []
    b = raw.reshape(-1, INFO_BYTES)
    for row in b:
        i32 = row[:8].view(np.int32)
        f64 = row[8:40].view(np.float64)
        tail = row[40:48].view(np.int32)
        out.append({"iters": int(i32[0]), "status": int(i32[1]), "status_name": STATUS.get(int(i32[1]), "?"),
                    "r_ref": float(f64[0]), "r0": float(f64[1]), "r_final": float(f64[2]),
                    "r_true": float(f64[3]), "start": START_NAMES.get(int(tail[0]), "?"),
                    "replaced": int(tail[1])})
    return out


@dataclass
class SolveResult:
    u: torch.Tensor
    info_dev: torch.Tensor
    history: torch.Tensor | None

    def info(self) -> list[dict]:
        """Per-field outcome (synchronises with the device)."""
        return decode_info(self.info_dev.cpu().numpy())


class Deconvolver:
    """A solver bound to one field shape, with its workspace allocated once.

    ``solve`` only launches kernels on the stream (no allocation when ``out``
    and ``info`` buffers are reused), so it can be timed or graph-captured.
    Each solve is one persistent launch that fills the GPU: run solves on one
    GPU one after another (one stream, or a batch in one call), not
    concurrently on several streams, where launches that split the GPU wait
    at their grid barriers until the wait bound ends them (GD_TIMEOUT).
    """

    def __init__(self, field_shape, ndim: int, dtype: torch.dtype, solver: str, device=None, h=None):
        self.lib = load()
        self.shape = tuple(field_shape)
        self.ndim = ndim
        self.dtype = dtype
        self.solver = solver
        self.grid = make_grid(self.shape, ndim, dtype, h)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        n = self._workspace_bytes()
        if n == 0:
            raise GdError(-1, "bad grid or solver")
        self.work = torch.empty(int(n), dtype=torch.uint8, device=self.device)
        self.batch = int(self.grid.batch)
        self.info_dev = torch.zeros(self.batch * INFO_BYTES, dtype=torch.uint8, device=self.device)
        self._fn = self._entry()

    # the C entry point and its workspace size; subclasses for other solves override these
    def _workspace_bytes(self) -> int:
        return self.lib.deconvolve_workspace_bytes(ctypes.byref(self.grid), SOLVERS[self.solver])

    def _entry(self):
        return getattr(self.lib, {"vc": "deconvolve_vancittert", "cg": "deconvolve_cg",
                                  "bicgstab": "deconvolve_bicgstab", "sd": "deconvolve_steepest_descent"}[self.solver])

    def solve(self, ubar: torch.Tensor, max_iter: int, tol: float = 0.0, init: str = "ubar",
              out: torch.Tensor | None = None, norm_ref: str = "r0ubar", history: torch.Tensor | None = None,
              wait_limit_us: int = 0, max_replace: int = 0, stream=None) -> SolveResult:
        """init: 'ubar' (the paper's start), 'zero', 'given' (the guess in
        ``out``) or 'warm' (the guess in ``out`` where its residual is below
        the ubar start's, else ubar).  max_replace: residual replacements
        allowed after the recursive residual meets tol (0: the library's
        default, negative: none)."""
        if tuple(ubar.shape) != self.shape or ubar.dtype != self.dtype or ubar.device != self.work.device:
            raise ValueError(f"ubar must have shape {self.shape} and dtype {self.dtype} on {self.work.device}")
        if init in ("given", "warm") and out is None:
            raise ValueError(f"init='{init}' reads the initial guess from `out`")
        u = _out(out, self.shape, ubar)
        o = _make_opts(max_iter, tol, init, norm_ref, _dev_ptr(history) if history is not None else None,
                       wait_limit_us, max_replace)
        if history is not None and (history.dtype != torch.float64 or history.numel() < self.batch * (max_iter + 1)
                                    or history.device != ubar.device):
            raise ValueError("history must be float64 with batch*(max_iter+1) entries, on ubar's device")
        rc = self._fn(ctypes.byref(self.grid), _dev_ptr(ubar), _dev_ptr(u), ctypes.byref(o),
                      self.work.data_ptr(), self.work.numel(), self.info_dev.data_ptr(), _stream_handle(stream))
        _check(rc)
        return SolveResult(u, self.info_dev, history)


def germano_filter(x: torch.Tensor, gamma: float, ndim: int = 2, out: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
    """y = G x with the paper's differential filter G = (I - delta^2 lap)^-1,
    transfer function 1 / (1 + (|k| / k_c)^2), k_c = gamma * min(n) / 2, applied
    through the library's FFTs (germano_filter_apply).  Power-of-two sizes."""
    lib = load()
    g = make_grid(x.shape, ndim, x.dtype)
    n = lib.germano_workspace_bytes(ctypes.byref(g), -1)
    if n == 0:
        raise GdError(-1, "bad grid (the differential filter needs power-of-two sizes)")
    work = torch.empty(int(n), dtype=torch.uint8, device=x.device)
    y = _out(out, x.shape, x)
    _check(lib.germano_filter_apply(ctypes.byref(g), float(gamma), _dev_ptr(x), _dev_ptr(y), work.data_ptr(),
                                    work.numel(), _stream_handle(stream)))
    return y


def energy_spectrum(x: torch.Tensor, ndim: int = 2, kpow: float = 0.0, stream=None) -> torch.Tensor:
    """Shell-summed spectrum 1/2 sum_{|k| ~ s} |k|^kpow |f_hat(k)|^2 of every
    field (energy_spectrum): a float64 tensor (..., nshells)."""
    lib = load()
    g = make_grid(x.shape, ndim, x.dtype)
    ns = lib.spectrum_shells(ctypes.byref(g))
    if ns == 0:
        raise GdError(-1, "bad grid (spectra need power-of-two sizes)")
    work = torch.empty(int(lib.spectrum_workspace_bytes(ctypes.byref(g))), dtype=torch.uint8, device=x.device)
    out = torch.empty(tuple(x.shape[:-ndim]) + (ns,), dtype=torch.float64, device=x.device)
    _check(lib.energy_spectrum(ctypes.byref(g), float(kpow), _dev_ptr(x), _dev_ptr(out), work.data_ptr(),
                               work.numel(), _stream_handle(stream)))
    return out


BAND_TAU = 1e-10   # default threshold of band_project, relative to the mean mode power of ubar


def band_project(ubar: torch.Tensor, u0: torch.Tensor, ndim: int = 2, tau: float = BAND_TAU,
                 work: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """u0 <- ubar + P (u0 - ubar) in place (band_project): P keeps the Fourier
    modes of each field where |ubar_hat|^2 > tau * mean |ubar_hat|^2.
    Power-of-two sizes.  Returns u0."""
    lib = load()
    if u0.shape != ubar.shape or u0.dtype != ubar.dtype:
        raise ValueError("ubar and u0 must match")
    g = make_grid(ubar.shape, ndim, ubar.dtype)
    n = int(lib.band_project_workspace_bytes(ctypes.byref(g)))
    if n == 0:
        raise GdError(-1, "bad grid (the band projection needs power-of-two sizes)")
    if work is None or work.numel() < n:
        work = torch.empty(n, dtype=torch.uint8, device=ubar.device)
    _check(lib.band_project(ctypes.byref(g), float(tau), _dev_ptr(ubar), _dev_ptr(u0), work.data_ptr(), work.numel(),
                            _stream_handle(stream)))
    return u0


def pdf_counts(x: torch.Tensor, lo: float, hi: float, nbins: int, ndim: int = 2, stream=None) -> torch.Tensor:
    """Counts of every field's values in nbins equal bins over [lo, hi]
    (pdf_counts): an int64 tensor (..., nbins)."""
    lib = load()
    g = make_grid(x.shape, ndim, x.dtype)
    out = torch.empty(tuple(x.shape[:-ndim]) + (int(nbins),), dtype=torch.int64, device=x.device)
    _check(lib.pdf_counts(ctypes.byref(g), float(lo), float(hi), int(nbins), _dev_ptr(x), _dev_ptr(out),
                          _stream_handle(stream)))
    return out


class BlockedVanCittert(Deconvolver):
    """Van Cittert with several passes per sweep (deconvolve_vancittert_blocked):
    same results as the "vc" solver, less memory traffic."""

    def __init__(self, field_shape, ndim: int, dtype: torch.dtype, device=None, h=None):
        super().__init__(field_shape, ndim, dtype, "vcb", device=device, h=h)
        self.passes_per_sweep = int(self.lib.vancittert_blocked_passes(ctypes.byref(self.grid)))

    def _workspace_bytes(self) -> int:
        return self.lib.vancittert_blocked_workspace_bytes(ctypes.byref(self.grid))

    def _entry(self):
        return self.lib.deconvolve_vancittert_blocked


class GermanoDeconvolver(Deconvolver):
    """Deconvolver for the differential filter with parameter gamma
    (deconvolve_germano): the solve runs on the Fourier coefficients."""

    def __init__(self, field_shape, ndim: int, dtype: torch.dtype, solver: str, gamma: float, device=None, h=None):
        self.gamma = float(gamma)
        super().__init__(field_shape, ndim, dtype, solver, device=device, h=h)

    def _workspace_bytes(self) -> int:
        # 0 also for sizes the FFTs do not take (not powers of two)
        return self.lib.germano_workspace_bytes(ctypes.byref(self.grid), SOLVERS[self.solver])

    def _entry(self):
        code, fn = SOLVERS[self.solver], self.lib.deconvolve_germano

        def call(grid, ub, u, o, work, wb, info, stream):
            return fn(code, grid, self.gamma, ub, u, o, work, wb, info, stream)
        return call

    def autotune(self, ubar: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> dict:
        """Time the launch configurations on these buffers and keep the
        fastest for later solves of this shape (deconvolve_germano_autotune)."""
        if tuple(ubar.shape) != self.shape or ubar.dtype != self.dtype or ubar.device != self.work.device:
            raise ValueError(f"ubar must have shape {self.shape} and dtype {self.dtype} on {self.work.device}")
        u = _out(out, self.shape, ubar)
        t = TuneInfo()
        _check(self.lib.deconvolve_germano_autotune(SOLVERS[self.solver], ctypes.byref(self.grid), self.gamma,
                                                    _dev_ptr(ubar), _dev_ptr(u), self.work.data_ptr(),
                                                    self.work.numel(), self.info_dev.data_ptr(),
                                                    _stream_handle(stream), ctypes.byref(t)))
        return _tune_dict(t)


def deconvolve_germano(solver: str, ubar: torch.Tensor, max_iter: int, gamma: float, tol: float = 0.0,
                       ndim: int = 2, init: str = "ubar", u0: torch.Tensor | None = None, norm_ref: str = "r0ubar",
                       history: bool = False, h=None, stream=None):
    """One-shot solve of G u = ubar with the differential filter.  Returns
    (u, infos, history or None); synchronises the stream."""
    d = GermanoDeconvolver(ubar.shape, ndim, ubar.dtype, solver, gamma, device=ubar.device, h=h)
    out = None
    if init in ("given", "warm"):
        if u0 is None:
            raise ValueError(f"init='{init}' needs u0")
        out = u0.clone()
    hist = None
    if history:
        hist = torch.full((d.batch, max_iter + 1), float("nan"), dtype=torch.float64, device=ubar.device)
    res = d.solve(ubar, max_iter, tol, init=init, out=out, norm_ref=norm_ref, history=hist, stream=stream)
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return res.u, res.info(), hist


def _make_opts(max_iter, tol, init, norm_ref, history, wait_limit_us, max_replace=0) -> Opts:
    o = Opts()
    o.max_iter = int(max_iter)
    o.init = INITS[init]
    o.norm_ref = NORM_REFS[norm_ref]
    o.max_replace = int(max_replace)
    o.tol = float(tol)
    o.history = history
    o.wait_limit_us = int(wait_limit_us)
    return o


def _tune_dict(t: TuneInfo) -> dict:
    return {k: (float(getattr(t, k)) if k.endswith("_ms") else int(getattr(t, k))) for k, _ in TuneInfo._fields_
            if k != "pad"}


def autotune(solver: str, ubar: torch.Tensor, ndim: int = 2, out: torch.Tensor | None = None, stream=None) -> dict:
    """Time the launch configurations for this (solver, shape, dtype) and keep
    the fastest for later solves of the same signature (deconvolve_autotune).
    ``out`` (or a scratch tensor) is overwritten.  Synchronous."""
    d = Deconvolver(ubar.shape, ndim, ubar.dtype, solver, device=ubar.device)
    u = _out(out, ubar.shape, ubar)
    t = TuneInfo()
    _check(d.lib.deconvolve_autotune(SOLVERS[solver], ctypes.byref(d.grid), _dev_ptr(ubar), _dev_ptr(u),
                                     d.work.data_ptr(), d.work.numel(), d.info_dev.data_ptr(),
                                     _stream_handle(stream), ctypes.byref(t)))
    return _tune_dict(t)


def _choice(tiles_per_wave=2, rows=0, tail_pct=0, interleave=0, wave_claims=0, blocks_per_cu=2,
            segments=0) -> TuneInfo:
    t = TuneInfo()
    t.tiles_per_wave, t.rows, t.tail_pct, t.interleave, t.wave_claims = (int(tiles_per_wave), int(rows), int(tail_pct),
                                                                         int(interleave), int(wave_claims))
    t.blocks_per_cu = int(blocks_per_cu)
    t.segments = int(segments)
    return t


def tune_set(solver: str, ubar: torch.Tensor, out: torch.Tensor, ndim: int = 2, **choice):
    """Pin the launch configuration for solves of `solver` on fields shaped
    like ubar whose input and output are aligned like ubar and out
    (gd_tune_set).  choice: tiles_per_wave, rows, tail_pct, interleave,
    wave_claims, blocks_per_cu (0: as many workgroups per CU as fit),
    segments (> 0: that many long tiles per column along the march axis)."""
    g = make_grid(ubar.shape, ndim, ubar.dtype)
    t = _choice(**choice)
    _check(load().gd_tune_set(SOLVERS[solver], ctypes.byref(g), _dev_ptr(ubar), _dev_ptr(out), ctypes.byref(t)))


def tune_reset():
    """Forget every tuning choice of this process (gd_tune_reset)."""
    load().gd_tune_reset()


@dataclass
class BatchResult:
    u: list
    info_dev: torch.Tensor
    history: list | None

    def info(self) -> list[dict]:
        """Per-instance outcome (synchronises with the device)."""
        return decode_info(self.info_dev.cpu().numpy())


class BatchDeconvolver:
    """Uneven batch: instance i is a 2D (ny, nx) or 3D (nz, ny, nx) field of
    its own size; all share solver and dtype.  One persistent launch solves
    them all (deconvolve_batch); ``solve`` only launches, so it can be timed or
    captured into a graph as long as the tensors it is given stay alive."""

    def __init__(self, shapes, dtype: torch.dtype, solver: str, device=None, h=None):
        self.lib = load()
        self.shapes = [tuple(int(v) for v in sh) for sh in shapes]
        if not self.shapes:
            raise ValueError("empty batch")
        self.dtype = dtype
        self.dt = F32 if dtype == torch.float32 else F64 if dtype == torch.float64 else -1
        if self.dt < 0:
            raise ValueError("fields must be float32 or float64")
        self.solver = solver
        self.count = len(self.shapes)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.list = (Instance * self.count)()
        for i, sh in enumerate(self.shapes):
            if len(sh) not in (2, 3):
                raise ValueError("instance shapes are (ny, nx) or (nz, ny, nx)")
            inst = self.list[i]
            inst.ndim = len(sh)
            rev = sh[::-1]
            for d in range(3):
                inst.n[d] = rev[d] if d < len(sh) else 1
                inst.h[d] = (h[i][d] if h is not None else 0.0) if d < len(sh) else 0.0
        n = self.lib.deconvolve_batch_workspace_bytes(SOLVERS[solver], self.dt, self.list, self.count)
        if n == 0:
            raise GdError(-1, "bad instance list or solver")
        self.work = torch.empty(int(n), dtype=torch.uint8, device=self.device)
        self.info_dev = torch.zeros(self.count * INFO_BYTES, dtype=torch.uint8, device=self.device)

    def _bind(self, ubars, us, histories):
        if len(ubars) != self.count or len(us) != self.count:
            raise ValueError(f"expected {self.count} fields")
        for i, (ub, u, sh) in enumerate(zip(ubars, us, self.shapes)):
            if tuple(ub.shape) != sh or tuple(u.shape) != sh or ub.dtype != self.dtype or u.dtype != self.dtype \
                    or ub.device != self.work.device or u.device != self.work.device:
                raise ValueError(f"instance {i}: fields must have shape {sh} and dtype {self.dtype} "
                                 f"on {self.work.device}")
            if histories is not None and histories[i].device != self.work.device:
                raise ValueError(f"instance {i}: history must be on {self.work.device}")
            self.list[i].ubar = _dev_ptr(ub)
            self.list[i].u = _dev_ptr(u)
            self.list[i].history = _dev_ptr(histories[i]) if histories is not None else None

    def solve(self, ubars, max_iter: int, tol: float = 0.0, init: str = "ubar", outs=None, norm_ref: str = "r0ubar",
              histories=None, wait_limit_us: int = 0, max_replace: int = 0, stream=None) -> BatchResult:
        if init in ("given", "warm") and outs is None:
            raise ValueError(f"init='{init}' reads the initial guesses from `outs`")
        us = [torch.empty_like(b) for b in ubars] if outs is None else list(outs)
        if histories is not None:
            if len(histories) != self.count:
                raise ValueError(f"expected {self.count} histories")
            for hst in histories:
                if hst.dtype != torch.float64 or hst.numel() < max_iter + 1:
                    raise ValueError("each history must be float64 with max_iter+1 entries")
        self._bind(ubars, us, histories)
        o = _make_opts(max_iter, tol, init, norm_ref, None, wait_limit_us, max_replace)
        _check(self.lib.deconvolve_batch(SOLVERS[self.solver], self.dt, self.list, self.count, ctypes.byref(o),
                                         self.work.data_ptr(), self.work.numel(), self.info_dev.data_ptr(),
                                         _stream_handle(stream)))
        return BatchResult(us, self.info_dev, histories)

    def tune_set(self, ubars, outs, **choice):
        """Pin this batch's launch configuration (gd_tune_set_batch)."""
        self._bind(ubars, outs, None)
        t = _choice(**choice)
        _check(self.lib.gd_tune_set_batch(SOLVERS[self.solver], self.dt, self.list, self.count, ctypes.byref(t)))

    def autotune(self, ubars, outs=None, stream=None) -> dict:
        """Tune this batch's launch (deconvolve_batch_autotune); ``outs`` are
        overwritten.  Synchronous."""
        us = [torch.empty_like(b) for b in ubars] if outs is None else list(outs)
        self._bind(ubars, us, None)
        t = TuneInfo()
        _check(self.lib.deconvolve_batch_autotune(SOLVERS[self.solver], self.dt, self.list, self.count,
                                                  self.work.data_ptr(), self.work.numel(), self.info_dev.data_ptr(),
                                                  _stream_handle(stream), ctypes.byref(t)))
        return _tune_dict(t)


def deconvolve_batch(solver: str, ubars, max_iter: int, tol: float = 0.0, init: str = "ubar", u0s=None,
                     norm_ref: str = "r0ubar", history: bool = False, wait_limit_us: int = 0, stream=None):
    """One-shot uneven-batch solve.  ``ubars``: list of 2D/3D tensors of one
    dtype.  Returns (list of u, infos, list of histories or None)."""
    b = BatchDeconvolver([t.shape for t in ubars], ubars[0].dtype, solver, device=ubars[0].device)
    outs = None
    if init in ("given", "warm"):
        if u0s is None:
            raise ValueError(f"init='{init}' needs u0s")
        outs = [t.clone() for t in u0s]
    hists = None
    if history:
        hists = [torch.full((max_iter + 1,), float("nan"), dtype=torch.float64, device=ubars[0].device)
                 for _ in ubars]
    res = b.solve(ubars, max_iter, tol, init=init, outs=outs, norm_ref=norm_ref, histories=hists,
                  wait_limit_us=wait_limit_us, stream=stream)
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return res.u, res.info(), hists


class WarmStart:
    """The learned warm start (warmstart_forward / warmstart_train_step): a
    periodic CNN (3x3 taps for ndim=2, 3x3x3 for ndim=3) whose output
    u0 = ubar + s * G^smooth f(ubar / s) starts a solve with init='warm' (the
    library falls back to ubar where u0 is no better).  With ``band`` (a
    band_project threshold, default BAND_TAU; None to skip) forward() keeps
    the correction inside ubar's Fourier support (power-of-two sizes).  Owns its
    FP32 parameters, Adam moments and step counter on the device.  ``params``:
    initial flat FP32/FP64 vector (for example synth.cnn_init_params(seed,
    ndim=ndim)).  Fields: (ny, nx) / (batch, ny, nx) in 2D, (nz, ny, nx) /
    (batch, nz, ny, nx) in 3D."""

    CHANNELS, LAYERS = 32, 6

    def __init__(self, params, device=None, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8, ndim: int = 2, smooth: int = 1, band: float | None = BAND_TAU):
        self.lib = load()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.ndim = ndim
        self.band = band
        self.net = Cnn()
        self.net.ndim, self.net.channels, self.net.layers = ndim, self.CHANNELS, self.LAYERS
        self.net.smooth = int(smooth)
        self.net.lr, self.net.beta1, self.net.beta2, self.net.eps = lr, beta1, beta2, eps
        n = int(self.lib.warmstart_param_count(ctypes.byref(self.net)))
        p = torch.as_tensor(np.asarray(params), dtype=torch.float32).reshape(-1)
        if p.numel() != n:
            raise ValueError(f"the network has {n} parameters, got {p.numel()}")
        self.params = p.to(self.device).contiguous()
        self.grad = torch.zeros_like(self.params)
        self.adam_m = torch.zeros_like(self.params)
        self.adam_v = torch.zeros_like(self.params)
        self.step = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.net.params, self.net.grad = self.params.data_ptr(), self.grad.data_ptr()
        self.net.adam_m, self.net.adam_v = self.adam_m.data_ptr(), self.adam_v.data_ptr()
        self.net.step = self.step.data_ptr()
        self._work = {}
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.device)

    def set_lr(self, lr: float):
        self.net.lr = float(lr)

    def _grid(self, x: torch.Tensor) -> Grid:
        if x.dim() not in (self.ndim, self.ndim + 1):
            raise ValueError(f"{self.ndim}D fields, with an optional leading batch dimension")
        return make_grid(x.shape, self.ndim, x.dtype)

    def _workspace(self, g: Grid, training: bool) -> torch.Tensor:
        key = (int(g.n[0]), int(g.n[1]), int(g.n[2]), int(g.batch), int(g.dtype), training)
        w = self._work.get(key)
        if w is None:
            n = self.lib.warmstart_workspace_bytes(ctypes.byref(self.net), ctypes.byref(g), int(training))
            if n == 0:
                raise GdError(-1, "bad network or grid")
            w = torch.empty(int(n), dtype=torch.uint8, device=self.device)
            self._work[key] = w
        return w

    def forward(self, ubar: torch.Tensor, out: torch.Tensor | None = None, stream=None,
                band: bool = True) -> torch.Tensor:
        """u0 for every field of ubar (launch only, no synchronisation); the
        band projection follows when self.band is set and ``band``."""
        g = self._grid(ubar)
        u0 = _out(out, ubar.shape, ubar)
        w = self._workspace(g, False)
        _check(self.lib.warmstart_forward(ctypes.byref(self.net), ctypes.byref(g), _dev_ptr(ubar), _dev_ptr(u0),
                                          w.data_ptr(), w.numel(), _stream_handle(stream)))
        if band and self.band is not None:
            key = ("band",) + tuple(ubar.shape) + (str(ubar.dtype),)
            bw = self._work.get(key)
            if bw is None:
                n = int(self.lib.band_project_workspace_bytes(ctypes.byref(g)))
                if n == 0:
                    raise GdError(-1, "the band projection needs power-of-two sizes (pass band=None)")
                bw = self._work[key] = torch.empty(n, dtype=torch.uint8, device=self.device)
            band_project(ubar, u0, self.ndim, self.band, work=bw, stream=stream)
        return u0

    def train_step(self, ubar: torch.Tensor, u: torch.Tensor, stream=None) -> torch.Tensor:
        """One Adam step on the pairs (ubar, u); returns the device loss (before
        the update).  Launch only."""
        if ubar.shape != u.shape or ubar.dtype != u.dtype or ubar.device != u.device:
            raise ValueError("ubar and u must match")
        g = self._grid(ubar)
        w = self._workspace(g, True)
        _check(self.lib.warmstart_train_step(ctypes.byref(self.net), ctypes.byref(g), _dev_ptr(ubar), _dev_ptr(u),
                                             w.data_ptr(), w.numel(), self.loss.data_ptr(), _stream_handle(stream)))
        return self.loss


def closure_stress(ubar: torch.Tensor, ustar: torch.Tensor, ndim: int, out: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
    """tau_ij = ubar_i ubar_j - G(u*_i u*_j) for i <= j (closure_stress).
    ubar, ustar: (..., ndim, [nz,] ny, nx) velocity fields (components in the
    dimension before the grid).  Returns (..., npairs, [nz,] ny, nx) with the
    pairs 11, 12, 22 (2D) or 11, 12, 13, 22, 23, 33 (3D).  Launch only."""
    if ubar.shape != ustar.shape or ubar.dtype != ustar.dtype:
        raise ValueError("ubar and ustar must match")
    if ubar.dim() < ndim + 1 or ubar.shape[-ndim - 1] != ndim:
        raise ValueError(f"the component dimension (before the grid) must have size {ndim}")
    lead = tuple(ubar.shape[:-ndim - 1])
    g = make_grid(lead + (1,) + tuple(ubar.shape[-ndim:]), ndim, ubar.dtype)
    np_ = ndim * (ndim + 1) // 2
    if ustar.device != ubar.device:
        raise ValueError("ubar and ustar must be on one device")
    tau = _out(out, lead + (np_,) + tuple(ubar.shape[-ndim:]), ubar)
    _check(load().closure_stress(ctypes.byref(g), _dev_ptr(ubar), _dev_ptr(ustar), _dev_ptr(tau),
                                 _stream_handle(stream)))
    return tau


def deconvolve(solver: str, ubar: torch.Tensor, max_iter: int, tol: float = 0.0, ndim: int = 2, init: str = "ubar",
               u0: torch.Tensor | None = None, norm_ref: str = "r0ubar", history: bool = False, h=None,
               wait_limit_us: int = 0, max_replace: int = 0, stream=None):
    """One-shot solve of G u = ubar.  Returns (u, infos, history or None).

    Synchronises the stream to read the per-field info records.
    """
    d = Deconvolver(ubar.shape, ndim, ubar.dtype, solver, device=ubar.device, h=h)
    out = None
    if init in ("given", "warm"):
        if u0 is None:
            raise ValueError(f"init='{init}' needs u0")
        out = u0.clone()
    hist = None
    if history:
        hist = torch.full((d.batch, max_iter + 1), float("nan"), dtype=torch.float64, device=ubar.device)
    res = d.solve(ubar, max_iter, tol, init=init, out=out, norm_ref=norm_ref, history=hist,
                  wait_limit_us=wait_limit_us, max_replace=max_replace, stream=stream)
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return res.u, res.info(), hist


def deconvolve_noalloc(solver: str, ubar: torch.Tensor, max_iter: int, info: torch.Tensor, tol: float = 0.0,
                       ndim: int = 2, init: str = "ubar", out: torch.Tensor | None = None, norm_ref: str = "r0ubar",
                       stream=None) -> torch.Tensor:
    """The solve with the library's fixed device workspace (deconvolve_noalloc):
    no allocation, no workspace argument.  ``info``: a device uint8 tensor of
    batch * INFO_BYTES (decode with decode_info after synchronising); ``out``:
    the result (read as the guess for init 'given' / 'warm').  Launch only.
    Calls on one GPU share one workspace: run them one after another."""
    lib = load()
    g = make_grid(ubar.shape, ndim, ubar.dtype)
    if info.dtype != torch.uint8 or info.numel() < int(g.batch) * INFO_BYTES or info.device != ubar.device:
        raise ValueError(f"info must be uint8 with batch*{INFO_BYTES} bytes on ubar's device")
    if init in ("given", "warm") and out is None:
        raise ValueError(f"init='{init}' reads the initial guess from `out`")
    u = _out(out, ubar.shape, ubar)
    o = _make_opts(max_iter, tol, init, norm_ref, None, 0)
    _check(lib.deconvolve_noalloc(SOLVERS[solver], ctypes.byref(g), _dev_ptr(ubar), _dev_ptr(u), ctypes.byref(o),
                                  _dev_ptr(info), _stream_handle(stream)))
    return u


def deconvolve_vancittert(ubar, max_iter, **kw):
    return deconvolve("vc", ubar, max_iter, **kw)


def deconvolve_cg(ubar, max_iter, **kw):
    return deconvolve("cg", ubar, max_iter, **kw)


def deconvolve_bicgstab(ubar, max_iter, **kw):
    return deconvolve("bicgstab", ubar, max_iter, **kw)


def deconvolve_steepest_descent(ubar, max_iter, **kw):
    return deconvolve("sd", ubar, max_iter, **kw)
