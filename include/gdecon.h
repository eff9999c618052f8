/*
 * gdecon.h -- C ABI of the MI355X deconvolution library (libgdecon.so).
 *
 * The library solves the approximate-deconvolution problem G u = ubar of
 * San & Vedula (Sec. 3, Eq. tau3) on periodic 2D and 3D grids.  G is the
 * separable 3-point trapezoidal low-pass filter with weights (1/4, 1/2, 1/4)
 * along every axis, applied matrix-free as a stencil; its Fourier transfer
 * function is prod_d cos^2(pi k_d / n_d).  The paper leaves G free (opening of
 * Sec. 4); it runs its own study with a spectral differential filter.
 *
 * Solvers: Van Cittert / Richardson (Algorithm 1), steepest descent
 * (Algorithm 2), conjugate gradient (Algorithm 3) and BiCGSTAB (Algorithm 4).
 *
 * Conventions for every entry point
 *   - Field pointers are DEVICE pointers.  Fields are C-contiguous with x
 *     fastest: 2D index i + nx*j, 3D index i + nx*(j + ny*k); field b of a
 *     batch starts at element b * nx*ny*nz.
 *   - The caller allocates and owns every buffer (inputs, outputs, workspace,
 *     info).  The library allocates no device memory and keeps no per-call
 *     state; its only global state is cached device properties and tuning
 *     choices, guarded by a mutex.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Every
 *     call is stream-ordered and returns without waiting for the GPU; results
 *     and `info` are valid once the stream has been synchronised.  A call
 *     launches only kernels (no memset or copy nodes), so it can be captured
 *     into a HIP graph.
 *   - Return value 0 = launched.  Negative values are argument or runtime
 *     errors detected BEFORE anything is launched (nothing is written then);
 *     gd_status_string() names them.  Convergence outcomes are not errors:
 *     they are reported per field in gd_info.status.
 *   - Inputs must not alias outputs (ubar vs u, x vs y).
 */
#ifndef GDECON_H
#define GDECON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* storage / arithmetic type of the fields */
enum { GD_F64 = 0, GD_F32 = 1 };

/* solvers: Algorithms 1-4 of the paper */
enum { GD_VANCITTERT = 0, GD_CG = 1, GD_BICGSTAB = 2, GD_STEEPEST_DESCENT = 3 };

/* initial guess: the paper's u0 = ubar (Algorithms 1-4), zero, the value
 * already in u (a warm start), or that value guarded by the paper's start:
 * with GD_INIT_WARM the solve starts from the guess in u only where its
 * residual ||ubar - G u0|| is finite and below ||ubar - G ubar||, and from
 * u0 = ubar otherwise (decided per field on the device; gd_info.start says
 * which start was used) */
enum { GD_INIT_UBAR = 0, GD_INIT_ZERO = 1, GD_INIT_GIVEN = 2, GD_INIT_WARM = 3 };

/* reference norm for the relative residual: ||ubar - G ubar|| (the paper's
 * initial residual, default) or ||ubar|| */
enum { GD_REF_R0UBAR = 0, GD_REF_UBAR = 1 };

/* return codes (negative) */
enum {
    GD_OK = 0,
    GD_EINVAL = -1,      /* bad ndim/dtype/size/enum, NULL pointer, aliasing */
    GD_EWORKSPACE = -2,  /* work == NULL or work_bytes too small */
    GD_EHIP = -3,        /* a HIP runtime call failed */
    GD_EALIGN = -4       /* workspace not 256-byte aligned */
};

/* per-field outcome, gd_info.status */
enum {
    GD_CONVERGED = 0,        /* ||r_n|| <= tol * r_ref, or r_n == 0 */
    GD_MAXITER = 1,          /* max_iter passes done (always the case for tol <= 0) */
    GD_BREAKDOWN_RHO = 2,    /* a zero denominator of alpha: (p,Gp), (f0,q), (r,Gr) or rho */
    GD_BREAKDOWN_OMEGA = 3,  /* BiCGSTAB: (t,t) == 0 with s != 0 */
    GD_NONFINITE = 4,        /* a NaN/Inf scalar (e.g. NaN in ubar) */
    GD_ZERO_REF = 5,         /* reference norm is zero: u = u0, no pass done */
    GD_TIMEOUT = 6,          /* the device-side grid barrier exceeded its wait bound */
    GD_STAGNATED = 7         /* the recursive residual met tol, but the true residual
                                ||ubar - G u|| stayed above tol * r_ref after every
                                residual replacement allowed (the rounding floor of
                                the storage precision) */
};

typedef struct gd_grid {
    int32_t ndim;   /* 2 or 3 */
    int32_t dtype;  /* GD_F64 or GD_F32 */
    int64_t n[3];   /* nx, ny, nz; each >= 1 (nz ignored when ndim == 2) */
    double h[3];    /* grid spacings for the inner product h^d sum a_i b_i
                       (the integral of Eq. inner); a value <= 0 means 2*pi/n */
    int64_t batch;  /* number of independent fields, >= 1, each with its own
                       scalars, iteration count and status */
} gd_grid;

typedef struct gd_opts {
    int32_t max_iter;   /* N: loop passes of Algorithms 1-4, >= 0 */
    int32_t init;       /* GD_INIT_* */
    int32_t norm_ref;   /* GD_REF_* */
    int32_t max_replace; /* residual replacements allowed per field: 0 = the
                           default (2), < 0 = none, > 0 = that many (see tol) */
    double tol;         /* > 0: after the first pass with ||r_n|| <= tol * r_ref
                           (r_n the recursive residual of the algorithm), the
                           true residual ||ubar - G u_n|| is evaluated in FP64
                           arithmetic; the field stops with GD_CONVERGED if it is
                           <= tol * r_ref too, else r is replaced by that true
                           residual, CG and BiCGSTAB restart from u_n (p = r,
                           BiCGSTAB's shadow f0 = r), and the iteration goes on.
                           When no replacement is left, the field stops with
                           GD_STAGNATED.  <= 0: run exactly max_iter passes
                           (unless a guard stops earlier) */
    double *history;    /* NULL, or device [batch][max_iter + 1] doubles:
                           history[b][n] = ||r_n|| (recursive residual,
                           h-weighted) for n <= iters; later entries untouched */
    int64_t wait_limit_us; /* bound on one grid-barrier wait; 0 = default
                              (10 s).  Exceeding it ends the kernel with
                              GD_TIMEOUT in every info. */
} gd_opts;

/* one per field, written by the device at the end of a solve (48 bytes) */
typedef struct gd_info {
    int32_t iters;   /* passes completed */
    int32_t status;  /* GD_CONVERGED ... */
    double r_ref;    /* reference norm */
    double r0;       /* ||r_0|| of the start used */
    double r_final;  /* ||r_iters|| (recursive residual) */
    double r_true;   /* ||ubar - G u|| recomputed at exit, FP64 arithmetic */
    int32_t start;   /* start used: GD_INIT_UBAR, GD_INIT_ZERO or GD_INIT_GIVEN
                        (GD_INIT_WARM resolves to GIVEN or, on fallback, UBAR) */
    int32_t replaced; /* residual replacements done */
} gd_info;

/*
 * y = G x for every field of the batch (the filter of Eq. tau3, applied as a
 * periodic stencil).  x, y: device, grid->batch fields of grid->dtype.
 * Errors: GD_EINVAL (bad grid, NULL, x == y).
 */
int filter_apply(const gd_grid *grid, const void *x, void *y, void *stream);

/*
 * Bytes of device workspace the solver needs for this grid (0 on a bad
 * grid/solver).  The workspace must be 256-byte aligned; its contents on entry
 * do not matter and are clobbered.
 */
size_t deconvolve_workspace_bytes(const gd_grid *grid, int32_t solver);

/*
 * Solve G u = ubar for every field of the batch.
 *   ubar  device, input, grid->batch fields (not modified)
 *   u     device, output; read on entry only when opts->init == GD_INIT_GIVEN
 *   opts  host pointer; see gd_opts
 *   work  device workspace of at least deconvolve_workspace_bytes() bytes
 *   info  device, grid->batch gd_info records (output)
 * Inner products, norms and the scalars alpha, beta, omega, rho are FP64 on the
 * device for both dtypes; with GD_F32 the stencil and the vector updates run in
 * FP32 (the precision mode).  The whole iteration loop, convergence test
 * included, runs on the device in one persistent launch.
 *
 * Van Cittert, Algorithm 1: u_{n+1} = u_n + r_n, r_{n+1} = r_n - G r_n.
 */
int deconvolve_vancittert(const gd_grid *grid, const void *ubar, void *u, const gd_opts *opts,
                          void *work, size_t work_bytes, gd_info *info, void *stream);

/* Conjugate gradient, Algorithm 3 (Eqs. cg1 - cg-b): alpha = rho/(p, Gp),
 * beta = rho_{n+1}/rho_n.  Same arguments as deconvolve_vancittert. */
int deconvolve_cg(const gd_grid *grid, const void *ubar, void *u, const gd_opts *opts,
                  void *work, size_t work_bytes, gd_info *info, void *stream);

/* BiCGSTAB, Algorithm 4, with the frozen shadow residual f0 = r0.  Same
 * arguments as deconvolve_vancittert.  If ||s|| <= tol * r_ref (or s == 0)
 * after the alpha half step, the solver takes u += alpha p, r = s and stops
 * with GD_CONVERGED. */
int deconvolve_bicgstab(const gd_grid *grid, const void *ubar, void *u, const gd_opts *opts,
                        void *work, size_t work_bytes, gd_info *info, void *stream);

/* Steepest descent, Algorithm 2 (Eq. sd-a): alpha = (r, r)/(r, Gr).  Same
 * arguments as deconvolve_vancittert. */
int deconvolve_steepest_descent(const gd_grid *grid, const void *ubar, void *u, const gd_opts *opts,
                                void *work, size_t work_bytes, gd_info *info, void *stream);

/*
 * ---- The solve without a workspace argument -----------------------------------
 *
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): the solve of
 * deconvolve_vancittert / _cg / _bicgstab / _steepest_descent (solver =
 * GD_VANCITTERT ... GD_STEEPEST_DESCENT) with its workspace (grid-barrier
 * state, per-field scalars, partial sums, work vectors) in a fixed device
 * array of deconvolve_noalloc_max_bytes() bytes (32 MiB) that the library
 * holds on every GPU it runs on until the process ends.  The caller passes
 * the inputs and outputs only; the arguments, results and info records are
 * those of the solver's own entry point, bit for bit.  Nothing is allocated:
 * the call launches the same kernels.  A solve whose workspace
 * (deconvolve_workspace_bytes) exceeds the array is rejected with
 * GD_EWORKSPACE before any launch: for BiCGSTAB that allows about 2^20 FP32
 * or 2^19 FP64 points in the whole batch.  Every call on one GPU uses that
 * GPU's one array, which keeps the last call's contents: calls that overlap
 * on one GPU (different streams, or host threads) race and corrupt each
 * other, so serialise them (one stream).  Errors: those of the solver's
 * entry point, GD_EWORKSPACE (too large), GD_EHIP.
 */
size_t deconvolve_noalloc_max_bytes(void);
int deconvolve_noalloc(int32_t solver, const gd_grid *grid, const void *ubar, void *u, const gd_opts *opts,
                       gd_info *info, void *stream);

/*
 * ---- Uneven batches: many independent fields of different sizes ----------
 *
 * One persistent launch solves every instance of the list, each with its own
 * grid, scalars, iteration count and status; the instances share the solver,
 * the dtype and the options.  Results equal what the single-grid entry points
 * compute for each instance up to the summation order of the dot products
 * (tiles are split differently), and are reproducible call to call.
 */
typedef struct gd_instance {
    int32_t ndim;        /* 2 or 3 */
    int32_t reserved;    /* set to 0 */
    int64_t n[3];        /* nx, ny, nz; each >= 1 (nz ignored when ndim == 2) */
    double h[3];         /* spacings of the inner product; <= 0 means 2*pi/n */
    const void *ubar;    /* device, input field (not modified) */
    void *u;             /* device, output field; read on entry only with
                            GD_INIT_GIVEN */
    double *history;     /* NULL or device [max_iter + 1] doubles (see gd_opts) */
} gd_instance;

/* Workspace bytes for a batch (0 on a bad list).  256-byte aligned buffer,
 * clobbered.  Depends only on the solver, dtype and the instance sizes. */
size_t deconvolve_batch_workspace_bytes(int32_t solver, int32_t dtype, const gd_instance *list, int32_t count);

/*
 * Solve G u = ubar for every instance of `list` (host array of `count`
 * descriptors, read during the call only) with `solver` (GD_VANCITTERT ...)
 * in one persistent launch on `stream`.  opts->history is ignored; each
 * instance names its own.  info: device, `count` records.  The instance
 * table is written into the workspace by kernels (no copy from host memory),
 * so the call can be captured into a HIP graph; a replay re-solves the same
 * pointers.  Errors: GD_EINVAL (bad list entry, overlapping fields, count < 1),
 * GD_EWORKSPACE, GD_EALIGN, GD_EHIP.
 */
int deconvolve_batch(int32_t solver, int32_t dtype, const gd_instance *list, int32_t count, const gd_opts *opts,
                     void *work, size_t work_bytes, gd_info *info, void *stream);

/*
 * ---- Autotuner -------------------------------------------------------------
 *
 * Times the candidate launch configurations of a solve (tile granularity:
 * target tiles per resident wave; the share of short tiles claimed at the end
 * of every sweep; the tile-pool layout; per-wave or per-workgroup tile
 * claims; workgroups per CU; 3D rows per tile where the uniform kernels offer
 * a choice) with short fixed-length trial solves on the caller's buffers and
 * remembers the fastest for this (solver, dtype, sizes) signature.  Later deconvolve_* / deconvolve_batch calls with the same
 * signature use it.  With the environment variable GD_TUNE_CACHE naming a
 * file, choices are also appended there and read back by later processes.
 * Synchronous (waits for the stream); not for use under graph capture.
 * `u` (every instance's u) is overwritten by the trials; `info` receives the
 * last trial's records.
 */
typedef struct gd_tune_info {
    int32_t candidates;      /* configurations timed */
    int32_t best;            /* index of the fastest */
    int32_t tiles_per_wave;  /* chosen tile granularity */
    int32_t rows;            /* chosen 3D rows per tile (0 = default rule) */
    int32_t tail_pct;        /* chosen percent of each column cut into short tiles */
    int32_t interleave;      /* chosen tile-pool layout: 0 contiguous shares
                                (halo reuse in L2), 1 interleaved over the XCDs */
    int32_t wave_claims;     /* 1: every wave claims its own tiles; 0: a
                                workgroup claims tiles for its four waves */
    int32_t blocks_per_cu;   /* chosen workgroups per CU of the persistent grid
                                (0 = as many as fit; at most 16) */
    int32_t segments;        /* chosen long tiles per column along the march
                                axis (1 .. 64), whatever the wave count; 0 =
                                as many as keep every resident wave busy.
                                Uniform solves only (uneven batches ignore
                                it); the tuner tries it for 3D fields. */
    int32_t pad;
    double best_ms;          /* trial time of the chosen configuration (the
                                leaders' round: solves of 8 Krylov or 20 Van
                                Cittert / steepest-descent passes) */
    double default_ms;       /* the same trial's time for the untuned default */
} gd_tune_info;

int deconvolve_autotune(int32_t solver, const gd_grid *grid, const void *ubar, void *u, void *work, size_t work_bytes,
                        gd_info *info, void *stream, gd_tune_info *out);
int deconvolve_batch_autotune(int32_t solver, int32_t dtype, const gd_instance *list, int32_t count, void *work,
                              size_t work_bytes, gd_info *info, void *stream, gd_tune_info *out);

/* Pin the launch configuration of a signature without timing anything (for
 * reproducible runs): later solves with the same solver, grid and pointer
 * alignment (the alignment of ubar and u decides the lane width), or the same
 * instance list, use `choice` (its tiles_per_wave, rows, tail_pct,
 * interleave, wave_claims, blocks_per_cu and segments; the timing fields are ignored).  Also written to the
 * GD_TUNE_CACHE file when it is set.  Errors: GD_EINVAL. */
int gd_tune_set(int32_t solver, const gd_grid *grid, const void *ubar, const void *u, const gd_tune_info *choice);
int gd_tune_set_batch(int32_t solver, int32_t dtype, const gd_instance *list, int32_t count,
                      const gd_tune_info *choice);

/* Forget every tuning choice made or loaded by this process. */
void gd_tune_reset(void);

/*
 * ---- Learned warm start -----------------------------------------------------
 *
 * The paper starts every deconvolution from u0 = ubar.  The warm start
 * predicts a better u0 with a small periodic convolutional network and hands
 * it to a solver with GD_INIT_WARM (the solver itself is unchanged; the
 * paper's start stays the fallback: a field whose predicted start has a
 * residual no smaller than ubar's, or a non-finite one, starts from ubar):
 *     s  = RMS of ubar over the field,  x0 = ubar / s,
 *     a_l = relu(conv_l(a_{l-1}))  for l = 1..5,   y = G^m conv_6(a_5),
 *     u0 = ubar + s * y,
 * conv_l a periodic 3x3 (gd_cnn.ndim == 2) or 3x3x3 (ndim == 3)
 * cross-correlation with bias, channels 1 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1,
 * G the trapezoidal deconvolution filter applied m = gd_cnn.smooth times (so
 * the correction lies in the range of G, like the paper's start ubar, and
 * the network's rounding noise is damped by G_hat^m where the fields have no
 * content).  Activations are bfloat16, the 32 -> 32 layers run on the matrix
 * cores with FP32 accumulation.  The grid's ndim must equal the network's;
 * batch = number of fields.  Before the solve, band_project (below) removes
 * the correction's content where ubar has none; the differential-filter
 * solve does that itself for a GD_INIT_WARM start.
 *
 * Parameters: one FP32 vector, layer by layer, each W[cout][tap][cin] with
 * tap = 3*(dy+1) + (dx+1) for the offset (dy, dx) in y and x (in 3D
 * 9*(dz+1) + 3*(dy+1) + (dx+1)), then bias[cout].
 */
typedef struct gd_cnn {
    int32_t ndim;      /* 2 or 3 */
    int32_t channels;  /* 32 */
    int32_t layers;    /* 6 */
    int32_t smooth;    /* m, applications of G to the network's output, 1 .. 8
                          (0 means 1) */
    float lr, beta1, beta2, eps;  /* Adam hyper-parameters (training only) */
    float *params;     /* device, warmstart_param_count() FP32 values (in/out) */
    float *grad;       /* device, same size, or NULL: the gradient of the last
                          training step is written here (else into the workspace) */
    float *adam_m;     /* device, same size, zero before the first step */
    float *adam_v;     /* device, same size, zero before the first step */
    int32_t *step;     /* device, one int: Adam steps taken (0 before the first) */
} gd_cnn;

/* Number of FP32 parameters (37601 in 2D, 112481 in 3D), or 0 for an
 * unsupported shape. */
int64_t warmstart_param_count(const gd_cnn *net);

/* Workspace bytes for warmstart_forward (training == 0) or
 * warmstart_train_step (training != 0) on this grid; 0 on bad arguments. */
size_t warmstart_workspace_bytes(const gd_cnn *net, const gd_grid *grid, int32_t training);

/* u0 = network(ubar) for every field of the batch.  ubar, u0: device fields of
 * grid->dtype (FP32 or FP64; the network itself runs in bfloat16/FP32).
 * Errors: GD_EINVAL (grid and network of different ndim, unsupported network
 * shape, NULL), GD_EWORKSPACE,
 * GD_EALIGN. */
int warmstart_forward(const gd_cnn *net, const gd_grid *grid, const void *ubar, void *u0, void *work,
                      size_t work_bytes, void *stream);

/* One training step on the pairs (ubar[b], u[b]): forward, the loss
 * mean over all points of (y - (u - ubar)/s)^2 written to *loss (device
 * double), backpropagation (gradient into net->grad when non-NULL), then one
 * Adam update of net->params (bias-corrected with *net->step + 1, after which
 * *net->step is incremented on the device).  Stream-ordered, capturable. */
int warmstart_train_step(const gd_cnn *net, const gd_grid *grid, const void *ubar, const void *u, void *work,
                         size_t work_bytes, double *loss, void *stream);

/*
 * ---- Van Cittert with several passes per sweep ----------------------------------
 *
 * Algorithm 1 with the trapezoidal stencil, computed K passes at a time
 * (temporal blocking): a tile of r with a K-point halo is advanced K passes in
 * LDS while u accumulates the residuals, so one read and one write of u and r
 * serve K passes.  Arguments, options, results and info records are those of
 * deconvolve_vancittert.  The stopping rule acts after every pass: a field
 * that stops inside a sweep has that sweep recomputed with the exact pass
 * count, so pass counts, statuses and histories match the one-pass solve.
 * Any grid size.  vancittert_blocked_passes() gives K (8 in 2D, 2 in 3D).
 * The call is a sequence of 2 ceil(max_iter / K) + 7 stream-ordered launches
 * (one more with a history), so max_iter is limited to 2^20 (GD_EINVAL
 * above); a launch after every field has stopped costs one state read per
 * tile.
 */
size_t vancittert_blocked_workspace_bytes(const gd_grid *grid);
int32_t vancittert_blocked_passes(const gd_grid *grid);
int deconvolve_vancittert_blocked(const gd_grid *grid, const void *ubar, void *u, const gd_opts *opts, void *work,
                                  size_t work_bytes, gd_info *info, void *stream);

/*
 * ---- The paper's differential filter ----------------------------------------
 *
 * The results section filters with G = (I - delta^2 lap)^-1 (Sec. 4, Eq. df),
 * applied through the FFT, with transfer function
 *     G_hat(k) = 1 / (1 + (|k| / k_c)^2),  delta = 1 / k_c,  k_c = gamma k_m
 * (Eq. df2); the domain is 2 pi periodic, so k is the integer wavenumber
 * vector, and k_m = min_d n_d / 2.  Sizes must be powers of two in [2, 4096]
 * (GD_F32) or [2, 2048] (GD_F64).  grid->h is used as in deconvolve_* (the
 * weight of the inner products).
 *
 * germano_workspace_bytes(grid, solver): bytes for deconvolve_germano with
 *   that solver, or with solver = -1 for germano_filter_apply; 0 if the grid
 *   is not supported.
 * germano_filter_apply(grid, gamma, x, y, work, work_bytes, stream):
 *   y = G x for every field of the batch (x, y device, same layout as
 *   filter_apply; they may be the same buffer).
 * deconvolve_germano(solver, grid, gamma, ubar, u, opts, work, work_bytes,
 *   info, stream): Algorithm 1, 2, 3 or 4 (solver = GD_VANCITTERT ...
 *   GD_STEEPEST_DESCENT) with this G, same arguments, options, results and
 *   info records as deconvolve_*.  The iteration runs on the Fourier
 *   coefficients (G diagonal there; inner products by Parseval's identity),
 *   between one forward FFT of ubar (and of u when opts->init is
 *   GD_INIT_GIVEN or GD_INIT_WARM) and one inverse FFT of the result; r_true
 *   is evaluated there too.  A GD_INIT_WARM start is band-projected on its
 *   coefficients first (band_project's P with tau = 1e-10, see below: free
 *   here), then judged against the ubar start.  Stream-ordered.
 * Errors: GD_EINVAL (unsupported size, gamma <= 0, NULL, overlaps),
 * GD_EWORKSPACE, GD_EALIGN (workspace not 256-byte aligned), GD_EHIP.
 */
size_t germano_workspace_bytes(const gd_grid *grid, int32_t solver);
int germano_filter_apply(const gd_grid *grid, double gamma, const void *x, void *y, void *work, size_t work_bytes,
                         void *stream);
int deconvolve_germano(int32_t solver, const gd_grid *grid, double gamma, const void *ubar, void *u,
                       const gd_opts *opts, void *work, size_t work_bytes, gd_info *info, void *stream);
/* As deconvolve_autotune, for deconvolve_germano with this grid and solver:
 * times the launch configurations of the solve on the Fourier coefficients
 * of ubar and remembers the fastest.  The trials run on the workspace: u
 * (non-NULL, as for deconvolve_germano) is not written, and ubar must not
 * overlap the workspace.  Synchronous. */
int deconvolve_germano_autotune(int32_t solver, const gd_grid *grid, double gamma, const void *ubar, void *u,
                                void *work, size_t work_bytes, gd_info *info, void *stream, gd_tune_info *out);

/*
 * ---- A-priori diagnostics -------------------------------------------------------
 *
 * The paper judges recovered fields by their energy spectra and by the PDFs
 * of their values (Sec. 4, the spectra and PDF figures of the 2D and 3D
 * cases).  With f_hat(k) = (1/N) sum_x f(x) exp(-i k.x) (integer wavenumbers
 * of the 2 pi periodic grid):
 *   energy_spectrum: out[b][s] = 1/2 sum over the wavenumbers whose |k|
 *     rounds to s of |k|^kpow |f_hat(k)|^2, s = 0 .. spectrum_shells() - 1
 *     (kpow = 0: the spectrum of f, summing to mean(f^2)/2; kpow = -2 turns a
 *     2D vorticity field into its kinetic energy spectrum, k = 0 then adding
 *     nothing).  Power-of-two sizes as for the differential filter.  out is
 *     device FP64 [batch][nshells]; work of spectrum_workspace_bytes().
 *   pdf_counts: counts[b][i] = number of points of field b whose value v has
 *     floor((v - lo) * (nbins / (hi - lo))) = i (evaluated in FP64), v = hi in
 *     the last bin, values outside [lo, hi] and NaN not counted.  Any grid
 *     size; 1 <= nbins <= 8192; counts is device int64 [batch][nbins],
 *     cleared by the call (by a kernel, so it can be captured).
 * Stream-ordered.  Errors: GD_EINVAL, GD_EWORKSPACE, GD_EALIGN, GD_EHIP.
 */
int32_t spectrum_shells(const gd_grid *grid);
size_t spectrum_workspace_bytes(const gd_grid *grid);
int energy_spectrum(const gd_grid *grid, double kpow, const void *x, double *out, void *work, size_t work_bytes,
                    void *stream);
int pdf_counts(const gd_grid *grid, double lo, double hi, int32_t nbins, const void *x, int64_t *counts,
               void *stream);

/*
 * ---- Band projection of a start ---------------------------------------------------
 *
 * G is diagonal in Fourier space for both filters (transfer functions
 * prod_d cos^2(pi k_d / n_d) and Eq. df2), so the
 * exact solution of G u = ubar has content only at the wavenumbers where ubar
 * has.  A start u0 that puts content anywhere else (a learned start's error)
 * leaves a residual there that the Krylov solvers remove slowly, because G_hat
 * is small outside the band of a filtered field.  band_project removes it:
 *     u0 <- ubar + P (u0 - ubar),
 * P keeping the Fourier modes k of field b with |ubar_hat(k)|^2 > tau * E_b,
 * E_b the mean of |ubar_hat(k)|^2 over all wavenumbers (Parseval: the mean of
 * ubar^2 times the point count), and zeroing the others.  tau = 0 keeps every
 * mode at which ubar is nonzero.  Computed by FFT (the differential filter's
 * transforms), in grid->dtype with FP64 power sums; power-of-two sizes as for
 * the differential filter.  ubar, u0: device fields of the grid (u0 in/out,
 * not overlapping ubar); work of band_project_workspace_bytes() (0 for an
 * unsupported grid).  Stream-ordered.
 * Errors: GD_EINVAL (size, tau < 0 or not finite, NULL, overlaps),
 * GD_EWORKSPACE, GD_EALIGN, GD_EHIP.
 */
size_t band_project_workspace_bytes(const gd_grid *grid);
int band_project(const gd_grid *grid, double tau, const void *ubar, void *u0, void *work, size_t work_bytes,
                 void *stream);

/*
 * ---- Closure stress ----------------------------------------------------------
 *
 * The sub-filter stress of the filtered equations, tau_ij = ubar_i ubar_j -
 * G(u_i u_j) (Sec. 2, Eq. fge3), closed by approximate deconvolution with the
 * deconvolved velocity u* in place of u (Sec. 3, Eq. tau3):
 *     tau_ij = ubar_i ubar_j - G(u*_i u*_j),   i <= j.
 * A velocity field has grid->ndim components; grid->batch is the number of
 * velocity fields.
 *   ubar, ustar  device, [batch][ndim][points] (component c of field b at
 *                offset (b * ndim + c) * points)
 *   tau          device, output, [batch][npairs][points], pairs in the order
 *                11, 12, 22 (2D) or 11, 12, 13, 22, 23, 33 (3D)
 * One fused pass; stream-ordered.  Errors: GD_EINVAL (bad grid, NULL, tau
 * overlapping an input), GD_EHIP.
 */
int closure_stress(const gd_grid *grid, const void *ubar, const void *ustar, void *tau, void *stream);

/* Human-readable name of a return code (< 0) or of a gd_info status (>= 0). */
const char *gd_status_string(int32_t code);

/* Text of the last error a call on this host thread returned (or ""). */
const char *gd_last_error(void);

/* Launch shape of the last solve launched from this host thread: tile lane
 * width (vw elements), rows per tile (R, 3D), planes per tile along the march
 * axis (L), tile count, and the persistent grid (workgroups, waves).  For
 * tests and performance reports. */
typedef struct gd_launch_info {
    int32_t variant, vw, R, reserved;
    int64_t L, tiles, blocks, waves;
} gd_launch_info;
int gd_last_launch(gd_launch_info *out);

/* Diagnostics: while set, every solve records, for its k-th grid barrier,
 * buf[4k] = first arrival, buf[4k+1] = last arrival, buf[4k+2] = release and
 * buf[4k+3] = latest per-field reduction, in device wall-clock ticks
 * (hipDeviceAttributeWallClockRate kHz), for 4k + 3 < capacity.  The caller
 * initialises buf (first arrival to UINT64_MAX, the others to 0) before each
 * solve.  buf: device memory of `capacity` uint64 entries; NULL switches
 * recording off. */
int gd_set_trace(uint64_t *buf, int64_t capacity);

#ifdef __cplusplus
}
#endif
#endif /* GDECON_H */
