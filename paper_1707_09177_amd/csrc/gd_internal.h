// gd_internal.h -- structures shared by the solver kernels and the host driver.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <climits>

#include "gd_device.h"
#include "gdecon.h"

namespace gd {

// Tile variants: a kernel is compiled for one (ndim, vw, R) shape, coded as
// ndim*100 + vw*10 + R, or for VAR_ALL (shape chosen per instance).  A uniform
// batch finds instance i by offsetting instance 0; kTableBit + shape is the
// same shape reading per-instance descriptors from a table (uneven batches
// whose instances share one shape); VAR_ALL always reads the table.
// kSpecBit + shape is the same shape run on a stored Fourier spectrum, with G
// the pointwise transfer function of the differential filter.
constexpr int VAR_ALL = 0;
constexpr int kTableBit = 1000;
constexpr int kSpecBit = 5000;
__host__ __device__ constexpr int var_code(int ndim, int vw, int R) { return ndim * 100 + vw * 10 + R; }
__host__ __device__ constexpr bool var_table(int c) { return c == VAR_ALL || (c % kSpecBit) >= kTableBit; }
__host__ __device__ constexpr bool var_spec(int c) { return c >= kSpecBit; }
__host__ __device__ constexpr int var_ndim(int c) { return (c % kTableBit) / 100; }
__host__ __device__ constexpr int var_vw(int c) { return (c / 10) % 10; }
__host__ __device__ constexpr int var_r(int c) { return c % 10; }

// solver vectors kept in the workspace (u and ubar are the caller's)
enum { V_R0 = 0, V_R1 = 1, V_P0 = 2, V_P1 = 3, V_Q0 = 4, V_Q1 = 5, V_F0 = 6, NVEC = 7 };

// sweeps of the persistent kernel
enum Phase : int {
    PH_RREF_UBAR = 0,  // ||ubar||^2
    PH_RREF_RES,       // ||ubar - G ubar||^2
    PH_INIT_UBAR,      // u0 = ubar
    PH_INIT_ZERO,      // u0 = 0
    PH_INIT_GIVEN,     // u0 from the caller
    PH_VC,             // Algorithm 1 pass
    PH_CG1,            // Algorithm 3: p, G p, (p, G p)
    PH_CG2,            // Algorithm 3: u, r, (r, r)
    PH_BIA,            // Algorithm 4: p, q = G p, (f0, q)
    PH_BIB,            // Algorithm 4: s, t = G s, (s,t) (t,t) (s,s)
    PH_BIC,            // Algorithm 4: u, r, (f0, r) (r, r)
    PH_SD1,            // Algorithm 2: (r, G r)
    PH_SD2,            // Algorithm 2: u, r, (r, r)
    PH_TRUE,           // ||ubar - G u||^2 in FP64, writes gd_info
    PH_VERIFY,         // ||ubar - G u||^2 in FP64 once the recursive residual met tol
    PH_REPLACE         // r = ubar - G u in FP64 arithmetic (stored), f0 = r, (r, r)
};

// Device descriptor of one field (instance) of a solve.
struct Inst {
    const void *ubar;
    void *u;
    void *vec[NVEC];
    double *hist;
    gd_info *info;
    Geo geo;
    int64_t tile0, ntiles;  // partial-sum slots [tile0, tile0 + ntiles) of this instance
    int64_t b0, s0;         // first long / short tile in the claim order (table mode)
    double hw;              // h^d of the inner product
    int32_t ndim, vw, R;
    // spectral solves: 1 / k_c^2 of the differential filter; the stored half
    // spectrum [k_z][k_y][row of nxs reals] has nxc = n_x / 2 + 1 complex
    // columns, and log2 n_y, log2 n_z (each point's wavenumber comes from its
    // index within the field, whatever tile geometry sweeps it)
    int32_t lny;
    double inv_kc2;
    int32_t nxc, nxs, lnz, pad;
};

// FP64 scalars of one instance, written by the wave that completes the
// instance's last tile of a sweep.  `cnt` counts the tiles of the current
// sweep that have published their partial sums.  The flags select which
// instances the control sweeps work on: `verify` (the recursive residual met
// tol: PH_VERIFY), `replace` (the true residual did not: PH_REPLACE),
// `restart` (the next pass starts a fresh Krylov sequence), `fallback` (a
// warm start's guess was rejected: PH_INIT_UBAR); `tknown` marks an instance
// whose info record is already written (PH_TRUE skips it).
struct alignas(128) State {
    double alpha, beta, omega, rho, rr, r_ref, r0;
    double r_ub;  // ||ubar - G ubar||: the warm start's acceptance bound
    int32_t iters, status, done, half;
    uint32_t cnt;
    int32_t verify, replace, restart, fallback, tknown, nrep, start;
};
static_assert(sizeof(State) == 128, "State is one 128-byte line");

// Grid-barrier state.  Workgroups arrive in NGRP groups (workgroup b is in
// group b % NGRP), each with its own counter and its own release flag on a
// separate 128-byte line, so that arrivals and polling spread over many
// memory channels instead of serialising on one address.
constexpr int NGRP = 32;
struct alignas(128) SyncLine {
    uint32_t v;
    uint32_t pad[31];
};
// Counters of instances in each control state, and their per-barrier
// snapshot: every workgroup takes its loop decisions from the snapshot of the
// barrier it has just passed, never from the live counters (which the next
// sweep's reductions already change).
struct alignas(128) Counts {
    int32_t active;    // instances still iterating
    int32_t verify;    // instances whose true residual is to be checked
    int32_t replace;   // instances whose residual is to be replaced
    int32_t fallback;  // warm starts rejected, to be restarted from ubar
    int32_t ntrue;     // finished instances that still need the exit true residual
    int32_t pad[27];
};
struct Sync {
    uint32_t top;    // groups complete at the current barrier
    uint32_t abort;  // set when a wait exceeded its bound
    uint32_t pad[30];
    Counts live;
    SyncLine cnt[NGRP];  // arrivals per group at the current barrier
    SyncLine gen[NGRP];  // completed barriers, one copy per group
    // tile pools of a sweep: the tiles are split into ng contiguous pools and
    // pool[par][p] counts the tiles of pool p taken so far in a sweep of
    // parity par (sweeps alternate between the two sets)
    SyncLine pool[2][NGRP];
    // the counters after barrier k, in slot k & 1
    Counts snap[2];
    // claims in each tile pool (written by the prep kernel for the launch's
    // pool count), read when a workgroup looks for pools to steal from
    int64_t pcnt[NGRP];
};

// A workgroup drains its own group's pool, then helps with the others.
constexpr int kSteal = NGRP;
// Target tiles per resident wave: the dynamic pools need several per wave to
// even out the per-wave speed differences at the end of a sweep.
constexpr int kTilesPerWave = 2;
// Percent of every column's planes cut into short tiles (claimed last).
constexpr int kTailPct = 15;
// Workgroups per CU of the persistent grid (0: as many as fit).  Two waves
// per SIMD measured faster than three for the 2D kernels, which fit three
// (16 x 2048^2 FP32: BiCGSTAB 4.47 against 4.89 ms, CG 3.72 against 4.66 ms);
// most 3D and uneven-batch kernels fit two anyway.
constexpr int kBlocksPerCu = 2;
constexpr int kMaxBlocksPerCu = 16;
// Largest tiles-per-column choice a launch configuration may pin.
constexpr int kMaxSegs = 64;

struct Params {
    Inst tmpl;            // uniform batch: instance 0 (others offset by stride)
    const Inst *table;    // uneven batch: one Inst per instance (device)
    State *st;
    Sync *sync;
    double *part;         // [tile][NACC] partial sums
    int64_t stride_bytes; // uniform batch: bytes between consecutive fields
    int64_t tiles_per_inst;
    int64_t total_tiles;
    int64_t big_total;    // tiles are claimed long ones first (all instances), then short ones
    int64_t wait_ticks;   // bound on one barrier wait, wall-clock ticks
    double tol;
    int32_t ninst, init, norm_ref, max_iter;
    int32_t hist_stride;
    int32_t max_replace;  // residual replacements per instance (0: none)
    // optional diagnostics: per barrier k, trace[4k..4k+3] = first arrival,
    // last arrival, release, latest instance completion (wall-clock ticks)
    unsigned long long *trace;
    int64_t trace_cap;
    int32_t steal;       // pools a wave visits (its own first)
    int32_t interleave;  // pool layout: 0 contiguous shares, 1 tiles pl, pl + ng, ...
    int32_t npools;      // tile pools of the launch: min(workgroups, NGRP)
    int32_t wave_claims; // 1: every wave claims its own tiles; 0: a workgroup claims for its waves
    int32_t solver;      // GD_VANCITTERT ... (where a replaced residual is stored)
    int32_t pad2;
};

// Launch configuration the autotuner chooses between: target tiles per
// resident wave (tile granularity) and, for 3D fields in the uniform kernels,
// rows per tile (0 = the default rule) and tiles per column along the march
// axis (0 = the wave-count rule).
struct TuneCfg {
    int tpw = kTilesPerWave;
    int rows = 0;
    int tail = kTailPct;
    int ilv = 0;  // interleaved tile pools
    int wc = 0;   // per-wave tile claims
    int bpc = kBlocksPerCu;  // workgroups per CU (0: as many as fit)
    int segs = 0;  // > 0: every column is cut into this many long tiles, whatever the wave count
};

// A solve on a stored Fourier spectrum (the differential filter); hw is the
// inner product's weight of the grid the spectrum came from.
struct SpecParams {
    double inv_kc2, hw;
    int64_t nxc, nxs;
    int32_t lny, lnz;
};

// Tile shape of a field: lanes hold vw consecutive x values, a 3D tile spans
// R rows, and a tile marches L planes.
struct TileShape {
    int vw;
    int R;
    int64_t L;
    int blocks_per_cu;  // 0 = as many as fit
};

constexpr int64_t kMinL = 8;
constexpr int64_t kMaxL = 512;

int64_t tiles_per_plane(int ndim, int64_t nx, int64_t ny, int vw, int R);
int64_t balanced_L(int64_t nmarch, int64_t cols, int64_t waves);

TileShape choose_tiles(int ndim, int64_t nx, int64_t ny, int64_t nz, int64_t batch, int tsize, bool aligned,
                       int solver, bool mixed);
// Tile shapes compiled into the single-shape kernels: 2D lanes of 16 bytes or
// of one element; 3D lanes of 16 bytes with 1, 2 or 4 rows per tile (4: two
// half-wave lane rows of two rows each), or of one element with 4 or 1 rows
// (fewer registers per row).
__host__ __device__ constexpr bool variant_ok(int tsize, int ndim, int vw, int R) {
    const int vm = 16 / tsize;
    if (ndim == 2) return R == 1 && (vw == vm || vw == 1);
    if (vw == vm) return R == 1 || R == 2 || R == 4;
    return vw == 1 && (R == 4 || R == 1);
}
// Shapes the VAR_ALL kernel (uneven batches) can run: one-row tiles, and in
// FP32 two-row 3D tiles of 16-byte lanes (their registers fit the two waves
// per SIMD the batch kernels run at; in FP64 they would not).
__host__ __device__ constexpr bool mixed_variant_ok(int tsize, int ndim, int vw, int R) {
    const int vm = 16 / tsize;
    if (ndim == 2) return R == 1 && (vw == vm || vw == 1);
    if (tsize == 4 && vw == vm && R == 2) return true;
    return (vw == vm || vw == 1) && R == 1;
}

// kernel entry points, one instantiation unit per dtype and solver
const void *solve_kernel_ptr(int dtype, int solver, int variant);
const void *filter_kernel_ptr(int dtype, int variant);
Geo make_geo(int ndim, int64_t nx, int64_t ny, int64_t nz, int vw, int R, int64_t L, int tail_pct);
int solve_uniform(int solver, const gd_grid *g, const void *ubar, void *u, const gd_opts *o, void *work,
                  size_t work_bytes, gd_info *info, void *stream, const TuneCfg *force, const SpecParams *spec);
int tune_uniform(int solver, const gd_grid *g, const void *ubar, void *u, void *work, size_t wb, gd_info *info,
                 void *stream, gd_tune_info *out, const SpecParams *spec);
int validate_grid(const gd_grid *g);
// n[0] * ... * n[ndim - 1] when every extent is >= 1 and the product is at
// most cap, else -1 (computed without overflow for any extents)
int64_t checked_points(const int64_t *n, int ndim, int64_t cap);
// largest batch * points a grid may describe: keeps every byte count of a
// call (fields, workspace) far from overflowing 64 bits
constexpr int64_t kMaxTotalPoints = int64_t(1) << 46;
double grid_weight(const gd_grid *g);
// error text for gd_last_error, then the code; every entry point reports through it
int fail(int code, const char *fmt, ...);
bool ranges_overlap(const void *a, size_t na, const void *b, size_t nb);
size_t align_up(size_t x, size_t a);
int validate_opts(const gd_opts *o);
void set_error_text(const char *msg);
int64_t geo_tiles(const Geo &g);

}  // namespace gd
