// gd_api.hip -- host driver and C ABI of libgdecon.so.
//
// Validates arguments, picks a tile shape, carves the caller's workspace and
// launches (1) a small prep kernel that clears the grid-barrier state and the
// per-field scalars and (2) one persistent solve kernel.  Both are plain kernel
// launches on the caller's stream, so a call can be captured into a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "gd_internal.h"
#include "gd_kernels.h"
#include "gdecon.h"

namespace gd {

const void *solve_kernels_f32_vc(int);
const void *solve_kernels_f32_cg(int);
const void *solve_kernels_f32_bicgstab(int);
const void *solve_kernels_f32_sd(int);
const void *solve_kernels_f64_vc(int);
const void *solve_kernels_f64_cg(int);
const void *solve_kernels_f64_bicgstab(int);
const void *solve_kernels_f64_sd(int);

const void *solve_kernel_ptr(int dtype, int solver, int variant) {
    if (dtype == GD_F32) {
        switch (solver) {
        case GD_VANCITTERT: return solve_kernels_f32_vc(variant);
        case GD_CG: return solve_kernels_f32_cg(variant);
        case GD_BICGSTAB: return solve_kernels_f32_bicgstab(variant);
        case GD_STEEPEST_DESCENT: return solve_kernels_f32_sd(variant);
        default: return nullptr;
        }
    }
    switch (solver) {
    case GD_VANCITTERT: return solve_kernels_f64_vc(variant);
    case GD_CG: return solve_kernels_f64_cg(variant);
    case GD_BICGSTAB: return solve_kernels_f64_bicgstab(variant);
    case GD_STEEPEST_DESCENT: return solve_kernels_f64_sd(variant);
    default: return nullptr;
    }
}

// Zero the barrier state and the per-instance scalars before a solve.
__global__ void prep_kernel(Params P) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        P.sync->top = 0;
        P.sync->abort = 0;
        P.sync->active = P.ninst;
    }
    if (i < 2) P.sync->snap[i].v = 0;
    if (i < NGRP) {
        P.sync->cnt[i].v = 0;
        P.sync->gen[i].v = 0;
        P.sync->pool[0][i].v = 0;
        P.sync->pool[1][i].v = 0;
    }
    if (i < P.ninst) {
        State s;
        s.alpha = s.beta = s.omega = 1.0;
        s.rho = s.rr = s.r_ref = s.r0 = 0.0;
        s.pad = 0.0;
        s.iters = 0;
        s.status = GD_MAXITER;
        s.done = 0;
        s.half = 0;
        s.cnt = 0;
        P.st[i] = s;
    }
}

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

struct DevProps {
    int ncu = 0;
    int64_t wall_khz = 0;
};
std::mutex g_mu;
std::map<int, DevProps> g_props;
std::map<const void *, int> g_occ;

int dev_props(DevProps *out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(GD_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_props.find(dev);
    if (it == g_props.end()) {
        DevProps p;
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1)
            return fail(GD_EHIP, "hipDeviceGetAttribute(MultiprocessorCount) failed");
        p.ncu = v;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) != hipSuccess || v <= 0) v = 100000;
        p.wall_khz = v;
        it = g_props.emplace(dev, p).first;
    }
    *out = it->second;
    return GD_OK;
}

// Resident workgroups per CU of a kernel (the persistent grid must not exceed
// this times the CU count, or the grid barrier could wait on workgroups that
// are not running).
int occupancy(const void *kernel) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_mu);
    static std::map<std::pair<int, const void *>, int> occ;
    auto key = std::make_pair(dev, kernel);
    auto it = occ.find(key);
    if (it != occ.end()) return it->second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, BLOCK, 0) != hipSuccess || nb < 1) nb = 1;
    occ[key] = nb;
    return nb;
}

bool vec_used(int solver, int v) {
    switch (solver) {
    case GD_VANCITTERT:
    case GD_STEEPEST_DESCENT: return v == V_R0 || v == V_R1;
    case GD_CG: return v == V_R0 || v == V_P0 || v == V_P1;
    case GD_BICGSTAB: return true;
    default: return false;
    }
}

int nvec_of(int solver) {
    int n = 0;
    for (int v = 0; v < NVEC; ++v) n += vec_used(solver, v);
    return n;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

const char *last_error() { return g_err.c_str(); }

thread_local gd_launch_info g_last_launch;
unsigned long long *g_trace = nullptr;
int64_t g_trace_cap = 0;

int validate_grid(const gd_grid *g) {
    if (!g) return fail(GD_EINVAL, "grid is NULL");
    if (g->ndim != 2 && g->ndim != 3) return fail(GD_EINVAL, "ndim must be 2 or 3 (got %d)", g->ndim);
    if (g->dtype != GD_F32 && g->dtype != GD_F64) return fail(GD_EINVAL, "dtype must be GD_F32 or GD_F64");
    for (int d = 0; d < g->ndim; ++d)
        if (g->n[d] < 1) return fail(GD_EINVAL, "n[%d] must be >= 1", d);
    if (g->batch < 1) return fail(GD_EINVAL, "batch must be >= 1");
    const int64_t npts = g->n[0] * g->n[1] * (g->ndim == 3 ? g->n[2] : 1);
    if (g->n[0] > (int64_t(1) << 31) || npts > (int64_t(1) << 40) || g->batch > (int64_t(1) << 30))
        return fail(GD_EINVAL, "field too large");
    return GD_OK;
}

int64_t grid_points(const gd_grid *g) { return g->n[0] * g->n[1] * (g->ndim == 3 ? g->n[2] : 1); }

double grid_weight(const gd_grid *g) {
    double w = 1.0;
    for (int d = 0; d < g->ndim; ++d) {
        const double h = g->h[d] > 0.0 ? g->h[d] : 2.0 * M_PI / (double)g->n[d];
        w *= h;
    }
    return w;
}

Geo make_geo(int ndim, int64_t nx, int64_t ny, int64_t nz, int vw, int R, int64_t L) {
    Geo g;
    g.nx = nx;
    if (ndim == 2) {
        g.nrows = 1;
        g.nmarch = ny;
        g.plane = nx;
        g.nrs = 1;
    } else {
        g.nrows = ny;
        g.nmarch = nz;
        g.plane = nx * ny;
        g.nrs = (ny + R - 1) / R;
    }
    g.nxs = (nx + (int64_t)WAVE * vw - 1) / ((int64_t)WAVE * vw);
    g.L = L;
    return g;
}

int64_t geo_tiles(const Geo &g) { return g.nxs * g.nrs * ((g.nmarch + g.L - 1) / g.L); }

// Upper bound on the tile count of any shape the library may pick for a field.
int64_t max_tiles(int ndim, int64_t nx, int64_t ny, int64_t nz) {
    return geo_tiles(make_geo(ndim, nx, ny, nz, 1, 1, kMinL));
}

size_t workspace_layout(const gd_grid *g, int solver, int64_t ninst, int64_t tiles_total_max, size_t *off_st,
                        size_t *off_part, size_t *off_vec, size_t *vec_bytes) {
    const size_t tsize = g->dtype == GD_F32 ? 4 : 8;
    size_t off = align_up(sizeof(Sync), 256);
    *off_st = off;
    off = align_up(off + (size_t)ninst * sizeof(State), 256);
    *off_part = off;
    off = align_up(off + (size_t)tiles_total_max * NACC * sizeof(double), 256);
    *off_vec = off;
    *vec_bytes = align_up((size_t)g->batch * (size_t)grid_points(g) * tsize, 256);
    off += (size_t)nvec_of(solver) * *vec_bytes;
    return off;
}

// Resident waves of the solve kernel for this variant (its persistent grid).
int solve_grid(int dtype, int solver, int variant, int blocks_per_cu, const void **kernel, int64_t *blocks_cap) {
    DevProps dp;
    int rc = dev_props(&dp);
    if (rc) return rc;
    const void *k = solve_kernel_ptr(dtype, solver, variant);
    if (!k) return fail(GD_EINVAL, "no kernel for solver %d variant %d", solver, variant);
    int occ = occupancy(k);
    if (blocks_per_cu > 0 && blocks_per_cu < occ) occ = blocks_per_cu;
    *kernel = k;
    *blocks_cap = (int64_t)occ * dp.ncu;
    return GD_OK;
}

int launch_solve(Params &P, const void *k, int64_t blocks_cap, hipStream_t stream) {
    DevProps dp;
    int rc = dev_props(&dp);
    if (rc) return rc;
    const int64_t want = (P.total_tiles + WPB - 1) / WPB;
    const int64_t blocks = std::max<int64_t>(1, std::min(want, blocks_cap));
    if (P.wait_ticks <= 0) P.wait_ticks = (int64_t)10 * 1000 * dp.wall_khz;  // 10 s
    const int prep_blocks = (int)((std::max<int64_t>(P.ninst, NGRP) + 255) / 256);
    hipLaunchKernelGGL(prep_kernel, dim3(prep_blocks), dim3(256), 0, stream, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(GD_EHIP, "prep launch: %s", hipGetErrorString(e));
    void *args[] = {&P};
    e = hipLaunchKernel(k, dim3((unsigned)blocks), dim3(BLOCK), args, 0, stream);
    if (e != hipSuccess) return fail(GD_EHIP, "solve launch: %s", hipGetErrorString(e));
    g_last_launch.blocks = blocks;
    g_last_launch.waves = blocks * WPB;
    g_last_launch.tiles = P.total_tiles;
    return GD_OK;
}

int64_t wait_ticks_of(const gd_opts *o) {
    if (!o || o->wait_limit_us <= 0) return 0;
    DevProps dp;
    if (dev_props(&dp)) return 0;
    const int64_t t = o->wait_limit_us * dp.wall_khz / 1000;
    return t < 1 ? 1 : t;
}

int validate_opts(const gd_opts *o) {
    if (!o) return fail(GD_EINVAL, "opts is NULL");
    if (o->max_iter < 0) return fail(GD_EINVAL, "max_iter must be >= 0");
    if (o->init < GD_INIT_UBAR || o->init > GD_INIT_GIVEN) return fail(GD_EINVAL, "bad init %d", o->init);
    if (o->norm_ref != GD_REF_R0UBAR && o->norm_ref != GD_REF_UBAR) return fail(GD_EINVAL, "bad norm_ref");
    if (std::isnan(o->tol)) return fail(GD_EINVAL, "tol is NaN");
    return GD_OK;
}

bool ranges_overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

int solve_common(int solver, const gd_grid *g, const void *ubar, void *u, const gd_opts *o, void *work,
                 size_t work_bytes, gd_info *info, void *stream) {
    int rc = validate_grid(g);
    if (rc) return rc;
    rc = validate_opts(o);
    if (rc) return rc;
    if (!ubar || !u || !info) return fail(GD_EINVAL, "ubar, u and info must be non-NULL");
    if (!work) return fail(GD_EWORKSPACE, "workspace is NULL");
    if ((uintptr_t)work % 256) return fail(GD_EALIGN, "workspace must be 256-byte aligned");
    const size_t tsize = g->dtype == GD_F32 ? 4 : 8;
    const int64_t npts = grid_points(g);
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->ndim == 3 ? g->n[2] : 1;
    const int64_t tmax = g->batch * max_tiles(g->ndim, nx, ny, nz);
    size_t off_st, off_part, off_vec, vec_bytes;
    const size_t need = workspace_layout(g, solver, g->batch, tmax, &off_st, &off_part, &off_vec, &vec_bytes);
    if (work_bytes < need) return fail(GD_EWORKSPACE, "workspace too small: need %zu bytes, got %zu", need, work_bytes);
    const size_t field_bytes = (size_t)g->batch * (size_t)npts * tsize;
    if (ranges_overlap(ubar, field_bytes, u, field_bytes)) return fail(GD_EINVAL, "ubar and u overlap");
    if (ranges_overlap(ubar, field_bytes, work, need)) return fail(GD_EINVAL, "ubar overlaps the workspace");
    if (ranges_overlap(u, field_bytes, work, need)) return fail(GD_EINVAL, "u overlaps the workspace");
    const bool aligned = ((uintptr_t)ubar % 16 == 0) && ((uintptr_t)u % 16 == 0);
    TileShape ts = choose_tiles(g->ndim, nx, ny, nz, g->batch, (int)tsize, aligned, solver, false);
    const int variant = var_code(g->ndim, ts.vw, ts.R);
    const void *kern = nullptr;
    int64_t blocks_cap = 0;
    rc = solve_grid(g->dtype, solver, variant, ts.blocks_per_cu, &kern, &blocks_cap);
    if (rc) return rc;
    // march length balanced over the waves the persistent grid will hold
    ts.L = balanced_L(g->ndim == 2 ? ny : nz, g->batch * tiles_per_plane(g->ndim, nx, ny, ts.vw, ts.R),
                      blocks_cap * WPB * kTilesPerWave);

    Params P;
    std::memset(&P, 0, sizeof P);
    Inst &I = P.tmpl;
    I.ubar = ubar;
    I.u = u;
    char *w = (char *)work;
    int slot = 0;
    for (int v = 0; v < NVEC; ++v) {
        if (vec_used(solver, v)) I.vec[v] = (void *)(w + off_vec + (size_t)(slot++) * vec_bytes);
        else I.vec[v] = nullptr;
    }
    I.hist = o->history;
    I.info = info;
    I.geo = make_geo(g->ndim, nx, ny, nz, ts.vw, ts.R, ts.L);
    I.tile0 = 0;
    I.ntiles = geo_tiles(I.geo);
    I.hw = grid_weight(g);
    I.ndim = g->ndim;
    I.vw = ts.vw;
    I.R = ts.R;
    P.table = nullptr;
    P.st = (State *)(w + off_st);
    P.sync = (Sync *)w;
    P.part = (double *)(w + off_part);
    P.stride_bytes = npts * (int64_t)tsize;
    P.tiles_per_inst = I.ntiles;
    P.total_tiles = I.ntiles * g->batch;
    P.wait_ticks = wait_ticks_of(o);
    P.tol = o->tol;
    P.ninst = (int32_t)g->batch;
    P.init = o->init;
    P.norm_ref = o->norm_ref;
    P.max_iter = o->max_iter;
    P.hist_stride = o->max_iter + 1;
    P.steal = kSteal;
    if (const char *e = getenv("GD_STEAL")) P.steal = std::max(0, atoi(e));
    P.trace = g_trace;
    P.trace_cap = g_trace_cap;
    rc = launch_solve(P, kern, blocks_cap, (hipStream_t)stream);
    if (rc == GD_OK) {
        g_last_launch.variant = variant;
        g_last_launch.vw = ts.vw;
        g_last_launch.R = ts.R;
        g_last_launch.L = ts.L;
    }
    return rc;
}

}  // namespace gd

using namespace gd;

extern "C" {

int filter_apply(const gd_grid *g, const void *x, void *y, void *stream) {
    int rc = validate_grid(g);
    if (rc) return rc;
    if (!x || !y) return fail(GD_EINVAL, "x and y must be non-NULL");
    const size_t tsize = g->dtype == GD_F32 ? 4 : 8;
    const int64_t npts = grid_points(g);
    const size_t bytes = (size_t)g->batch * (size_t)npts * tsize;
    if (ranges_overlap(x, bytes, y, bytes)) return fail(GD_EINVAL, "x and y must not overlap");
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->ndim == 3 ? g->n[2] : 1;
    const bool aligned = ((uintptr_t)x % 16 == 0) && ((uintptr_t)y % 16 == 0);
    const TileShape ts = choose_tiles(g->ndim, nx, ny, nz, g->batch, (int)tsize, aligned, -1, false);
    Inst I;
    std::memset(&I, 0, sizeof I);
    I.ubar = x;
    I.u = y;
    I.geo = make_geo(g->ndim, nx, ny, nz, ts.vw, ts.R, ts.L);
    I.ndim = g->ndim;
    I.vw = ts.vw;
    I.R = ts.R;
    const int64_t tpi = geo_tiles(I.geo);
    int64_t total = tpi * g->batch;
    const int64_t blocks = (total + WPB - 1) / WPB;
    if (blocks > 0x7fffffff) return fail(GD_EINVAL, "grid too large");
    const void *k = filter_kernel_ptr(g->dtype, var_code(g->ndim, ts.vw, ts.R));
    if (!k) return fail(GD_EINVAL, "no filter kernel for this tile shape");
    int64_t stride = npts;
    void *args[] = {&I, &stride, (void *)&tpi, &total};
    hipError_t e = hipLaunchKernel(k, dim3((unsigned)blocks), dim3(BLOCK), args, 0, (hipStream_t)stream);
    if (e != hipSuccess) return fail(GD_EHIP, "filter launch: %s", hipGetErrorString(e));
    return GD_OK;
}

size_t deconvolve_workspace_bytes(const gd_grid *g, int32_t solver) {
    if (validate_grid(g)) return 0;
    if (solver < GD_VANCITTERT || solver > GD_STEEPEST_DESCENT) return 0;
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->ndim == 3 ? g->n[2] : 1;
    size_t a, b, c, d;
    return workspace_layout(g, solver, g->batch, g->batch * max_tiles(g->ndim, nx, ny, nz), &a, &b, &c, &d);
}

int deconvolve_vancittert(const gd_grid *g, const void *ubar, void *u, const gd_opts *o, void *work, size_t wb,
                          gd_info *info, void *stream) {
    return solve_common(GD_VANCITTERT, g, ubar, u, o, work, wb, info, stream);
}

int deconvolve_cg(const gd_grid *g, const void *ubar, void *u, const gd_opts *o, void *work, size_t wb,
                  gd_info *info, void *stream) {
    return solve_common(GD_CG, g, ubar, u, o, work, wb, info, stream);
}

int deconvolve_bicgstab(const gd_grid *g, const void *ubar, void *u, const gd_opts *o, void *work, size_t wb,
                        gd_info *info, void *stream) {
    return solve_common(GD_BICGSTAB, g, ubar, u, o, work, wb, info, stream);
}

int deconvolve_steepest_descent(const gd_grid *g, const void *ubar, void *u, const gd_opts *o, void *work, size_t wb,
                                gd_info *info, void *stream) {
    return solve_common(GD_STEEPEST_DESCENT, g, ubar, u, o, work, wb, info, stream);
}

const char *gd_status_string(int32_t code) {
    switch (code) {
    case GD_OK: return "GD_OK / GD_CONVERGED";
    case GD_EINVAL: return "GD_EINVAL";
    case GD_EWORKSPACE: return "GD_EWORKSPACE";
    case GD_EHIP: return "GD_EHIP";
    case GD_EALIGN: return "GD_EALIGN";
    case GD_MAXITER: return "GD_MAXITER";
    case GD_BREAKDOWN_RHO: return "GD_BREAKDOWN_RHO";
    case GD_BREAKDOWN_OMEGA: return "GD_BREAKDOWN_OMEGA";
    case GD_NONFINITE: return "GD_NONFINITE";
    case GD_ZERO_REF: return "GD_ZERO_REF";
    case GD_TIMEOUT: return "GD_TIMEOUT";
    default: return "unknown";
    }
}

const char *gd_last_error(void) { return gd::last_error(); }

int gd_set_trace(uint64_t *buf, int64_t capacity) {
    gd::g_trace = reinterpret_cast<unsigned long long *>(buf);
    gd::g_trace_cap = buf ? capacity : 0;
    return GD_OK;
}

int gd_last_launch(gd_launch_info *out) {
    if (!out) return GD_EINVAL;
    *out = gd::g_last_launch;
    return GD_OK;
}

}  // extern "C"
