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
#include <vector>

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
        Counts c;
        memset(&c, 0, sizeof c);
        c.active = P.ninst;
        P.sync->live = c;
    }
    if (i < 2) {
        Counts z;
        memset(&z, 0, sizeof z);
        P.sync->snap[i] = z;
    }
    if (i < NGRP) {
        int64_t c = 0;  // claims in pool i (the kernel's pool layouts)
        const int64_t ng = P.npools, ntot = P.total_tiles, nb = P.big_total, ns = ntot - nb;
        if (i < ng) c = P.interleave ? (ntot - i + ng - 1) / ng : (nb * (i + 1) / ng - nb * i / ng) + (ns * (i + 1) / ng - ns * i / ng);
        P.sync->pcnt[i] = c;
        P.sync->cnt[i].v = 0;
        P.sync->gen[i].v = 0;
        P.sync->pool[0][i].v = 0;
        P.sync->pool[1][i].v = 0;
    }
    if (i < P.ninst) {
        State s;
        s.alpha = s.beta = s.omega = 1.0;
        s.rho = s.rr = s.r_ref = s.r0 = 0.0;
        s.r_ub = 0.0;
        s.iters = 0;
        s.status = GD_MAXITER;
        s.done = 0;
        s.half = 0;
        s.cnt = 0;
        s.verify = s.replace = s.restart = s.fallback = s.tknown = s.nrep = 0;
        s.start = P.init == GD_INIT_WARM ? GD_INIT_GIVEN : P.init;
        P.st[i] = s;
    }
}

namespace {
thread_local std::string g_err;
}  // namespace

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

namespace {

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

}  // namespace

const char *last_error() { return g_err.c_str(); }

// Error text for the other translation units of the library (the warm-start
// network), so that gd_last_error() reports every entry point.
void set_error_text(const char *msg) { g_err = msg; }

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
    const int64_t npts = checked_points(g->n, g->ndim, int64_t(1) << 40);
    if (npts < 0 || g->n[0] > (int64_t(1) << 31) || g->batch > (int64_t(1) << 30) ||
        g->batch > kMaxTotalPoints / npts)
        return fail(GD_EINVAL, "field too large");
    return GD_OK;
}

int64_t checked_points(const int64_t *n, int ndim, int64_t cap) {
    int64_t p = 1;
    for (int d = 0; d < ndim; ++d) {
        if (n[d] < 1 || n[d] > cap / p) return -1;
        p *= n[d];
    }
    return p;
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

// Tile geometry of a field.  Every column (x segment x row tile) is cut into
// long tiles of L planes and, over roughly the last tail_pct percent of its
// planes, short tiles of L2 = L / 4 planes (at least kMinL): the short tiles
// are claimed last, so the end of a sweep, when waves finish at different
// times, is made of work that finishes quickly.
Geo make_geo(int ndim, int64_t nx, int64_t ny, int64_t nz, int vw, int R, int64_t L, int tail_pct) {
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
    const int64_t tc = ndim == 3 ? tile_cols(vw, R) : (int64_t)WAVE * vw;  // x columns per tile
    g.nxs = (nx + tc - 1) / tc;
    g.L = L;
    const int64_t cols = g.nxs * g.nrs;
    const int64_t L2 = std::max<int64_t>(kMinL, L / 4);
    const int64_t nlong = tail_pct > 0 ? (g.nmarch * (100 - tail_pct) / 100) / L : 0;
    if (tail_pct > 0 && L2 < L && nlong >= 1 && nlong * L < g.nmarch) {
        g.L2 = L2;
        g.mb = nlong * L;
        g.nbig = cols * nlong;
    } else {  // long tiles only
        g.L2 = L;
        g.mb = g.nmarch;
        g.nbig = cols * ((g.nmarch + L - 1) / L);
    }
    return g;
}

int64_t geo_tiles(const Geo &g) {
    const int64_t rest = g.nmarch - g.mb;
    return g.nbig + (rest > 0 ? g.nxs * g.nrs * ((rest + g.L2 - 1) / g.L2) : 0);
}

// Upper bound on the tile count of any shape the library may pick for a field.
int64_t max_tiles(int ndim, int64_t nx, int64_t ny, int64_t nz) {
    // long tiles cover at most nmarch / kMinL segments, short ones add at most one more
    const Geo g = make_geo(ndim, nx, ny, nz, 1, 1, kMinL, 0);
    return g.nxs * g.nrs * ((g.nmarch + kMinL - 1) / kMinL + 1);
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
    P.npools = (int32_t)std::min<int64_t>(blocks, NGRP);
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
    if (o->init < GD_INIT_UBAR || o->init > GD_INIT_WARM) return fail(GD_EINVAL, "bad init %d", o->init);
    if (o->norm_ref != GD_REF_R0UBAR && o->norm_ref != GD_REF_UBAR) return fail(GD_EINVAL, "bad norm_ref");
    if (std::isnan(o->tol)) return fail(GD_EINVAL, "tol is NaN");
    return GD_OK;
}

// residual replacements per instance that the options allow
int32_t replacements_of(const gd_opts *o) {
    constexpr int32_t kDefaultReplace = 2;
    return o->max_replace == 0 ? kDefaultReplace : std::max<int32_t>(0, o->max_replace);
}

bool ranges_overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

// ---- tuning choices ----------------------------------------------------------

std::mutex g_tune_mu;
std::map<std::string, TuneCfg> g_tune;
bool g_tune_loaded = false;

const char *tune_file() {
    const char *f = getenv("GD_TUNE_CACHE");
    return (f && *f) ? f : nullptr;
}

// caller holds g_tune_mu
void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *f = tune_file();
    if (!f) return;
    FILE *fp = fopen(f, "r");
    if (!fp) return;
    char line[1024];
    while (fgets(line, sizeof line, fp)) {
        char key[900];
        int tpw = 0, rows = 0, tail = 0, ilv = 0, wc = 0, bpc = kBlocksPerCu, segs = 0;
        const int nf = sscanf(line, "%899s %d %d %d %d %d %d %d", key, &tpw, &rows, &tail, &ilv, &wc, &bpc, &segs);
        if (nf >= 6 && tpw >= 1 && tpw <= 64 && rows >= 0 && rows <= 4 && tail >= 0 && tail <= 50 &&
            (ilv == 0 || ilv == 1) && (wc == 0 || wc == 1) && bpc >= 0 && bpc <= kMaxBlocksPerCu && segs >= 0 &&
            segs <= kMaxSegs) {
            TuneCfg c;
            c.tpw = tpw;
            c.rows = rows;
            c.tail = tail;
            c.ilv = ilv;
            c.wc = wc;
            c.bpc = bpc;
            c.segs = segs;
            g_tune[key] = c;
        }
    }
    fclose(fp);
}

bool tune_lookup(const std::string &key, TuneCfg *out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

void tune_store(const std::string &key, const TuneCfg &c) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    g_tune[key] = c;
    if (const char *f = tune_file()) {
        if (FILE *fp = fopen(f, "a")) {
            fprintf(fp, "%s %d %d %d %d %d %d %d\n", key.c_str(), c.tpw, c.rows, c.tail, c.ilv, c.wc, c.bpc, c.segs);
            fclose(fp);
        }
    }
}

std::string device_tag() {
    DevProps dp;
    if (dev_props(&dp)) return "dev?";
    char b[64];
    snprintf(b, sizeof b, "cu%d", dp.ncu);
    return b;
}

std::string key_uniform(int solver, const gd_grid *g, bool aligned) {
    char b[256];
    snprintf(b, sizeof b, "U:%s:s%d:t%d:d%d:%lldx%lldx%lld:b%lld:a%d", device_tag().c_str(), solver, g->dtype, g->ndim,
             (long long)g->n[0], (long long)g->n[1], (long long)(g->ndim == 3 ? g->n[2] : 1), (long long)g->batch,
             aligned ? 1 : 0);
    return b;
}

// ---- uniform batches -----------------------------------------------------------

int solve_uniform(int solver, const gd_grid *g, const void *ubar, void *u, const gd_opts *o, void *work,
                  size_t work_bytes, gd_info *info, void *stream, const TuneCfg *force, const SpecParams *spec) {
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
    TuneCfg cfg;
    if (force) cfg = *force;
    else tune_lookup(key_uniform(solver, g, aligned) + (spec ? ":spec" : ""), &cfg);
    TileShape ts = choose_tiles(g->ndim, nx, ny, nz, g->batch, (int)tsize, aligned, solver, false);
    if (g->ndim == 3 && cfg.rows > 0 && variant_ok((int)tsize, 3, ts.vw, cfg.rows) && (cfg.rows == 1 || ny >= cfg.rows))
        ts.R = cfg.rows;
    if (spec) {  // pointwise sweeps over a spectrum: whole 16-byte lanes, one row per tile
        ts.vw = 16 / (int)tsize;
        ts.R = 1;
    }
    const int variant = (spec ? kSpecBit : 0) + var_code(g->ndim, ts.vw, ts.R);
    const void *kern = nullptr;
    int64_t blocks_cap = 0;
    rc = solve_grid(g->dtype, solver, variant, cfg.bpc, &kern, &blocks_cap);
    if (rc) return rc;
    // march length balanced over the waves the persistent grid will hold
    ts.L = balanced_L(g->ndim == 2 ? ny : nz, g->batch * tiles_per_plane(g->ndim, nx, ny, ts.vw, ts.R),
                      blocks_cap * WPB * std::max(1, cfg.tpw));
    if (cfg.segs > 0) {  // a fixed number of long tiles per column
        const int64_t nm = g->ndim == 2 ? ny : nz;
        ts.L = std::min<int64_t>(kMaxL, std::max<int64_t>(kMinL, (nm + cfg.segs - 1) / cfg.segs));
    }

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
    I.geo = make_geo(g->ndim, nx, ny, nz, ts.vw, ts.R, ts.L, cfg.tail);
    I.tile0 = 0;
    I.ntiles = geo_tiles(I.geo);
    I.hw = grid_weight(g);
    I.ndim = g->ndim;
    I.vw = ts.vw;
    I.R = ts.R;
    if (spec) {
        I.hw = spec->hw;
        I.inv_kc2 = spec->inv_kc2;
        I.nxc = (int32_t)spec->nxc;
        I.nxs = (int32_t)spec->nxs;
        I.lny = spec->lny;
        I.lnz = spec->lnz;
    }
    P.table = nullptr;
    P.st = (State *)(w + off_st);
    P.sync = (Sync *)w;
    P.part = (double *)(w + off_part);
    P.stride_bytes = npts * (int64_t)tsize;
    P.tiles_per_inst = I.ntiles;
    P.total_tiles = I.ntiles * g->batch;
    P.big_total = I.geo.nbig * g->batch;
    P.wait_ticks = wait_ticks_of(o);
    P.tol = o->tol;
    P.ninst = (int32_t)g->batch;
    P.init = o->init;
    P.norm_ref = o->norm_ref;
    P.max_iter = o->max_iter;
    P.hist_stride = o->max_iter + 1;
    P.max_replace = replacements_of(o);
    P.solver = solver;
    P.steal = kSteal;
    if (const char *e = getenv("GD_STEAL")) P.steal = std::max(0, atoi(e));
    P.interleave = cfg.ilv;
    P.wave_claims = cfg.wc;
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

// ---- uneven batches ----------------------------------------------------------

// Instance descriptors are written into the workspace by this kernel, whose
// argument carries up to kTableChunk of them: the values travel with the
// launch itself, so no host buffer has to outlive the call or a captured graph.
constexpr int kTableChunk = 12;
struct TableChunk {
    Inst inst[kTableChunk];
    Inst *dst;
    int32_t n;
    int32_t pad;
};
static_assert(sizeof(Inst) % 8 == 0, "Inst is copied in 8-byte words");
static_assert(sizeof(TableChunk) <= 3072, "kernel argument too large");

__global__ void table_kernel(TableChunk c) {
    constexpr int words = (int)(sizeof(Inst) / 8);
    const uint64_t *src = reinterpret_cast<const uint64_t *>(c.inst);
    uint64_t *dst = reinterpret_cast<uint64_t *>(c.dst);
    for (int k = threadIdx.x; k < c.n * words; k += blockDim.x) dst[k] = src[k];
}

struct BatchLayout {
    size_t off_st, off_tab, off_part, off_vec, total;
    int64_t tiles_max;
};

int64_t inst_points(const gd_instance &d) { return d.n[0] * d.n[1] * (d.ndim == 3 ? d.n[2] : 1); }

int validate_instance(const gd_instance &d, int i) {
    if (d.ndim != 2 && d.ndim != 3) return fail(GD_EINVAL, "instance %d: ndim must be 2 or 3", i);
    for (int k = 0; k < d.ndim; ++k)
        if (d.n[k] < 1) return fail(GD_EINVAL, "instance %d: n[%d] must be >= 1", i, k);
    if (checked_points(d.n, d.ndim, int64_t(1) << 40) < 0 || d.n[0] > (int64_t(1) << 31))
        return fail(GD_EINVAL, "instance %d: field too large", i);
    return GD_OK;
}

// every instance valid, and all of them together within kMaxTotalPoints
int validate_instances(const gd_instance *list, int32_t count) {
    int64_t tot = 0;
    for (int i = 0; i < count; ++i) {
        const int rc = validate_instance(list[i], i);
        if (rc) return rc;
        tot += inst_points(list[i]);  // each at most 2^40: no overflow before the test below
        if (tot > kMaxTotalPoints) return fail(GD_EINVAL, "the instances hold too many points");
    }
    return GD_OK;
}

BatchLayout batch_layout(int solver, int dtype, const gd_instance *list, int32_t count) {
    const size_t tsize = dtype == GD_F32 ? 4 : 8;
    BatchLayout L;
    size_t off = align_up(sizeof(Sync), 256);
    L.off_st = off;
    off = align_up(off + (size_t)count * sizeof(State), 256);
    L.off_tab = off;
    off = align_up(off + (size_t)count * sizeof(Inst), 256);
    L.tiles_max = 0;
    for (int i = 0; i < count; ++i) {
        const gd_instance &d = list[i];
        L.tiles_max += max_tiles(d.ndim, d.n[0], d.n[1], d.ndim == 3 ? d.n[2] : 1);
    }
    L.off_part = off;
    off = align_up(off + (size_t)L.tiles_max * NACC * sizeof(double), 256);
    L.off_vec = off;
    for (int i = 0; i < count; ++i) off += (size_t)nvec_of(solver) * align_up((size_t)inst_points(list[i]) * tsize, 256);
    L.total = off;
    return L;
}

std::string key_batch(int solver, int dtype, const gd_instance *list, int32_t count) {
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the sizes and alignments
    auto mix = [&](uint64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (v >> (8 * b)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    for (int i = 0; i < count; ++i) {
        const gd_instance &d = list[i];
        mix((uint64_t)d.ndim);
        for (int k = 0; k < 3; ++k) mix((uint64_t)(k < d.ndim ? d.n[k] : 1));
        mix((((uintptr_t)d.ubar | (uintptr_t)d.u) % 16 == 0) ? 1 : 0);
    }
    char b[256];
    snprintf(b, sizeof b, "B:%s:s%d:t%d:c%d:%016llx", device_tag().c_str(), solver, dtype, count, (unsigned long long)h);
    return b;
}

// Every u must be disjoint from every other field (inputs may be shared).
int check_batch_overlaps(int dtype, const gd_instance *list, int32_t count, const void *work, size_t need) {
    const size_t tsize = dtype == GD_F32 ? 4 : 8;
    struct Iv {
        uintptr_t a, b;
        bool out;
        int i;
    };
    std::vector<Iv> iv;
    iv.reserve(2 * (size_t)count);
    for (int i = 0; i < count; ++i) {
        const size_t bytes = (size_t)inst_points(list[i]) * tsize;
        iv.push_back({(uintptr_t)list[i].ubar, (uintptr_t)list[i].ubar + bytes, false, i});
        iv.push_back({(uintptr_t)list[i].u, (uintptr_t)list[i].u + bytes, true, i});
        if (ranges_overlap(list[i].ubar, bytes, work, need) || ranges_overlap(list[i].u, bytes, work, need))
            return fail(GD_EINVAL, "instance %d overlaps the workspace", i);
    }
    std::sort(iv.begin(), iv.end(), [](const Iv &x, const Iv &y) { return x.a < y.a; });
    uintptr_t end_any = 0, end_out = 0;
    for (const Iv &c : iv) {
        if (c.a < end_out || (c.out && c.a < end_any))
            return fail(GD_EINVAL, "instance %d: an output field overlaps another field", c.i);
        end_any = std::max(end_any, c.b);
        if (c.out) end_out = std::max(end_out, c.b);
    }
    return GD_OK;
}

int solve_batch(int solver, int dtype, const gd_instance *list, int32_t count, const gd_opts *o, void *work,
                size_t work_bytes, gd_info *info, void *stream, const TuneCfg *force) {
    if (solver < GD_VANCITTERT || solver > GD_STEEPEST_DESCENT) return fail(GD_EINVAL, "bad solver %d", solver);
    if (dtype != GD_F32 && dtype != GD_F64) return fail(GD_EINVAL, "dtype must be GD_F32 or GD_F64");
    if (!list || count < 1) return fail(GD_EINVAL, "the instance list is empty");
    int rc = validate_opts(o);
    if (rc) return rc;
    if (!info) return fail(GD_EINVAL, "info must be non-NULL");
    if ((rc = validate_instances(list, count))) return rc;
    for (int i = 0; i < count; ++i) {
        if (!list[i].ubar || !list[i].u) return fail(GD_EINVAL, "instance %d: ubar and u must be non-NULL", i);
    }
    if (!work) return fail(GD_EWORKSPACE, "workspace is NULL");
    if ((uintptr_t)work % 256) return fail(GD_EALIGN, "workspace must be 256-byte aligned");
    const BatchLayout lay = batch_layout(solver, dtype, list, count);
    if (work_bytes < lay.total)
        return fail(GD_EWORKSPACE, "workspace too small: need %zu bytes, got %zu", lay.total, work_bytes);
    if ((rc = check_batch_overlaps(dtype, list, count, work, lay.total))) return rc;

    const int tsize = dtype == GD_F32 ? 4 : 8;
    const int vm = 16 / tsize;
    std::vector<Inst> tab((size_t)count);
    bool same = true;
    for (int i = 0; i < count; ++i) {
        const gd_instance &d = list[i];
        const bool al = ((uintptr_t)d.ubar % 16 == 0) && ((uintptr_t)d.u % 16 == 0);
        Inst &I = tab[i];
        std::memset(&I, 0, sizeof I);
        I.ndim = d.ndim;
        I.vw = (al && d.n[0] % vm == 0 && d.n[0] >= vm) ? vm : 1;
        I.R = (I.ndim == 3 && mixed_variant_ok(tsize, 3, I.vw, 2) && d.n[1] >= 2) ? 2 : 1;
        if (I.ndim != tab[0].ndim || I.vw != tab[0].vw || I.R != tab[0].R) same = false;
    }
    const int variant = (same && tab[0].vw == vm) ? kTableBit + var_code(tab[0].ndim, vm, tab[0].R) : VAR_ALL;
    TuneCfg cfg;
    if (force) cfg = *force;
    else tune_lookup(key_batch(solver, dtype, list, count), &cfg);
    const void *kern = nullptr;
    int64_t blocks_cap = 0;
    if ((rc = solve_grid(dtype, solver, variant, cfg.bpc, &kern, &blocks_cap))) return rc;

    // Tiles of about equal size across instances: target points per tile from
    // the total work and the tiles the grid should hold.
    double ptot = 0;
    for (int i = 0; i < count; ++i) ptot += (double)inst_points(list[i]);
    const double target_tiles = (double)blocks_cap * WPB * std::max(1, cfg.tpw);
    const double pts_per_tile = std::max(1.0, ptot / target_tiles);
    char *w = (char *)work;
    size_t voff = lay.off_vec;
    int64_t tile0 = 0, big0 = 0, small0 = 0;
    for (int i = 0; i < count; ++i) {
        const gd_instance &d = list[i];
        Inst &I = tab[i];
        const int64_t nx = d.n[0], ny = d.n[1], nz = d.ndim == 3 ? d.n[2] : 1;
        const int64_t nmarch = d.ndim == 2 ? ny : nz;
        const double row_pts = (double)WAVE * I.vw * I.R;
        int64_t L = (int64_t)std::llround(pts_per_tile / row_pts);
        L = std::min<int64_t>(std::max<int64_t>(L, kMinL), kMaxL);
        const int64_t nseg = std::max<int64_t>(1, (nmarch + L - 1) / L);
        L = std::max<int64_t>(kMinL, (nmarch + nseg - 1) / nseg);
        I.ubar = d.ubar;
        I.u = d.u;
        const size_t vb = align_up((size_t)inst_points(d) * tsize, 256);
        int slot = 0;
        for (int v = 0; v < NVEC; ++v) I.vec[v] = vec_used(solver, v) ? (void *)(w + voff + (size_t)(slot++) * vb) : nullptr;
        voff += (size_t)nvec_of(solver) * vb;
        I.hist = d.history;
        I.info = info + i;
        I.geo = make_geo(d.ndim, nx, ny, nz, I.vw, I.R, L, cfg.tail);
        I.tile0 = tile0;
        I.ntiles = geo_tiles(I.geo);
        tile0 += I.ntiles;
        I.b0 = big0;
        I.s0 = small0;
        big0 += I.geo.nbig;
        small0 += I.ntiles - I.geo.nbig;
        gd_grid gi;
        std::memset(&gi, 0, sizeof gi);
        gi.ndim = d.ndim;
        for (int k = 0; k < 3; ++k) {
            gi.n[k] = d.n[k];
            gi.h[k] = d.h[k];
        }
        I.hw = grid_weight(&gi);
    }
    if (tile0 > lay.tiles_max) return fail(GD_EINVAL, "internal: tile count exceeds the workspace bound");

    Inst *dtab = (Inst *)(w + lay.off_tab);
    for (int i = 0; i < count; i += kTableChunk) {
        TableChunk c;
        std::memset(&c, 0, sizeof c);
        c.n = std::min(kTableChunk, count - i);
        std::memcpy(c.inst, &tab[i], (size_t)c.n * sizeof(Inst));
        c.dst = dtab + i;
        hipLaunchKernelGGL(table_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(GD_EHIP, "table launch: %s", hipGetErrorString(e));
    }

    Params P;
    std::memset(&P, 0, sizeof P);
    P.table = dtab;
    P.st = (State *)(w + lay.off_st);
    P.sync = (Sync *)w;
    P.part = (double *)(w + lay.off_part);
    P.total_tiles = tile0;
    P.big_total = big0;
    P.wait_ticks = wait_ticks_of(o);
    P.tol = o->tol;
    P.ninst = count;
    P.init = o->init;
    P.norm_ref = o->norm_ref;
    P.max_iter = o->max_iter;
    P.max_replace = replacements_of(o);
    P.solver = solver;
    P.steal = kSteal;
    if (const char *e = getenv("GD_STEAL")) P.steal = std::max(0, atoi(e));
    P.interleave = cfg.ilv;
    P.wave_claims = cfg.wc;
    P.trace = g_trace;
    P.trace_cap = g_trace_cap;
    rc = launch_solve(P, kern, blocks_cap, (hipStream_t)stream);
    if (rc == GD_OK) {
        g_last_launch.variant = variant;
        g_last_launch.vw = same ? tab[0].vw : 0;
        g_last_launch.R = same ? tab[0].R : 0;
        g_last_launch.L = count == 1 ? tab[0].geo.L : 0;
    }
    return rc;
}

// ---- autotuner ---------------------------------------------------------------

// A later candidate must beat the best so far by this fraction: the leaders'
// times are minima of five runs, which repeat to about 0.3 %, so 0.5 %
// separates them (a 2 % margin had kept a configuration 1.6 % slower).
constexpr double kTuneMargin = 0.005;

// Time each candidate with short fixed-length solves (4 Krylov or 10 Van
// Cittert / steepest-descent passes; one warm-up, then the best of three),
// then time the four fastest again on solves twice as long, round-robin,
// best of five each, and return the index of the fastest; candidate 0 (the
// untuned default) is always among them.  The first round's noise is of the
// order of the differences between the leaders, and the longer solves rank
// them as full solves do, where init and exit weigh less: 3 x 256^3 BiCGSTAB
// with two tiles per column trails 52-plane tiles in some 4-pass trials but
// leads by 2 % in full solves.  launch(cfg, long_trial) runs one trial.
template <typename Launch>
int time_candidates(const std::vector<TuneCfg> &cands, Launch &&launch, hipStream_t stream, gd_tune_info *out) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(GD_EHIP, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(GD_EHIP, "hipEventCreate failed");
    }
    int rc = GD_OK;
    auto time_once = [&](size_t c, bool long_trial, double &ms_out) -> int {
        (void)hipEventRecord(e0, stream);
        int r = launch(cands[c], long_trial);
        if (r) return r;
        (void)hipEventRecord(e1, stream);
        if (hipEventSynchronize(e1) != hipSuccess) return fail(GD_EHIP, "hipEventSynchronize failed");
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms_out = ms;
        return GD_OK;
    };
    std::vector<double> t(cands.size(), 1e30);
    for (size_t c = 0; c < cands.size() && rc == GD_OK; ++c) {
        if ((rc = launch(cands[c], false))) break;
        for (int rep = 0; rep < 3 && rc == GD_OK; ++rep) {
            double ms = 0;
            if ((rc = time_once(c, false, ms)) == GD_OK) t[c] = std::min(t[c], ms);
        }
    }
    // second round over the leaders (the default always among them)
    std::vector<size_t> order(cands.size());
    for (size_t c = 0; c < order.size(); ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return t[a] < t[b]; });
    std::vector<size_t> lead(order.begin(), order.begin() + std::min<size_t>(4, order.size()));
    if (std::find(lead.begin(), lead.end(), (size_t)0) == lead.end() && !cands.empty()) lead.push_back(0);
    std::sort(lead.begin(), lead.end());
    std::vector<double> t2(cands.size(), 1e30);
    for (int rep = 0; rep < 5 && rc == GD_OK; ++rep)
        for (size_t c : lead) {
            double ms = 0;
            if ((rc = time_once(c, true, ms))) break;
            t2[c] = std::min(t2[c], ms);
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    // a later candidate must win by a clear margin: ties within the trial
    // noise keep the earlier (default-like, contiguous-pool) configuration
    int best = -1;
    double best_ms = 0;
    for (size_t c : lead)
        if (best < 0 || t2[c] < best_ms * (1.0 - kTuneMargin)) {
            best = (int)c;
            best_ms = t2[c];
        }
    if (out) {
        out->candidates = (int32_t)cands.size();
        out->best = best;
        out->tiles_per_wave = cands[best].tpw;
        out->rows = cands[best].rows;
        out->tail_pct = cands[best].tail;
        out->interleave = cands[best].ilv;
        out->wave_claims = cands[best].wc;
        out->blocks_per_cu = cands[best].bpc;
        out->segments = cands[best].segs;
        out->best_ms = best_ms;
        out->default_ms = t2.empty() ? 0.0 : t2[0];
    }
    return best;
}

gd_opts trial_opts(int solver, bool long_trial = false) {
    gd_opts o;
    std::memset(&o, 0, sizeof o);
    // enough passes that the sweeps, not init and exit, decide (Van Cittert
    // and steepest descent passes move a third to a half of a Krylov pass)
    o.max_iter = (solver == GD_VANCITTERT || solver == GD_STEEPEST_DESCENT) ? 10 : 4;
    if (long_trial) o.max_iter *= 2;
    o.init = GD_INIT_UBAR;
    o.norm_ref = GD_REF_R0UBAR;
    o.tol = 0.0;
    return o;
}

const int kTpwCands[] = {kTilesPerWave, 1, 3, 4, 6};
const int kTailCands[] = {kTailPct, 0, 25};
const int kBpcCands[] = {kBlocksPerCu, 0};

// Time the launch configurations of a uniform solve (on a stored spectrum
// when `spec` is set) and remember the fastest.
int tune_uniform(int solver, const gd_grid *g, const void *ubar, void *u, void *work, size_t wb, gd_info *info,
                 void *stream, gd_tune_info *out, const SpecParams *spec) {
    int rc = validate_grid(g);
    if (rc) return rc;
    if (solver < GD_VANCITTERT || solver > GD_STEEPEST_DESCENT) return fail(GD_EINVAL, "bad solver %d", solver);
    const gd_opts o = trial_opts(solver), o2 = trial_opts(solver, true);
    std::vector<TuneCfg> cands;
    std::vector<int> rows = {0};
    if (g->ndim == 3 && !spec) rows = {0, 1, 2, 4};
    for (int bp : kBpcCands)
        for (int r : rows)
            for (int t : kTpwCands)
                for (int tl : kTailCands)
                    for (int il = 0; il < 2; ++il)
                        for (int wc = 0; wc < 2; ++wc) {
                            TuneCfg c;
                            c.tpw = t;
                            c.rows = r;
                            c.tail = tl;
                            c.ilv = il;
                            c.wc = wc;
                            c.bpc = bp;
                            cands.push_back(c);
                        }
    // 3D stencil sweeps: a few long tiles per column, all marching the same
    // plane ranges, even where that leaves CUs idle (3 x 256^3 FP32
    // BiCGSTAB: two tiles per column on 192 workgroups, 5.19 ms, against
    // 5.30 ms for the wave-count rule's 52-plane tiles on 480)
    if (g->ndim == 3 && !spec)
        for (int bp : {kBlocksPerCu, 1})
            for (int r : rows)
                for (int sg = 1; sg <= 4; ++sg) {
                    TuneCfg c;
                    c.tpw = 1;
                    c.rows = r;
                    c.tail = 0;
                    c.bpc = bp;
                    c.segs = sg;
                    cands.push_back(c);
                }
    // every candidate must launch; a shape the field cannot use falls back to
    // the default rule inside solve_uniform, so duplicates are harmless
    auto launch = [&](const TuneCfg &c, bool long_trial) {
        return solve_uniform(solver, g, ubar, u, long_trial ? &o2 : &o, work, wb, info, stream, &c, spec);
    };
    const int best = time_candidates(cands, launch, (hipStream_t)stream, out);
    if (best < 0) return best;
    const bool aligned = ((uintptr_t)ubar % 16 == 0) && ((uintptr_t)u % 16 == 0);
    tune_store(key_uniform(solver, g, aligned) + (spec ? ":spec" : ""), cands[best]);
    return GD_OK;
}

// ---- the solve without a workspace argument ------------------------------------

// The workspace of deconvolve_noalloc: a fixed device array (one copy per GPU,
// held until the process ends).  In host code `scratch` names a host-side
// stand-in, not device memory: kernels get the device address that
// hipGetSymbolAddress returns for the current device, kept per device.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch;
}  // namespace

// Device address of this GPU's scratch array, looked up once per device.
int scratch_address(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(GD_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it == g_scratch.end()) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return fail(GD_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        it = g_scratch.emplace(dev, ptr).first;
    }
    *out = it->second;
    return GD_OK;
}

}  // namespace gd

using namespace gd;

extern "C" {

size_t deconvolve_noalloc_max_bytes(void) { return kScratchBytes; }

int deconvolve_noalloc(int32_t solver, const gd_grid *g, const void *ubar, void *u, const gd_opts *o, gd_info *info,
                       void *stream) {
    if (solver < GD_VANCITTERT || solver > GD_STEEPEST_DESCENT) return fail(GD_EINVAL, "bad solver %d", solver);
    int rc = validate_grid(g);
    if (rc) return rc;
    const size_t need = deconvolve_workspace_bytes(g, solver);
    if (need == 0 || need > kScratchBytes)
        return fail(GD_EWORKSPACE, "this solve needs %zu bytes of workspace; deconvolve_noalloc holds %zu", need,
                    kScratchBytes);
    void *work = nullptr;
    if ((rc = scratch_address(&work))) return rc;
    return solve_uniform(solver, g, ubar, u, o, work, kScratchBytes, info, stream, nullptr, nullptr);
}

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
    I.geo = make_geo(g->ndim, nx, ny, nz, ts.vw, ts.R, ts.L, 0);
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
    return solve_uniform(GD_VANCITTERT, g, ubar, u, o, work, wb, info, stream, nullptr, nullptr);
}

int deconvolve_cg(const gd_grid *g, const void *ubar, void *u, const gd_opts *o, void *work, size_t wb,
                  gd_info *info, void *stream) {
    return solve_uniform(GD_CG, g, ubar, u, o, work, wb, info, stream, nullptr, nullptr);
}

int deconvolve_bicgstab(const gd_grid *g, const void *ubar, void *u, const gd_opts *o, void *work, size_t wb,
                        gd_info *info, void *stream) {
    return solve_uniform(GD_BICGSTAB, g, ubar, u, o, work, wb, info, stream, nullptr, nullptr);
}

int deconvolve_steepest_descent(const gd_grid *g, const void *ubar, void *u, const gd_opts *o, void *work, size_t wb,
                                gd_info *info, void *stream) {
    return solve_uniform(GD_STEEPEST_DESCENT, g, ubar, u, o, work, wb, info, stream, nullptr, nullptr);
}

size_t deconvolve_batch_workspace_bytes(int32_t solver, int32_t dtype, const gd_instance *list, int32_t count) {
    if (solver < GD_VANCITTERT || solver > GD_STEEPEST_DESCENT) return 0;
    if ((dtype != GD_F32 && dtype != GD_F64) || !list || count < 1) return 0;
    if (validate_instances(list, count)) return 0;
    return batch_layout(solver, dtype, list, count).total;
}

int deconvolve_batch(int32_t solver, int32_t dtype, const gd_instance *list, int32_t count, const gd_opts *o,
                     void *work, size_t wb, gd_info *info, void *stream) {
    return solve_batch(solver, dtype, list, count, o, work, wb, info, stream, nullptr);
}

int deconvolve_autotune(int32_t solver, const gd_grid *g, const void *ubar, void *u, void *work, size_t wb,
                        gd_info *info, void *stream, gd_tune_info *out) {
    return tune_uniform(solver, g, ubar, u, work, wb, info, stream, out, nullptr);
}

int deconvolve_batch_autotune(int32_t solver, int32_t dtype, const gd_instance *list, int32_t count, void *work,
                              size_t wb, gd_info *info, void *stream, gd_tune_info *out) {
    const gd_opts o = trial_opts(solver), o2 = trial_opts(solver, true);
    std::vector<TuneCfg> cands;
    for (int bp : kBpcCands)
        for (int t : kTpwCands)
            for (int tl : kTailCands)
                for (int il = 0; il < 2; ++il)
                    for (int wc = 0; wc < 2; ++wc) {
                        TuneCfg c;
                        c.tpw = t;
                        c.tail = tl;
                        c.ilv = il;
                        c.wc = wc;
                        c.bpc = bp;
                        cands.push_back(c);
                    }
    auto launch = [&](const TuneCfg &c, bool long_trial) {
        return solve_batch(solver, dtype, list, count, long_trial ? &o2 : &o, work, wb, info, stream, &c);
    };
    const int best = time_candidates(cands, launch, (hipStream_t)stream, out);
    if (best < 0) return best;
    tune_store(key_batch(solver, dtype, list, count), cands[best]);
    return GD_OK;
}

static int tune_choice(const gd_tune_info *c, TuneCfg *cfg) {
    if (!c) return fail(GD_EINVAL, "choice is NULL");
    if (c->tiles_per_wave < 1 || c->tiles_per_wave > 64 || c->rows < 0 || c->rows > 4 || c->tail_pct < 0 ||
        c->tail_pct > 50 || (c->interleave != 0 && c->interleave != 1) || (c->wave_claims != 0 && c->wave_claims != 1) ||
        c->blocks_per_cu < 0 || c->blocks_per_cu > kMaxBlocksPerCu || c->segments < 0 || c->segments > kMaxSegs)
        return fail(GD_EINVAL, "launch configuration out of range");
    cfg->tpw = c->tiles_per_wave;
    cfg->rows = c->rows;
    cfg->tail = c->tail_pct;
    cfg->ilv = c->interleave;
    cfg->wc = c->wave_claims;
    cfg->bpc = c->blocks_per_cu;
    cfg->segs = c->segments;
    return GD_OK;
}

int gd_tune_set(int32_t solver, const gd_grid *g, const void *ubar, const void *u, const gd_tune_info *choice) {
    int rc = validate_grid(g);
    if (rc) return rc;
    if (solver < GD_VANCITTERT || solver > GD_STEEPEST_DESCENT) return fail(GD_EINVAL, "bad solver %d", solver);
    TuneCfg cfg;
    if ((rc = tune_choice(choice, &cfg))) return rc;
    const bool aligned = ((uintptr_t)ubar % 16 == 0) && ((uintptr_t)u % 16 == 0);
    tune_store(key_uniform(solver, g, aligned), cfg);
    return GD_OK;
}

int gd_tune_set_batch(int32_t solver, int32_t dtype, const gd_instance *list, int32_t count,
                      const gd_tune_info *choice) {
    if (solver < GD_VANCITTERT || solver > GD_STEEPEST_DESCENT) return fail(GD_EINVAL, "bad solver %d", solver);
    if ((dtype != GD_F32 && dtype != GD_F64) || !list || count < 1) return fail(GD_EINVAL, "bad instance list");
    int rc = validate_instances(list, count);
    if (rc) return rc;
    TuneCfg cfg;
    if ((rc = tune_choice(choice, &cfg))) return rc;
    tune_store(key_batch(solver, dtype, list, count), cfg);
    return GD_OK;
}

void gd_tune_reset(void) {
    std::lock_guard<std::mutex> lk(gd::g_tune_mu);
    gd::g_tune.clear();
    gd::g_tune_loaded = true;  // a cache file is not read again after a reset
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
    case GD_STAGNATED: return "GD_STAGNATED";
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
