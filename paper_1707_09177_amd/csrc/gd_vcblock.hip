// gd_vcblock.hip -- Van Cittert with K passes per sweep (temporal blocking).
//
// Algorithm 1 (u_{n+1} = u_n + r_n, r_{n+1} = r_n - G r_n, Eqs. adm2 and ric)
// needs the stencil only for r, and u just accumulates the residuals.  So a
// workgroup loads a tile of r_n with a K-point halo into LDS, and runs K passes
// there.  The valid region shrinks by one point per pass, so after K passes
// the tile interior holds r_{n+K}.  u_n + r_n + ... + r_{n+K-1} accumulates in
// registers, and ||r_{n+j}||^2 is summed over the interior for every j.  One
// sweep reads r (with its halo) and u, and writes r and u: about 4 + halo
// field accesses for K passes, against 4 K for one pass per sweep.
//
// The stopping rule still acts after every pass.  After each sweep launch a
// small kernel sums every field's K partial norms per pass in tile order and
// applies the rule pass by pass.  When the field stops at pass j < K inside
// the sweep, the sweep is redone from its inputs with j passes: u and r
// ping-pong between two buffer sets, and later sweeps skip a finished field,
// so those inputs are intact.  Pass counts, statuses and residual histories
// are those of the one-pass-per-sweep solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "gd_internal.h"

namespace gdvcb {

using gd::fail;

inline size_t align_up_256(size_t x) { return gd::align_up(x, 256); }

// Tile shapes: interior TX x TY (x TZ) and K passes per sweep, sized so that
// two LDS copies of the tile with its halo fit in 64 KB and a halo row
// (TX + 2K points) is a whole number of 64-lane waves.
template <typename T, int NDIM> struct Shape;
template <> struct Shape<float, 2> {
    static constexpr int TX = 112, TY = 32, TZ = 1, K = 8;
};
template <> struct Shape<double, 2> {
    static constexpr int TX = 48, TY = 32, TZ = 1, K = 8;
};
template <> struct Shape<float, 3> {
    static constexpr int TX = 32, TY = 8, TZ = 8, K = 2;
};
template <> struct Shape<double, 3> {
    static constexpr int TX = 16, TY = 8, TZ = 8, K = 2;
};

constexpr int kMaxK = 8;

struct alignas(128) VState {
    double r_ref, r0, r_last;
    int32_t iters, status, done, redo;  // redo: passes of the sweep to recompute
    int32_t parity;                     // buffer set holding the current u, r
    uint32_t pad;
};

// fields still iterating (the sweeps' fast exit) and fields with a sweep to recompute
struct alignas(128) Global {
    int32_t active, redo;
};

struct Args {
    Global *glob;
    const void *ubar;
    void *u[2], *r[2];
    double *part;     // [field][tile][kMaxK + 1]
    VState *st;
    double *hist;     // [field][max_iter + 1] or NULL
    gd_info *info;
    int64_t nx, ny, nz, npts;
    int64_t tx, ty, tz, tiles;  // tiles per axis / per field
    int64_t nfields;
    double tol;
    int32_t max_iter, init, norm_ref, steps;
};

// periodic index; the common case (already in range) takes no division
__device__ __forceinline__ int64_t wrapi(int64_t v, int64_t n) {
    if (v >= 0 && v < n) return v;
    const int64_t m = (int64_t)((int32_t)v % (int32_t)n);  // |v| < 2^31 for every field accepted
    return m < 0 ? m + n : m;
}

// Tile t of a field: origin and which interior points lie in the field.
struct TileOrg {
    int64_t x0, y0, z0;
};
__device__ __forceinline__ TileOrg tile_org(const Args &A, int64_t t, int TX, int TY, int TZ) {
    TileOrg o;
    o.x0 = (t % A.tx) * TX;
    o.y0 = ((t / A.tx) % A.ty) * TY;
    o.z0 = (t / (A.tx * A.ty)) * TZ;
    return o;
}

// Load a field region [x0-h, x0+TX+h) x ... (periodic) into LDS, x fastest:
// a wave per row, lanes along x.
template <typename T, int NDIM, int RX, int RY, int RZ>
__device__ __forceinline__ void load_region(T *dst, const T *src, const Args &A, const TileOrg &o, int h) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int row = wave; row < RY * RZ; row += 4) {
        const int iy = row % RY, iz = row / RY;
        const int64_t gy = wrapi(o.y0 + iy - h, A.ny);
        const int64_t gz = NDIM == 3 ? wrapi(o.z0 + iz - h, A.nz) : 0;
        const T *srow = src + (gz * A.ny + gy) * A.nx;
        T *drow = dst + row * RX;
        for (int ix = lane; ix < RX; ix += 64) drow[ix] = srow[wrapi(o.x0 + ix - h, A.nx)];
    }
}

// y = x - G x on the region shrunk by s points per side, reading x, writing y
// (a wave per row, lanes along x).
template <typename T, int NDIM, int RX, int RY, int RZ>
__device__ __forceinline__ void step(const T *x, T *y, int s) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int zlo = NDIM == 3 ? s : 0, zhi = NDIM == 3 ? RZ - s : 1;
    const int ny = RY - 2 * s;
    for (int iz = zlo; iz < zhi; ++iz)
        for (int iy = s + wave; iy < s + ny; iy += 4)
            for (int ix = s + lane; ix < RX - s; ix += 64) {
                const int c = (iz * RY + iy) * RX + ix;
                auto row = [&](int off) {
                    const T *p = x + c + off;
                    return T(0.5) * p[0] + T(0.25) * (p[-1] + p[1]);
                };
                auto plane = [&](int off) { return T(0.5) * row(off) + T(0.25) * (row(off - RX) + row(off + RX)); };
                T g;
                if constexpr (NDIM == 2) g = plane(0);
                else g = T(0.5) * plane(0) + T(0.25) * (plane(-RX * RY) + plane(RX * RY));
                y[c] = x[c] - g;
            }
}

__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double s = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return s;
}

// sums over the field's tiles, in tile order per thread, then threads in order
__device__ __forceinline__ double field_sum(const double *part, int64_t tiles, int j, double *red) {
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < tiles; t += 256) s += part[t * (kMaxK + 1) + j];
    return block_sum(s, red);
}

__device__ __forceinline__ int stop_rule(double rn, double tol, double r_ref, int n, int max_iter, int *status) {
    if (!isfinite(rn)) {
        *status = GD_NONFINITE;
        return 1;
    }
    if (rn == 0.0 || (tol > 0.0 && rn <= tol * r_ref)) {
        *status = GD_CONVERGED;
        return 1;
    }
    if (n >= max_iter) {
        *status = GD_MAXITER;
        return 1;
    }
    return 0;
}

// Initial guess, r0 = ubar - G u0, ||r0||^2, and the reference norm's square
// when it is not ||r0|| (partials j = 0 and 1).
template <typename T, int NDIM>
__global__ __launch_bounds__(256) void k_vcb_init(Args A) {
    using S = Shape<T, NDIM>;
    constexpr int RX = S::TX + 2, RY = S::TY + 2, RZ = NDIM == 3 ? S::TZ + 2 : 1;
    __shared__ T a[RX * RY * RZ], b[RX * RY * RZ];
    __shared__ double red[4];
    const int64_t f = blockIdx.x / A.tiles, t = blockIdx.x % A.tiles;
    const T *ub = static_cast<const T *>(A.ubar) + f * A.npts;
    T *u = static_cast<T *>(A.u[0]) + f * A.npts;
    T *r = static_cast<T *>(A.r[0]) + f * A.npts;
    const TileOrg o = tile_org(A, t, S::TX, S::TY, S::TZ);
    // G u0 over the interior (u0 = ubar, 0 or the caller's u)
    if (A.init == GD_INIT_GIVEN) load_region<T, NDIM, RX, RY, RZ>(a, u, A, o, 1);
    else load_region<T, NDIM, RX, RY, RZ>(a, ub, A, o, 1);
    __syncthreads();
    step<T, NDIM, RX, RY, RZ>(a, b, 1);  // b = a - G a
    __syncthreads();
    double rr = 0.0, rf = 0.0;
    constexpr int NI = S::TX * S::TY * S::TZ;
    for (int i = threadIdx.x; i < NI; i += 256) {
        const int ix = i % S::TX, iy = (i / S::TX) % S::TY, iz = i / (S::TX * S::TY);
        const int64_t gx = o.x0 + ix, gy = o.y0 + iy, gz = o.z0 + iz;
        if (gx >= A.nx || gy >= A.ny || (NDIM == 3 && gz >= A.nz)) continue;
        const int c = ((NDIM == 3 ? iz + 1 : 0) * RY + iy + 1) * RX + ix + 1;
        const int64_t g = (gz * A.ny + gy) * A.nx + gx;
        const T ubv = A.init == GD_INIT_GIVEN ? ub[g] : a[c];  // the tile holds ubar unless u0 is given
        T rv;
        if (A.init == GD_INIT_UBAR) {
            rv = b[c];  // ubar - G ubar
            u[g] = ubv;
        } else if (A.init == GD_INIT_ZERO) {
            rv = ubv;
            u[g] = T(0);
        } else {
            rv = ubv - (a[c] - b[c]);  // ubar - G u0
        }
        r[g] = rv;
        rr += double(rv) * double(rv);
        if (A.norm_ref == GD_REF_UBAR) rf += double(ubv) * double(ubv);
        else if (A.init != GD_INIT_UBAR) rf += double(b[c]) * double(b[c]);  // needs G ubar: below
    }
    if (A.norm_ref == GD_REF_R0UBAR && A.init == GD_INIT_GIVEN) {
        // a held u0: recompute ubar - G ubar for the reference norm
        __syncthreads();
        load_region<T, NDIM, RX, RY, RZ>(a, ub, A, o, 1);
        __syncthreads();
        step<T, NDIM, RX, RY, RZ>(a, b, 1);
        __syncthreads();
        rf = 0.0;
        for (int i = threadIdx.x; i < NI; i += 256) {
            const int ix = i % S::TX, iy = (i / S::TX) % S::TY, iz = i / (S::TX * S::TY);
            if (o.x0 + ix >= A.nx || o.y0 + iy >= A.ny || (NDIM == 3 && o.z0 + iz >= A.nz)) continue;
            const int c = ((NDIM == 3 ? iz + 1 : 0) * RY + iy + 1) * RX + ix + 1;
            rf += double(b[c]) * double(b[c]);
        }
    }
    const double srr = block_sum(rr, red), srf = block_sum(rf, red);
    double *pp = A.part + (f * A.tiles + t) * (kMaxK + 1);
    if (threadIdx.x == 0) {
        pp[0] = srr;
        pp[1] = srf;
    }
}

// Per field, after the init launch: r0, the reference norm, the guards and the
// stopping rule at pass 0.  One workgroup per field; partials summed in tile order.
__global__ __launch_bounds__(256) void k_vcb_init_reduce(Args A) {
    __shared__ double red[4];
    const int64_t f = blockIdx.x;
    VState *st = A.st + f;
    const double r0sq = field_sum(A.part + f * A.tiles * (kMaxK + 1), A.tiles, 0, red);
    const double rfsq = field_sum(A.part + f * A.tiles * (kMaxK + 1), A.tiles, 1, red);
    if (threadIdx.x != 0) return;
    const double r0 = sqrt(r0sq);
    const double r_ref = (A.norm_ref == GD_REF_R0UBAR && A.init == GD_INIT_UBAR) ? r0 : sqrt(rfsq);
    st->r0 = r0;
    st->r_ref = r_ref;
    st->r_last = r0;
    int status = GD_MAXITER, done;
    if (!isfinite(r_ref)) {
        status = GD_NONFINITE;
        done = 1;
    } else if (r_ref == 0.0) {
        status = GD_ZERO_REF;
        done = 1;
    } else {
        done = stop_rule(r0, A.tol, r_ref, 0, A.max_iter, &status);
    }
    st->status = status;
    st->done = done;
    if (done) atomicAdd(&A.glob->active, -1);
    if (A.hist) A.hist[f * (A.max_iter + 1)] = r0;
}

// One sweep of up to K passes over every tile (REDO: recompute a stopped
// field's last sweep with its recorded pass count).  A grid of resident
// workgroups strides over the tiles, so a launch whose fields have all
// stopped costs one state read per tile.
template <typename T, int NDIM, bool REDO>
__global__ __launch_bounds__(256) void k_vcb_sweep(Args A) {
    using S = Shape<T, NDIM>;
    constexpr int K = S::K;
    constexpr int RX = S::TX + 2 * K, RY = S::TY + 2 * K, RZ = NDIM == 3 ? S::TZ + 2 * K : 1;
    constexpr int NI = S::TX * S::TY * S::TZ;
    constexpr int PER = (NI + 255) / 256;  // interior points per thread
    __shared__ T a[RX * RY * RZ], b[RX * RY * RZ];
    __shared__ double red[4];
    __shared__ int skip, passes, par, any;
    // the state is only written between launches (by the reduction kernels)
    if (threadIdx.x == 0) any = REDO ? A.glob->redo : A.glob->active;
    __syncthreads();
    if (any <= 0) return;  // every field has stopped (or nothing to recompute)
    int64_t fcur = -1;
    for (int64_t bt = blockIdx.x; bt < A.nfields * A.tiles; bt += gridDim.x) {
        const int64_t f = bt / A.tiles, t = bt % A.tiles;
        VState *st = A.st + f;
        if (f != fcur) {
            __syncthreads();
            if (threadIdx.x == 0) {
                skip = REDO ? st->redo == 0 : st->done != 0;
                passes = REDO ? st->redo : A.steps;
                par = st->parity;
            }
            __syncthreads();
            fcur = f;
        }
        if (skip) continue;
        const int p = par;
        const int steps = passes;
        const T *rin = static_cast<const T *>(A.r[p]) + f * A.npts;
        const T *uin = static_cast<const T *>(A.u[p]) + f * A.npts;
        T *rout = static_cast<T *>(A.r[1 - p]) + f * A.npts;
        T *uout = static_cast<T *>(A.u[1 - p]) + f * A.npts;
        const TileOrg o = tile_org(A, t, S::TX, S::TY, S::TZ);
        load_region<T, NDIM, RX, RY, RZ>(a, rin, A, o, K);
        // the thread's interior points: LDS index, field index, in-field flag
        int li[PER];
        int64_t gi[PER];
        bool in[PER];
        T uacc[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = threadIdx.x + 256 * q;
            const int ix = i % S::TX, iy = (i / S::TX) % S::TY, iz = i / (S::TX * S::TY);
            const int64_t gx = o.x0 + ix, gy = o.y0 + iy, gz = o.z0 + iz;
            in[q] = i < NI && gx < A.nx && gy < A.ny && (NDIM == 2 || gz < A.nz);
            li[q] = ((NDIM == 3 ? iz + K : 0) * RY + iy + K) * RX + ix + K;
            gi[q] = (gz * A.ny + gy) * A.nx + gx;
            uacc[q] = in[q] ? uin[gi[q]] : T(0);
        }
        __syncthreads();
        double nrm[kMaxK];
        T *x = a, *y = b;
        for (int j = 0; j < steps; ++j) {
#pragma unroll
            for (int q = 0; q < PER; ++q)
                if (in[q]) uacc[q] += x[li[q]];  // u_{n+j+1} = u_{n+j} + r_{n+j}
            // pass j leaves r valid on the region shrunk by K - steps + j + 1
            // points per side: the interior after the last pass
            step<T, NDIM, RX, RY, RZ>(x, y, K - steps + j + 1);
            __syncthreads();
            double sum = 0.0;
#pragma unroll
            for (int q = 0; q < PER; ++q)
                if (in[q]) sum += double(y[li[q]]) * double(y[li[q]]);
            nrm[j] = sum;
            T *tmp = x;
            x = y;
            y = tmp;
        }
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (in[q]) {
                uout[gi[q]] = uacc[q];
                rout[gi[q]] = x[li[q]];
            }
        double *pp = A.part + (f * A.tiles + t) * (kMaxK + 1);
        for (int j = 0; j < steps; ++j) {
            const double sj = block_sum(nrm[j], red);
            if (threadIdx.x == 0) pp[j] = sj;
        }
    }
}

// Per field, after a sweep launch: the residual norm of every pass of the
// sweep (partials summed in tile order), the stopping rule pass by pass, and
// the state for the next launch.
template <bool REDO>
__global__ __launch_bounds__(256) void k_vcb_sweep_reduce(Args A) {
    __shared__ double red[4];
    const int64_t f = blockIdx.x;
    VState *st = A.st + f;
    if (REDO ? st->redo == 0 : st->done != 0) return;  // uniform across the workgroup
    const int steps = REDO ? st->redo : A.steps;
    double tot[kMaxK];
    for (int j = 0; j < steps; ++j) tot[j] = field_sum(A.part + f * A.tiles * (kMaxK + 1), A.tiles, j, red);
    if (threadIdx.x != 0) return;
    const int p = st->parity;
    if (REDO) {
        st->r_last = sqrt(tot[steps - 1]);
        st->parity = 1 - p;
        st->redo = 0;
        atomicAdd(&A.glob->redo, -1);
        return;
    }
    const int n0 = st->iters;
    int status = GD_MAXITER;
    for (int j = 0; j < steps; ++j) {
        const int n = n0 + j + 1;
        const double rn = sqrt(tot[j]);
        if (A.hist) A.hist[f * (A.max_iter + 1) + n] = rn;
        if (stop_rule(rn, A.tol, st->r_ref, n, A.max_iter, &status)) {
            st->iters = n;
            st->status = status;
            st->r_last = rn;
            if (j + 1 < steps) {  // stopped inside the sweep: recompute j + 1 passes
                st->redo = j + 1;
                atomicAdd(&A.glob->redo, 1);
            } else {
                st->parity = 1 - p;
            }
            st->done = 1;
            atomicAdd(&A.glob->active, -1);
            return;
        }
    }
    st->iters = n0 + steps;
    st->r_last = sqrt(tot[steps - 1]);
    st->parity = 1 - p;
}

// Exit: the true residual ||ubar - G u|| of the final u, the info record, and
// u moved to the caller's buffer when it ended in the workspace copy.
template <typename T, int NDIM>
__global__ __launch_bounds__(256) void k_vcb_finish(Args A, double hw_sqrt) {
    using S = Shape<T, NDIM>;
    constexpr int RX = S::TX + 2, RY = S::TY + 2, RZ = NDIM == 3 ? S::TZ + 2 : 1;
    constexpr int NI = S::TX * S::TY * S::TZ;
    __shared__ T a[RX * RY * RZ], b[RX * RY * RZ];
    __shared__ double red[4];
    const int64_t f = blockIdx.x / A.tiles, t = blockIdx.x % A.tiles;
    const VState *st = A.st + f;
    const int p = st->parity;
    const T *ub = static_cast<const T *>(A.ubar) + f * A.npts;
    const T *uf = static_cast<const T *>(A.u[p]) + f * A.npts;
    T *uc = static_cast<T *>(A.u[0]) + f * A.npts;
    const TileOrg o = tile_org(A, t, S::TX, S::TY, S::TZ);
    load_region<T, NDIM, RX, RY, RZ>(a, uf, A, o, 1);
    __syncthreads();
    step<T, NDIM, RX, RY, RZ>(a, b, 1);  // b = u - G u
    __syncthreads();
    double s = 0.0;
    for (int i = threadIdx.x; i < NI; i += 256) {
        const int ix = i % S::TX, iy = (i / S::TX) % S::TY, iz = i / (S::TX * S::TY);
        const int64_t gx = o.x0 + ix, gy = o.y0 + iy, gz = o.z0 + iz;
        if (gx >= A.nx || gy >= A.ny || (NDIM == 3 && gz >= A.nz)) continue;
        const int c = ((NDIM == 3 ? iz + 1 : 0) * RY + iy + 1) * RX + ix + 1;
        const int64_t g = (gz * A.ny + gy) * A.nx + gx;
        const double d = double(ub[g]) - (double(a[c]) - double(b[c]));  // ubar - G u
        s += d * d;
        if (p != 0) uc[g] = a[c];  // the result ended in the workspace copy
    }
    const double ss = block_sum(s, red);
    if (threadIdx.x == 0) A.part[(f * A.tiles + t) * (kMaxK + 1) + kMaxK] = ss;
}

__global__ __launch_bounds__(256) void k_vcb_finish_reduce(Args A, double hw_sqrt) {
    __shared__ double red[4];
    const int64_t f = blockIdx.x;
    const VState *st = A.st + f;
    const double tsq = field_sum(A.part + f * A.tiles * (kMaxK + 1), A.tiles, kMaxK, red);
    if (threadIdx.x != 0) return;
    gd_info &I = A.info[f];
    I.iters = st->iters;
    I.status = st->status;
    I.r_ref = st->r_ref * hw_sqrt;
    I.r0 = st->r0 * hw_sqrt;
    I.r_final = st->r_last * hw_sqrt;
    I.r_true = sqrt(tsq) * hw_sqrt;
    I.start = A.init;
    I.replaced = 0;
}

// history entries are norms without the spacing weight until scaled here
__global__ void k_vcb_hist_scale(double *hist, int64_t n, double w) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        hist[i] *= w;
}

__global__ void k_vcb_prep(VState *st, Global *glob, int64_t nfields) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        glob->active = (int32_t)nfields;
        glob->redo = 0;
    }
    if (i < nfields) {
        st[i].done = 0;
        st[i].redo = 0;
        st[i].parity = 0;
        st[i].iters = 0;
    }
}


template <typename T, int NDIM>
void tiles_of(const gd_grid *g, int64_t &tx, int64_t &ty, int64_t &tz) {
    using S = Shape<T, NDIM>;
    tx = (g->n[0] + S::TX - 1) / S::TX;
    ty = (g->n[1] + S::TY - 1) / S::TY;
    tz = NDIM == 3 ? (g->n[2] + S::TZ - 1) / S::TZ : 1;
}

// the host issues two launches per sweep of K passes, up to max_iter passes
constexpr int kMaxBlockedIter = 1 << 20;

struct Layout {
    size_t glob, st, part, r0, r1, u1, total;
    int64_t tiles;
};

Layout layout(const gd_grid *g) {
    Layout L;
    int64_t tx, ty, tz;
    if (g->dtype == GD_F32) {
        if (g->ndim == 2) tiles_of<float, 2>(g, tx, ty, tz);
        else tiles_of<float, 3>(g, tx, ty, tz);
    } else {
        if (g->ndim == 2) tiles_of<double, 2>(g, tx, ty, tz);
        else tiles_of<double, 3>(g, tx, ty, tz);
    }
    L.tiles = tx * ty * tz;
    const size_t ts = g->dtype == GD_F32 ? 4 : 8;
    const size_t fb = align_up_256((size_t)g->batch * g->n[0] * g->n[1] * (g->ndim == 3 ? g->n[2] : 1) * ts);
    size_t off = 0;
    L.glob = off;
    off = align_up_256(off + sizeof(Global));
    L.st = off;
    off = align_up_256(off + (size_t)g->batch * sizeof(VState));
    L.part = off;
    off = align_up_256(off + (size_t)g->batch * L.tiles * (kMaxK + 1) * sizeof(double));
    L.r0 = off;
    L.r1 = off + fb;
    L.u1 = off + 2 * fb;
    L.total = off + 3 * fb;
    return L;
}

template <typename T, int NDIM>
int run(const gd_grid *g, const void *ubar, void *u, const gd_opts *o, void *work, const Layout &L, gd_info *info,
        hipStream_t st) {
    using S = Shape<T, NDIM>;
    Args A;
    std::memset(&A, 0, sizeof A);
    char *w = (char *)work;
    A.ubar = ubar;
    A.u[0] = u;
    A.u[1] = w + L.u1;
    A.r[0] = w + L.r0;
    A.r[1] = w + L.r1;
    A.part = (double *)(w + L.part);
    A.st = (VState *)(w + L.st);
    A.glob = (Global *)(w + L.glob);
    A.hist = o->history;
    A.info = info;
    A.nx = g->n[0];
    A.ny = g->n[1];
    A.nz = NDIM == 3 ? g->n[2] : 1;
    A.npts = A.nx * A.ny * A.nz;
    tiles_of<T, NDIM>(g, A.tx, A.ty, A.tz);
    A.tiles = L.tiles;
    A.nfields = g->batch;
    A.tol = o->tol;
    A.max_iter = o->max_iter;
    A.init = o->init;
    A.norm_ref = o->norm_ref;
    const int64_t nblk = g->batch * A.tiles;
    if (nblk > 0x7fffffff) return fail(GD_EINVAL, "field too large");
    // resident workgroups of the sweep kernel: its persistent grid
    int dev = 0, ncu = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_vcb_sweep<T, NDIM, false>, 256, 0) != hipSuccess)
        return fail(GD_EHIP, "device query failed");
    const unsigned sweep_blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nblk, (int64_t)std::max(occ, 1) * ncu));
    hipLaunchKernelGGL(k_vcb_prep, dim3((unsigned)((g->batch + 255) / 256)), dim3(256), 0, st, A.st, A.glob, g->batch);
    const dim3 per_field((unsigned)g->batch);
    hipLaunchKernelGGL((k_vcb_init<T, NDIM>), dim3((unsigned)nblk), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_vcb_init_reduce, per_field, dim3(256), 0, st, A);
    for (int done = 0; done < o->max_iter; done += S::K) {
        A.steps = std::min(S::K, o->max_iter - done);
        hipLaunchKernelGGL((k_vcb_sweep<T, NDIM, false>), dim3(sweep_blocks), dim3(256), 0, st, A);
        hipLaunchKernelGGL(k_vcb_sweep_reduce<false>, per_field, dim3(256), 0, st, A);
    }
    A.steps = 0;
    hipLaunchKernelGGL((k_vcb_sweep<T, NDIM, true>), dim3(sweep_blocks), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_vcb_sweep_reduce<true>, per_field, dim3(256), 0, st, A);
    // norms above are plain sums; the inner product carries the spacing weight h^d
    const double hw = gd::grid_weight(g);
    hipLaunchKernelGGL((k_vcb_finish<T, NDIM>), dim3((unsigned)nblk), dim3(256), 0, st, A, sqrt(hw));
    hipLaunchKernelGGL(k_vcb_finish_reduce, per_field, dim3(256), 0, st, A, sqrt(hw));
    if (o->history) {
        const int64_t nh = g->batch * (int64_t)(o->max_iter + 1);
        hipLaunchKernelGGL(k_vcb_hist_scale, dim3((unsigned)std::min<int64_t>((nh + 255) / 256, 4096)), dim3(256), 0,
                           st, o->history, nh, sqrt(hw));
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GD_OK : fail(GD_EHIP, "blocked Van Cittert launch: %s", hipGetErrorString(e));
}


}  // namespace gdvcb

using namespace gdvcb;

extern "C" {

size_t vancittert_blocked_workspace_bytes(const gd_grid *g) {
    if (gd::validate_grid(g)) return 0;
    return layout(g).total;
}

int32_t vancittert_blocked_passes(const gd_grid *g) {
    if (gd::validate_grid(g)) return 0;
    if (g->ndim == 2) return g->dtype == GD_F32 ? Shape<float, 2>::K : Shape<double, 2>::K;
    return g->dtype == GD_F32 ? Shape<float, 3>::K : Shape<double, 3>::K;
}

int deconvolve_vancittert_blocked(const gd_grid *g, const void *ubar, void *u, const gd_opts *o, void *work,
                                  size_t wb, gd_info *info, void *stream) {
    int rc = gd::validate_grid(g);
    if (rc) return rc;
    if ((rc = gd::validate_opts(o))) return rc;
    if (o->init == GD_INIT_WARM) return fail(GD_EINVAL, "the blocked Van Cittert takes the ubar, zero or given start");
    if (o->max_iter > kMaxBlockedIter)
        return fail(GD_EINVAL, "max_iter must be at most %d (the host launches every sweep)", kMaxBlockedIter);
    if (!ubar || !u || !info) return fail(GD_EINVAL, "ubar, u and info must be non-NULL");
    if (!work) return fail(GD_EWORKSPACE, "workspace is NULL");
    if ((uintptr_t)work % 256) return fail(GD_EALIGN, "workspace must be 256-byte aligned");
    for (int d = 0; d < g->ndim; ++d)
        if (g->n[d] >= (int64_t(1) << 30)) return fail(GD_EINVAL, "n[%d] must be below 2^30", d);
    const Layout L = layout(g);
    if (wb < L.total) return fail(GD_EWORKSPACE, "workspace too small: need %zu bytes, got %zu", L.total, wb);
    const size_t fb = (size_t)g->batch * g->n[0] * g->n[1] * (g->ndim == 3 ? g->n[2] : 1) * (g->dtype == GD_F32 ? 4 : 8);
    if (gd::ranges_overlap(ubar, fb, u, fb)) return fail(GD_EINVAL, "ubar and u overlap");
    if (gd::ranges_overlap(ubar, fb, work, L.total) || gd::ranges_overlap(u, fb, work, L.total))
        return fail(GD_EINVAL, "a field overlaps the workspace");
    hipStream_t st = (hipStream_t)stream;
    if (g->dtype == GD_F32)
        return g->ndim == 2 ? run<float, 2>(g, ubar, u, o, work, L, info, st) : run<float, 3>(g, ubar, u, o, work, L, info, st);
    return g->ndim == 2 ? run<double, 2>(g, ubar, u, o, work, L, info, st) : run<double, 3>(g, ubar, u, o, work, L, info, st);
}

}  // extern "C"
