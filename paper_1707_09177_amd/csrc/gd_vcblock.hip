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
    int32_t next;                       // passes of the field's next sweep
    int32_t nshort;                     // sweeps shortened to a predicted stop so far
};

// Sweeps a field may shorten to the passes its residual's decay rate predicts
// to the tolerance (the host launches this many sweeps beyond max_iter / K).
constexpr int kShortSweeps = 2;

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
    int64_t tx, ty, tz, tiles;  // tiles per axis / per field (init and exit kernels; 2D sweeps)
    int64_t mx, my, mz, stiles; // 3D sweeps: column tiles per axis / per field (the z march)
    int64_t pslots;             // partial-sum slots per field: max(tiles, stiles)
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
    double *pp = A.part + (f * A.pslots + t) * (kMaxK + 1);
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
    const double r0sq = field_sum(A.part + f * A.pslots * (kMaxK + 1), A.tiles, 0, red);
    const double rfsq = field_sum(A.part + f * A.pslots * (kMaxK + 1), A.tiles, 1, red);
    if (threadIdx.x != 0) return;
    const double r0 = sqrt(r0sq);
    const double r_ref = (A.norm_ref == GD_REF_R0UBAR && A.init == GD_INIT_UBAR) ? r0 : sqrt(rfsq);
    st->r0 = r0;
    st->r_ref = r_ref;
    st->r_last = r0;
    st->next = A.steps;
    st->nshort = 0;
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
                passes = REDO ? st->redo : st->next;
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
        double *pp = A.part + (f * A.pslots + t) * (kMaxK + 1);
        for (int j = 0; j < steps; ++j) {
            const double sj = block_sum(nrm[j], red);
            if (threadIdx.x == 0) pp[j] = sj;
        }
    }
}

// 3D sweeps march along z (2.5D blocking).  A workgroup owns a column of
// TX x TY interior points and TZ interior planes; it loads r_n one plane at
// a time with a K-point periodic halo in x and y (the planes K below and
// above the chunk included), and every pass j = 1 .. K runs one plane behind
// the pass before it: r_{n+j} on plane p needs r_{n+j-1} on planes p-1, p, p+1.
// Per plane and pass, the x-y part of G (9 weights) is applied from LDS to
// the previous pass's plane, and the z part from a window of three such
// planes that each thread keeps in registers for the points it owns; so LDS
// holds one plane per pass, not a 3D block with halo in z, and r is read
// once (plus x-y halo) and written once per K passes.
constexpr int kMarchThreads = 512;

// sum over the march kernel's workgroup, waves in order
__device__ __forceinline__ double march_block_sum(double v, double *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kMarchThreads / 64; ++w) t += red[w];
    __syncthreads();
    return t;
}

template <typename T> struct MShape;
template <> struct MShape<float> {
    static constexpr int TX = 64, TY = 32, TZ = 32;
};
template <> struct MShape<double> {
    static constexpr int TX = 32, TY = 32, TZ = 32;
};

template <typename T, bool REDO>
__global__ __launch_bounds__(kMarchThreads) void k_vcb_march(Args A) {
    using S = MShape<T>;
    constexpr int K = Shape<T, 3>::K;
    constexpr int RX = S::TX + 2 * K, RY = S::TY + 2 * K, NP = RX * RY;  // a loaded plane (interior + halo)
    constexpr int CX = RX - 2, NC = CX * (RY - 2);                         // points a pass computes
    constexpr int NT = kMarchThreads, PL = (NP + NT - 1) / NT, PC = (NC + NT - 1) / NT;
    __shared__ T buf[K][NP];  // plane of r_{n+j} being consumed, j = 0 .. K-1
    __shared__ double red[NT / 64];
    __shared__ int skip, passes, par, any;
    if (threadIdx.x == 0) any = REDO ? A.glob->redo : A.glob->active;
    __syncthreads();
    if (any <= 0) return;
    const int tid = threadIdx.x;
    const int64_t plane = A.nx * A.ny;
    int64_t fcur = -1;
    for (int64_t bt = blockIdx.x; bt < A.nfields * A.stiles; bt += gridDim.x) {
        const int64_t f = bt / A.stiles, t = bt % A.stiles;
        VState *st = A.st + f;
        if (f != fcur) {
            __syncthreads();
            if (tid == 0) {
                skip = REDO ? st->redo == 0 : st->done != 0;
                passes = REDO ? st->redo : st->next;
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
        const int64_t x0 = (t % A.mx) * S::TX, y0 = ((t / A.mx) % A.my) * S::TY, z0 = (t / (A.mx * A.my)) * S::TZ;
        const int64_t zlo = z0 - K;
        // loaded points: in-plane offsets of the region (periodic; a plane
        // holds fewer than 2^31 points, the host checks)
        uint32_t lo[PL];
#pragma unroll
        for (int q = 0; q < PL; ++q) {
            const int i = min(tid + NT * q, NP - 1);
            lo[q] = (uint32_t)(wrapi(y0 + i / RX - K, A.ny) * A.nx + wrapi(x0 + i % RX - K, A.nx));
        }
        // computed points: LDS index, interior flag, in-plane offset
        int li[PC];
        bool in[PC];
        uint32_t go[PC];
#pragma unroll
        for (int q = 0; q < PC; ++q) {
            const int i = tid + NT * q;
            const int cx = i % CX + 1, cy = i / CX + 1;  // region coordinates
            li[q] = i < NC ? cy * RX + cx : RX + 1;
            const int64_t gx = x0 + cx - K, gy = y0 + cy - K;
            in[q] = i < NC && cx >= K && cx < K + S::TX && cy >= K && cy < K + S::TY && gx < A.nx && gy < A.ny;
            go[q] = in[q] ? (uint32_t)(gy * A.nx + gx) : 0u;
        }
        // per pass j: the x-y filtered planes of r_{n+j-1} (window of three)
        // and its values on the two latest planes, at the thread's points
        T F[K][3][PC], Cv[K][2][PC];
        T uacc[K + 1][PC];  // u_n + r_n + ... on the planes in flight (newest last)
        double nrm[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            nrm[j] = 0.0;
#pragma unroll
            for (int q = 0; q < PC; ++q) F[j][0][q] = F[j][1][q] = F[j][2][q] = Cv[j][0][q] = Cv[j][1][q] = T(0);
        }
#pragma unroll
        for (int k = 0; k <= K; ++k)
#pragma unroll
            for (int q = 0; q < PC; ++q) uacc[k][q] = T(0);
        T pre[PL];
        {
            const T *src = rin + wrapi(zlo, A.nz) * plane;
#pragma unroll
            for (int q = 0; q < PL; ++q) pre[q] = src[lo[q]];
        }
        const int nstep = S::TZ + K + steps;  // the last interior plane leaves pass `steps` at step nstep - 1
        for (int s = 0; s < nstep; ++s) {
            const int64_t zs = zlo + s;  // plane entering as r_n
            __syncthreads();             // every read of buf from the previous step is done
#pragma unroll
            for (int q = 0; q < PL; ++q)
                if (tid + NT * q < NP) buf[0][tid + NT * q] = pre[q];
            // u_n on this plane starts its accumulator
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int q = 0; q < PC; ++q) uacc[k][q] = uacc[k + 1][q];
            {
                const bool inz = zs >= z0 && zs < z0 + S::TZ && zs < A.nz;
                const T *src = uin + (inz ? zs : 0) * plane;
#pragma unroll
                for (int q = 0; q < PC; ++q) uacc[K][q] = (inz && in[q]) ? src[go[q]] : T(0);
            }
            if (s + 1 < nstep) {  // prefetch the next plane of r_n
                const T *src = rin + wrapi(zs + 1, A.nz) * plane;
#pragma unroll
                for (int q = 0; q < PL; ++q) pre[q] = src[lo[q]];
            }
            __syncthreads();
#pragma unroll
            for (int j = 1; j <= K; ++j) {
                if (j > steps) break;
                // pass j - 1 holds plane zs - (j - 1) in buf[j - 1] (from this step)
                if (s < 2 * (j - 1)) break;  // ... from step 2 (j - 1) on
#pragma unroll
                for (int q = 0; q < PC; ++q) {
                    const T *b = &buf[j - 1][li[q]];
                    auto rowf = [&](int o) { return T(0.5) * b[o] + T(0.25) * (b[o - 1] + b[o + 1]); };
                    F[j - 1][0][q] = F[j - 1][1][q];
                    F[j - 1][1][q] = F[j - 1][2][q];
                    F[j - 1][2][q] = T(0.5) * rowf(0) + T(0.25) * (rowf(-RX) + rowf(RX));
                    Cv[j - 1][0][q] = Cv[j - 1][1][q];
                    Cv[j - 1][1][q] = b[0];
                }
                if (s < 2 * j) break;  // the window of pass j - 1 is complete from step 2 j on
                // r_{n+j} on plane pz = zs - j
                const int64_t pz = zs - j;
                const bool inz = pz >= z0 && pz < z0 + S::TZ && pz < A.nz;
                T v[PC];
#pragma unroll
                for (int q = 0; q < PC; ++q) {
                    const T c = Cv[j - 1][0][q];
                    v[q] = c - (T(0.5) * F[j - 1][1][q] + T(0.25) * (F[j - 1][0][q] + F[j - 1][2][q]));
                    if (inz && in[q]) {
                        uacc[K - j][q] += c;  // u_{n+j} = u_{n+j-1} + r_{n+j-1}
                        nrm[j - 1] += double(v[q]) * double(v[q]);
                    }
                }
                if (j == steps) {
                    if (inz) {
#pragma unroll
                        for (int q = 0; q < PC; ++q)
                            if (in[q]) {
                                rout[pz * plane + go[q]] = v[q];
                                uout[pz * plane + go[q]] = uacc[K - j][q];
                            }
                    }
                    break;
                }
                // buf[j] was last read in the previous step, before this step's first barrier
#pragma unroll
                for (int q = 0; q < PC; ++q)
                    if (tid + NT * q < NC) buf[j][li[q]] = v[q];
                __syncthreads();
            }
        }
        double *pp = A.part + (f * A.pslots + t) * (kMaxK + 1);
        for (int j = 0; j < steps; ++j) {
            const double sj = march_block_sum(nrm[j], red);
            if (tid == 0) pp[j] = sj;
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
    const int steps = REDO ? st->redo : st->next;
    double tot[kMaxK];
    for (int j = 0; j < steps; ++j) tot[j] = field_sum(A.part + f * A.pslots * (kMaxK + 1), A.stiles, j, red);
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
    const double r_now = sqrt(tot[steps - 1]);
    const double r_prev = steps >= 2 ? sqrt(tot[steps - 2]) : st->r_last;
    st->r_last = r_now;
    st->parity = 1 - p;
    // The next sweep runs all A.steps passes or, at most kShortSweeps times
    // per field, the passes the last decay rate predicts to the tolerance
    // (Algorithm 1's residual shrinks by a nearly constant factor per pass
    // once its slowest mode dominates), so that the stop falls on a sweep's
    // last pass and nothing is recomputed.  A wrong prediction costs a short
    // sweep or a recomputation; the stopping rule itself is unchanged.
    int nx = A.steps;
    if (A.tol > 0.0 && st->nshort < kShortSweeps && r_now > 0.0 && r_now < r_prev) {
        const double need = log(A.tol * st->r_ref / r_now) / log(r_now / r_prev);
        if (need >= 0.0 && need < (double)A.steps) {
            nx = max(1, (int)ceil(need));
            ++st->nshort;
        }
    }
    st->next = min(nx, A.max_iter - st->iters);
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
    if (threadIdx.x == 0) A.part[(f * A.pslots + t) * (kMaxK + 1) + kMaxK] = ss;
}

__global__ __launch_bounds__(256) void k_vcb_finish_reduce(Args A, double hw_sqrt) {
    __shared__ double red[4];
    const int64_t f = blockIdx.x;
    const VState *st = A.st + f;
    const double tsq = field_sum(A.part + f * A.pslots * (kMaxK + 1), A.tiles, kMaxK, red);
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
    int64_t tiles, stiles, pslots;
};

// column tiles of the 3D z march
template <typename T>
void march_tiles_of(const gd_grid *g, int64_t &mx, int64_t &my, int64_t &mz) {
    using S = MShape<T>;
    mx = (g->n[0] + S::TX - 1) / S::TX;
    my = (g->n[1] + S::TY - 1) / S::TY;
    mz = (g->n[2] + S::TZ - 1) / S::TZ;
}

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
    L.stiles = L.tiles;
    if (g->ndim == 3) {
        int64_t mx, my, mz;
        if (g->dtype == GD_F32) march_tiles_of<float>(g, mx, my, mz);
        else march_tiles_of<double>(g, mx, my, mz);
        L.stiles = mx * my * mz;
    }
    L.pslots = std::max(L.tiles, L.stiles);
    const size_t ts = g->dtype == GD_F32 ? 4 : 8;
    const size_t fb = align_up_256((size_t)g->batch * g->n[0] * g->n[1] * (g->ndim == 3 ? g->n[2] : 1) * ts);
    size_t off = 0;
    L.glob = off;
    off = align_up_256(off + sizeof(Global));
    L.st = off;
    off = align_up_256(off + (size_t)g->batch * sizeof(VState));
    L.part = off;
    off = align_up_256(off + (size_t)g->batch * L.pslots * (kMaxK + 1) * sizeof(double));
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
    A.stiles = L.stiles;
    A.pslots = L.pslots;
    if constexpr (NDIM == 3) march_tiles_of<T>(g, A.mx, A.my, A.mz);
    A.nfields = g->batch;
    A.tol = o->tol;
    A.max_iter = o->max_iter;
    A.init = o->init;
    A.norm_ref = o->norm_ref;
    const int64_t nblk = g->batch * A.tiles, sblk = g->batch * A.stiles;
    if (nblk > 0x7fffffff) return fail(GD_EINVAL, "field too large");
    // resident workgroups of the sweep kernel: its persistent grid
    auto sweep_fn = [] {
        if constexpr (NDIM == 3) return k_vcb_march<T, false>;
        else return k_vcb_sweep<T, NDIM, false>;
    }();
    int dev = 0, ncu = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, sweep_fn, NDIM == 3 ? kMarchThreads : 256, 0) != hipSuccess)
        return fail(GD_EHIP, "device query failed");
    const unsigned sweep_blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(sblk, (int64_t)std::max(occ, 1) * ncu));
    auto launch_sweep = [&](bool redo) {
        if constexpr (NDIM == 3) {
            if (redo) hipLaunchKernelGGL((k_vcb_march<T, true>), dim3(sweep_blocks), dim3(kMarchThreads), 0, st, A);
            else hipLaunchKernelGGL((k_vcb_march<T, false>), dim3(sweep_blocks), dim3(kMarchThreads), 0, st, A);
        } else {
            if (redo) hipLaunchKernelGGL((k_vcb_sweep<T, NDIM, true>), dim3(sweep_blocks), dim3(256), 0, st, A);
            else hipLaunchKernelGGL((k_vcb_sweep<T, NDIM, false>), dim3(sweep_blocks), dim3(256), 0, st, A);
        }
    };
    // passes per sweep (a field's own count, at most this, is set by the
    // reduce kernels)
    A.steps = std::min(S::K, o->max_iter);
    hipLaunchKernelGGL(k_vcb_prep, dim3((unsigned)((g->batch + 255) / 256)), dim3(256), 0, st, A.st, A.glob, g->batch);
    const dim3 per_field((unsigned)g->batch);
    hipLaunchKernelGGL((k_vcb_init<T, NDIM>), dim3((unsigned)nblk), dim3(256), 0, st, A);
    hipLaunchKernelGGL(k_vcb_init_reduce, per_field, dim3(256), 0, st, A);
    // enough sweeps for max_iter passes, also for a field that shortened
    // kShortSweeps of them (each runs at least one pass)
    const int nsweeps = o->max_iter > 0 ? (o->max_iter + S::K - 1) / S::K + kShortSweeps : 0;
    for (int k = 0; k < nsweeps; ++k) {
        launch_sweep(false);
        hipLaunchKernelGGL(k_vcb_sweep_reduce<false>, per_field, dim3(256), 0, st, A);
    }
    launch_sweep(true);
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
    if (g->ndim == 3 && g->n[0] * g->n[1] >= (int64_t(1) << 31))
        return fail(GD_EINVAL, "a 3D plane must hold fewer than 2^31 points");
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
