// gd_closure.hip -- the approximate-deconvolution closure stress.
//
// The filtered equations of motion need the sub-filter stress
// tau_ij = ubar_i ubar_j - G(u_i u_j) (Sec. 2, Eq. fge3); approximate
// deconvolution closes it with the deconvolved velocity u* in place of the
// unknown u (Sec. 3, the AD form of Eq. tau3):
//     tau_ij = ubar_i ubar_j - G(u*_i u*_j),   i <= j,
// 3 pairs in 2D (11, 12, 22), 6 in 3D (11, 12, 13, 22, 23, 33).
//
// One fused pass that marches along the slowest axis (z in 3D, y in 2D).  A
// workgroup owns an in-plane tile (3D: 64 x 8 points, each thread two
// consecutive rows; 2D: a row segment of 256) and a run of planes.  For every
// plane it stages the products u*_i u*_j of the tile and its one-point halo in
// LDS, filters them in-plane there, keeps three filtered planes per pair in
// registers for the march-axis pass, and writes every tau_ij of the plane
// behind.  The next plane's u* loads are issued before the current plane is
// filtered.  HBM traffic: u* (halo re-reads mostly hit L2), ubar and tau, each
// once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "gd_internal.h"

namespace gdclosure {

// Periodic index for v in [-1, n].
__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Periodic index of a halo column or row of a ragged tile: v in [-1, n] wraps;
// beyond n lie points outside the field whose values no output uses, clamped
// to stay in bounds.
__device__ __forceinline__ int wrap_halo(int v, int n) { return v < 0 ? v + n : (v == n ? 0 : (v > n ? n - 1 : v)); }

template <int NDIM>
struct Shape;
template <>
struct Shape<3> {
    static constexpr int TX = 64, RPT = 2;  // tile width; rows per thread
    static constexpr bool XCD = true;       // x/y neighbour tiles on one XCD share halo lines in its L2
};
template <>
struct Shape<2> {
    static constexpr int TX = 256, RPT = 1;
    static constexpr bool XCD = false;      // only two halo points per row: nothing to share
};

template <typename T, int NDIM>
__global__ __launch_bounds__(256) void k_closure(const T *ubar, const T *ustar, T *tau, int nx, int ny, int nz,
                                                 int tiles_x, int tiles_y, int segs, int seg, int nblocks) {
    using S = Shape<NDIM>;
    constexpr int NC = NDIM, NP = NDIM * (NDIM + 1) / 2;  // velocity / stress components
    constexpr int TX = S::TX, RPT = S::RPT;
    constexpr int TYW = 256 / TX;                         // thread rows
    constexpr int TY = TYW * RPT;                         // tile rows (3D)
    constexpr int HX = TX + 2, HY = NDIM == 3 ? TY + 2 : 1;
    constexpr int NS = HX * HY, SPT = (NS + 255) / 256;   // staged points per plane; per thread
    static_assert(NDIM == 3 || (TYW == 1 && RPT == 1), "2D tiles are row segments");
    __shared__ T prod[NP][NS];
    const int tid = threadIdx.x;
    int lin = blockIdx.x;
    if (S::XCD) {  // workgroups are dealt round-robin over the 8 XCDs: give each a contiguous range
        const int per = nblocks / 8, rem = nblocks % 8, xcd = lin % 8, k = lin / 8;
        lin = xcd * per + min(xcd, rem) + k;
    }
    const int tx = lin % tiles_x;
    lin /= tiles_x;
    const int ty = lin % tiles_y;
    lin /= tiles_y;
    const int sg = lin % segs;
    const int64_t f = lin / segs;                         // velocity field of the batch
    const int lx = tid % TX, ly = tid / TX;
    const int x0 = tx * TX, y0 = ty * TY;
    const int x = x0 + lx, yb = NDIM == 3 ? y0 + ly * RPT : 0;
    const int nm = NDIM == 3 ? nz : ny;                   // march extent
    const int64_t pstride = NDIM == 3 ? (int64_t)nx * ny : nx;
    const int64_t npts = pstride * nm;
    const T *us = ustar + f * NC * npts;
    const T *ub = ubar + f * NC * npts;
    T *tf = tau + f * NP * npts;
    int64_t soff[SPT];                                    // in-plane offsets of this thread's staged points
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        const int s = tid + 256 * k;
        const int gx = wrap_halo(x0 + s % HX - 1, nx);
        const int gy = NDIM == 3 ? wrap_halo(y0 + s / HX - 1, ny) : 0;
        soff[k] = (int64_t)gy * nx + gx;
    }
    const int m0 = sg * seg, m1 = min(nm, m0 + seg);
    T st[SPT][NC];
    auto stage = [&](int m) {
        const int64_t base = (int64_t)wrap(m, nm) * pstride;
#pragma unroll
        for (int k = 0; k < SPT; ++k)
            if (k + 1 < SPT || tid + 256 * k < NS)
#pragma unroll
                for (int c = 0; c < NC; ++c) st[k][c] = us[c * npts + base + soff[k]];
    };
    stage(m0 - 1);
    T h0[RPT][NP], h1[RPT][NP], h2[RPT][NP];              // in-plane filtered products of planes m-2, m-1, m
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int k = 0; k < NP; ++k) h0[r][k] = h1[r][k] = h2[r][k] = T(0);
    for (int m = m0 - 1; m <= m1; ++m) {
        __syncthreads();  // the previous plane's products have been read
#pragma unroll
        for (int k = 0; k < SPT; ++k)
            if (k + 1 < SPT || tid + 256 * k < NS) {
                int q = 0;
#pragma unroll
                for (int a = 0; a < NC; ++a)
#pragma unroll
                    for (int b = a; b < NC; ++b) prod[q++][tid + 256 * k] = st[k][a] * st[k][b];
            }
        __syncthreads();
        if (m < m1) stage(m + 1);
        const bool outm = m > m0 && x < nx;               // plane m-1 has both march neighbours now
        T v[RPT][NC];
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            if (outm && (NDIM == 2 || yb + r < ny))
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    v[r][c] = ub[c * npts + (int64_t)(m - 1) * pstride + (int64_t)(yb + r) * nx + x];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            T xr[RPT + 2];                                // x pass of rows yb-1 .. yb+RPT
#pragma unroll
            for (int j = 0; j < (NDIM == 3 ? RPT + 2 : 1); ++j) {
                const T *p = &prod[k][(ly * RPT + j) * HX + lx];
                xr[j] = T(0.5) * p[1] + T(0.25) * (p[0] + p[2]);
            }
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const T hn = NDIM == 3 ? T(0.5) * xr[r + 1] + T(0.25) * (xr[r] + xr[r + 2]) : xr[0];
                h0[r][k] = h1[r][k];
                h1[r][k] = h2[r][k];
                h2[r][k] = hn;
            }
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            if (outm && (NDIM == 2 || yb + r < ny)) {
                const int64_t i = (int64_t)(m - 1) * pstride + (int64_t)(yb + r) * nx + x;
                int k = 0;
#pragma unroll
                for (int a = 0; a < NC; ++a)
#pragma unroll
                    for (int b = a; b < NC; ++b, ++k)  // tau is written once and not re-read here
                        __builtin_nontemporal_store(
                            v[r][a] * v[r][b] - (T(0.5) * h1[r][k] + T(0.25) * (h0[r][k] + h2[r][k])),
                            &tf[k * npts + i]);
            }
    }
}

// Planes per workgroup: the longest run (64 in 2D, 32 in 3D, at least 4) that
// still gives the launch enough workgroups (2048 in 2D; 512 in 3D, where the
// tiles are larger and a long march amortises the halo planes).
template <int NDIM>
int choose_seg(int64_t tiles, int nm) {
    int seg = NDIM == 3 ? 32 : 64;
    const int64_t want = NDIM == 3 ? 512 : 2048;
    while (seg > 4 && tiles * ((nm + seg - 1) / seg) < want) seg /= 2;
    return seg;
}

template <typename T, int NDIM>
int launch(const T *ub, const T *us, T *tau, int64_t nx, int64_t ny, int64_t nz, int64_t batch, hipStream_t st) {
    constexpr int TX = Shape<NDIM>::TX, TY = 256 / TX * Shape<NDIM>::RPT;
    const int64_t tiles_x = (nx + TX - 1) / TX, tiles_y = NDIM == 3 ? (ny + TY - 1) / TY : 1;
    const int nm = (int)(NDIM == 3 ? nz : ny);
    const int seg = choose_seg<NDIM>(tiles_x * tiles_y * batch, nm);
    const int64_t segs = (nm + seg - 1) / seg;
    const int64_t blocks = tiles_x * tiles_y * segs * batch;
    if (blocks > 0x7fffffff) return -1;
    hipLaunchKernelGGL((k_closure<T, NDIM>), dim3((unsigned)blocks), dim3(256), 0, st, ub, us, tau, (int)nx, (int)ny,
                       (int)nz, (int)tiles_x, (int)tiles_y, (int)segs, seg, (int)blocks);
    return 0;
}

using gd::fail;


}  // namespace gdclosure

using namespace gdclosure;

extern "C" {

int closure_stress(const gd_grid *g, const void *ubar, const void *ustar, void *tau, void *stream) {
    if (!g) return fail(GD_EINVAL, "grid is NULL");
    if (g->ndim != 2 && g->ndim != 3) return fail(GD_EINVAL, "ndim must be 2 or 3");
    if (g->dtype != GD_F32 && g->dtype != GD_F64) return fail(GD_EINVAL, "dtype must be GD_F32 or GD_F64");
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->ndim == 3 ? g->n[2] : 1;
    if (nx < 1 || ny < 1 || nz < 1 || g->batch < 1) return fail(GD_EINVAL, "sizes must be >= 1");
    const int64_t npts = gd::checked_points(g->n, g->ndim, int64_t(1) << 36);
    if (nx >= (1 << 30) || ny >= (1 << 30) || nz >= (1 << 30) || npts < 0 || g->batch > gd::kMaxTotalPoints / npts)
        return fail(GD_EINVAL, "field too large");
    if (!ubar || !ustar || !tau) return fail(GD_EINVAL, "ubar, ustar and tau must be non-NULL");
    const size_t ts = g->dtype == GD_F32 ? 4 : 8;
    const int nc = g->ndim, np = nc * (nc + 1) / 2;
    const size_t in_bytes = (size_t)g->batch * nc * nx * ny * nz * ts, out_bytes = (size_t)g->batch * np * nx * ny * nz * ts;
    if (gd::ranges_overlap(tau, out_bytes, ubar, in_bytes) || gd::ranges_overlap(tau, out_bytes, ustar, in_bytes))
        return fail(GD_EINVAL, "tau overlaps an input");
    hipStream_t st = (hipStream_t)stream;
    int rc;
    if (g->dtype == GD_F32)
        rc = g->ndim == 2 ? launch<float, 2>((const float *)ubar, (const float *)ustar, (float *)tau, nx, ny, nz, g->batch, st)
                          : launch<float, 3>((const float *)ubar, (const float *)ustar, (float *)tau, nx, ny, nz, g->batch, st);
    else
        rc = g->ndim == 2
                 ? launch<double, 2>((const double *)ubar, (const double *)ustar, (double *)tau, nx, ny, nz, g->batch, st)
                 : launch<double, 3>((const double *)ubar, (const double *)ustar, (double *)tau, nx, ny, nz, g->batch, st);
    if (rc != 0) return fail(GD_EINVAL, "grid too large");
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(GD_EHIP, "closure launch: %s", hipGetErrorString(e));
    return GD_OK;
}

}  // extern "C"
