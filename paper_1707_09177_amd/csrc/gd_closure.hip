// gd_closure.hip -- the approximate-deconvolution closure stress.
//
// The filtered equations of motion need the sub-filter stress
// tau_ij = ubar_i ubar_j - G(u_i u_j) (Sec. 2, Eq. fge3); approximate
// deconvolution closes it with the deconvolved velocity u* in place of the
// unknown u (Sec. 3, the AD form of Eq. tau3):
//     tau_ij = ubar_i ubar_j - G(u*_i u*_j),   i <= j,
// 3 pairs in 2D (11, 12, 22), 6 in 3D (11, 12, 13, 22, 23, 33).
//
// One fused pass: a workgroup owns a 32 x 8 column of the field and marches
// along z.  For every plane it stages the products u*_i u*_j of the tile and
// its one-point halo in LDS, filters them in x and y there, keeps three
// filtered planes in registers for the z pass, and writes every tau_ij of the
// plane behind.  HBM traffic: the u* components (with the halo of the tile),
// the ubar components and the tau outputs, each once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "gdecon.h"

namespace gd {
void set_error_text(const char *msg);
}

namespace gdclosure {

constexpr int TXC = 32, TYC = 8;                // tile of one workgroup (one thread per column)
constexpr int HXC = TXC + 2, HYC = TYC + 2;     // tile with its halo
constexpr int kZSeg = 32;                       // planes per workgroup along z

// Periodic index for v in [-1, n].
__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Periodic index of a halo column or row of a ragged tile: v in [-1, n] wraps;
// beyond n lie points outside the field whose values no output uses, clamped
// to stay in bounds.
__device__ __forceinline__ int wrap_halo(int v, int n) { return v < 0 ? v + n : (v == n ? 0 : (v > n ? n - 1 : v)); }

template <typename T, int NDIM>
__global__ __launch_bounds__(256) void k_closure(const T *ubar, const T *ustar, T *tau, int nx, int ny, int nz,
                                                 int tiles_x, int tiles_y, int zsegs) {
    constexpr int NC = NDIM;                    // velocity components
    constexpr int NP = NDIM * (NDIM + 1) / 2;   // stress components
    __shared__ T prod[NP][HYC * HXC];
    const int tid = threadIdx.x;
    const int lx = tid % TXC, ly = tid / TXC;
    int blk = blockIdx.x;
    const int tx = blk % tiles_x;
    blk /= tiles_x;
    const int ty = blk % tiles_y;
    blk /= tiles_y;
    const int zs = blk % zsegs;
    const int64_t f = blk / zsegs;              // field of the batch
    const int x0 = tx * TXC, y0 = ty * TYC;
    const int x = x0 + lx, y = y0 + ly;
    const bool act = x < nx && y < ny;
    const int64_t plane = (int64_t)nx * ny, npts = plane * nz;
    const T *us = ustar + f * NC * npts;
    const T *ub = ubar + f * NC * npts;
    T *tf = tau + f * NP * npts;
    const int z0 = NDIM == 3 ? zs * kZSeg : 0;
    const int z1 = NDIM == 3 ? std::min(nz, z0 + kZSeg) : 1;
    T h0[NP], h1[NP], h2[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) h0[k] = h1[k] = h2[k] = T(0);
    const int mlo = NDIM == 3 ? z0 - 1 : 0, mhi = NDIM == 3 ? z1 : 0;
    for (int m = mlo; m <= mhi; ++m) {
        const int mw = NDIM == 3 ? wrap(m, nz) : 0;
        __syncthreads();  // the previous plane's products have been read
        for (int q = tid; q < HYC * HXC; q += 256) {
            const int hy = q / HXC, hx = q % HXC;
            const int gy = wrap_halo(y0 + hy - 1, ny), gx = wrap_halo(x0 + hx - 1, nx);
            const int64_t i = (int64_t)mw * plane + (int64_t)gy * nx + gx;
            T v[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) v[c] = us[c * npts + i];
            int k = 0;
#pragma unroll
            for (int a = 0; a < NC; ++a)
#pragma unroll
                for (int b = a; b < NC; ++b) prod[k++][q] = v[a] * v[b];
        }
        __syncthreads();
        // x and y passes of the filter at this thread's point
        T hn[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            auto row = [&](int r) {
                const T *p = &prod[k][(ly + r) * HXC + lx];
                return T(0.5) * p[1] + T(0.25) * (p[0] + p[2]);
            };
            hn[k] = T(0.5) * row(1) + T(0.25) * (row(0) + row(2));
        }
        if constexpr (NDIM == 2) {
            if (act) {
                const int64_t i = (int64_t)y * nx + x;
                T v[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) v[c] = ub[c * npts + i];
                int k = 0;
#pragma unroll
                for (int a = 0; a < NC; ++a)
#pragma unroll
                    for (int b = a; b < NC; ++b, ++k) tf[k * npts + i] = v[a] * v[b] - hn[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                h0[k] = h1[k];
                h1[k] = h2[k];
                h2[k] = hn[k];
            }
            // z pass: plane m-1 has both of its neighbours now
            if (m > z0 && act) {
                const int64_t i = (int64_t)(m - 1) * plane + (int64_t)y * nx + x;
                T v[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) v[c] = ub[c * npts + i];
                int k = 0;
#pragma unroll
                for (int a = 0; a < NC; ++a)
#pragma unroll
                    for (int b = a; b < NC; ++b, ++k)
                        tf[k * npts + i] = v[a] * v[b] - (T(0.5) * h1[k] + T(0.25) * (h0[k] + h2[k]));
            }
        }
    }
}

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    gd::set_error_text(buf);
    return code;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

}  // namespace gdclosure

using namespace gdclosure;

extern "C" {

int closure_stress(const gd_grid *g, const void *ubar, const void *ustar, void *tau, void *stream) {
    if (!g) return fail(GD_EINVAL, "grid is NULL");
    if (g->ndim != 2 && g->ndim != 3) return fail(GD_EINVAL, "ndim must be 2 or 3");
    if (g->dtype != GD_F32 && g->dtype != GD_F64) return fail(GD_EINVAL, "dtype must be GD_F32 or GD_F64");
    const int64_t nx = g->n[0], ny = g->n[1], nz = g->ndim == 3 ? g->n[2] : 1;
    if (nx < 1 || ny < 1 || nz < 1 || g->batch < 1) return fail(GD_EINVAL, "sizes must be >= 1");
    if (nx >= (1 << 30) || ny >= (1 << 30) || nz >= (1 << 30) || nx * ny * nz > (int64_t(1) << 36))
        return fail(GD_EINVAL, "field too large");
    if (!ubar || !ustar || !tau) return fail(GD_EINVAL, "ubar, ustar and tau must be non-NULL");
    const size_t ts = g->dtype == GD_F32 ? 4 : 8;
    const int nc = g->ndim, np = nc * (nc + 1) / 2;
    const size_t in_bytes = (size_t)g->batch * nc * nx * ny * nz * ts, out_bytes = (size_t)g->batch * np * nx * ny * nz * ts;
    if (overlap(tau, out_bytes, ubar, in_bytes) || overlap(tau, out_bytes, ustar, in_bytes))
        return fail(GD_EINVAL, "tau overlaps an input");
    const int tiles_x = (int)((nx + TXC - 1) / TXC), tiles_y = (int)((ny + TYC - 1) / TYC);
    const int zsegs = g->ndim == 3 ? (int)((nz + kZSeg - 1) / kZSeg) : 1;
    const int64_t blocks = (int64_t)tiles_x * tiles_y * zsegs * g->batch;
    if (blocks > 0x7fffffff) return fail(GD_EINVAL, "grid too large");
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)blocks), block(256);
    if (g->dtype == GD_F32) {
        if (g->ndim == 2)
            hipLaunchKernelGGL((k_closure<float, 2>), grid, block, 0, st, (const float *)ubar, (const float *)ustar,
                               (float *)tau, (int)nx, (int)ny, (int)nz, tiles_x, tiles_y, zsegs);
        else
            hipLaunchKernelGGL((k_closure<float, 3>), grid, block, 0, st, (const float *)ubar, (const float *)ustar,
                               (float *)tau, (int)nx, (int)ny, (int)nz, tiles_x, tiles_y, zsegs);
    } else {
        if (g->ndim == 2)
            hipLaunchKernelGGL((k_closure<double, 2>), grid, block, 0, st, (const double *)ubar,
                               (const double *)ustar, (double *)tau, (int)nx, (int)ny, (int)nz, tiles_x, tiles_y, zsegs);
        else
            hipLaunchKernelGGL((k_closure<double, 3>), grid, block, 0, st, (const double *)ubar,
                               (const double *)ustar, (double *)tau, (int)nx, (int)ny, (int)nz, tiles_x, tiles_y, zsegs);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(GD_EHIP, "closure launch: %s", hipGetErrorString(e));
    return GD_OK;
}

}  // extern "C"
