// gd_device.h -- device building blocks of the deconvolution library (gfx950).
//
// Layout of the work: a field (2D: ny rows of nx; 3D: nz planes of ny rows of
// nx) is cut into tiles.  One wavefront (64 lanes) owns one tile and marches
// it along the slowest axis (y in 2D, z in 3D).  A lane holds VW consecutive
// x values (VW*4 or VW*8 = 16 bytes for the wide variant), so a wave reads
// 64*VW contiguous elements per row with one coalesced 16-byte load per lane.
// The filter G = Gx Gy (Gz), with 1D weights (1/4, 1/2, 1/4), is evaluated
// separably:
//   * x: neighbours inside the wave come from the adjacent lanes (ds_bpermute
//     shuffles); the two lanes at the segment edges load their outer neighbour
//     with periodic wrap-around;
//   * y (3D only): a tile spans R rows; R+2 rows (one halo row on each side)
//     are x-filtered per plane and combined in registers;
//   * the march axis: a rolling window of three x(y)-filtered planes.
// Every element of the stencil input is loaded once per tile from HBM (plus
// the halo rows/planes of the tile), and the output of plane m-1 is produced
// as soon as plane m has been read.
//
// The stencil input S of a sweep is not necessarily a stored field: the
// Krylov sweeps evaluate it on the fly from several fields (for example
// p_{n+1} = r_n + beta (p_n - omega q_n) in BiCGSTAB), so the fused sweep
// writes p_{n+1} and q_{n+1} = G p_{n+1} in the same pass.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gd {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int WPB = BLOCK / WAVE;
constexpr int NACC = 3;  // partial sums per tile and phase

// vector widths: 16-byte lanes
template <typename T> struct VMax { static constexpr int v = 16 / sizeof(T); };

template <typename T, int VW>
__device__ __forceinline__ void vld(const T *__restrict__ p, T (&v)[VW]) {
    if constexpr (VW == 1) {
        v[0] = *p;
    } else {
        typedef T vt __attribute__((ext_vector_type(VW)));
        vt x = *reinterpret_cast<const vt *>(p);
#pragma unroll
        for (int k = 0; k < VW; ++k) v[k] = x[k];
    }
}

template <typename T, int VW>
__device__ __forceinline__ void vst(T *__restrict__ p, const T (&v)[VW]) {
    if constexpr (VW == 1) {
        *p = v[0];
    } else {
        typedef T vt __attribute__((ext_vector_type(VW)));
        vt x;
#pragma unroll
        for (int k = 0; k < VW; ++k) x[k] = v[k];
        *reinterpret_cast<vt *>(p) = x;
    }
}

template <typename C>
__device__ __forceinline__ C shfl_up1(C v) { return __shfl_up(v, 1, WAVE); }
template <typename C>
__device__ __forceinline__ C shfl_down1(C v) { return __shfl_down(v, 1, WAVE); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// Geometry of one field as the march sees it.
struct Geo {
    int64_t nx;      // row length
    int64_t nrows;   // rows per plane (1 in 2D, ny in 3D)
    int64_t nmarch;  // planes along the march axis (ny in 2D, nz in 3D)
    int64_t plane;   // elements per plane (nx in 2D, nx*ny in 3D)
    int64_t nxs;     // x segments of WAVE*VW columns
    int64_t nrs;     // row tiles of R rows (1 in 2D)
    int64_t L;       // planes per tile along the march axis
};

// March one tile with the separable stencil.
//   op.src(idx, s[VW])  stencil input at VW consecutive points (aligned idx)
//   op.src1(idx)        stencil input at one point
//   op.out(idx, s, g, acc)  consume the centre value s and g = (G S) there
// NDIM 2: R must be 1 (no in-plane y).
template <int NDIM, int VW, int R, typename C, class Op>
__device__ __forceinline__ void march_tile(const Geo &g, int64_t lt, Op &op, double (&acc)[NACC], int lane) {
    static_assert(NDIM == 3 || R == 1, "2D tiles are one row wide");
    constexpr int HR = NDIM == 3 ? R + 2 : 1;
    const int64_t nx = g.nx;
    const int64_t xs = lt % g.nxs;
    const int64_t rest = lt / g.nxs;
    const int64_t rs = rest % g.nrs;
    const int64_t ms = rest / g.nrs;
    const int64_t seg0 = xs * (WAVE * VW);
    const int64_t x0 = seg0 + (int64_t)lane * VW;
    const bool act = x0 < nx;
    const int64_t seg_end = (seg0 + WAVE * VW < nx) ? seg0 + WAVE * VW : nx;
    const int last_lane = (int)((seg_end - seg0 + VW - 1) / VW) - 1;
    const int64_t xl = x0 == 0 ? nx - 1 : x0 - 1;
    const int64_t xr = (x0 + VW >= nx) ? 0 : x0 + VW;
    const int64_t row0 = rs * R;
    const int64_t m0 = ms * g.L;
    const int64_t m1 = (m0 + g.L < g.nmarch) ? m0 + g.L : g.nmarch;

    int64_t rowoff[HR];
#pragma unroll
    for (int h = 0; h < HR; ++h) {
        if constexpr (NDIM == 3) {
            int64_t row = (row0 + h - 1) % g.nrows;
            if (row < 0) row += g.nrows;
            rowoff[h] = row * nx;
        } else {
            rowoff[h] = 0;
        }
    }

    C W0[R][VW], W1[R][VW], W2[R][VW], S1[R][VW], S2[R][VW];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < VW; ++k) W0[r][k] = W1[r][k] = W2[r][k] = S1[r][k] = S2[r][k] = C(0);

    for (int64_t m = m0 - 1; m <= m1; ++m) {
        const int64_t mw = m < 0 ? m + g.nmarch : (m >= g.nmarch ? m - g.nmarch : m);
        C hx[HR][VW], sc[HR][VW];
#pragma unroll
        for (int h = 0; h < HR; ++h) {
            const int64_t base = mw * g.plane + rowoff[h];
            if (act) {
                op.src(base + x0, sc[h]);
            } else {
#pragma unroll
                for (int k = 0; k < VW; ++k) sc[h][k] = C(0);
            }
            C left = shfl_up1(sc[h][VW - 1]);
            C right = shfl_down1(sc[h][0]);
            if (lane == 0) left = op.src1(base + xl);
            if (lane == last_lane) right = op.src1(base + xr);
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                const C l = k == 0 ? left : sc[h][k - 1];
                const C rr = k == VW - 1 ? right : sc[h][k + 1];
                hx[h][k] = C(0.5) * sc[h][k] + C(0.25) * (l + rr);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                W0[r][k] = W1[r][k];
                W1[r][k] = W2[r][k];
                S1[r][k] = S2[r][k];
                if constexpr (NDIM == 3) {
                    W2[r][k] = C(0.5) * hx[r + 1][k] + C(0.25) * (hx[r][k] + hx[r + 2][k]);
                    S2[r][k] = sc[r + 1][k];
                } else {
                    W2[r][k] = hx[0][k];
                    S2[r][k] = sc[0][k];
                }
            }
        if (m > m0 && act) {
            const int64_t mo = m - 1;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (NDIM == 2 || row0 + r < g.nrows) {
                    C gv[VW];
#pragma unroll
                    for (int k = 0; k < VW; ++k) gv[k] = C(0.5) * W1[r][k] + C(0.25) * (W0[r][k] + W2[r][k]);
                    op.out(mo * g.plane + (row0 + r) * nx + x0, S1[r], gv, acc);
                }
            }
        }
    }
}

// Pointwise pass over a tile (sweeps that need no stencil).
template <int NDIM, int VW, int R, typename C, class Op>
__device__ __forceinline__ void point_tile(const Geo &g, int64_t lt, Op &op, double (&acc)[NACC], int lane) {
    const int64_t xs = lt % g.nxs;
    const int64_t rest = lt / g.nxs;
    const int64_t rs = rest % g.nrs;
    const int64_t ms = rest / g.nrs;
    const int64_t x0 = xs * (WAVE * VW) + (int64_t)lane * VW;
    if (x0 >= g.nx) return;
    const int64_t row0 = rs * R;
    const int64_t m0 = ms * g.L;
    const int64_t m1 = (m0 + g.L < g.nmarch) ? m0 + g.L : g.nmarch;
    C zero[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) zero[k] = C(0);
    for (int64_t m = m0; m < m1; ++m)
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (NDIM == 2 || row0 + r < g.nrows) op.out(m * g.plane + (row0 + r) * g.nx + x0, zero, zero, acc);
}

}  // namespace gd
