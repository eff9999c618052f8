// gd_device.h -- device building blocks of the deconvolution library (gfx950).
//
// Layout of the work: a field (2D: ny rows of nx; 3D: nz planes of ny rows of
// nx) is cut into tiles.  One wavefront (64 lanes) owns one tile and marches
// it along the slowest axis (y in 2D, z in 3D).  A lane holds VW consecutive
// x values (16-byte lanes for the wide variant), so a wave reads 64*VW
// contiguous elements of a row with one coalesced load per lane.  The filter
// G = Gx Gy (Gz), with 1D weights (1/4, 1/2, 1/4), is evaluated separably:
//   * x: each lane also loads its two outer neighbours (x0-1 and x0+VW, with
//     periodic wrap); they sit in the cache lines the wave is already
//     reading, so they cost L1/L2 bandwidth, not HBM bandwidth;
//   * y (3D only): a tile spans R rows; R+2 rows (one halo row each side) are
//     x-filtered per plane and combined in registers;
//   * the march axis: a rolling window of three x(y)-filtered planes.
// All loads are branch-free (inactive lanes read a valid clamped address and
// discard the value) and software-pipelined one plane ahead: the inputs of
// plane m+1 and the centre-only fields of plane m are in flight while plane m
// is filtered and plane m-1 is written.
//
// The stencil input S of a sweep need not be a stored field: the Krylov
// sweeps evaluate it pointwise from several fields (for example
// p_{n+1} = r_n + beta (p_n - omega q_n) in BiCGSTAB), so one fused pass both
// forms p_{n+1} and applies G to it.
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

// Non-temporal load for operands a sweep reads exactly once (no halo reuse):
// they then crowd L2 less, which the stencil inputs' halo rows reuse
// (2048^2 x 16 BiCGSTAB 4.86 -> 4.47 ms, CG 4.24 -> 4.03 ms).
template <typename T, int VW>
__device__ __forceinline__ void vld_nt(const T *__restrict__ p, T (&v)[VW]) {
    if constexpr (VW == 1) {
        v[0] = __builtin_nontemporal_load(p);
    } else {
        typedef T vt __attribute__((ext_vector_type(VW)));
        vt x = __builtin_nontemporal_load(reinterpret_cast<const vt *>(p));
#pragma unroll
        for (int k = 0; k < VW; ++k) v[k] = x[k];
    }
}

// Non-temporal (streaming) stores.  A sweep's outputs are read again only in
// the next sweep, long after they have left L2; streaming them measured
// faster (2048^2 x 16 BiCGSTAB 4.99 -> 4.87 ms), most likely because less
// dirty data is left for the grid barrier's release fence to write back.
template <typename T, int VW>
__device__ __forceinline__ void vst(T *__restrict__ p, const T (&v)[VW]) {
    if constexpr (VW == 1) {
        __builtin_nontemporal_store(v[0], p);
    } else {
        typedef T vt __attribute__((ext_vector_type(VW)));
        vt x;
#pragma unroll
        for (int k = 0; k < VW; ++k) x[k] = v[k];
        __builtin_nontemporal_store(x, reinterpret_cast<vt *>(p));
    }
}

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
    int64_t L;       // planes per long tile along the march axis
    int64_t L2;      // planes per short tile (the tail of every column)
    int64_t mb;      // planes [0, mb) are cut into long tiles, [mb, nmarch) into short ones
    int64_t nbig;    // long tiles of the field (they come first in the tile order)
};

template <int N> struct Arr { static constexpr int n = N > 0 ? N : 1; };

// Tile position of a lane.
struct TilePos {
    int64_t x0, xc, xl, xr, row0, m0, m1;
    bool act;
};

template <int VW, int R>
__device__ __forceinline__ TilePos tile_pos(const Geo &g, int64_t lt, int lane) {
    TilePos p;
    const int64_t cols = g.nxs * g.nrs;
    int64_t c, mend;
    if (lt < g.nbig) {  // long tiles: planes [0, mb)
        c = lt % cols;
        p.m0 = (lt / cols) * g.L;
        mend = p.m0 + g.L;
        if (mend > g.mb) mend = g.mb;
    } else {  // short tiles: planes [mb, nmarch)
        const int64_t l2 = lt - g.nbig;
        c = l2 % cols;
        p.m0 = g.mb + (l2 / cols) * g.L2;
        mend = p.m0 + g.L2;
    }
    p.m1 = mend < g.nmarch ? mend : g.nmarch;
    const int64_t xs = c % g.nxs;
    const int64_t rs = c / g.nxs;
    p.x0 = xs * (WAVE * VW) + (int64_t)lane * VW;
    p.act = p.x0 < g.nx;
    p.xc = p.act ? p.x0 : g.nx - VW;  // a valid column for inactive lanes
    p.xl = p.xc == 0 ? g.nx - 1 : p.xc - 1;
    p.xr = (p.xc + VW >= g.nx) ? p.xc + VW - g.nx : p.xc + VW;
    p.row0 = rs * R;
    return p;
}

// March one tile with the separable stencil.
//   Op::NI stencil-input fields op.in[f]; op.mix(v[NI]) forms S at a point
//   Op::NO centre-only fields op.oin[f], loaded for every output point
//   op.out(idx, s[VW], g[VW], o[NO][VW], acc) consumes S, G S and the centre
//   fields at VW consecutive output points
// NDIM 2: R must be 1 (no in-plane y).
template <int NDIM, int VW, int R, typename T, typename C, class Op>
__device__ __forceinline__ void march_tile(const Geo &g, int64_t lt, const Op &op, double (&acc)[NACC], int lane) {
    static_assert(NDIM == 3 || R == 1, "2D tiles are one row wide");
    constexpr int HR = NDIM == 3 ? R + 2 : 1;
    constexpr int NI = Arr<Op::NI>::n;
    constexpr int NO = Arr<Op::NO>::n;
    const TilePos p = tile_pos<VW, R>(g, lt, lane);
    const int64_t nx = g.nx;

    int64_t rowoff[HR];
#pragma unroll
    for (int h = 0; h < HR; ++h) {
        if constexpr (NDIM == 3) {
            int64_t row = (p.row0 + h - 1) % g.nrows;
            if (row < 0) row += g.nrows;
            rowoff[h] = row * nx;
        } else {
            rowoff[h] = 0;
        }
    }
    int64_t orow[R];  // output rows, clamped so that loads stay in the field
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t row = p.row0 + r;
        orow[r] = (row < g.nrows ? row : g.nrows - 1) * nx;
    }

    auto wrapm = [&](int64_t m) -> int64_t { return m < 0 ? m + g.nmarch : (m >= g.nmarch ? m - g.nmarch : m); };

    // raw stencil inputs of one plane: centre vector and the two x neighbours
    T cv[HR][NI][VW], cl[HR][NI], cr[HR][NI];
    auto load_in = [&](int64_t mw, T (&v)[HR][NI][VW], T (&l)[HR][NI], T (&r)[HR][NI]) {
#pragma unroll
        for (int h = 0; h < HR; ++h) {
            const int64_t base = mw * g.plane + rowoff[h];
#pragma unroll
            for (int f = 0; f < Op::NI; ++f) {
                vld<T, VW>(op.in[f] + base + p.xc, v[h][f]);
                l[h][f] = op.in[f][base + p.xl];
                r[h][f] = op.in[f][base + p.xr];
            }
        }
    };
    T co[R][NO][VW];
    auto load_out = [&](int64_t m, T (&o)[R][NO][VW]) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int f = 0; f < Op::NO; ++f) vld_nt<T, VW>(op.oin[f] + m * g.plane + orow[r] + p.xc, o[r][f]);
    };

    C W0[R][VW], W1[R][VW], W2[R][VW], S1[R][VW], S2[R][VW];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < VW; ++k) W0[r][k] = W1[r][k] = W2[r][k] = S1[r][k] = S2[r][k] = C(0);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int f = 0; f < NO; ++f)
#pragma unroll
            for (int k = 0; k < VW; ++k) co[r][f][k] = T(0);

    load_in(wrapm(p.m0 - 1), cv, cl, cr);
    for (int64_t m = p.m0 - 1; m <= p.m1; ++m) {
        // prefetch: inputs of plane m+1, centre fields of plane m
        T nv[HR][NI][VW], nl[HR][NI], nr[HR][NI];
        T no[R][NO][VW];
        if (m < p.m1) load_in(wrapm(m + 1), nv, nl, nr);
        if (m >= p.m0 && m < p.m1) load_out(m, no);

        // x(y)-filter plane m
        C sc[HR][VW], hx[HR][VW];
#pragma unroll
        for (int h = 0; h < HR; ++h) {
            C left, right;
            {
                T a[NI], b[NI];
#pragma unroll
                for (int f = 0; f < NI; ++f) {
                    a[f] = cl[h][f];
                    b[f] = cr[h][f];
                }
                left = op.mix(a);
                right = op.mix(b);
            }
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                T a[NI];
#pragma unroll
                for (int f = 0; f < NI; ++f) a[f] = cv[h][f][k];
                sc[h][k] = op.mix(a);
            }
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
        // output plane m-1 (its centre fields were loaded one step ago)
        if (m > p.m0) {
            const int64_t mo = m - 1;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (p.act && (NDIM == 2 || p.row0 + r < g.nrows)) {
                    C gv[VW];
#pragma unroll
                    for (int k = 0; k < VW; ++k) gv[k] = C(0.5) * W1[r][k] + C(0.25) * (W0[r][k] + W2[r][k]);
                    op.out(mo * g.plane + (p.row0 + r) * nx + p.x0, S1[r], gv, co[r], acc);
                }
            }
        }
        // rotate the prefetch buffers
#pragma unroll
        for (int h = 0; h < HR; ++h)
#pragma unroll
            for (int f = 0; f < NI; ++f) {
                cl[h][f] = nl[h][f];
                cr[h][f] = nr[h][f];
#pragma unroll
                for (int k = 0; k < VW; ++k) cv[h][f][k] = nv[h][f][k];
            }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int f = 0; f < NO; ++f)
#pragma unroll
                for (int k = 0; k < VW; ++k) co[r][f][k] = no[r][f][k];
    }
}

// Pointwise pass over a tile (sweeps that need no stencil): only centre fields.
template <int NDIM, int VW, int R, typename T, typename C, class Op>
__device__ __forceinline__ void point_tile(const Geo &g, int64_t lt, const Op &op, double (&acc)[NACC], int lane) {
    constexpr int NO = Arr<Op::NO>::n;
    const TilePos p = tile_pos<VW, R>(g, lt, lane);
    if (!p.act) return;
    C zero[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) zero[k] = C(0);
    for (int64_t m = p.m0; m < p.m1; ++m)
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (NDIM == 2 || p.row0 + r < g.nrows) {
                const int64_t i = m * g.plane + (p.row0 + r) * g.nx + p.x0;
                T o[NO][VW];
#pragma unroll
                for (int f = 0; f < Op::NO; ++f) vld_nt<T, VW>(op.oin[f] + i, o[f]);
                op.out(i, zero, zero, o, acc);
            }
}

}  // namespace gd
