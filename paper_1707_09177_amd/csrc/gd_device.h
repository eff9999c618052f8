// gd_device.h -- device building blocks of the deconvolution library (gfx950).
//
// Layout of the work: a field (2D: ny rows of nx; 3D: nz planes of ny rows of
// nx) is cut into tiles.  One wavefront (64 lanes) owns one tile and marches
// it along the slowest axis (y in 2D, z in 3D).  A lane holds VW consecutive
// x values (16-byte lanes for the wide variant), so a wave reads 64*VW
// contiguous elements of a row with one coalesced load per lane.  The filter
// G = Gx Gy (Gz), with 1D weights (1/4, 1/2, 1/4), is evaluated separably:
//   * x: in 3D the neighbours x0-1 and x0+VW of a lane's points are the
//     edge points of the lanes beside it, passed across by full-wave DPP
//     shifts; the periodic neighbours outside the wave's span are loaded by
//     lane 0 (left) and by the lane after the last active one, or lane 63
//     (right).  In 2D each lane loads its two neighbours itself (L1 hits);
//   * y (3D only): a tile spans R rows; R+2 rows (one halo row each side) are
//     x-filtered per plane and combined in registers;
//   * the march axis: a rolling window of three x(y)-filtered planes.
// The stencil input S of a sweep need not be a stored field: the Krylov
// sweeps evaluate it pointwise from several fields (for example
// p_{n+1} = r_n + beta (p_n - omega q_n) in BiCGSTAB), so one fused pass both
// forms p_{n+1} and applies G to it.  Loads are branch-free (inactive lanes
// read a valid clamped address and discard the value).  A tile's planes, rows
// and x segment are the same in every lane (scalar registers), and a lane's
// loads address a plane as a scalar base plus a 32-bit byte offset.
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

// Lane rows of a tile: a 3D tile of 16-byte lanes and R = 4 rows is two
// half-waves of 32 lanes stacked in y, each lane holding two rows (the rows
// between the halves are passed across instead of loaded twice); every other
// tile is one row of 64 lanes, each lane holding R rows.
__host__ __device__ constexpr int tile_lane_rows(int vw, int R) { return (vw > 1 && R == 4) ? 2 : 1; }
// x columns a tile spans
__host__ __device__ constexpr int tile_cols(int vw, int R) { return WAVE / tile_lane_rows(vw, R) * vw; }

// Tile position of a lane.  seg0 (the tile's first column), m0 and m1 are
// the same in every lane of the wave; so is row0 (the lane's first row) in a
// one-lane-row tile.
struct TilePos {
    int64_t x0, xc, xl, xr, seg0, row0, m0, m1;
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
    constexpr int LY = tile_lane_rows(VW, R), LX = WAVE / LY;
    const int lx = lane & (LX - 1), ly = lane / LX;
    p.seg0 = xs * (LX * VW);
    p.x0 = p.seg0 + (int64_t)lx * VW;
    p.act = p.x0 < g.nx;
    p.xc = p.act ? p.x0 : g.nx - VW;  // a valid column for inactive lanes
    p.xl = p.xc == 0 ? g.nx - 1 : p.xc - 1;
    p.xr = (p.xc + VW >= g.nx) ? p.xc + VW - g.nx : p.xc + VW;
    p.row0 = rs * R + ly * (R / LY);
    return p;
}

// base + byte_off: a wave-uniform base (scalar registers) plus a 32-bit
// per-lane byte offset, the form of a global load with a scalar base address
template <typename T>
__device__ __forceinline__ const T *at_off(const T *base, uint32_t byte_off) {
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}

// Full-wave DPP shifts by one lane (GFX9 wave_shr:1 / wave_shl:1): lane i
// receives lane i-1's (from_left) or lane i+1's (from_right) value; the lane
// without a source keeps `v`.  64-bit values move as two 32-bit halves.
template <int CTRL, typename C>
__device__ __forceinline__ C dpp_shift(C v) {
    if constexpr (sizeof(C) == 4) {
        const int x = __builtin_bit_cast(int, v);
        return __builtin_bit_cast(C, __builtin_amdgcn_update_dpp(x, x, CTRL, 0xf, 0xf, false));
    } else {
        static_assert(sizeof(C) == 8, "32- or 64-bit lanes");
        const long long x = __builtin_bit_cast(long long, v);
        const int lo = (int)(x & 0xffffffffll), hi = (int)(x >> 32);
        const int a = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
        const int b = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
        return __builtin_bit_cast(C, (long long)(((unsigned long long)(unsigned)b << 32) | (unsigned)a));
    }
}
constexpr int kDppWaveShr1 = 0x138;  // lane i <- lane i - 1
constexpr int kDppWaveShl1 = 0x130;  // lane i <- lane i + 1

// 2D march (one row per plane): the x neighbours are per-lane loads of the
// points beside the lane's vector (hits in L1: the neighbouring lanes load
// the same lines), with the next plane's loads and the next output's centre
// fields issued a whole step ahead.  In 2D this measured faster than the
// cross-lane form below (2048^2 x 16 BiCGSTAB 4.47 vs 4.62 ms): a plane is a
// single row, so the extra loads are few and the wave has registers to spare
// for two planes in flight.
template <int VW, typename T, typename C, class Op>
__device__ __forceinline__ void march_row(const Geo &g, int64_t lt, const Op &op, double (&acc)[NACC], int lane) {
    constexpr int NI = Arr<Op::NI>::n;
    constexpr int NO = Arr<Op::NO>::n;
    const TilePos p = tile_pos<VW, 1>(g, lt, lane);
    auto wrapm = [&](int64_t m) -> int64_t { return m < 0 ? m + g.nmarch : (m >= g.nmarch ? m - g.nmarch : m); };

    // a plane is one row: loads address it as a uniform base plus 32-bit byte offsets
    const uint32_t oc = (uint32_t)(p.xc * (int64_t)sizeof(T));
    const uint32_t ol = (uint32_t)(p.xl * (int64_t)sizeof(T));
    const uint32_t orr = (uint32_t)(p.xr * (int64_t)sizeof(T));
    // raw stencil inputs of one plane: the lane's vector and its two x neighbours
    auto load_in = [&](int64_t mw, T (&v)[NI][VW], T (&l)[NI], T (&r)[NI]) {
#pragma unroll
        for (int f = 0; f < Op::NI; ++f) {
            const T *pb = op.in[f] + mw * g.plane;
            vld<T, VW>(at_off(pb, oc), v[f]);
            l[f] = *at_off(pb, ol);
            r[f] = *at_off(pb, orr);
        }
    };
    auto load_out = [&](int64_t m, T (&o)[NO][VW]) {
#pragma unroll
        for (int f = 0; f < Op::NO; ++f) vld_nt<T, VW>(at_off(op.oin[f] + m * g.plane, oc), o[f]);
    };

    // the x-filtered rows of planes m-2, m-1, m (G_y combines them)
    C W0[VW], W1[VW], W2[VW], SA[VW], SB[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) W0[k] = W1[k] = W2[k] = SA[k] = SB[k] = C(0);
    // ping-pong buffers (the march is unrolled by two, so no buffer is copied
    // from one step to the next): plane loads and centre fields
    T vA[NI][VW], lA[NI], rA[NI], vB[NI][VW], lB[NI], rB[NI], oA[NO][VW], oB[NO][VW];
#pragma unroll
    for (int f = 0; f < NO; ++f)
#pragma unroll
        for (int k = 0; k < VW; ++k) oA[f][k] = oB[f][k] = T(0);

    // step m: plane m is in (cv, cl, cr); plane m + 1's loads go to (nv, nl,
    // nr), plane m's centre fields to no; co holds plane m - 1's, sprev S(m-1).
    // The loads are unconditional (the last step reloads its own plane and the
    // first and last load unused centre fields, from cache), so no register
    // array needs a copy for a path that skips them.
    auto step = [&](int64_t m, T (&cv)[NI][VW], T (&cl)[NI], T (&cr)[NI], T (&nv)[NI][VW], T (&nl)[NI],
                    T (&nr)[NI], T (&co)[NO][VW], T (&no)[NO][VW], C (&sprev)[VW], C (&scur)[VW]) {
        load_in(wrapm(m < p.m1 ? m + 1 : m), nv, nl, nr);
        load_out(m < p.m0 ? p.m0 : (m < p.m1 ? m : p.m1 - 1), no);

        // x-filter plane m
        C hx[VW], left, right;
        {
            T a[NI], b[NI];
#pragma unroll
            for (int f = 0; f < NI; ++f) {
                a[f] = cl[f];
                b[f] = cr[f];
            }
            left = op.mix(a);
            right = op.mix(b);
        }
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            T a[NI];
#pragma unroll
            for (int f = 0; f < NI; ++f) a[f] = cv[f][k];
            scur[k] = op.mix(a);
        }
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            const C l = k == 0 ? left : scur[k - 1];
            const C rr = k == VW - 1 ? right : scur[k + 1];
            hx[k] = C(0.5) * scur[k] + C(0.25) * (l + rr);
        }
        C gv[VW];
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            W0[k] = W1[k];
            W1[k] = W2[k];
            W2[k] = hx[k];
            gv[k] = C(0.5) * W1[k] + C(0.25) * (W0[k] + W2[k]);
        }
        // output plane m-1 (its centre fields were loaded one step ago)
        if (m > p.m0 && p.act) op.out((m - 1) * g.plane + p.x0, sprev, gv, co, acc);
    };

    load_in(wrapm(p.m0 - 1), vA, lA, rA);
    for (int64_t m = p.m0 - 1; m <= p.m1; m += 2) {
        step(m, vA, lA, rA, vB, lB, rB, oB, oA, SB, SA);
        if (m + 1 <= p.m1) step(m + 1, vB, lB, rB, vA, lA, rA, oA, oB, SA, SB);
    }
}

// 3D march: a tile spans R rows of a plane, and R + 2 rows (one halo row
// each side) are x-filtered per plane and combined in y in registers.  The x
// neighbours cross lanes by DPP; the next plane's loads are in flight while a
// plane is filtered.  Must be called by the whole wave.
template <int VW, int R, typename T, typename C, class Op>
__device__ __forceinline__ void march_slab(const Geo &g, int64_t lt, const Op &op, double (&acc)[NACC], int lane) {
    constexpr int HR = R + 2;
    constexpr int NI = Arr<Op::NI>::n;
    constexpr int NO = Arr<Op::NO>::n;
    const TilePos p = tile_pos<VW, R>(g, lt, lane);
    const int64_t nx = g.nx;

    int64_t rowoff[HR];
#pragma unroll
    for (int h = 0; h < HR; ++h) {
        int64_t row = (p.row0 + h - 1) % g.nrows;
        if (row < 0) row += g.nrows;
        rowoff[h] = row * nx;
    }
    int64_t orow[R];  // output rows, clamped so that loads stay in the field
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t row = p.row0 + r;
        orow[r] = (row < g.nrows ? row : g.nrows - 1) * nx;
    }

    // the wave's x span: lanes 0 .. last hold field points (a field's last
    // segment may be partial; nx is a multiple of VW); the same in every lane
    const int64_t seg0 = p.seg0;
    const int64_t nseg = nx - seg0 < (int64_t)WAVE * VW ? nx - seg0 : (int64_t)WAVE * VW;
    const int last = (int)(nseg / VW) - 1;
    // the periodic neighbours outside the span: lane 0 loads the left one; the
    // right one is loaded by lane last + 1 (a lane without points of its own)
    // when the span is partial, else by lane last = 63
    const bool full = last == WAVE - 1;
    const int redge = full ? last : last + 1;
    const int64_t xleft = seg0 == 0 ? nx - 1 : seg0 - 1;
    const int64_t xright = seg0 + nseg >= nx ? seg0 + nseg - nx : seg0 + nseg;
    const int64_t xe = lane == 0 ? xleft : (lane == redge ? xright : p.xc);

    auto wrapm = [&](int64_t m) -> int64_t { return m < 0 ? m + g.nmarch : (m >= g.nmarch ? m - g.nmarch : m); };

    // Loads address a plane as a uniform base (scalar registers) plus a
    // 32-bit byte offset per lane (a plane holds less than 4 GiB; the host
    // checks), so a lane keeps one offset per row, not a 64-bit address per
    // row and field.
    uint32_t vo[HR], eo[HR], oo[R];
#pragma unroll
    for (int h = 0; h < HR; ++h) {
        vo[h] = (uint32_t)((rowoff[h] + p.xc) * (int64_t)sizeof(T));
        eo[h] = (uint32_t)((rowoff[h] + xe) * (int64_t)sizeof(T));
    }
#pragma unroll
    for (int r = 0; r < R; ++r) oo[r] = (uint32_t)((orow[r] + p.xc) * (int64_t)sizeof(T));
    auto at = [](const T *base, uint32_t byte_off) { return at_off(base, byte_off); };

    // raw stencil inputs of the plane in flight: the lane's vectors and edge points
    T raw[HR][NI][VW], rawe[HR][NI];
    auto load_in = [&](int64_t mw) {
#pragma unroll
        for (int f = 0; f < Op::NI; ++f) {
            const T *pb = op.in[f] + mw * g.plane;
#pragma unroll
            for (int h = 0; h < HR; ++h) {
                vld<T, VW>(at(pb, vo[h]), raw[h][f]);
                // every lane loads (no exec-mask branch); lanes other than the
                // two edge lanes read their own first point, already in L1
                rawe[h][f] = *at(pb, eo[h]);
            }
        }
    };
    T co[R][NO][VW];  // centre fields of the plane the next output comes from
    auto load_out = [&](int64_t m) {
#pragma unroll
        for (int f = 0; f < Op::NO; ++f) {
            const T *pb = op.oin[f] + m * g.plane;
#pragma unroll
            for (int r = 0; r < R; ++r) vld_nt<T, VW>(at(pb, oo[r]), co[r][f]);
        }
    };

    // the in-plane filtered planes m-2, m-1, m (G_z combines them); S1 holds
    // S(m-1) until its output
    C W0[R][VW], W1[R][VW], W2[R][VW], S1[R][VW];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < VW; ++k) W0[r][k] = W1[r][k] = W2[r][k] = S1[r][k] = C(0);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int f = 0; f < NO; ++f)
#pragma unroll
            for (int k = 0; k < VW; ++k) co[r][f][k] = T(0);

    load_in(wrapm(p.m0 - 1));
    for (int64_t m = p.m0 - 1; m <= p.m1; ++m) {
        // form S on plane m from its arrived loads (issued one step ago)
        C sm[HR][VW], se[HR], sr[HR];
#pragma unroll
        for (int h = 0; h < HR; ++h) {
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                T a[NI];
#pragma unroll
                for (int f = 0; f < NI; ++f) a[f] = raw[h][f][k];
                sm[h][k] = op.mix(a);
            }
            se[h] = op.mix(rawe[h]);
            // lane last's right neighbour: its own edge point on a full span,
            // else lane last + 1's
            sr[h] = full ? se[h] : dpp_shift<kDppWaveShl1>(se[h]);
        }
        // plane m + 1 into the registers just freed.  The scheduler may not
        // hoist these loads above the use of plane m's values, and they are
        // unconditional (the last step reloads its own plane, from cache): the
        // loads then reuse the same registers, with no copy at the end of the
        // step.
        __builtin_amdgcn_sched_barrier(0);
        load_in(wrapm(m < p.m1 ? m + 1 : m));

        // x-filter the R + 2 rows of plane m, then y and z
        C hx[HR][VW];
#pragma unroll
        for (int h = 0; h < HR; ++h) {
            C left = dpp_shift<kDppWaveShr1>(sm[h][VW - 1]);
            C right = dpp_shift<kDppWaveShl1>(sm[h][0]);
            if (lane == 0) left = se[h];
            if (lane == last) right = sr[h];
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                const C l = k == 0 ? left : sm[h][k - 1];
                const C rr = k == VW - 1 ? right : sm[h][k + 1];
                hx[h][k] = C(0.5) * sm[h][k] + C(0.25) * (l + rr);
            }
        }
        C gv[R][VW];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                W0[r][k] = W1[r][k];
                W1[r][k] = W2[r][k];
                W2[r][k] = C(0.5) * hx[r + 1][k] + C(0.25) * (hx[r][k] + hx[r + 2][k]);
                gv[r][k] = C(0.5) * W1[r][k] + C(0.25) * (W0[r][k] + W2[r][k]);
            }
        // output plane m - 1 (its centre fields were loaded one step ago)
        if (m > p.m0) {
            const int64_t mo = m - 1;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (p.act && p.row0 + r < g.nrows)
                    op.out(mo * g.plane + (p.row0 + r) * nx + p.x0, S1[r], gv[r], co[r], acc);
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < VW; ++k) S1[r][k] = sm[r + 1][k];
        // centre fields of plane m, for the next step's output (unconditional
        // too: the first and the last step load a neighbouring plane of the
        // tile, unused)
        __builtin_amdgcn_sched_barrier(0);
        load_out(m < p.m0 ? p.m0 : (m < p.m1 ? m : p.m1 - 1));
    }
}

// 3D march of a two-lane-row tile (16-byte lanes, R = 4): lanes 0-31 hold
// rows row0, row0 + 1 of 32 x-segments and lanes 32-63 the next two rows.
// Each lane loads its two rows and one more: the row above the tile (lower
// half) or the row below it (upper half); the rows between the halves cross
// by a lane exchange (lane i <-> i ^ 32) of x-filtered values.  So a lane
// loads 3 rows per 2 output rows (the one-lane-row tile of R = 2: 4).
// x neighbours cross lanes by DPP within each half.  Must be called by the
// whole wave.
template <int VW, typename T, typename C, class Op>
__device__ __forceinline__ void march_pair(const Geo &g, int64_t lt, const Op &op, double (&acc)[NACC], int lane) {
    constexpr int R = 4, RY = 2, LX = WAVE / 2;
    constexpr int NI = Arr<Op::NI>::n;
    constexpr int NO = Arr<Op::NO>::n;
    const TilePos p = tile_pos<VW, R>(g, lt, lane);
    const int lx = lane & (LX - 1);
    const bool upper = lane >= LX;
    const int64_t nx = g.nx;
    auto wrow = [&](int64_t row) -> int64_t {
        row %= g.nrows;
        return row < 0 ? row + g.nrows : row;
    };
    // rows a lane loads: its own two (periodically wrapped: a row past the
    // field's end is a neighbour's halo, not an output) and the extra one
    int64_t rowoff[3];
    rowoff[0] = wrow(p.row0) * nx;
    rowoff[1] = wrow(p.row0 + 1) * nx;
    rowoff[2] = wrow(upper ? p.row0 + 2 : p.row0 - 1) * nx;

    // a half's x span: lanes 0 .. last of the half hold field points; the
    // periodic neighbours outside it are loaded by the half's lane 0 (left)
    // and by its lane last + 1, or last = 31 on a full span (right)
    const int64_t seg0 = p.seg0;
    const int64_t nseg = nx - seg0 < (int64_t)LX * VW ? nx - seg0 : (int64_t)LX * VW;
    const int last = (int)(nseg / VW) - 1;
    const bool full = last == LX - 1;
    const int redge = full ? last : last + 1;
    const int64_t xleft = seg0 == 0 ? nx - 1 : seg0 - 1;
    const int64_t xright = seg0 + nseg >= nx ? seg0 + nseg - nx : seg0 + nseg;
    const int64_t xe = lx == 0 ? xleft : (lx == redge ? xright : p.xc);

    auto wrapm = [&](int64_t m) -> int64_t { return m < 0 ? m + g.nmarch : (m >= g.nmarch ? m - g.nmarch : m); };
    uint32_t vo[3], eo[3];
#pragma unroll
    for (int h = 0; h < 3; ++h) {
        vo[h] = (uint32_t)((rowoff[h] + p.xc) * (int64_t)sizeof(T));
        eo[h] = (uint32_t)((rowoff[h] + xe) * (int64_t)sizeof(T));
    }

    // raw stencil inputs of two planes in flight (double-buffered: plane m + 2
    // is loaded while plane m is filtered)
    T rawA[3][NI][VW], raweA[3][NI], rawB[3][NI][VW], raweB[3][NI];
    auto load_in = [&](int64_t mw, T (&raw)[3][NI][VW], T (&rawe)[3][NI]) {
#pragma unroll
        for (int f = 0; f < Op::NI; ++f) {
            const T *pb = op.in[f] + mw * g.plane;
#pragma unroll
            for (int h = 0; h < 3; ++h) {
                vld<T, VW>(at_off(pb, vo[h]), raw[h][f]);
                rawe[h][f] = *at_off(pb, eo[h]);
            }
        }
    };
    T co[RY][NO][VW];
    auto load_out = [&](int64_t m) {
#pragma unroll
        for (int f = 0; f < Op::NO; ++f) {
            const T *pb = op.oin[f] + m * g.plane;
#pragma unroll
            for (int r = 0; r < RY; ++r) vld_nt<T, VW>(at_off(pb, vo[r]), co[r][f]);
        }
    };

    C W0[RY][VW], W1[RY][VW], W2[RY][VW], S1[RY][VW];
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int k = 0; k < VW; ++k) W0[r][k] = W1[r][k] = W2[r][k] = S1[r][k] = C(0);
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int f = 0; f < NO; ++f)
#pragma unroll
            for (int k = 0; k < VW; ++k) co[r][f][k] = T(0);

    // one step: filter plane m from `raw` (loaded two steps ago), then reuse
    // its registers for plane m + 2 (the last steps reload plane m1, from cache)
    auto step = [&](int64_t m, T (&raw)[3][NI][VW], T (&rawe)[3][NI]) {
        C sm[3][VW], se[3], sr[3];
#pragma unroll
        for (int h = 0; h < 3; ++h) {
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                T a[NI];
#pragma unroll
                for (int f = 0; f < NI; ++f) a[f] = raw[h][f][k];
                sm[h][k] = op.mix(a);
            }
            se[h] = op.mix(rawe[h]);
            sr[h] = full ? se[h] : dpp_shift<kDppWaveShl1>(se[h]);
        }
        __builtin_amdgcn_sched_barrier(0);
        load_in(wrapm(m + 2 <= p.m1 ? m + 2 : p.m1), raw, rawe);

        // x-filter the three rows (DPP across the whole wave; the halves'
        // edge lanes take their own loads instead)
        C hx[3][VW];
#pragma unroll
        for (int h = 0; h < 3; ++h) {
            C left = dpp_shift<kDppWaveShr1>(sm[h][VW - 1]);
            C right = dpp_shift<kDppWaveShl1>(sm[h][0]);
            if (lx == 0) left = se[h];
            if (lx == last) right = sr[h];
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                const C l = k == 0 ? left : sm[h][k - 1];
                const C rr = k == VW - 1 ? right : sm[h][k + 1];
                hx[h][k] = C(0.5) * sm[h][k] + C(0.25) * (l + rr);
            }
        }
        // the row below own row 1 (lower half) is the upper half's own row 0;
        // the row above own row 0 (upper half) is the lower half's own row 1
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            const C send = upper ? hx[0][k] : hx[1][k];
            const C recv = __shfl_xor(send, LX, WAVE);
            const C above0 = upper ? recv : hx[2][k];
            const C below1 = upper ? hx[2][k] : recv;
            W0[0][k] = W1[0][k];
            W1[0][k] = W2[0][k];
            W2[0][k] = C(0.5) * hx[0][k] + C(0.25) * (above0 + hx[1][k]);
            W0[1][k] = W1[1][k];
            W1[1][k] = W2[1][k];
            W2[1][k] = C(0.5) * hx[1][k] + C(0.25) * (hx[0][k] + below1);
        }
        C gv[RY][VW];
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int k = 0; k < VW; ++k) gv[r][k] = C(0.5) * W1[r][k] + C(0.25) * (W0[r][k] + W2[r][k]);
        // output plane m - 1 (its centre fields were loaded one step ago)
        if (m > p.m0) {
            const int64_t mo = m - 1;
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                if (p.act && p.row0 + r < g.nrows)
                    op.out(mo * g.plane + (p.row0 + r) * nx + p.x0, S1[r], gv[r], co[r], acc);
            }
        }
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int k = 0; k < VW; ++k) S1[r][k] = sm[r][k];
        __builtin_amdgcn_sched_barrier(0);
        load_out(m < p.m0 ? p.m0 : (m < p.m1 ? m : p.m1 - 1));
    };

    // planes m0 - 1 .. m1 (the two halo planes included), two in flight
    load_in(wrapm(p.m0 - 1), rawA, raweA);
    load_in(wrapm(p.m0 <= p.m1 ? p.m0 : p.m1), rawB, raweB);
    for (int64_t m = p.m0 - 1; m <= p.m1; m += 2) {
        step(m, rawA, raweA);
        if (m + 1 <= p.m1) step(m + 1, rawB, raweB);
    }
}

// March one tile with the separable stencil.
//   Op::NI stencil-input fields op.in[f]; op.mix(v[NI]) forms S at a point
//   Op::NO centre-only fields op.oin[f], loaded for every output point
//   op.out(idx, s[VW], g[VW], o[NO][VW], acc) consumes S, G S and the centre
//   fields at VW consecutive output points
// NDIM 2: R must be 1 (no in-plane y).  Must be called by the whole wave.
template <int NDIM, int VW, int R, typename T, typename C, class Op>
__device__ __forceinline__ void march_tile(const Geo &g, int64_t lt, const Op &op, double (&acc)[NACC], int lane) {
    static_assert(NDIM == 3 || R == 1, "2D tiles are one row wide");
    if constexpr (NDIM == 2)
        march_row<VW, T, C>(g, lt, op, acc, lane);
    else if constexpr (tile_lane_rows(VW, R) == 2)
        march_pair<VW, T, C>(g, lt, op, acc, lane);
    else
        march_slab<VW, R, T, C>(g, lt, op, acc, lane);
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
    constexpr int RY = R / tile_lane_rows(VW, R);  // rows per lane
    for (int64_t m = p.m0; m < p.m1; ++m)
#pragma unroll
        for (int r = 0; r < RY; ++r)
            if (NDIM == 2 || p.row0 + r < g.nrows) {
                const int64_t i = m * g.plane + (p.row0 + r) * g.nx + p.x0;
                T o[NO][VW];
#pragma unroll
                for (int f = 0; f < Op::NO; ++f) vld_nt<T, VW>(op.oin[f] + i, o[f]);
                op.out(i, zero, zero, o, acc);
            }
}

}  // namespace gd
