// gd_ops.h -- the fused sweeps of the four solvers.
//
// Each sweep is a functor used by march_tile / point_tile:
//   NI, in[]   fields the stencil input S is formed from; mix() forms S at a
//              point from their values there (S itself is never stored)
//   NO, oin[]  fields read only at the output point
//   out()      receives S, G S and the centre fields at VW consecutive points,
//              writes the sweep's vector updates and accumulates its inner
//              products in FP64
// The sweeps follow Algorithms 1-4 of the paper with the vector updates fused
// around each application of G; each inner product (a, b) = h^d sum a_i b_i
// is completed by the grid barrier that follows the sweep.
#pragma once

#include "gd_device.h"

namespace gd {

template <typename T, typename C, int VW>
__device__ __forceinline__ void store_c(T *p, const C (&v)[VW]) {
    T t[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) t[k] = T(v[k]);
    vst<T, VW>(p, t);
}

// y = G x (the filter itself)
template <typename T, typename C, int VW>
struct OpFilter {
    static constexpr int NI = 1, NO = 0;
    const T *in[1];
    const T *oin[1];
    T *y;
    __device__ C mix(const T (&v)[1]) const { return C(v[0]); }
    __device__ void out(int64_t i, const C (&)[VW], const C (&g)[VW], const T (&)[1][VW], double (&)[NACC]) const {
        store_c<T, C, VW>(y + i, g);
    }
};

// acc0 += (ubar - G x)^2  (true residual; reference norm ||ubar - G ubar||),
// acc1 += ubar^2 (read only by the reference sweep, which needs both norms)
template <typename T, typename C, int VW>
struct OpResNorm {
    static constexpr int NI = 1, NO = 1;
    const T *in[1];   // x
    const T *oin[1];  // ubar
    __device__ C mix(const T (&v)[1]) const { return C(v[0]); }
    __device__ void out(int64_t, const C (&)[VW], const C (&g)[VW], const T (&o)[1][VW], double (&acc)[NACC]) const {
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            const double d = double(o[0][k]) - double(g[k]);
            acc[0] += d * d;
            acc[1] += double(o[0][k]) * double(o[0][k]);
        }
    }
};

// acc0 += ubar^2  (reference norm ||ubar||), pointwise
template <typename T, typename C, int VW>
struct OpNormUbar {
    static constexpr int NI = 0, NO = 1;
    const T *in[1];
    const T *oin[1];  // ubar
    __device__ void out(int64_t, const C (&)[VW], const C (&)[VW], const T (&o)[1][VW], double (&acc)[NACC]) const {
#pragma unroll
        for (int k = 0; k < VW; ++k) acc[0] += double(o[0][k]) * double(o[0][k]);
    }
};

// u0 = ubar, r0 = ubar - G ubar, f0 = r0 (BiCGSTAB); acc0 = (r0, r0)
template <typename T, typename C, int VW>
struct OpInitUbar {
    static constexpr int NI = 1, NO = 0;
    const T *in[1];  // ubar
    const T *oin[1];
    T *u, *r, *f0;
    __device__ C mix(const T (&v)[1]) const { return C(v[0]); }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], const T (&)[1][VW], double (&acc)[NACC]) const {
        C rv[VW];
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            rv[k] = s[k] - g[k];
            acc[0] += double(rv[k]) * double(rv[k]);
        }
        store_c<T, C, VW>(u + i, s);
        store_c<T, C, VW>(r + i, rv);
        if (f0) store_c<T, C, VW>(f0 + i, rv);
    }
};

// u0 given: r0 = ubar - G u0, f0 = r0
template <typename T, typename C, int VW>
struct OpInitGiven {
    static constexpr int NI = 1, NO = 1;
    const T *in[1];   // u0
    const T *oin[1];  // ubar
    T *r, *f0;
    __device__ C mix(const T (&v)[1]) const { return C(v[0]); }
    __device__ void out(int64_t i, const C (&)[VW], const C (&g)[VW], const T (&o)[1][VW], double (&acc)[NACC]) const {
        C rv[VW];
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            rv[k] = C(o[0][k]) - g[k];
            acc[0] += double(rv[k]) * double(rv[k]);
        }
        store_c<T, C, VW>(r + i, rv);
        if (f0) store_c<T, C, VW>(f0 + i, rv);
    }
};

// u0 = 0: r0 = ubar, f0 = ubar (pointwise)
template <typename T, typename C, int VW>
struct OpInitZero {
    static constexpr int NI = 0, NO = 1;
    const T *in[1];
    const T *oin[1];  // ubar
    T *u, *r, *f0;
    __device__ void out(int64_t i, const C (&)[VW], const C (&)[VW], const T (&o)[1][VW], double (&acc)[NACC]) const {
        T z[VW];
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            z[k] = T(0);
            acc[0] += double(o[0][k]) * double(o[0][k]);
        }
        vst<T, VW>(u + i, z);
        vst<T, VW>(r + i, o[0]);
        if (f0) vst<T, VW>(f0 + i, o[0]);
    }
};

// Van Cittert pass (Algorithm 1): u += r; r' = r - G r; acc0 = (r', r')
template <typename T, typename C, int VW>
struct OpVC {
    static constexpr int NI = 1, NO = 1;
    const T *in[1];   // r
    const T *oin[1];  // u
    T *rn, *u;
    __device__ C mix(const T (&v)[1]) const { return C(v[0]); }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], const T (&o)[1][VW], double (&acc)[NACC]) const {
        C uv[VW], rv[VW];
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            uv[k] = C(o[0][k]) + s[k];
            rv[k] = s[k] - g[k];
            acc[0] += double(rv[k]) * double(rv[k]);
        }
        store_c<T, C, VW>(u + i, uv);
        store_c<T, C, VW>(rn + i, rv);
    }
};

// CG sweep 1 (Algorithm 3), first pass: p0 = r0; d = G p0; acc0 = (p0, d)
template <typename T, typename C, int VW>
struct OpCG1First {
    static constexpr int NI = 1, NO = 0;
    const T *in[1];  // r
    const T *oin[1];
    T *pn;
    __device__ C mix(const T (&v)[1]) const { return C(v[0]); }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], const T (&)[1][VW], double (&acc)[NACC]) const {
#pragma unroll
        for (int k = 0; k < VW; ++k) acc[0] += double(s[k]) * double(g[k]);
        store_c<T, C, VW>(pn + i, s);
    }
};

// CG sweep 1, later passes: p' = r + beta p; d = G p'; acc0 = (p', d)
template <typename T, typename C, int VW>
struct OpCG1 {
    static constexpr int NI = 2, NO = 0;
    const T *in[2];  // r, p
    const T *oin[1];
    T *pn;
    C beta;
    __device__ C mix(const T (&v)[2]) const { return C(v[0]) + beta * C(v[1]); }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], const T (&)[1][VW], double (&acc)[NACC]) const {
#pragma unroll
        for (int k = 0; k < VW; ++k) acc[0] += double(s[k]) * double(g[k]);
        store_c<T, C, VW>(pn + i, s);
    }
};

// CG sweep 2: u += alpha p; r -= alpha G p (G p recomputed); acc0 = (r, r)
template <typename T, typename C, int VW>
struct OpCG2 {
    static constexpr int NI = 1, NO = 2;
    const T *in[1];   // p
    const T *oin[2];  // u, r
    T *u, *r;
    C alpha;
    __device__ C mix(const T (&v)[1]) const { return C(v[0]); }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], const T (&o)[2][VW], double (&acc)[NACC]) const {
        C uv[VW], rv[VW];
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            uv[k] = C(o[0][k]) + alpha * s[k];
            rv[k] = C(o[1][k]) - alpha * g[k];
            acc[0] += double(rv[k]) * double(rv[k]);
        }
        store_c<T, C, VW>(u + i, uv);
        store_c<T, C, VW>(r + i, rv);
    }
};

// BiCGSTAB sweep A (Algorithm 4), first pass: p1 = r0 (p0 = q0 = 0);
// q1 = G p1; acc0 = (f0, q1)
template <typename T, typename C, int VW>
struct OpBiAFirst {
    static constexpr int NI = 1, NO = 1;
    const T *in[1];   // r
    const T *oin[1];  // f0
    T *pn, *qn;
    __device__ C mix(const T (&v)[1]) const { return C(v[0]); }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], const T (&o)[1][VW], double (&acc)[NACC]) const {
#pragma unroll
        for (int k = 0; k < VW; ++k) acc[0] += double(o[0][k]) * double(g[k]);
        store_c<T, C, VW>(pn + i, s);
        store_c<T, C, VW>(qn + i, g);
    }
};

// BiCGSTAB sweep A: p' = r + beta (p - omega q); q' = G p'; acc0 = (f0, q')
template <typename T, typename C, int VW>
struct OpBiA {
    static constexpr int NI = 3, NO = 1;
    const T *in[3];   // r, p, q
    const T *oin[1];  // f0
    T *pn, *qn;
    C beta, omega;
    __device__ C mix(const T (&v)[3]) const { return C(v[0]) + beta * (C(v[1]) - omega * C(v[2])); }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], const T (&o)[1][VW], double (&acc)[NACC]) const {
#pragma unroll
        for (int k = 0; k < VW; ++k) acc[0] += double(o[0][k]) * double(g[k]);
        store_c<T, C, VW>(pn + i, s);
        store_c<T, C, VW>(qn + i, g);
    }
};

// BiCGSTAB sweep B: s = r - alpha q, t = G s (both on the fly);
// acc = (s, t), (t, t), (s, s)
template <typename T, typename C, int VW>
struct OpBiB {
    static constexpr int NI = 2, NO = 0;
    const T *in[2];  // r, q
    const T *oin[1];
    C alpha;
    __device__ C mix(const T (&v)[2]) const { return C(v[0]) - alpha * C(v[1]); }
    __device__ void out(int64_t, const C (&s)[VW], const C (&g)[VW], const T (&)[1][VW], double (&acc)[NACC]) const {
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            acc[0] += double(s[k]) * double(g[k]);
            acc[1] += double(g[k]) * double(g[k]);
            acc[2] += double(s[k]) * double(s[k]);
        }
    }
};

// BiCGSTAB sweep C: s, t recomputed; u += alpha p + omega s; r' = s - omega t;
// acc = (f0, r'), (r', r')
template <typename T, typename C, int VW>
struct OpBiC {
    static constexpr int NI = 2, NO = 3;
    const T *in[2];   // r, q
    const T *oin[3];  // u, p, f0
    T *u, *rn;
    C alpha, omega;
    __device__ C mix(const T (&v)[2]) const { return C(v[0]) - alpha * C(v[1]); }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], const T (&o)[3][VW], double (&acc)[NACC]) const {
        C uv[VW], rv[VW];
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            uv[k] = C(o[0][k]) + (alpha * C(o[1][k]) + omega * s[k]);
            rv[k] = s[k] - omega * g[k];
            acc[0] += double(o[2][k]) * double(rv[k]);
            acc[1] += double(rv[k]) * double(rv[k]);
        }
        store_c<T, C, VW>(u + i, uv);
        store_c<T, C, VW>(rn + i, rv);
    }
};

// Steepest descent sweep 1 (Algorithm 2): acc0 = (r, G r)
template <typename T, typename C, int VW>
struct OpSD1 {
    static constexpr int NI = 1, NO = 0;
    const T *in[1];  // r
    const T *oin[1];
    __device__ C mix(const T (&v)[1]) const { return C(v[0]); }
    __device__ void out(int64_t, const C (&s)[VW], const C (&g)[VW], const T (&)[1][VW], double (&acc)[NACC]) const {
#pragma unroll
        for (int k = 0; k < VW; ++k) acc[0] += double(s[k]) * double(g[k]);
    }
};

// Steepest descent sweep 2: u += alpha r; r' = r - alpha G r; acc0 = (r', r')
template <typename T, typename C, int VW>
struct OpSD2 {
    static constexpr int NI = 1, NO = 1;
    const T *in[1];   // r
    const T *oin[1];  // u
    T *rn, *u;
    C alpha;
    __device__ C mix(const T (&v)[1]) const { return C(v[0]); }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], const T (&o)[1][VW], double (&acc)[NACC]) const {
        C uv[VW], rv[VW];
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            uv[k] = C(o[0][k]) + alpha * s[k];
            rv[k] = s[k] - alpha * g[k];
            acc[0] += double(rv[k]) * double(rv[k]);
        }
        store_c<T, C, VW>(u + i, uv);
        store_c<T, C, VW>(rn + i, rv);
    }
};

}  // namespace gd
