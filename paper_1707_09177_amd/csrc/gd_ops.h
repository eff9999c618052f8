// gd_ops.h -- the fused sweeps of the four solvers.
//
// Each sweep is a functor used by march_tile / point_tile: `src` evaluates
// the stencil input S at a point, `out` receives S and G S at an output point,
// does the sweep's vector updates there and accumulates its inner products in
// FP64.  The sweeps follow Algorithms 1-4 of the paper with the vector
// updates fused around each application of G; every inner product
// (a, b) = h^d sum a_i b_i is completed by the grid barrier that follows the
// sweep.
#pragma once

#include "gd_device.h"

namespace gd {

// ---- helpers on VW-wide registers
template <typename T, typename C, int VW>
__device__ __forceinline__ void load_c(const T *p, C (&v)[VW]) {
    T t[VW];
    vld<T, VW>(p, t);
#pragma unroll
    for (int k = 0; k < VW; ++k) v[k] = C(t[k]);
}

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
    const T *x;
    T *y;
    __device__ void src(int64_t i, C (&s)[VW]) const { load_c<T, C, VW>(x + i, s); }
    __device__ C src1(int64_t i) const { return C(x[i]); }
    __device__ void out(int64_t i, const C (&)[VW], const C (&g)[VW], double (&)[NACC]) const {
        store_c<T, C, VW>(y + i, g);
    }
};

// acc0 += (ubar - G x)^2  (true residual; reference norm ||ubar - G ubar||)
template <typename T, typename C, int VW>
struct OpResNorm {
    const T *x;
    const T *ub;
    __device__ void src(int64_t i, C (&s)[VW]) const { load_c<T, C, VW>(x + i, s); }
    __device__ C src1(int64_t i) const { return C(x[i]); }
    __device__ void out(int64_t i, const C (&)[VW], const C (&g)[VW], double (&acc)[NACC]) const {
        C b[VW];
        load_c<T, C, VW>(ub + i, b);
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            const double d = double(b[k]) - double(g[k]);
            acc[0] += d * d;
        }
    }
};

// acc0 += ubar^2  (reference norm ||ubar||), pointwise
template <typename T, typename C, int VW>
struct OpNormUbar {
    const T *ub;
    __device__ void src(int64_t, C (&)[VW]) const {}
    __device__ C src1(int64_t) const { return C(0); }
    __device__ void out(int64_t i, const C (&)[VW], const C (&)[VW], double (&acc)[NACC]) const {
        T b[VW];
        vld<T, VW>(ub + i, b);
#pragma unroll
        for (int k = 0; k < VW; ++k) acc[0] += double(b[k]) * double(b[k]);
    }
};

// u0 = ubar, r0 = ubar - G ubar, f0 = r0 (BiCGSTAB); acc0 = (r0, r0)
template <typename T, typename C, int VW>
struct OpInitUbar {
    const T *ub;
    T *u, *r, *f0;
    __device__ void src(int64_t i, C (&s)[VW]) const { load_c<T, C, VW>(ub + i, s); }
    __device__ C src1(int64_t i) const { return C(ub[i]); }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], double (&acc)[NACC]) const {
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
    const T *u, *ub;
    T *r, *f0;
    __device__ void src(int64_t i, C (&s)[VW]) const { load_c<T, C, VW>(u + i, s); }
    __device__ C src1(int64_t i) const { return C(u[i]); }
    __device__ void out(int64_t i, const C (&)[VW], const C (&g)[VW], double (&acc)[NACC]) const {
        C b[VW], rv[VW];
        load_c<T, C, VW>(ub + i, b);
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            rv[k] = b[k] - g[k];
            acc[0] += double(rv[k]) * double(rv[k]);
        }
        store_c<T, C, VW>(r + i, rv);
        if (f0) store_c<T, C, VW>(f0 + i, rv);
    }
};

// u0 = 0: r0 = ubar, f0 = ubar (pointwise)
template <typename T, typename C, int VW>
struct OpInitZero {
    const T *ub;
    T *u, *r, *f0;
    __device__ void src(int64_t, C (&)[VW]) const {}
    __device__ C src1(int64_t) const { return C(0); }
    __device__ void out(int64_t i, const C (&)[VW], const C (&)[VW], double (&acc)[NACC]) const {
        T b[VW], z[VW];
        vld<T, VW>(ub + i, b);
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            z[k] = T(0);
            acc[0] += double(b[k]) * double(b[k]);
        }
        vst<T, VW>(u + i, z);
        vst<T, VW>(r + i, b);
        if (f0) vst<T, VW>(f0 + i, b);
    }
};

// Van Cittert pass (Algorithm 1): u += r; r' = r - G r; acc0 = (r', r')
template <typename T, typename C, int VW>
struct OpVC {
    const T *r;
    T *rn, *u;
    __device__ void src(int64_t i, C (&s)[VW]) const { load_c<T, C, VW>(r + i, s); }
    __device__ C src1(int64_t i) const { return C(r[i]); }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], double (&acc)[NACC]) const {
        C uv[VW], rv[VW];
        load_c<T, C, VW>(u + i, uv);
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            uv[k] += s[k];
            rv[k] = s[k] - g[k];
            acc[0] += double(rv[k]) * double(rv[k]);
        }
        store_c<T, C, VW>(u + i, uv);
        store_c<T, C, VW>(rn + i, rv);
    }
};

// CG sweep 1 (Algorithm 3): p' = r + beta p (p' = r on the first pass);
// d = G p'; acc0 = (p', d)
template <typename T, typename C, int VW>
struct OpCG1 {
    const T *r, *po;
    T *pn;
    C beta;
    bool first;
    __device__ void src(int64_t i, C (&s)[VW]) const {
        load_c<T, C, VW>(r + i, s);
        if (!first) {
            C pv[VW];
            load_c<T, C, VW>(po + i, pv);
#pragma unroll
            for (int k = 0; k < VW; ++k) s[k] = s[k] + beta * pv[k];
        }
    }
    __device__ C src1(int64_t i) const { return first ? C(r[i]) : C(r[i]) + beta * C(po[i]); }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], double (&acc)[NACC]) const {
#pragma unroll
        for (int k = 0; k < VW; ++k) acc[0] += double(s[k]) * double(g[k]);
        store_c<T, C, VW>(pn + i, s);
    }
};

// CG sweep 2: u += alpha p; r -= alpha G p (G p recomputed); acc0 = (r, r)
template <typename T, typename C, int VW>
struct OpCG2 {
    const T *p;
    T *r, *u;
    C alpha;
    __device__ void src(int64_t i, C (&s)[VW]) const { load_c<T, C, VW>(p + i, s); }
    __device__ C src1(int64_t i) const { return C(p[i]); }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], double (&acc)[NACC]) const {
        C uv[VW], rv[VW];
        load_c<T, C, VW>(u + i, uv);
        load_c<T, C, VW>(r + i, rv);
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            uv[k] += alpha * s[k];
            rv[k] -= alpha * g[k];
            acc[0] += double(rv[k]) * double(rv[k]);
        }
        store_c<T, C, VW>(u + i, uv);
        store_c<T, C, VW>(r + i, rv);
    }
};

// BiCGSTAB sweep A (Algorithm 4): p' = r + beta (p - omega q) (p' = r on the
// first pass, where p0 = q0 = 0); q' = G p'; acc0 = (f0, q')
template <typename T, typename C, int VW>
struct OpBiA {
    const T *r, *po, *qo, *f0;
    T *pn, *qn;
    C beta, omega;
    bool first;
    __device__ void src(int64_t i, C (&s)[VW]) const {
        load_c<T, C, VW>(r + i, s);
        if (!first) {
            C pv[VW], qv[VW];
            load_c<T, C, VW>(po + i, pv);
            load_c<T, C, VW>(qo + i, qv);
#pragma unroll
            for (int k = 0; k < VW; ++k) s[k] = s[k] + beta * (pv[k] - omega * qv[k]);
        }
    }
    __device__ C src1(int64_t i) const {
        return first ? C(r[i]) : C(r[i]) + beta * (C(po[i]) - omega * C(qo[i]));
    }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], double (&acc)[NACC]) const {
        C fv[VW];
        load_c<T, C, VW>(f0 + i, fv);
#pragma unroll
        for (int k = 0; k < VW; ++k) acc[0] += double(fv[k]) * double(g[k]);
        store_c<T, C, VW>(pn + i, s);
        store_c<T, C, VW>(qn + i, g);
    }
};

// BiCGSTAB sweep B: s = r - alpha q, t = G s (both on the fly);
// acc = (s, t), (t, t), (s, s)
template <typename T, typename C, int VW>
struct OpBiB {
    const T *r, *q;
    C alpha;
    __device__ void src(int64_t i, C (&s)[VW]) const {
        C qv[VW];
        load_c<T, C, VW>(r + i, s);
        load_c<T, C, VW>(q + i, qv);
#pragma unroll
        for (int k = 0; k < VW; ++k) s[k] = s[k] - alpha * qv[k];
    }
    __device__ C src1(int64_t i) const { return C(r[i]) - alpha * C(q[i]); }
    __device__ void out(int64_t, const C (&s)[VW], const C (&g)[VW], double (&acc)[NACC]) const {
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
    const T *r, *q, *p, *f0;
    T *u, *rn;
    C alpha, omega;
    __device__ void src(int64_t i, C (&s)[VW]) const {
        C qv[VW];
        load_c<T, C, VW>(r + i, s);
        load_c<T, C, VW>(q + i, qv);
#pragma unroll
        for (int k = 0; k < VW; ++k) s[k] = s[k] - alpha * qv[k];
    }
    __device__ C src1(int64_t i) const { return C(r[i]) - alpha * C(q[i]); }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], double (&acc)[NACC]) const {
        C uv[VW], pv[VW], fv[VW], rv[VW];
        load_c<T, C, VW>(u + i, uv);
        load_c<T, C, VW>(p + i, pv);
        load_c<T, C, VW>(f0 + i, fv);
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            uv[k] += alpha * pv[k] + omega * s[k];
            rv[k] = s[k] - omega * g[k];
            acc[0] += double(fv[k]) * double(rv[k]);
            acc[1] += double(rv[k]) * double(rv[k]);
        }
        store_c<T, C, VW>(u + i, uv);
        store_c<T, C, VW>(rn + i, rv);
    }
};

// Steepest descent sweep 1 (Algorithm 2): acc0 = (r, G r)
template <typename T, typename C, int VW>
struct OpSD1 {
    const T *r;
    __device__ void src(int64_t i, C (&s)[VW]) const { load_c<T, C, VW>(r + i, s); }
    __device__ C src1(int64_t i) const { return C(r[i]); }
    __device__ void out(int64_t, const C (&s)[VW], const C (&g)[VW], double (&acc)[NACC]) const {
#pragma unroll
        for (int k = 0; k < VW; ++k) acc[0] += double(s[k]) * double(g[k]);
    }
};

// Steepest descent sweep 2: u += alpha r; r' = r - alpha G r; acc0 = (r', r')
template <typename T, typename C, int VW>
struct OpSD2 {
    const T *r;
    T *rn, *u;
    C alpha;
    __device__ void src(int64_t i, C (&s)[VW]) const { load_c<T, C, VW>(r + i, s); }
    __device__ C src1(int64_t i) const { return C(r[i]); }
    __device__ void out(int64_t i, const C (&s)[VW], const C (&g)[VW], double (&acc)[NACC]) const {
        C uv[VW], rv[VW];
        load_c<T, C, VW>(u + i, uv);
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            uv[k] += alpha * s[k];
            rv[k] = s[k] - alpha * g[k];
            acc[0] += double(rv[k]) * double(rv[k]);
        }
        store_c<T, C, VW>(u + i, uv);
        store_c<T, C, VW>(rn + i, rv);
    }
};

}  // namespace gd
