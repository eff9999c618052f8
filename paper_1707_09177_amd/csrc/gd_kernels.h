// gd_kernels.h -- the persistent solver kernel and the filter kernel.
//
// One launch runs a whole solve for a batch of fields ("instances").  The grid
// holds at most as many workgroups as can be resident at once, every wave
// loops over tiles, and the sweeps of Algorithms 1-4 are separated by a grid
// barrier.  Each tile publishes its FP64 partial inner products and counts
// itself done for its instance; the wave that completes an instance's last
// tile sums that instance's partials in tile order (so results are bitwise
// reproducible and independent of which wave ran which tile) and updates its
// scalars (alpha, beta, omega, rho, convergence test, guards, residual
// history).  Instances therefore finish their reductions in parallel, and the
// grid barrier itself only orders the sweeps.  The iteration loop, including
// the stopping test, never returns to the host.
#pragma once
#include <hip/hip_runtime.h>

#include "gd_device.h"
#include "gd_ops.h"
#include "gd_internal.h"
#include "gdecon.h"

namespace gd {

// ------------------------------------------------------------ device state
// s_waitcnt vmcnt(0): block until every vector-memory operation this wave
// has issued (stores and cache invalidations included) has completed.  GFX9 encoding:
// vmcnt = 0, expcnt = 7 and lgkmcnt = 15 (the latter two: no wait).
__device__ __forceinline__ void wait_vm_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ __forceinline__ int ld_i32(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_f64(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// v, which is the same in every lane, as a value the compiler knows to be
// wave-uniform (kept in scalar registers, with scalar branches on it)
__device__ __forceinline__ int64_t wave_uniform(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <bool TABLE>
static __device__ __forceinline__ Inst get_inst(const Params &P, int i) {
    if constexpr (TABLE) return P.table[i];
    Inst I = P.tmpl;
    const int64_t off = (int64_t)i * P.stride_bytes;
    I.ubar = (const char *)I.ubar + off;
    I.u = (char *)I.u + off;
#pragma unroll
    for (int v = 0; v < NVEC; ++v)
        if (I.vec[v]) I.vec[v] = (char *)I.vec[v] + off;
    if (I.hist) I.hist += (int64_t)i * P.hist_stride;
    I.info += i;
    I.tile0 = (int64_t)i * P.tiles_per_inst;
    return I;
}

// Tile t of the claim order -> instance, and the instance's local tile lt.
// Claims take every instance's long tiles first, then the short ones, so the
// end of a sweep is made of short tiles.
template <bool TABLE>
static __device__ __forceinline__ int locate(const Params &P, int64_t t, int64_t &lt) {
    if constexpr (!TABLE) {
        const int64_t nb = P.tmpl.geo.nbig;
        if (t < P.big_total) {
            lt = t % nb;
            return (int)(t / nb);
        }
        const int64_t ns = P.tiles_per_inst - nb;
        const int64_t t2 = t - P.big_total;
        lt = nb + t2 % ns;
        return (int)(t2 / ns);
    } else {
        const bool big = t < P.big_total;
        const int64_t key = big ? t : t - P.big_total;
        int lo = 0, hi = P.ninst - 1;
        while (lo < hi) {  // last instance whose range starts at or before key
            const int mid = (lo + hi + 1) >> 1;
            const int64_t v = big ? P.table[mid].b0 : P.table[mid].s0;
            if (v <= key) lo = mid;
            else hi = mid - 1;
        }
        lt = big ? key - P.table[lo].b0 : P.table[lo].geo.nbig + (key - P.table[lo].s0);
        return lo;
    }
}

// Call f.template operator()<NDIM, VW, R>() for the instance's tile variant.
// VS is one variant code (a kernel specialised to one tile shape) or VAR_ALL
// (a kernel for uneven batches that picks the shape per instance among the
// shapes mixed_variant_ok() accepts).
template <typename T, int VS, class F>
__device__ __forceinline__ void with_variant(const Inst &I, F &&f) {
    if constexpr (VS != VAR_ALL) {
        f.template operator()<var_ndim(VS), var_vw(VS), var_r(VS)>();
    } else {
        constexpr int VM = VMax<T>::v;
        if (I.ndim == 2) {
            if (I.vw == VM) f.template operator()<2, VM, 1>();
            else f.template operator()<2, 1, 1>();
        } else if (I.vw == VM) {
            if constexpr (mixed_variant_ok((int)sizeof(T), 3, VM, 2)) {
                if (I.R == 2) f.template operator()<3, VM, 2>();
                else f.template operator()<3, VM, 1>();
            } else {
                f.template operator()<3, VM, 1>();
            }
        } else {
            f.template operator()<3, 1, 1>();
        }
    }
}

template <int PH> struct PhaseNacc { static constexpr int v = 1; };
template <> struct PhaseNacc<PH_BIB> { static constexpr int v = 3; };
template <> struct PhaseNacc<PH_BIC> { static constexpr int v = 2; };
template <> struct PhaseNacc<PH_RREF_RES> { static constexpr int v = 2; };

__host__ __device__ constexpr inline int phase_nacc(int ph) {
    return ph == PH_BIB ? 3 : ((ph == PH_BIC || ph == PH_RREF_RES) ? 2 : 1);
}

// Pointwise pass over a tile of a stored half spectrum (the differential
// filter): G S = G_hat(k) S at every point, G_hat = 1 / (1 + |k|^2 / k_c^2).
// The spectrum is [k_z][k_y][row of nxs reals, (re, im) pairs, k_x = 0 ..
// nxc - 1, then zero padding] per field; the tile geometry may present it
// with any row length, so each point's wavenumber comes from its index i in
// the field: i = (k_z n_y + k_y) nxs + 2 k_x (+ 1 for the imaginary part).
// A lane's VW elements lie in one stored row (nxs and the lane offset are
// multiples of VW).  G_hat is taken as 0 on the padding.
template <int NDIM, int VW, int R, typename T, typename C, class Op>
__device__ __forceinline__ void spectral_tile(const Inst &I, int64_t lt, const Op &op, double (&acc)[NACC],
                                              int lane) {
    constexpr int NI = Arr<Op::NI>::n;
    constexpr int NO = Arr<Op::NO>::n;
    const Geo &g = I.geo;
    const TilePos p = tile_pos<VW, R>(g, lt, lane);
    if (!p.act) return;
    const C ikc2 = C(I.inv_kc2);
    const int64_t ny = int64_t(1) << I.lny, nz = int64_t(1) << I.lnz;
    const int64_t nxs = I.nxs;
    const double inv_nxs = 1.0 / (double)nxs;
    auto sk = [](int64_t k, int64_t n) -> int64_t { return 2 * k <= n ? k : k - n; };
    // one row at a time, its loads issued one step ahead
    const int64_t nrow_steps = (p.m1 - p.m0) * R;
    auto index_of = [&](int64_t q, int64_t &m, int64_t &row) {
        m = p.m0 + q / R;
        row = p.row0 + q % R;
    };
    T v[NI][VW], o[NO][VW];
    auto load = [&](int64_t q, T (&vv)[NI][VW], T (&oo)[NO][VW]) {
        int64_t m, row;
        index_of(q, m, row);
        if (NDIM == 3 && row >= g.nrows) row = g.nrows - 1;  // loads stay in the field
        const int64_t i = m * g.plane + row * g.nx + p.x0;
#pragma unroll
        for (int f = 0; f < Op::NI; ++f) vld<T, VW>(op.in[f] + i, vv[f]);
#pragma unroll
        for (int f = 0; f < Op::NO; ++f) vld_nt<T, VW>(op.oin[f] + i, oo[f]);
    };
    if (nrow_steps > 0) load(0, v, o);
    for (int64_t q = 0; q < nrow_steps; ++q) {
        T nv[NI][VW], no[NO][VW];
        if (q + 1 < nrow_steps) load(q + 1, nv, no);
        int64_t m, row;
        index_of(q, m, row);
        if (NDIM == 2 || row < g.nrows) {
            const int64_t i = m * g.plane + row * g.nx + p.x0;
            // stored row s = i / nxs, exactly: a double-precision estimate, then one correction
            int64_t srow = (int64_t)((double)i * inv_nxs);
            int64_t off = i - srow * nxs;
            if (off < 0) {
                --srow;
                off += nxs;
            } else if (off >= nxs) {
                ++srow;
                off -= nxs;
            }
            const int64_t ky = srow & (ny - 1), kz = srow >> I.lny;
            const int64_t a = sk(ky, ny), b = sk(kz, nz);
            const C kyz2 = C(a * a + b * b);
            C s[VW], gv[VW];
#pragma unroll
            for (int k = 0; k < VW; ++k) {
                T av[NI];
#pragma unroll
                for (int f = 0; f < NI; ++f) av[f] = v[f][k];
                s[k] = op.mix(av);
                const int64_t kx = (off + k) >> 1;
                const C gh = kx >= I.nxc ? C(0) : C(1) / (C(1) + (C(kx * kx) + kyz2) * ikc2);
                gv[k] = gh * s[k];
            }
            op.out(i, s, gv, o, acc);
        }
#pragma unroll
        for (int f = 0; f < NI; ++f)
#pragma unroll
            for (int k = 0; k < VW; ++k) v[f][k] = nv[f][k];
#pragma unroll
        for (int f = 0; f < NO; ++f)
#pragma unroll
            for (int k = 0; k < VW; ++k) o[f][k] = no[f][k];
    }
}

// One tile of a sweep that applies G: the stencil march, or on a stored
// spectrum the pointwise transfer function.
template <int VS, int NDIM, int VW, int R, typename T, typename C, class Op>
__device__ __forceinline__ void g_tile(const Inst &I, int64_t lt, const Op &op, double (&acc)[NACC], int lane) {
    if constexpr (var_spec(VS)) spectral_tile<NDIM, VW, R, T, C>(I, lt, op, acc, lane);
    else march_tile<NDIM, VW, R, T, C>(I.geo, lt, op, acc, lane);
}

// One tile of one sweep.
template <typename T, int VS, int PH>
__device__ __forceinline__ void tile_body(const Params &P, const Inst &I, const State *S, int it, int64_t lt,
                                          double (&acc)[NACC], int lane) {
    const T alpha = T(ld_f64(&S->alpha));
    const T beta = T(ld_f64(&S->beta));
    const T omega = T(ld_f64(&S->omega));
    const bool odd = (it & 1) != 0;
    // the first pass of a Krylov sequence: the solve's first, or the first
    // after a residual replacement (the same value in every lane)
    const bool first = it == 0 || __builtin_amdgcn_readfirstlane(ld_i32(&S->restart)) != 0;
    T *const V[NVEC] = {static_cast<T *>(I.vec[0]), static_cast<T *>(I.vec[1]), static_cast<T *>(I.vec[2]),
                        static_cast<T *>(I.vec[3]), static_cast<T *>(I.vec[4]), static_cast<T *>(I.vec[5]),
                        static_cast<T *>(I.vec[6])};
    // ping-pong buffers: X(base) is the current one, Y(base) the next one
    // (a bitwise blend, so that the pair is never indexed through memory)
    const uintptr_t sel = odd ? ~uintptr_t(0) : uintptr_t(0);
    auto blend = [&](T *a, T *b) -> T * {
        return reinterpret_cast<T *>((reinterpret_cast<uintptr_t>(a) & ~sel) | (reinterpret_cast<uintptr_t>(b) & sel));
    };
    auto X = [&](int base) -> T * { return blend(V[base], V[base + 1]); };
    auto Y = [&](int base) -> T * { return blend(V[base + 1], V[base]); };
    const T *ub = static_cast<const T *>(I.ubar);
    T *u = static_cast<T *>(I.u);
    with_variant<T, VS>(I, [&]<int NDIM, int VW, int R>() {
        const Geo &g = I.geo;
        if constexpr (PH == PH_RREF_UBAR) {
            OpNormUbar<T, T, VW> op{{nullptr}, {ub}};
            point_tile<NDIM, VW, R, T, T>(g, lt, op, acc, lane);
        } else if constexpr (PH == PH_RREF_RES) {
            OpResNorm<T, T, VW> op{{ub}, {ub}};
            g_tile<VS, NDIM, VW, R, T, T>(I, lt, op, acc, lane);
        } else if constexpr (PH == PH_TRUE) {
            OpResNorm<T, double, VW> op{{u}, {ub}};
            g_tile<VS, NDIM, VW, R, T, double>(I, lt, op, acc, lane);
        } else if constexpr (PH == PH_INIT_UBAR) {
            OpInitUbar<T, T, VW> op{{ub}, {nullptr}, u, V[V_R0], V[V_F0]};
            g_tile<VS, NDIM, VW, R, T, T>(I, lt, op, acc, lane);
        } else if constexpr (PH == PH_INIT_ZERO) {
            OpInitZero<T, T, VW> op{{nullptr}, {ub}, u, V[V_R0], V[V_F0]};
            point_tile<NDIM, VW, R, T, T>(g, lt, op, acc, lane);
        } else if constexpr (PH == PH_INIT_GIVEN) {
            OpInitGiven<T, T, VW> op{{u}, {ub}, V[V_R0], V[V_F0]};
            g_tile<VS, NDIM, VW, R, T, T>(I, lt, op, acc, lane);
        } else if constexpr (PH == PH_VC) {
            OpVC<T, T, VW> op{{X(V_R0)}, {u}, Y(V_R0), u};
            g_tile<VS, NDIM, VW, R, T, T>(I, lt, op, acc, lane);
        } else if constexpr (PH == PH_CG1) {
            if (first) {
                OpCG1First<T, T, VW> op{{V[V_R0]}, {nullptr}, Y(V_P0)};
                g_tile<VS, NDIM, VW, R, T, T>(I, lt, op, acc, lane);
            } else {
                OpCG1<T, T, VW> op{{V[V_R0], X(V_P0)}, {nullptr}, Y(V_P0), beta};
                g_tile<VS, NDIM, VW, R, T, T>(I, lt, op, acc, lane);
            }
        } else if constexpr (PH == PH_CG2) {
            OpCG2<T, T, VW> op{{Y(V_P0)}, {u, V[V_R0]}, u, V[V_R0], alpha};
            g_tile<VS, NDIM, VW, R, T, T>(I, lt, op, acc, lane);
        } else if constexpr (PH == PH_BIA) {
            if (first) {
                OpBiAFirst<T, T, VW> op{{X(V_R0)}, {V[V_F0]}, Y(V_P0), Y(V_Q0)};
                g_tile<VS, NDIM, VW, R, T, T>(I, lt, op, acc, lane);
            } else {
                OpBiA<T, T, VW> op{{X(V_R0), X(V_P0), X(V_Q0)}, {V[V_F0]}, Y(V_P0), Y(V_Q0), beta, omega};
                g_tile<VS, NDIM, VW, R, T, T>(I, lt, op, acc, lane);
            }
        } else if constexpr (PH == PH_BIB) {
            OpBiB<T, T, VW> op{{X(V_R0), Y(V_Q0)}, {nullptr}, alpha};
            g_tile<VS, NDIM, VW, R, T, T>(I, lt, op, acc, lane);
        } else if constexpr (PH == PH_BIC) {
            OpBiC<T, T, VW> op{{X(V_R0), Y(V_Q0)}, {u, Y(V_P0), V[V_F0]}, u, Y(V_R0), alpha, omega};
            g_tile<VS, NDIM, VW, R, T, T>(I, lt, op, acc, lane);
        } else if constexpr (PH == PH_SD1) {
            OpSD1<T, T, VW> op{{X(V_R0)}, {nullptr}};
            g_tile<VS, NDIM, VW, R, T, T>(I, lt, op, acc, lane);
        } else if constexpr (PH == PH_SD2) {
            OpSD2<T, T, VW> op{{X(V_R0)}, {u}, Y(V_R0), u, alpha};
            g_tile<VS, NDIM, VW, R, T, T>(I, lt, op, acc, lane);
        } else if constexpr (PH == PH_VERIFY) {
            OpResNorm<T, double, VW> op{{u}, {ub}};
            g_tile<VS, NDIM, VW, R, T, double>(I, lt, op, acc, lane);
        } else if constexpr (PH == PH_REPLACE) {
            // `it` is the index of the pass that follows: the residual goes
            // where that pass reads it (CG updates r in place; the others
            // ping-pong it)
            T *rdst = P.solver == GD_CG ? V[V_R0] : X(V_R0);
            OpInitGiven<T, double, VW> op{{u}, {ub}, rdst, V[V_F0]};
            g_tile<VS, NDIM, VW, R, T, double>(I, lt, op, acc, lane);
        }
    });
}

// ------------------------------------------------ scalar recurrences (FP64)
// Counters of the control states (Sync::live), changed by the single lane
// that completes an instance's reduction.
__device__ __forceinline__ void count(int32_t *c, int d) {
    __hip_atomic_fetch_add(c, d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The instance stops; its exit true residual is still to be computed (PH_TRUE).
static __device__ __forceinline__ void finish(const Params &P, State *S, int status) {
    S->status = status;
    S->done = 1;
    count(&P.sync->live.active, -1);
    count(&P.sync->live.ntrue, 1);
}

// The instance stops with its true residual rt already known: its info
// record is written here and PH_TRUE skips it.
static __device__ __forceinline__ void finish_known(const Params &P, const Inst &I, State *S, int status, double rt) {
    S->status = status;
    S->done = 1;
    S->tknown = 1;
    count(&P.sync->live.active, -1);
    gd_info out;
    out.iters = S->iters;
    out.status = status;
    out.r_ref = S->r_ref;
    out.r0 = S->r0;
    out.r_final = sqrt(S->rr);
    out.r_true = rt;
    out.start = S->start;
    out.replaced = S->nrep;
    *I.info = out;
}

// Stopping test after `n` completed passes with residual norm rn.  When the
// recursive residual meets the tolerance after a pass, the instance goes to
// the true-residual check (PH_VERIFY) instead of stopping; the initial
// residual (n = 0) is computed directly and needs no check.
static __device__ __forceinline__ bool stop_check(const Params &P, State *S, double rn, int n) {
    if (!isfinite(rn)) { finish(P, S, GD_NONFINITE); return true; }
    if (rn == 0.0 || (P.tol > 0.0 && rn <= P.tol * S->r_ref)) {
        if (n > 0 && P.tol > 0.0) {
            S->verify = 1;
            count(&P.sync->live.verify, 1);
        } else {
            finish(P, S, GD_CONVERGED);
        }
        return true;
    }
    if (n >= P.max_iter) { finish(P, S, GD_MAXITER); return true; }
    return false;
}

static __device__ __forceinline__ void update_scalars(const Params &P, const Inst &I, State *S, int ph, const double (&sum)[NACC]) {
    const double hw = I.hw;
    switch (ph) {
    case PH_RREF_UBAR:
        S->r_ref = sqrt(hw * sum[0]);
        break;
    case PH_RREF_RES:
        // ||ubar - G ubar|| (the warm start's acceptance bound) and ||ubar||
        S->r_ub = sqrt(hw * sum[0]);
        S->r_ref = P.norm_ref == GD_REF_UBAR ? sqrt(hw * sum[1]) : S->r_ub;
        break;
    case PH_INIT_UBAR:
    case PH_INIT_ZERO:
    case PH_INIT_GIVEN: {
        const double rr = hw * sum[0];
        const double r0 = sqrt(rr);
        if (ph == PH_INIT_GIVEN && P.init == GD_INIT_WARM && (!isfinite(r0) || !(r0 < S->r_ub))) {
            // the guess is no better than the paper's start: restart from ubar
            S->fallback = 1;
            count(&P.sync->live.fallback, 1);
            break;
        }
        if (ph == PH_INIT_UBAR && S->fallback) {
            S->fallback = 0;
            count(&P.sync->live.fallback, -1);
        }
        if (ph == PH_INIT_UBAR && P.norm_ref == GD_REF_R0UBAR) S->r_ref = r0;
        S->start = ph == PH_INIT_UBAR ? GD_INIT_UBAR : (ph == PH_INIT_ZERO ? GD_INIT_ZERO : GD_INIT_GIVEN);
        S->r0 = r0;
        S->rr = rr;
        S->iters = 0;
        if (I.hist) I.hist[0] = r0;  // index 0 <= max_iter
        // Algorithm 3: rho_0 = (r0, r0).  Algorithm 4: alpha = omega = rho = 1
        // and rho_1 = (f0, r0) = (r0, r0) since f0 = r0.
        S->alpha = 1.0;
        S->omega = 1.0;
        S->beta = 0.0;
        S->rho = rr;
        if (!isfinite(S->r_ref)) finish(P, S, GD_NONFINITE);
        else if (S->r_ref == 0.0) finish(P, S, GD_ZERO_REF);
        else stop_check(P, S, r0, 0);
        break;
    }
    case PH_VC:
    case PH_SD2: {
        const double rr = hw * sum[0];
        S->iters += 1;
        S->rr = rr;
        S->restart = 0;
        if (I.hist && S->iters <= P.max_iter) I.hist[S->iters] = sqrt(rr);
        stop_check(P, S, sqrt(rr), S->iters);
        break;
    }
    case PH_SD1: {
        const double rd = hw * sum[0];
        if (!isfinite(rd)) finish(P, S, GD_NONFINITE);
        else if (rd == 0.0) finish(P, S, GD_BREAKDOWN_RHO);
        else S->alpha = S->rr / rd;
        break;
    }
    case PH_CG1: {
        const double pd = hw * sum[0];
        S->restart = 0;
        if (!isfinite(pd)) finish(P, S, GD_NONFINITE);
        else if (pd == 0.0) finish(P, S, GD_BREAKDOWN_RHO);
        else S->alpha = S->rho / pd;
        break;
    }
    case PH_CG2: {
        const double rho_new = hw * sum[0];
        S->iters += 1;
        S->rr = rho_new;
        if (I.hist && S->iters <= P.max_iter) I.hist[S->iters] = sqrt(rho_new);
        if (!stop_check(P, S, sqrt(rho_new), S->iters)) {
            S->beta = rho_new / S->rho;
            S->rho = rho_new;
        }
        break;
    }
    case PH_BIA: {
        const double fq = hw * sum[0];
        S->restart = 0;
        if (!isfinite(fq)) finish(P, S, GD_NONFINITE);
        else if (fq == 0.0) finish(P, S, GD_BREAKDOWN_RHO);
        else S->alpha = S->rho / fq;  // rho holds rho_{n+1} = (f0, r_n)
        break;
    }
    case PH_BIB: {
        const double st = hw * sum[0], tt = hw * sum[1], ss = hw * sum[2];
        if (!isfinite(st) || !isfinite(tt) || !isfinite(ss)) {
            finish(P, S, GD_NONFINITE);
            break;
        }
        const double thr = P.tol > 0.0 ? P.tol * S->r_ref : 0.0;
        const int half = (ss == 0.0) || (sqrt(ss) <= thr);
        if (!half && tt == 0.0) {
            finish(P, S, GD_BREAKDOWN_OMEGA);
            break;
        }
        S->half = half;
        S->omega = half ? 0.0 : st / tt;
        break;
    }
    case PH_BIC: {
        const double fr = hw * sum[0], rr = hw * sum[1];
        S->iters += 1;
        S->rr = rr;
        if (I.hist && S->iters <= P.max_iter) I.hist[S->iters] = sqrt(rr);
        if (S->half) {
            // s met the tolerance after the alpha half step: u += alpha p, r = s
            if (!isfinite(rr)) finish(P, S, GD_NONFINITE);
            else if (P.tol > 0.0) {
                S->verify = 1;
                count(&P.sync->live.verify, 1);
            } else {
                finish(P, S, GD_CONVERGED);
            }
            break;
        }
        if (stop_check(P, S, sqrt(rr), S->iters)) break;
        if (!isfinite(fr)) finish(P, S, GD_NONFINITE);
        else if (fr == 0.0) finish(P, S, GD_BREAKDOWN_RHO);
        else {
            S->beta = (S->alpha / S->omega) * (fr / S->rho);
            S->rho = fr;
        }
        break;
    }
    case PH_VERIFY: {
        // the true residual of the iterate whose recursive residual met tol
        const double rt = sqrt(hw * sum[0]);
        S->verify = 0;
        count(&P.sync->live.verify, -1);
        if (!isfinite(rt)) finish_known(P, I, S, GD_NONFINITE, rt);
        else if (rt <= P.tol * S->r_ref) finish_known(P, I, S, GD_CONVERGED, rt);
        else if (S->iters >= P.max_iter) finish_known(P, I, S, GD_MAXITER, rt);
        else if (S->nrep >= P.max_replace) finish_known(P, I, S, GD_STAGNATED, rt);
        else {
            S->replace = 1;
            count(&P.sync->live.replace, 1);
        }
        break;
    }
    case PH_REPLACE: {
        // r (and BiCGSTAB's shadow f0) now hold ubar - G u: the Krylov
        // sequence restarts from the current iterate, as from a given start
        const double rr = hw * sum[0];
        S->replace = 0;
        count(&P.sync->live.replace, -1);
        S->nrep += 1;
        S->restart = 1;
        S->half = 0;
        S->rr = rr;
        S->rho = rr;
        S->alpha = 1.0;
        S->omega = 1.0;
        S->beta = 0.0;
        break;
    }
    case PH_TRUE: {
        gd_info out;
        out.iters = S->iters;
        out.status = S->status;
        out.r_ref = S->r_ref;
        out.r0 = S->r0;
        out.r_final = sqrt(S->rr);
        out.r_true = sqrt(hw * sum[0]);
        out.start = S->start;
        out.replaced = S->nrep;
        *I.info = out;
        break;
    }
    default:
        break;
    }
}

// Sum instance i's per-tile partials in tile order and advance its scalars.
// Run by the whole wave that completed the instance's last tile.
template <bool TABLE>
static __device__ void complete_instance(const Params &P, const Inst &I, State *S, int ph, int lane,
                                         uint32_t epoch) {
    const int nacc = phase_nacc(ph);
    double sum[NACC] = {0.0, 0.0, 0.0};
    for (int64_t t = lane; t < I.ntiles; t += WAVE) {
#pragma unroll
        for (int k = 0; k < NACC; ++k)
            if (k < nacc) sum[k] += ld_f64(&P.part[(I.tile0 + t) * NACC + k]);
    }
#pragma unroll
    for (int k = 0; k < NACC; ++k) sum[k] = wave_sum(sum[k]);
    if (lane == 0) {
        update_scalars(P, I, S, ph, sum);
        __hip_atomic_store(&S->cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (P.trace && 4 * (int64_t)epoch + 3 < P.trace_cap)
            atomicMax(&P.trace[4 * epoch + 3], (unsigned long long)wall_clock64());
    }
}

// Whether sweep PH leaves instance S alone: the control sweeps work only on
// the instances flagged for them, PH_TRUE on those without a known true
// residual, the others on the instances still iterating.
template <int PH>
__device__ __forceinline__ bool skip_instance(const Params &P, const State *S) {
    if constexpr (PH == PH_TRUE) return ld_i32(&S->tknown) != 0;
    else if constexpr (PH == PH_VERIFY) return ld_i32(&S->verify) == 0;
    else if constexpr (PH == PH_REPLACE) return ld_i32(&S->replace) == 0;
    else if constexpr (PH == PH_INIT_UBAR) return P.init == GD_INIT_WARM ? ld_i32(&S->fallback) == 0 : ld_i32(&S->done) != 0;
    else return ld_i32(&S->done) != 0;
}

// One tile of a sweep: march it, publish its partials, count it done, and
// finish the instance's reduction if it was the instance's last tile.
template <typename T, int VS, int PH>
__device__ __forceinline__ void run_tile(const Params &P, int it, uint32_t epoch, int64_t t, int lane) {
    constexpr int nacc = PhaseNacc<PH>::v;
    // the tile, and with it the instance, the tile's planes and rows and the
    // plane addresses of the march, are the same in every lane
    t = wave_uniform(t);
    int64_t lt = 0;
    const int i = locate<var_table(VS)>(P, t, lt);
    State *S = &P.st[i];
    // instances the sweep does not work on skip their tiles (a wave-uniform decision)
    if (__builtin_amdgcn_readfirstlane(skip_instance<PH>(P, S) ? 1 : 0) != 0) return;
    const Inst I = get_inst<var_table(VS)>(P, i);
    double acc[NACC] = {0.0, 0.0, 0.0};
    tile_body<T, VS, PH>(P, I, S, it, lt, acc, lane);
    // publish this tile's partials, then count the tile done
#pragma unroll
    for (int k2 = 0; k2 < nacc; ++k2) {
        const double v = wave_sum(acc[k2]);
        // agent-coherent store (no L2 write-back of unrelated lines needed)
        if (lane == 0)
            __hip_atomic_store(&P.part[(I.tile0 + lt) * NACC + k2], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // wait until this wave's partial stores have completed, then count the
    // tile; the completing wave reads the partials with agent-coherent loads
    // after it has seen the full count
    wait_vm_stores();
    uint32_t prev = 0;
    if (lane == 0) prev = __hip_atomic_fetch_add(&S->cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    prev = (uint32_t)__builtin_amdgcn_readfirstlane(prev);
    if (prev == (uint32_t)I.ntiles - 1) complete_instance<var_table(VS)>(P, I, S, PH, lane, epoch);
}

// One sweep.  With P.steal > 0 the tiles come from the sweep's pools: a
// workgroup drains its own group's pool, then the others that still hold
// tiles.  Per-workgroup claims (P.wave_claims == 0): thread 0 claims WPB
// consecutive tiles with one atomic and hands them out through LDS, so the
// decision to move on is the same for the whole workgroup; per-wave claims:
// every wave claims its own.  With P.steal == 0, wave w takes tiles w, w + W,
// ... (W waves).  A tile's result does not depend on which wave runs it.
// Every mode feeds one call site of run_tile, so the tile body is inlined
// once (16 x 2048^2 BiCGSTAB at fixed launch shapes: 4.51 ms, against 4.74 ms
// with a loop and a call site per mode; in 3D and in uneven batches the body
// is larger still).
template <typename T, int VS, int PH>
__device__ __forceinline__ void run_phase(const Params &P, int it, uint32_t epoch) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t ntot = P.total_tiles;
    __shared__ int64_t s_base;
    __shared__ uint32_t s_left[NGRP];
    const uint32_t nb = gridDim.x;
    const uint32_t ng = nb < (uint32_t)NGRP ? nb : (uint32_t)NGRP;
    const uint32_t grp = blockIdx.x % NGRP;
    // Pool pl owns a contiguous share of the long tiles and a contiguous share
    // of the short ones and hands out its long tiles first: neighbouring tiles
    // (which share halo planes and rows) stay on one XCD and its L2, and the
    // end of a sweep is made of short tiles.  Interleaved layout: pool pl
    // hands out tiles pl, pl + ng, ... instead (spreads each field over every
    // XCD, at the cost of halo reuse in L2).
    const int64_t nbig = P.big_total, nsmall = ntot - P.big_total;
    const bool ilv = P.interleave != 0;
    const bool dyn = P.steal > 0;
    const bool wc = P.wave_claims != 0;
    const uint32_t hmax = dyn ? ((uint32_t)P.steal < ng ? (uint32_t)P.steal : ng) : 0;
    int64_t next = (int64_t)blockIdx.x * WPB + wave;  // static mode
    const int64_t stride = (int64_t)gridDim.x * WPB;
    uint32_t h = 0, pl = 0;  // pool being drained: the h-th visited
    bool open = false;
    int64_t blo = 0, bcnt = 0, slo = 0, cnt = 0;
    for (;;) {
        int64_t t;
        if (!dyn) {
            if (next >= ntot) break;
            t = next;
            next += stride;
        } else {
            if (!open) {
                if (h >= hmax) break;
                pl = (grp + h) % ng;
                if (h == 1) {
                    // Own pool empty: read every pool's counter at once (one
                    // round trip) and steal only from pools that still had
                    // tiles.  Counters only grow, so a pool seen empty stays
                    // empty and is skipped.
                    __syncthreads();
                    if (threadIdx.x < ng) {
                        const uint32_t q = threadIdx.x;
                        const uint32_t c = __hip_atomic_load(&P.sync->pool[epoch & 1][q].v, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                        s_left[q] = (int64_t)c < P.sync->pcnt[q] ? 1u : 0u;
                    }
                    __syncthreads();
                }
                if (h > 0 && s_left[pl] == 0) {  // the flags do not change: the same choice in every wave
                    ++h;
                    continue;
                }
                blo = nbig * pl / ng;
                bcnt = nbig * (pl + 1) / ng - blo;
                slo = nbig + nsmall * pl / ng;
                cnt = ilv ? (ntot - (int64_t)pl + ng - 1) / ng : bcnt + (nsmall * (pl + 1) / ng - nsmall * pl / ng);
                open = true;
            }
            uint32_t *ctr = &P.sync->pool[epoch & 1][pl].v;
            int64_t k;
            if (wc) {
                // All lanes take part in the atomic (lane 0 adds 1, the
                // others 0) and lane 0's result is the claim, so the claim
                // has no lane-dependent branch: one taken under
                // `if (lane == 0)` and broadcast was turned by the compiler
                // into a loop that re-read an old claim.
                const uint32_t r = __hip_atomic_fetch_add(ctr, lane == 0 ? 1u : 0u, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                k = (int64_t)__builtin_amdgcn_readfirstlane(r);
                if (k >= cnt) {  // same value in every lane
                    open = false;
                    ++h;
                    continue;
                }
            } else {
                __syncthreads();  // every wave has read the previous round's s_base
                if (threadIdx.x == 0)
                    s_base = (int64_t)__hip_atomic_fetch_add(ctr, (uint32_t)WPB, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                __syncthreads();
                const int64_t base = (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)s_base);
                if (base >= cnt) {  // same decision in every wave of the workgroup
                    open = false;
                    ++h;
                    continue;
                }
                k = base + wave;
                if (k >= cnt) continue;  // no tile for this wave in this round
            }
            t = ilv ? (int64_t)pl + k * ng : (k < bcnt ? blo + k : slo + (k - bcnt));
        }
        run_tile<T, VS, PH>(P, it, epoch, t, lane);
    }
}

template <bool TABLE>
static __device__ __forceinline__ void mark_timeout(const Params &P) {
    __hip_atomic_store(&P.sync->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int i = 0; i < P.ninst; ++i) {
        const Inst I = get_inst<TABLE>(P, i);
        I.info->status = GD_TIMEOUT;
        I.info->iters = P.st[i].iters;
    }
}

// Grid barrier between sweeps.  Returns false when the run was aborted (a
// wait exceeded its bound).
//
// Arrival is two-level: a workgroup counts itself in its group; the last of a
// group counts the group at the top; the last group's last workgroup writes
// the next generation into every group's release flag, and each workgroup
// polls only its own group's flag.
//
// Memory ordering across the 8 XCDs (each with its own L2): thread 0 of every
// workgroup issues one agent-scope release fence (L2 write-back) before it
// arrives, waits with relaxed loads (no cache maintenance while others are
// still streaming), and issues one agent-scope acquire fence after the wait.
// The workgroup's other waves share the CU's caches and are ordered behind
// thread 0 by the workgroup barrier.
// The counters of the control states after a barrier (the snapshot every
// workgroup reads, so that all take the same path).
struct Snap {
    int active, verify, replace, fallback, ntrue;
};

template <bool TABLE>
static __device__ __forceinline__ int grid_sync(const Params &P, uint32_t &epoch, Snap &sn) {
    __shared__ int s_last, s_abort;
    __shared__ Snap s_snap;
    __syncthreads();
    const uint32_t nb = gridDim.x;
    const uint32_t ng = nb < (uint32_t)NGRP ? nb : (uint32_t)NGRP;
    const uint32_t grp = blockIdx.x % NGRP;
    Sync *sy = P.sync;
    if (threadIdx.x == 0) {
        const bool tr = P.trace && 4 * (int64_t)epoch + 3 < P.trace_cap;
        if (tr) {
            const unsigned long long now = wall_clock64();
            atomicMin(&P.trace[4 * epoch + 0], now);
            atomicMax(&P.trace[4 * epoch + 1], now);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t gsize = (nb - grp + NGRP - 1) / NGRP;
        const uint32_t c = __hip_atomic_fetch_add(&sy->cnt[grp].v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int last = 0;
        if (c == gsize - 1) {
            __hip_atomic_store(&sy->cnt[grp].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            const uint32_t t = __hip_atomic_fetch_add(&sy->top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (t == ng - 1) {
                __hip_atomic_store(&sy->top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                last = 1;
            }
        }
        int ab = 0;
        if (!last) {
            const int64_t t0 = wall_clock64();
            int nap = 1;
            while (__hip_atomic_load(&sy->gen[grp].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) {
                if (__hip_atomic_load(&sy->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ab = 1;
                    break;
                }
                if (wall_clock64() - t0 > P.wait_ticks) {
                    mark_timeout<TABLE>(P);
                    ab = 1;
                    break;
                }
                // back off up to ~0.5 us between polls
                if (nap < 16) {
                    __builtin_amdgcn_s_sleep(1);
                    ++nap;
                } else {
                    __builtin_amdgcn_s_sleep(8);
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        // let the cache invalidation complete before the other waves of the
        // workgroup, released by the barrier below, issue their loads
        wait_vm_stores();
        s_last = last;
        s_abort = ab;
        if (!last && !ab) {
            const Counts *c = &sy->snap[epoch & 1];
            s_snap.active = __hip_atomic_load(&c->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_snap.verify = __hip_atomic_load(&c->verify, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_snap.replace = __hip_atomic_load(&c->replace, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_snap.fallback = __hip_atomic_load(&c->fallback, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_snap.ntrue = __hip_atomic_load(&c->ntrue, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    if (s_abort) return -1;
    if (s_last && threadIdx.x < WAVE) {
        // every workgroup has arrived: every tile of the sweep and every
        // instance reduction is done, so the counters are final for this barrier
        if (threadIdx.x == 0) {
            Counts *c = &sy->snap[epoch & 1];
            auto take = [&](int32_t *live, int32_t *snap) {
                const int v = __hip_atomic_load(live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(snap, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return v;
            };
            s_snap.active = take(&sy->live.active, &c->active);
            s_snap.verify = take(&sy->live.verify, &c->verify);
            s_snap.replace = take(&sy->live.replace, &c->replace);
            s_snap.fallback = take(&sy->live.fallback, &c->fallback);
            s_snap.ntrue = take(&sy->live.ntrue, &c->ntrue);
            if (P.trace && 4 * (int64_t)epoch + 3 < P.trace_cap) P.trace[4 * epoch + 2] = wall_clock64();
        }
        // the sweep just finished is done with its pool set; the sweep after
        // next uses it again
        for (uint32_t k = threadIdx.x; k < (uint32_t)NGRP; k += WAVE)
            __hip_atomic_store(&sy->pool[epoch & 1][k].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        for (uint32_t k = threadIdx.x; k < ng; k += WAVE)
            __hip_atomic_store(&sy->gen[k].v, epoch + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();  // s_snap is set; no wave of this workgroup runs ahead
    // uniform values (scalar registers), read in every later loop decision
    sn.active = __builtin_amdgcn_readfirstlane(s_snap.active);
    sn.verify = __builtin_amdgcn_readfirstlane(s_snap.verify);
    sn.replace = __builtin_amdgcn_readfirstlane(s_snap.replace);
    sn.fallback = __builtin_amdgcn_readfirstlane(s_snap.fallback);
    sn.ntrue = __builtin_amdgcn_readfirstlane(s_snap.ntrue);
    ++epoch;
    return sn.active;
}

// Waves per SIMD the kernels of a variant must reach: two for FP32, whose
// kernels fit the 256 registers of two waves without spilling (the two-row
// 3D BiCGSTAB kernel only just); FP64 keeps the count its registers give (its
// two-row and four-row 3D kernels would spill).  The FP32 four-row 3D
// BiCGSTAB kernel (344) is the exception: with two planes of loads in
// flight it needs a few registers more than two waves allow, and its tuned
// launch on 3 x 256^3 runs one wave per SIMD anyway (two tiles per column,
// one workgroup per CU: 5.12 -> 5.09 ms without the two spilled registers).
template <typename T, int SOLVER, int VS>
constexpr int kMinWavesPerEU = (sizeof(T) == 4 && !(SOLVER == GD_BICGSTAB && VS == 344)) ? 2 : 1;

template <typename T, int SOLVER, int VS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kMinWavesPerEU<T, SOLVER, VS>))) void solve_kernel(
    Params P) {
    constexpr bool TB = var_table(VS);
    uint32_t epoch = 0;
    Snap sn;
    // reference norm when it is not the initial residual itself (a warm start
    // also needs ||ubar - G ubar||, its acceptance bound)
    if (P.norm_ref == GD_REF_UBAR && P.init != GD_INIT_WARM) {
        run_phase<T, VS, PH_RREF_UBAR>(P, 0, epoch);
        if (grid_sync<TB>(P, epoch, sn) < 0) return;
    } else if (P.init != GD_INIT_UBAR) {
        run_phase<T, VS, PH_RREF_RES>(P, 0, epoch);
        if (grid_sync<TB>(P, epoch, sn) < 0) return;
    }
    // initial guess and residual
    if (P.init == GD_INIT_UBAR) run_phase<T, VS, PH_INIT_UBAR>(P, 0, epoch);
    else if (P.init == GD_INIT_ZERO) run_phase<T, VS, PH_INIT_ZERO>(P, 0, epoch);
    else run_phase<T, VS, PH_INIT_GIVEN>(P, 0, epoch);
    int act = grid_sync<TB>(P, epoch, sn);
    if (act < 0) return;
    // warm starts no better than ubar restart from ubar
    if (sn.fallback > 0) {
        run_phase<T, VS, PH_INIT_UBAR>(P, 0, epoch);
        if ((act = grid_sync<TB>(P, epoch, sn)) < 0) return;
    }
    // every workgroup sees the same snapshot after each barrier, so all take
    // the same path through the loops
    int it = 0;
    for (;;) {
        while (it < P.max_iter && act > 0) {
            if constexpr (SOLVER == GD_VANCITTERT) {
                run_phase<T, VS, PH_VC>(P, it, epoch);
                if ((act = grid_sync<TB>(P, epoch, sn)) < 0) return;
            } else if constexpr (SOLVER == GD_CG) {
                run_phase<T, VS, PH_CG1>(P, it, epoch);
                if (grid_sync<TB>(P, epoch, sn) < 0) return;
                run_phase<T, VS, PH_CG2>(P, it, epoch);
                if ((act = grid_sync<TB>(P, epoch, sn)) < 0) return;
            } else if constexpr (SOLVER == GD_BICGSTAB) {
                run_phase<T, VS, PH_BIA>(P, it, epoch);
                if (grid_sync<TB>(P, epoch, sn) < 0) return;
                run_phase<T, VS, PH_BIB>(P, it, epoch);
                if (grid_sync<TB>(P, epoch, sn) < 0) return;
                run_phase<T, VS, PH_BIC>(P, it, epoch);
                if ((act = grid_sync<TB>(P, epoch, sn)) < 0) return;
            } else {
                run_phase<T, VS, PH_SD1>(P, it, epoch);
                if (grid_sync<TB>(P, epoch, sn) < 0) return;
                run_phase<T, VS, PH_SD2>(P, it, epoch);
                if ((act = grid_sync<TB>(P, epoch, sn)) < 0) return;
            }
            ++it;
            if (sn.verify > 0) break;
        }
        if (sn.verify == 0) break;
        // instances whose recursive residual met tol: their true residual
        // decides; where it is above tol, the residual is replaced by it
        run_phase<T, VS, PH_VERIFY>(P, it, epoch);
        if ((act = grid_sync<TB>(P, epoch, sn)) < 0) return;
        if (sn.replace > 0) {
            run_phase<T, VS, PH_REPLACE>(P, it, epoch);
            if ((act = grid_sync<TB>(P, epoch, sn)) < 0) return;
        }
    }
    // exit true residual of the instances that stopped otherwise
    if (sn.ntrue > 0) {
        run_phase<T, VS, PH_TRUE>(P, 0, epoch);
        grid_sync<TB>(P, epoch, sn);
    }
}

// filter_apply: one wave per tile, no reduction.
template <typename T, int VS>
__global__ __launch_bounds__(BLOCK) void filter_kernel(Inst tmpl, int64_t stride_elems, int64_t tiles_per_inst,
                                                       int64_t total_tiles) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t t = (int64_t)blockIdx.x * WPB + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (t >= total_tiles) return;
    const int64_t b = t / tiles_per_inst;
    const T *x = static_cast<const T *>(tmpl.ubar) + b * stride_elems;
    T *y = static_cast<T *>(tmpl.u) + b * stride_elems;
    double acc[NACC] = {0.0, 0.0, 0.0};
    with_variant<T, VS>(tmpl, [&]<int NDIM, int VW, int R>() {
        OpFilter<T, T, VW> op{{x}, {nullptr}, y};
        march_tile<NDIM, VW, R, T, T>(tmpl.geo, t - b * tiles_per_inst, op, acc, lane);
    });
}

}  // namespace gd
