// gd_kernels.h -- the persistent solver kernel and the filter kernel.
//
// One launch runs a whole solve for a batch of fields ("instances").  The grid
// holds at most as many workgroups as can be resident at once, every wave
// loops over tiles, and the sweeps of Algorithms 1-4 are separated by a grid
// barrier.  The last workgroup to reach a barrier sums the per-tile FP64
// partial inner products of every instance in a fixed order (so results are
// bitwise reproducible and independent of which wave ran which tile),
// updates that instance's scalars (alpha, beta, omega, rho, convergence test,
// guards, residual history) and releases the others.  The iteration loop,
// including the stopping test, therefore never returns to the host.
#pragma once
#include <hip/hip_runtime.h>

#include "gd_device.h"
#include "gd_ops.h"
#include "gd_internal.h"
#include "gdecon.h"

namespace gd {

// ------------------------------------------------------------ device state
__device__ __forceinline__ int ld_i32(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_f64(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

static __device__ __forceinline__ Inst get_inst(const Params &P, int i) {
    if (P.table) return P.table[i];
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

static __device__ __forceinline__ int inst_of(const Params &P, int64_t t) {
    if (!P.table) return (int)(t / P.tiles_per_inst);
    int lo = 0, hi = P.ninst - 1;
    while (lo < hi) {  // last instance with tile0 <= t
        const int mid = (lo + hi + 1) >> 1;
        if (P.table[mid].tile0 <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
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
            if (I.R == 2) f.template operator()<3, VM, 2>();
            else f.template operator()<3, VM, 1>();
        } else {
            f.template operator()<3, 1, 1>();
        }
    }
}

template <int PH> struct PhaseNacc { static constexpr int v = 1; };
template <> struct PhaseNacc<PH_BIB> { static constexpr int v = 3; };
template <> struct PhaseNacc<PH_BIC> { static constexpr int v = 2; };

__host__ __device__ constexpr inline int phase_nacc(int ph) { return ph == PH_BIB ? 3 : (ph == PH_BIC ? 2 : 1); }

// One tile of one sweep.
template <typename T, int VS, int PH>
__device__ __forceinline__ void tile_body(const Inst &I, const State *S, int it, int64_t lt, double (&acc)[NACC],
                                          int lane) {
    const T alpha = T(ld_f64(&S->alpha));
    const T beta = T(ld_f64(&S->beta));
    const T omega = T(ld_f64(&S->omega));
    const bool odd = (it & 1) != 0;
    T *const *V = reinterpret_cast<T *const *>(I.vec);
    // ping-pong buffers: X(base) is the current one, Y(base) the next one
    auto X = [&](int base) -> T * { return odd ? V[base + 1] : V[base]; };
    auto Y = [&](int base) -> T * { return odd ? V[base] : V[base + 1]; };
    const T *ub = static_cast<const T *>(I.ubar);
    T *u = static_cast<T *>(I.u);
    with_variant<T, VS>(I, [&]<int NDIM, int VW, int R>() {
        if constexpr (PH == PH_RREF_UBAR) {
            OpNormUbar<T, T, VW> op{ub};
            point_tile<NDIM, VW, R, T>(I.geo, lt, op, acc, lane);
        } else if constexpr (PH == PH_RREF_RES) {
            OpResNorm<T, T, VW> op{ub, ub};
            march_tile<NDIM, VW, R, T>(I.geo, lt, op, acc, lane);
        } else if constexpr (PH == PH_TRUE) {
            OpResNorm<T, double, VW> op{u, ub};
            march_tile<NDIM, VW, R, double>(I.geo, lt, op, acc, lane);
        } else if constexpr (PH == PH_INIT_UBAR) {
            OpInitUbar<T, T, VW> op{ub, u, V[V_R0], V[V_F0]};
            march_tile<NDIM, VW, R, T>(I.geo, lt, op, acc, lane);
        } else if constexpr (PH == PH_INIT_ZERO) {
            OpInitZero<T, T, VW> op{ub, u, V[V_R0], V[V_F0]};
            point_tile<NDIM, VW, R, T>(I.geo, lt, op, acc, lane);
        } else if constexpr (PH == PH_INIT_GIVEN) {
            OpInitGiven<T, T, VW> op{u, ub, V[V_R0], V[V_F0]};
            march_tile<NDIM, VW, R, T>(I.geo, lt, op, acc, lane);
        } else if constexpr (PH == PH_VC) {
            OpVC<T, T, VW> op{X(V_R0), Y(V_R0), u};
            march_tile<NDIM, VW, R, T>(I.geo, lt, op, acc, lane);
        } else if constexpr (PH == PH_CG1) {
            OpCG1<T, T, VW> op{V[V_R0], X(V_P0), Y(V_P0), beta, it == 0};
            march_tile<NDIM, VW, R, T>(I.geo, lt, op, acc, lane);
        } else if constexpr (PH == PH_CG2) {
            OpCG2<T, T, VW> op{Y(V_P0), V[V_R0], u, alpha};
            march_tile<NDIM, VW, R, T>(I.geo, lt, op, acc, lane);
        } else if constexpr (PH == PH_BIA) {
            OpBiA<T, T, VW> op{X(V_R0), X(V_P0), X(V_Q0), V[V_F0],
                               Y(V_P0), Y(V_Q0), beta, omega, it == 0};
            march_tile<NDIM, VW, R, T>(I.geo, lt, op, acc, lane);
        } else if constexpr (PH == PH_BIB) {
            OpBiB<T, T, VW> op{X(V_R0), Y(V_Q0), alpha};
            march_tile<NDIM, VW, R, T>(I.geo, lt, op, acc, lane);
        } else if constexpr (PH == PH_BIC) {
            OpBiC<T, T, VW> op{X(V_R0), Y(V_Q0), Y(V_P0), V[V_F0], u, Y(V_R0), alpha, omega};
            march_tile<NDIM, VW, R, T>(I.geo, lt, op, acc, lane);
        } else if constexpr (PH == PH_SD1) {
            OpSD1<T, T, VW> op{X(V_R0)};
            march_tile<NDIM, VW, R, T>(I.geo, lt, op, acc, lane);
        } else if constexpr (PH == PH_SD2) {
            OpSD2<T, T, VW> op{X(V_R0), Y(V_R0), u, alpha};
            march_tile<NDIM, VW, R, T>(I.geo, lt, op, acc, lane);
        }
    });
}

template <typename T, int VS, int PH>
__device__ void run_phase(const Params &P, int it) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t wave_gid = (int64_t)blockIdx.x * WPB + (threadIdx.x >> 6);
    const int64_t nwaves = (int64_t)gridDim.x * WPB;
    constexpr int nacc = PhaseNacc<PH>::v;
    for (int64_t t = wave_gid; t < P.total_tiles; t += nwaves) {
        const int i = inst_of(P, t);
        const State *S = &P.st[i];
        if (PH != PH_TRUE && ld_i32(&S->done)) continue;
        const Inst I = get_inst(P, i);
        double acc[NACC] = {0.0, 0.0, 0.0};
        tile_body<T, VS, PH>(I, S, it, t - I.tile0, acc, lane);
#pragma unroll
        for (int k = 0; k < nacc; ++k) {
            const double v = wave_sum(acc[k]);
            if (lane == 0) P.part[t * NACC + k] = v;
        }
    }
}

// ------------------------------------------------ scalar recurrences (FP64)
static __device__ __forceinline__ void finish(State *S, int status) {
    S->status = status;
    S->done = 1;
}

// Stopping test after `n` completed passes with residual norm rn.
static __device__ __forceinline__ bool stop_check(const Params &P, State *S, double rn, int n) {
    if (!isfinite(rn)) { finish(S, GD_NONFINITE); return true; }
    if (rn == 0.0 || (P.tol > 0.0 && rn <= P.tol * S->r_ref)) { finish(S, GD_CONVERGED); return true; }
    if (n >= P.max_iter) { finish(S, GD_MAXITER); return true; }
    return false;
}

static __device__ __forceinline__ void update_scalars(const Params &P, const Inst &I, State *S, int ph, int solver, const double (&sum)[NACC]) {
    const double hw = I.hw;
    switch (ph) {
    case PH_RREF_UBAR:
    case PH_RREF_RES:
        S->r_ref = sqrt(hw * sum[0]);
        break;
    case PH_INIT_UBAR:
    case PH_INIT_ZERO:
    case PH_INIT_GIVEN: {
        const double rr = hw * sum[0];
        const double r0 = sqrt(rr);
        if (ph == PH_INIT_UBAR && P.norm_ref == GD_REF_R0UBAR) S->r_ref = r0;
        S->r0 = r0;
        S->rr = rr;
        S->iters = 0;
        if (I.hist) I.hist[0] = r0;
        // Algorithm 3: rho_0 = (r0, r0).  Algorithm 4: alpha = omega = rho = 1
        // and rho_1 = (f0, r0) = (r0, r0) since f0 = r0.
        S->alpha = 1.0;
        S->omega = 1.0;
        S->beta = 0.0;
        S->rho = rr;
        if (!isfinite(S->r_ref)) finish(S, GD_NONFINITE);
        else if (S->r_ref == 0.0) finish(S, GD_ZERO_REF);
        else stop_check(P, S, r0, 0);
        break;
    }
    case PH_VC:
    case PH_SD2: {
        const double rr = hw * sum[0];
        S->iters += 1;
        S->rr = rr;
        if (I.hist) I.hist[S->iters] = sqrt(rr);
        stop_check(P, S, sqrt(rr), S->iters);
        break;
    }
    case PH_SD1: {
        const double rd = hw * sum[0];
        if (!isfinite(rd)) finish(S, GD_NONFINITE);
        else if (rd == 0.0) finish(S, GD_BREAKDOWN_RHO);
        else S->alpha = S->rr / rd;
        break;
    }
    case PH_CG1: {
        const double pd = hw * sum[0];
        if (!isfinite(pd)) finish(S, GD_NONFINITE);
        else if (pd == 0.0) finish(S, GD_BREAKDOWN_RHO);
        else S->alpha = S->rho / pd;
        break;
    }
    case PH_CG2: {
        const double rho_new = hw * sum[0];
        S->iters += 1;
        S->rr = rho_new;
        if (I.hist) I.hist[S->iters] = sqrt(rho_new);
        if (!stop_check(P, S, sqrt(rho_new), S->iters)) {
            S->beta = rho_new / S->rho;
            S->rho = rho_new;
        }
        break;
    }
    case PH_BIA: {
        const double fq = hw * sum[0];
        if (!isfinite(fq)) finish(S, GD_NONFINITE);
        else if (fq == 0.0) finish(S, GD_BREAKDOWN_RHO);
        else S->alpha = S->rho / fq;  // rho holds rho_{n+1} = (f0, r_n)
        break;
    }
    case PH_BIB: {
        const double st = hw * sum[0], tt = hw * sum[1], ss = hw * sum[2];
        if (!isfinite(st) || !isfinite(tt) || !isfinite(ss)) {
            finish(S, GD_NONFINITE);
            break;
        }
        const double thr = P.tol > 0.0 ? P.tol * S->r_ref : 0.0;
        const int half = (ss == 0.0) || (sqrt(ss) <= thr);
        if (!half && tt == 0.0) {
            finish(S, GD_BREAKDOWN_OMEGA);
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
        if (I.hist) I.hist[S->iters] = sqrt(rr);
        if (S->half) {
            finish(S, isfinite(rr) ? GD_CONVERGED : GD_NONFINITE);
            break;
        }
        if (stop_check(P, S, sqrt(rr), S->iters)) break;
        if (!isfinite(fr)) finish(S, GD_NONFINITE);
        else if (fr == 0.0) finish(S, GD_BREAKDOWN_RHO);
        else {
            S->beta = (S->alpha / S->omega) * (fr / S->rho);
            S->rho = fr;
        }
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
        *I.info = out;
        break;
    }
    default:
        break;
    }
    (void)solver;
}

// Executed by the whole last-arriving workgroup.
static __device__ void reduce_update(const Params &P, int ph, int solver) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (WAVE - 1);
    __shared__ int s_act[WPB];
    const int nacc = phase_nacc(ph);
    int act = 0;
    for (int i = wave; i < P.ninst; i += WPB) {
        State *S = &P.st[i];
        if (ph != PH_TRUE && ld_i32(&S->done)) continue;
        const Inst I = get_inst(P, i);
        double sum[NACC] = {0.0, 0.0, 0.0};
        for (int64_t t = lane; t < I.ntiles; t += WAVE) {
#pragma unroll
            for (int k = 0; k < NACC; ++k)
                if (k < nacc) sum[k] += ld_f64(&P.part[(I.tile0 + t) * NACC + k]);
        }
#pragma unroll
        for (int k = 0; k < NACC; ++k) sum[k] = wave_sum(sum[k]);
        if (lane == 0) {
            update_scalars(P, I, S, ph, solver, sum);
            if (ph != PH_TRUE && !S->done) ++act;
        }
    }
    if (lane == 0) s_act[wave] = act;
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0;
        for (int w = 0; w < WPB; ++w) a += s_act[w];
        __hip_atomic_store(&P.sync->active, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

static __device__ void mark_timeout(const Params &P) {
    __hip_atomic_store(&P.sync->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int i = 0; i < P.ninst; ++i) {
        const Inst I = get_inst(P, i);
        I.info->status = GD_TIMEOUT;
        I.info->iters = P.st[i].iters;
    }
}

// Grid barrier that also finishes the sweep's reductions.  Returns false when
// the run was aborted (a wait exceeded its bound).
static __device__ bool grid_sync(const Params &P, uint32_t &epoch, int ph, int solver) {
    __shared__ int s_last, s_abort;
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t prev = __hip_atomic_fetch_add(&P.sync->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        const int last = prev == gridDim.x - 1;
        int ab = 0;
        if (!last) {
            const int64_t t0 = wall_clock64();
            while (__hip_atomic_load(&P.sync->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == epoch) {
                if (__hip_atomic_load(&P.sync->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    ab = 1;
                    break;
                }
                if (wall_clock64() - t0 > P.wait_ticks) {
                    mark_timeout(P);
                    ab = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        s_last = last;
        s_abort = ab;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (s_abort) return false;
    if (s_last) {
        reduce_update(P, ph, solver);
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_store(&P.sync->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&P.sync->gen, epoch + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    ++epoch;
    return true;
}

__device__ __forceinline__ int active_count(const Params &P) {
    return __hip_atomic_load(&P.sync->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T, int SOLVER, int VS>
__global__ __launch_bounds__(BLOCK) void solve_kernel(Params P) {
    uint32_t epoch = 0;
    // reference norm when it is not the initial residual itself
    if (P.norm_ref == GD_REF_UBAR) {
        run_phase<T, VS, PH_RREF_UBAR>(P, 0);
        if (!grid_sync(P, epoch, PH_RREF_UBAR, SOLVER)) return;
    } else if (P.init != GD_INIT_UBAR) {
        run_phase<T, VS, PH_RREF_RES>(P, 0);
        if (!grid_sync(P, epoch, PH_RREF_RES, SOLVER)) return;
    }
    // initial guess and residual
    if (P.init == GD_INIT_UBAR) {
        run_phase<T, VS, PH_INIT_UBAR>(P, 0);
        if (!grid_sync(P, epoch, PH_INIT_UBAR, SOLVER)) return;
    } else if (P.init == GD_INIT_ZERO) {
        run_phase<T, VS, PH_INIT_ZERO>(P, 0);
        if (!grid_sync(P, epoch, PH_INIT_ZERO, SOLVER)) return;
    } else {
        run_phase<T, VS, PH_INIT_GIVEN>(P, 0);
        if (!grid_sync(P, epoch, PH_INIT_GIVEN, SOLVER)) return;
    }
    for (int it = 0; it < P.max_iter && active_count(P) > 0; ++it) {
        if constexpr (SOLVER == GD_VANCITTERT) {
            run_phase<T, VS, PH_VC>(P, it);
            if (!grid_sync(P, epoch, PH_VC, SOLVER)) return;
        } else if constexpr (SOLVER == GD_CG) {
            run_phase<T, VS, PH_CG1>(P, it);
            if (!grid_sync(P, epoch, PH_CG1, SOLVER)) return;
            run_phase<T, VS, PH_CG2>(P, it);
            if (!grid_sync(P, epoch, PH_CG2, SOLVER)) return;
        } else if constexpr (SOLVER == GD_BICGSTAB) {
            run_phase<T, VS, PH_BIA>(P, it);
            if (!grid_sync(P, epoch, PH_BIA, SOLVER)) return;
            run_phase<T, VS, PH_BIB>(P, it);
            if (!grid_sync(P, epoch, PH_BIB, SOLVER)) return;
            run_phase<T, VS, PH_BIC>(P, it);
            if (!grid_sync(P, epoch, PH_BIC, SOLVER)) return;
        } else {
            run_phase<T, VS, PH_SD1>(P, it);
            if (!grid_sync(P, epoch, PH_SD1, SOLVER)) return;
            run_phase<T, VS, PH_SD2>(P, it);
            if (!grid_sync(P, epoch, PH_SD2, SOLVER)) return;
        }
    }
    run_phase<T, VS, PH_TRUE>(P, 0);
    grid_sync(P, epoch, PH_TRUE, SOLVER);
}

// filter_apply: one wave per tile, no reduction.
template <typename T, int VS>
__global__ __launch_bounds__(BLOCK) void filter_kernel(Inst tmpl, int64_t stride_elems, int64_t tiles_per_inst,
                                                       int64_t total_tiles) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t t = (int64_t)blockIdx.x * WPB + (threadIdx.x >> 6);
    if (t >= total_tiles) return;
    const int64_t b = t / tiles_per_inst;
    const T *x = static_cast<const T *>(tmpl.ubar) + b * stride_elems;
    T *y = static_cast<T *>(tmpl.u) + b * stride_elems;
    double acc[NACC] = {0.0, 0.0, 0.0};
    with_variant<T, VS>(tmpl, [&]<int NDIM, int VW, int R>() {
        OpFilter<T, T, VW> op{x, y};
        march_tile<NDIM, VW, R, T>(tmpl.geo, t - b * tiles_per_inst, op, acc, lane);
    });
}


}  // namespace gd
