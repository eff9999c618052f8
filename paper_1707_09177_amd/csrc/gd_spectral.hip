// gd_spectral.hip -- the paper's differential filter and the solve with it.
//
// The results section filters with G = (I - delta^2 lap)^-1, applied through
// the FFT, whose transfer function is G_hat(k) = 1 / (1 + (|k| / k_c)^2),
// delta = 1 / k_c, k_c = gamma k_m (Sec. 4, Eqs. df and df2; k_m, the highest
// wavenumber the grid resolves, is taken as min_d n_d / 2, the domain is
// 2 pi periodic so wavenumbers are integers).
//
// G is diagonal in Fourier space, and Algorithms 1-4 use G only through
// products G x, linear combinations and inner products.  So the solve runs on
// Fourier coefficients: one forward FFT of ubar (and of a given u0), every
// pass of the persistent solve kernel with G x = G_hat(k) x(k) evaluated
// pointwise, and one inverse FFT of u.  Inner products carry over through
// Parseval's identity: the half spectrum of a real field is stored scaled by
// c(k) = sqrt(w(k_x) / N) (w = 1 on the k_x = 0 and k_x = n_x / 2 columns,
// 2 elsewhere, N the point count), so the plain dot product of two stored
// spectra, real and imaginary parts taken as separate reals, equals
// sum_x a(x) b(x).  The persistent solve kernel therefore runs unchanged, on
// a real array of 2 (n_x / 2 + 1) columns per row (padded to a whole number
// of 16-byte lanes; the padding stays zero).
//
// FFTs: power-of-two lengths.  Rows (x) use the half-length complex
// transform of the even/odd-packed real row plus the standard split; y and z
// transform strided columns, a workgroup taking a few adjacent columns so
// that its loads are contiguous runs of them.  Each transform is decimation
// in time in LDS after a bit-reversed load, two radix-2 stages at a time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "gd_internal.h"
#include "gd_twiddle.h"

namespace gdspec {

using gd::fail;

inline size_t align_up_256(size_t x) { return gd::align_up(x, 256); }

__constant__ gdtw::Table c_tw = gdtw::make_table();

struct TableF {
    float2 v[gdtw::kTwN / 2];
};
constexpr TableF make_table_f() {
    TableF t{};
    const gdtw::Table d = gdtw::make_table();
    for (int k = 0; k < gdtw::kTwN / 2; ++k) t.v[k] = float2{float(d.v[k].re), float(d.v[k].im)};
    return t;
}
__constant__ TableF c_twf = make_table_f();

template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };

template <typename T>
__device__ __forceinline__ typename V2<T>::t cmul(typename V2<T>::t a, typename V2<T>::t b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// exp(-+2 pi i k / n), k < n / 2 (n a power of two <= kTwN), from the table
template <typename T, bool INV>
__device__ __forceinline__ typename V2<T>::t tw(int k, int tstride) {
    if constexpr (sizeof(T) == 4) {
        const float2 c = c_twf.v[k * tstride];
        return {c.x, INV ? -c.y : c.y};
    } else {
        const gdtw::Cd c = c_tw.v[k * tstride];
        return {c.re, INV ? -c.im : c.im};
    }
}

// exp(-+2 pi i k / n) for 0 <= k <= n (used by the real-row split)
template <typename T, bool INV>
__device__ __forceinline__ typename V2<T>::t tw_full(int k, int n) {
    const int half = n / 2;
    if (k == half) return {T(-1), T(0)};
    if (k == n) return {T(1), T(0)};
    if (k < half) return tw<T, INV>(k, gdtw::kTwN / n);
    typename V2<T>::t w = tw<T, INV>(k - half, gdtw::kTwN / n);
    return {-w.x, -w.y};
}

__device__ __forceinline__ int bitrev(int j, int logn) { return logn == 0 ? 0 : (int)(__brev((unsigned)j) >> (32 - logn)); }

// In-place DIT transforms of the cw = 2^logcw columns of length n stored
// buf[j * cw + c], already in bit-reversed order: one radix-2 stage when
// log2 n is odd, then pairs of radix-2 stages fused into radix-4 butterflies
// held in registers (half the LDS round trips and barriers).
template <typename T, bool INV>
__device__ __forceinline__ void lds_fft(typename V2<T>::t *buf, int n, int logn, int logcw) {
    using V = typename V2<T>::t;
    const int cmask = (1 << logcw) - 1;
    auto at = [&](int i, int c) -> V & { return buf[(i << logcw) + c]; };
    int s = 1;
    if (logn & 1) {
        for (int b = threadIdx.x; b < (n / 2) << logcw; b += 256) {
            const int c = b & cmask, i0 = (b >> logcw) << 1;
            const V a = at(i0, c), x = at(i0 + 1, c);
            at(i0, c) = {a.x + x.x, a.y + x.y};
            at(i0 + 1, c) = {a.x - x.x, a.y - x.y};
        }
        __syncthreads();
        s = 2;
    }
    for (; s < logn; s += 2) {
        const int h = 1 << (s - 1);
        const int ts1 = gdtw::kTwN >> s, ts2 = gdtw::kTwN >> (s + 1);
        for (int b = threadIdx.x; b < (n / 4) << logcw; b += 256) {
            const int c = b & cmask, bb = b >> logcw;
            const int pos = bb & (h - 1);
            const int i0 = ((bb >> (s - 1)) << (s + 1)) + pos;
            const V x0 = at(i0, c), x1 = at(i0 + h, c), x2 = at(i0 + 2 * h, c), x3 = at(i0 + 3 * h, c);
            const V w1 = tw<T, INV>(pos, ts1), w2 = tw<T, INV>(pos, ts2);
            // stage s: pairs (x0, x1) and (x2, x3), twiddle W_2h^pos
            V t = cmul<T>(x1, w1);
            const V a0 = {x0.x + t.x, x0.y + t.y}, a1 = {x0.x - t.x, x0.y - t.y};
            t = cmul<T>(x3, w1);
            const V a2 = {x2.x + t.x, x2.y + t.y}, a3 = {x2.x - t.x, x2.y - t.y};
            // stage s+1: pairs (a0, a2) with W_4h^pos, (a1, a3) with W_4h^(pos+h) = W_4h^pos (-+i)
            t = cmul<T>(a2, w2);
            at(i0, c) = {a0.x + t.x, a0.y + t.y};
            at(i0 + 2 * h, c) = {a0.x - t.x, a0.y - t.y};
            t = cmul<T>(a3, w2);
            t = INV ? V{-t.y, t.x} : V{t.y, -t.x};
            at(i0 + h, c) = {a1.x + t.x, a1.y + t.y};
            at(i0 + 3 * h, c) = {a1.x - t.x, a1.y - t.y};
        }
        __syncthreads();
    }
}

// Multipliers applied to the spectrum (see the file comment).
enum Mul : int { MUL_NONE = 0, MUL_C = 1, MUL_INV_CN = 2, MUL_GHAT_N = 3 };

struct SpecMap {
    int64_t nx, ny, nz;  // logical grid
    int64_t nxh;         // complex columns per stored row (padded)
    int64_t nxc;         // nx / 2 + 1
    double inv_kc2, npts;
    int ndim, axis;      // axis of this column pass: 1 (y) or 2 (z)
    int mul;
};

__device__ __forceinline__ int64_t signed_k(int64_t k, int64_t n) { return k <= n / 2 ? k : k - n; }

// multiplier at spectral index (kx, ky, kz)
__device__ __forceinline__ double mul_at(const SpecMap &m, int64_t kx, int64_t ky, int64_t kz) {
    if (kx >= m.nxc) return 0.0;  // padding columns
    const double w = (kx == 0 || 2 * kx == m.nx) ? 1.0 : 2.0;
    switch (m.mul) {
    case MUL_C: return sqrt(w / m.npts);
    case MUL_INV_CN: return 1.0 / sqrt(w * m.npts);
    case MUL_GHAT_N: {
        const double a = (double)signed_k(ky, m.ny), b = (double)signed_k(kz, m.nz);
        const double k2 = (double)(kx * kx) + a * a + b * b;
        return 1.0 / ((1.0 + k2 * m.inv_kc2) * m.npts);
    }
    default: return 1.0;
    }
}

// Complex transforms of length n along the middle axis of a [outer][n][inner]
// array of complex values, cw adjacent inner columns per workgroup (in place).
// The multiplier (if any) is applied after a forward / before an inverse
// transform.
template <typename T, bool INV>
__global__ __launch_bounds__(256) void k_fft_cols(T *data, int64_t inner, int n, int logn, int logcw, int64_t nchunks,
                                                  SpecMap m) {
    using V = typename V2<T>::t;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    V *buf = reinterpret_cast<V *>(lds_raw);
    const int cw = 1 << logcw;
    // workgroups are dealt round-robin over the 8 XCDs: give each XCD a
    // contiguous range, so that the chunks sharing a cache line share an L2
    int64_t lin = blockIdx.x;
    {
        const int64_t nb = gridDim.x, per = nb / 8, rem = nb % 8, xcd = lin % 8, k = lin / 8;
        lin = xcd * per + (xcd < rem ? xcd : rem) + k;
    }
    const int64_t chunk = lin % nchunks, o = lin / nchunks;
    const int64_t i0 = chunk * cw;
    const int ncols = (int)std::min<int64_t>(cw, inner - i0);
    V *base = reinterpret_cast<V *>(data) + (o * n) * inner + i0;
    auto mult = [&](int j, int c) -> double {
        const int64_t ii = i0 + c;
        if (m.axis == 1) return mul_at(m, ii, j, m.ndim == 3 ? o % m.nz : 0);
        return mul_at(m, ii % m.nxh, ii / m.nxh, j);
    };
    for (int idx = threadIdx.x; idx < n << logcw; idx += 256) {
        const int c = idx & (cw - 1), j = idx >> logcw;
        V v = {T(0), T(0)};
        if (c < ncols) {
            v = base[(int64_t)j * inner + c];
            if (INV && m.mul != MUL_NONE) {
                const T s = T(mult(j, c));
                v = {v.x * s, v.y * s};
            }
        }
        buf[(bitrev(j, logn) << logcw) + c] = v;
    }
    __syncthreads();
    lds_fft<T, INV>(buf, n, logn, logcw);
    for (int idx = threadIdx.x; idx < n << logcw; idx += 256) {
        const int c = idx & (cw - 1), j = idx >> logcw;
        if (c >= ncols) continue;
        V v = buf[(j << logcw) + c];
        if (!INV && m.mul != MUL_NONE) {
            const T s = T(mult(j, c));
            v = {v.x * s, v.y * s};
        }
        base[(int64_t)j * inner + c] = v;
    }
}

// Forward real rows: x (rows of nx reals) -> X (rows of nxh complex values:
// k = 0 .. nx/2, then zero padding).  rpw rows per workgroup.
template <typename T>
__global__ __launch_bounds__(256) void k_rfft_rows(const T *x, T *X, int64_t nrows, int nx, int logn2, int64_t nxh,
                                                   int logrpw) {
    using V = typename V2<T>::t;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    V *buf = reinterpret_cast<V *>(lds_raw);
    const int n2 = nx / 2, rpw = 1 << logrpw;
    const int64_t r0 = (int64_t)blockIdx.x * rpw;
    const int nr = (int)std::min<int64_t>(rpw, nrows - r0);
    const V *src = reinterpret_cast<const V *>(x + r0 * nx);  // z[j] = x[2j] + i x[2j+1]
    for (int idx = threadIdx.x; idx < n2 << logrpw; idx += 256) {
        const int r = idx >> logn2, j = idx & (n2 - 1);
        buf[(bitrev(j, logn2) << logrpw) + r] = r < nr ? src[(int64_t)r * n2 + j] : V{T(0), T(0)};
    }
    __syncthreads();
    lds_fft<T, false>(buf, n2, logn2, logrpw);
    V *dst = reinterpret_cast<V *>(X) + r0 * nxh;
    for (int idx = threadIdx.x; idx < (int)nxh * nr; idx += 256) {
        const int r = idx / (int)nxh, k = idx % (int)nxh;
        V out = {T(0), T(0)};
        if (k <= n2) {
            // X[k] = (Z[k] + conj Z[n2-k]) / 2 - i/2 exp(-2 pi i k / nx) (Z[k] - conj Z[n2-k])
            const V zk = buf[((k & (n2 - 1)) << logrpw) + r];
            const V zm0 = buf[(((n2 - k) & (n2 - 1)) << logrpw) + r];
            const V zm = {zm0.x, -zm0.y};
            const V e = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y + zm.y)};
            const V d = {T(0.5) * (zk.x - zm.x), T(0.5) * (zk.y - zm.y)};
            const V w = tw_full<T, false>(k, nx);
            const V wd = cmul<T>(w, d);  // times -i: (a + ib)(-i) = b - ia
            out = {e.x + wd.y, e.y - wd.x};
        }
        dst[(int64_t)r * nxh + k] = out;
    }
}

// Inverse real rows: X (rows of nxh complex, k = 0 .. nx/2 used) -> x, the
// unnormalised inverse (nx times the inverse DFT along x).
template <typename T>
__global__ __launch_bounds__(256) void k_irfft_rows(const T *X, T *x, int64_t nrows, int nx, int logn2, int64_t nxh,
                                                    int logrpw) {
    using V = typename V2<T>::t;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    V *buf = reinterpret_cast<V *>(lds_raw);
    const int n2 = nx / 2, rpw = 1 << logrpw;
    const int64_t r0 = (int64_t)blockIdx.x * rpw;
    const int nr = (int)std::min<int64_t>(rpw, nrows - r0);
    const V *src = reinterpret_cast<const V *>(X) + r0 * nxh;
    const int np = n2 / 2 + 1;  // pairs (k, n2 - k), k = 0 .. n2/2
    for (int idx = threadIdx.x; idx < np * rpw; idx += 256) {
        const int r = idx / np, k = idx % np;
        V a = {T(0), T(0)}, b = {T(0), T(0)};
        if (r < nr) {
            a = src[(int64_t)r * nxh + k];
            b = src[(int64_t)r * nxh + (n2 - k)];
        }
        // Z[k] = (X[k] + conj X[n2-k]) + i exp(2 pi i k / nx) (X[k] - conj X[n2-k])
        auto z_of = [&](V xk, V xm, int kk) -> V {
            const V s = {xk.x + xm.x, xk.y - xm.y};
            const V d = {xk.x - xm.x, xk.y + xm.y};
            const V wd = cmul<T>(tw_full<T, true>(kk, nx), d);
            return {s.x - wd.y, s.y + wd.x};  // s + i wd
        };
        if (k < n2) buf[(bitrev(k, logn2) << logrpw) + r] = z_of(a, b, k);
        if (k != 0 && n2 - k != k) buf[(bitrev(n2 - k, logn2) << logrpw) + r] = z_of(b, a, n2 - k);
    }
    __syncthreads();
    lds_fft<T, true>(buf, n2, logn2, logrpw);
    V *dst = reinterpret_cast<V *>(x + r0 * nx);
    for (int idx = threadIdx.x; idx < n2 * nr; idx += 256) {
        const int r = idx >> logn2, j = idx & (n2 - 1);
        dst[(int64_t)r * n2 + j] = buf[(j << logrpw) + r];
    }
}

constexpr size_t kLdsBudget = 64 * 1024;
// column transforms: a smaller share, so that more workgroups are resident
constexpr size_t kColLds = 32 * 1024;

int ilog2(int64_t n) {
    int l = 0;
    while ((int64_t(1) << l) < n) ++l;
    return l;
}

bool pow2(int64_t n) { return n >= 2 && (n & (n - 1)) == 0; }

// Geometry of the stored half spectrum of a grid.
struct Spec {
    int ndim;
    int64_t nx, ny, nz, batch;
    int64_t nxc, nxs, nxh;  // complex columns, stored reals per row, stored complex per row
    int64_t elems;          // stored reals of the batch
    size_t tsize;
};

Spec spec_of(const gd_grid *g) {
    Spec s;
    s.ndim = g->ndim;
    s.nx = g->n[0];
    s.ny = g->n[1];
    s.nz = g->ndim == 3 ? g->n[2] : 1;
    s.batch = g->batch;
    s.tsize = g->dtype == GD_F32 ? 4 : 8;
    const int64_t lane = 16 / (int64_t)s.tsize;  // reals per 16-byte lane
    s.nxc = s.nx / 2 + 1;
    s.nxs = (2 * s.nxc + lane - 1) / lane * lane;
    s.nxh = s.nxs / 2;
    s.elems = s.batch * s.nz * s.ny * s.nxs;
    return s;
}

int validate_spec_grid(const gd_grid *g) {
    int rc = gd::validate_grid(g);
    if (rc) return rc;
    const int64_t maxn = g->dtype == GD_F32 ? 4096 : 2048;
    for (int d = 0; d < g->ndim; ++d)
        if (!pow2(g->n[d]) || g->n[d] > maxn)
            return fail(GD_EINVAL, "the differential filter needs power-of-two sizes in [2, %lld] (n[%d] = %lld)",
                        (long long)maxn, d, (long long)g->n[d]);
    return GD_OK;
}

double inv_kc2_of(const gd_grid *g, double gamma) {
    int64_t nmin = g->n[0];
    for (int d = 1; d < g->ndim; ++d) nmin = std::min<int64_t>(nmin, g->n[d]);
    const double kc = gamma * (double)nmin / 2.0;
    return 1.0 / (kc * kc);
}

SpecMap map_of(const Spec &s, int axis, int mul, double inv_kc2) {
    SpecMap m;
    m.nx = s.nx;
    m.ny = s.ny;
    m.nz = s.nz;
    m.nxh = s.nxh;
    m.nxc = s.nxc;
    m.inv_kc2 = inv_kc2;
    m.npts = (double)(s.nx * s.ny * s.nz);
    m.ndim = s.ndim;
    m.axis = axis;
    m.mul = mul;
    return m;
}

template <typename T>
int launch_cols(const Spec &s, T *data, int axis, bool inv, int mul, double inv_kc2, hipStream_t st) {
    const int64_t n = axis == 1 ? s.ny : s.nz;
    const int64_t inner = axis == 1 ? s.nxh : s.ny * s.nxh;
    const int64_t outer = axis == 1 ? s.batch * s.nz : s.batch;
    const size_t cs = 2 * sizeof(T);
    int logcw = 0;  // adjacent columns per workgroup: a power of two, up to 16, within the LDS budget
    while (logcw < 4 && (int64_t(2) << logcw) <= inner && (size_t)n * (size_t(2) << logcw) * cs <= kColLds) ++logcw;
    const int cw = 1 << logcw;
    const int64_t nchunks = (inner + cw - 1) / cw;
    const int64_t blocks = outer * nchunks;
    if (blocks > 0x7fffffff) return fail(GD_EINVAL, "grid too large for the FFT");
    const SpecMap m = map_of(s, axis, mul, inv_kc2);
    const size_t lds = (size_t)n * cw * cs;
    if (inv)
        hipLaunchKernelGGL((k_fft_cols<T, true>), dim3((unsigned)blocks), dim3(256), lds, st, data, inner, (int)n,
                           ilog2(n), logcw, nchunks, m);
    else
        hipLaunchKernelGGL((k_fft_cols<T, false>), dim3((unsigned)blocks), dim3(256), lds, st, data, inner, (int)n,
                           ilog2(n), logcw, nchunks, m);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GD_OK : fail(GD_EHIP, "FFT column launch: %s", hipGetErrorString(e));
}

// log2 of the rows per workgroup of the row transforms: enough rows for two
// radix-4 butterflies (n2 / 4 per row) per thread, within the LDS share
template <typename T>
int log_rows_per_wg(const Spec &s) {
    const int64_t n2 = s.nx / 2;
    int l = 0;
    while ((std::max<int64_t>(1, n2 / 4) << l) < 512 && (n2 << (l + 1)) * 2 * (int64_t)sizeof(T) <= (int64_t)kColLds)
        ++l;
    return l;
}

// real fields x -> stored half spectrum X (scaled by c(k) when `scaled`, by
// G_hat / N when `ghat`)
template <typename T>
int forward(const Spec &s, const T *x, T *X, int mul, double inv_kc2, hipStream_t st) {
    const int64_t nrows = s.batch * s.nz * s.ny;
    const int lr = log_rows_per_wg<T>(s), rpw = 1 << lr;
    const int64_t blocks = (nrows + rpw - 1) / rpw;
    const size_t lds = (size_t)(s.nx / 2) * rpw * 2 * sizeof(T);
    hipLaunchKernelGGL((k_rfft_rows<T>), dim3((unsigned)blocks), dim3(256), lds, st, x, X, nrows, (int)s.nx,
                       ilog2(s.nx / 2), s.nxh, lr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(GD_EHIP, "FFT row launch: %s", hipGetErrorString(e));
    int rc;
    if (s.ndim == 2) return launch_cols<T>(s, X, 1, false, mul, inv_kc2, st);
    if ((rc = launch_cols<T>(s, X, 1, false, MUL_NONE, inv_kc2, st))) return rc;
    return launch_cols<T>(s, X, 2, false, mul, inv_kc2, st);
}

// stored half spectrum X (overwritten) -> real fields x
template <typename T>
int inverse(const Spec &s, T *X, T *x, int mul, double inv_kc2, hipStream_t st) {
    int rc;
    if (s.ndim == 3) {
        if ((rc = launch_cols<T>(s, X, 2, true, mul, inv_kc2, st))) return rc;
        if ((rc = launch_cols<T>(s, X, 1, true, MUL_NONE, inv_kc2, st))) return rc;
    } else if ((rc = launch_cols<T>(s, X, 1, true, mul, inv_kc2, st))) {
        return rc;
    }
    const int64_t nrows = s.batch * s.nz * s.ny;
    const int lr = log_rows_per_wg<T>(s), rpw = 1 << lr;
    const int64_t blocks = (nrows + rpw - 1) / rpw;
    const size_t lds = (size_t)(s.nx / 2) * rpw * 2 * sizeof(T);
    hipLaunchKernelGGL((k_irfft_rows<T>), dim3((unsigned)blocks), dim3(256), lds, st, X, x, nrows, (int)s.nx,
                       ilog2(s.nx / 2), s.nxh, lr);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GD_OK : fail(GD_EHIP, "FFT row launch: %s", hipGetErrorString(e));
}


// The grid the persistent solve kernel sweeps over the stored spectrum.  Its
// sweeps are pointwise, so the spectrum of a field (nz ny rows of nxs reals)
// is presented as rows of W reals, W the largest power of two up to 8192 that
// divides the field: every 256-real wave segment is then full (rows of nxs =
// n_x + 2 or + 4 reals would end in a nearly empty segment, half of all
// segments at n_x = 256).  Small fields keep the stored rows.
gd_grid spectral_grid(const gd_grid *g, const Spec &s) {
    gd_grid v = *g;
    const int64_t total = s.nz * s.ny * s.nxs;
    int64_t W = 1;
    while (W < 8192 && total % (2 * W) == 0) W *= 2;
    if (W >= 1024 && total / W >= 16) {
        v.ndim = 2;
        v.n[0] = W;
        v.n[1] = total / W;
        v.n[2] = 1;
    } else {
        v.n[0] = s.nxs;
    }
    for (int d = 0; d < 3; ++d) v.h[d] = 0.0;  // the weight travels in SpecParams
    return v;
}

gd::SpecParams spec_params(const gd_grid *g, const Spec &s, double inv_kc2) {
    gd::SpecParams sp;
    sp.inv_kc2 = inv_kc2;
    sp.hw = gd::grid_weight(g);
    sp.nxc = s.nxc;
    sp.nxs = s.nxs;
    sp.lny = ilog2(s.ny);
    sp.lnz = ilog2(s.nz);
    return sp;
}


// ---- a-priori diagnostics: energy spectra and PDFs ---------------------------

// nearest integer to sqrt(k2) for integer k2 >= 0, decided in integer arithmetic
__host__ __device__ inline int64_t shell_of(int64_t k2) {
    int64_t s = (int64_t)sqrt((double)k2);
    if ((2 * s + 1) * (2 * s + 1) <= 4 * k2) ++s;
    if (s > 0 && (2 * s - 1) * (2 * s - 1) > 4 * k2) --s;
    return s;
}

int64_t num_shells(const Spec &s) {
    const int64_t a = s.nx / 2, b = s.ny / 2, c = s.ndim == 3 ? s.nz / 2 : 0;
    return shell_of(a * a + b * b + c * c) + 1;
}

// |k|^kpow = (k^2)^(kpow/2) for k^2 >= 1.  For kpow/2 = ipow, an integer in
// [-2, 2] (kIpowNone otherwise), the power is formed from the integer k^2 by
// exact products and at most one correctly rounded division instead of pow().
constexpr int kIpowNone = 99;
__device__ __forceinline__ double kpow_of(int64_t k2, double kpow, int ipow) {
    if (ipow == kIpowNone) return pow((double)k2, 0.5 * kpow);
    const double x = (double)k2;  // k^2 < 2^26 here, so x * x is exact
    const double r = (ipow == 2 || ipow == -2) ? x * x : x;
    return ipow > 0 ? r : 1.0 / r;
}

// Partial shell sums of one chunk of rows of one field's stored spectrum:
// 1/2 w(k_x) |X / N|^2 |k|^p per coefficient, accumulated per shell in LDS.
// A wave takes whole rows; along a row |k| grows with k_x, so the lanes of a
// wave hold nondecreasing shells, summed by a segmented scan before one LDS
// update per segment.  Every wave of the workgroup (blockDim.x / 64 of them)
// has its own bins, which no other wave touches, and adds into them in
// program order; the waves' bins are then summed in wave order.  So the
// result does not depend on timing.
template <typename T>
__global__ __launch_bounds__(256) void k_spectrum_part(const T *X, double *part, int64_t rows_per_field,
                                                       int64_t rows_per_chunk, int64_t nchunks, int64_t nshells, Spec s,
                                                       double kpow, int ipow) {
    using V = typename V2<T>::t;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int nwaves = (int)(blockDim.x >> 6);
    double *all_bins = reinterpret_cast<double *>(lds_raw);
    for (int64_t i = threadIdx.x; i < nwaves * nshells; i += blockDim.x) all_bins[i] = 0.0;
    __syncthreads();
    const int64_t b = blockIdx.x / nchunks, ch = blockIdx.x % nchunks;
    const int64_t row0 = ch * rows_per_chunk, row1 = std::min(rows_per_field, row0 + rows_per_chunk);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double *bins = all_bins + wave * nshells;
    const V *F = reinterpret_cast<const V *>(X) + b * rows_per_field * s.nxh;
    const double inv_n2 = 1.0 / ((double)(s.nx * s.ny * s.nz) * (double)(s.nx * s.ny * s.nz));
    for (int64_t row = row0 + wave; row < row1; row += nwaves) {
        const int64_t ky = row % s.ny, kz = row / s.ny;
        const int64_t a = ky <= s.ny / 2 ? ky : ky - s.ny, c = kz <= s.nz / 2 ? kz : kz - s.nz;
        const int64_t kyz2 = a * a + c * c;
        for (int64_t kx0 = 0; kx0 < s.nxc; kx0 += 64) {
            const int64_t kx = kx0 + lane;
            double v = 0.0;
            int64_t key = -1;
            if (kx < s.nxc) {
                const V z = F[row * s.nxh + kx];
                const int64_t k2 = kx * kx + kyz2;
                const double w = (kx == 0 || 2 * kx == s.nx) ? 0.5 : 1.0;
                double kp = 1.0;
                if (kpow != 0.0) kp = k2 > 0 ? kpow_of(k2, kpow, ipow) : 0.0;
                v = w * ((double)z.x * (double)z.x + (double)z.y * (double)z.y) * inv_n2 * kp;
                key = shell_of(k2);
            }
            // segmented inclusive scan over equal, contiguous keys
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const double ov = __shfl_up(v, off, 64);
                const int64_t ok = __shfl_up(key, off, 64);
                if (lane >= off && ok == key) v += ov;
            }
            // one lane per segment: distinct bins within this update
            const int64_t next = __shfl_down(key, 1, 64);
            if (key >= 0 && (lane == 63 || next != key)) bins[key] += v;
        }
    }
    __syncthreads();
    double *dst = part + (b * nchunks + ch) * nshells;
    for (int64_t i = threadIdx.x; i < nshells; i += blockDim.x) {
        double acc = all_bins[i];
        for (int w = 1; w < nwaves; ++w) acc += all_bins[w * nshells + i];
        dst[i] = acc;
    }
}

// out[b][s] = sum over the chunks' partial sums: one workgroup per (field,
// shell), thread j adding chunks j, j + 256, ... in order, then a fixed tree
// over the threads, so the result does not depend on timing.
__global__ __launch_bounds__(256) void k_spectrum_reduce(const double *part, double *out, int64_t nchunks,
                                                         int64_t nshells, int64_t batch) {
    __shared__ double red[256];
    for (int64_t t = blockIdx.x; t < batch * nshells; t += gridDim.x) {
        const int64_t b = t / nshells, sh = t % nshells;
        double acc = 0.0;
        for (int64_t c = threadIdx.x; c < nchunks; c += 256) acc += part[(b * nchunks + c) * nshells + sh];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[t] = red[0];
        __syncthreads();
    }
}

// blocks of 256 threads for a grid-stride loop over n items
unsigned stride_blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

// ---- band projection of a start ---------------------------------------------

// Energy of each field from its unnormalized half spectrum: part[b][c] = sum
// over chunk c of field b's stored modes of w(kx) |X|^2 (w = 1 on the kx = 0
// and kx = nx / 2 columns, 2 elsewhere, 0 on the padding), each workgroup a
// fixed tree over its threads, so the result does not depend on timing.
template <typename T, bool SCALED = false>
__global__ __launch_bounds__(256) void k_band_power(const T *X, double *part, int64_t per_field, int64_t nchunks,
                                                    Spec s) {
    using V = typename V2<T>::t;
    __shared__ double red[256];
    const int64_t b = blockIdx.y, ch = blockIdx.x;
    const int64_t len = (per_field + nchunks - 1) / nchunks;
    const int64_t i0 = ch * len, i1 = std::min(per_field, i0 + len);
    const V *F = reinterpret_cast<const V *>(X) + b * per_field;
    double acc = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const int64_t kx = i % s.nxh;
        if (kx < s.nxc) {
            const V z = F[i];
            // a Parseval-scaled spectrum (SCALED) already carries w in its values
            const double w = SCALED ? 1.0 : ((kx == 0 || 2 * kx == s.nx) ? 1.0 : 2.0);
            acc += w * ((double)z.x * (double)z.x + (double)z.y * (double)z.y);
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[b * nchunks + ch] = red[0];
}

// X0 <- (X0 - XB) / N on the modes where |XB|^2 > tau E_b, 0 elsewhere, with
// E_b = (1/N) sum_k w |XB|^2 the mean of |XB(k)|^2 over all N wavenumbers of
// field b (= sum_x ubar^2, Parseval).  The 1/N makes the unnormalized
// inverse transform the inverse.
template <typename T>
__global__ __launch_bounds__(256) void k_band_mask(T *X0, const T *XB, const double *part, int64_t per_field,
                                                   int64_t nchunks, Spec s, double tau) {
    using V = typename V2<T>::t;
    __shared__ double thr;
    const int64_t b = blockIdx.y;
    const double n = (double)(s.nx * s.ny * s.nz);
    if (threadIdx.x == 0) {
        double e = 0.0;
        for (int64_t c = 0; c < nchunks; ++c) e += part[b * nchunks + c];
        thr = tau * (e / n);
    }
    __syncthreads();
    const double t = thr, inv_n = 1.0 / n;
    V *F0 = reinterpret_cast<V *>(X0) + b * per_field;
    const V *FB = reinterpret_cast<const V *>(XB) + b * per_field;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < per_field; i += (int64_t)gridDim.x * 256) {
        const int64_t kx = i % s.nxh;
        const V zb = FB[i], z0 = F0[i];
        const double p = (double)zb.x * (double)zb.x + (double)zb.y * (double)zb.y;
        V r;
        r.x = r.y = T(0);
        if (kx < s.nxc && p > t) {
            r.x = (T)(((double)z0.x - (double)zb.x) * inv_n);
            r.y = (T)(((double)z0.y - (double)zb.y) * inv_n);
        }
        F0[i] = r;
    }
}

// The same projection on the Parseval-scaled spectra the differential-filter
// solve holds (S = sqrt(w(kx) / N) X, and part from k_band_power<T, true>
// sums to sum_x ubar^2 = E): U <- U where |X_B|^2 = |S_B|^2 N / w > tau E,
// U <- S_B elsewhere (the start keeps ubar's coefficients there, so
// start - ubar has no content outside ubar's support).
template <typename T>
__global__ __launch_bounds__(256) void k_band_keep(T *U, const T *UB, const double *part, int64_t per_field,
                                                   int64_t nchunks, Spec s, double tau) {
    using V = typename V2<T>::t;
    __shared__ double e_sh;
    const int64_t b = blockIdx.y;
    if (threadIdx.x == 0) {
        double e = 0.0;
        for (int64_t c = 0; c < nchunks; ++c) e += part[b * nchunks + c];
        e_sh = e;
    }
    __syncthreads();
    const double te = tau * e_sh / (double)(s.nx * s.ny * s.nz);
    V *F = reinterpret_cast<V *>(U) + b * per_field;
    const V *FB = reinterpret_cast<const V *>(UB) + b * per_field;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < per_field; i += (int64_t)gridDim.x * 256) {
        const int64_t kx = i % s.nxh;
        if (kx >= s.nxc) continue;  // padding stays zero
        const V zb = FB[i];
        const double w = (kx == 0 || 2 * kx == s.nx) ? 1.0 : 2.0;
        const double p = (double)zb.x * (double)zb.x + (double)zb.y * (double)zb.y;
        if (!(p > te * w)) F[i] = zb;
    }
}

// u0 += ubar
template <typename T>
__global__ __launch_bounds__(256) void k_band_add(T *u0, const T *ubar, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) u0[i] += ubar[i];
}

// threshold of the band projection a warm start of the differential-filter
// solve gets (relative to the mean mode power of ubar)
constexpr double kWarmBandTau = 1e-10;

// chunks per field of the band power sums: about 4096 stored modes each, at most 256
int64_t band_chunks(const Spec &s) {
    const int64_t per_field = s.nz * s.ny * s.nxh;
    return std::max<int64_t>(1, std::min<int64_t>(256, per_field / 4096));
}

template <typename T>
int band_project_run(const Spec &s, double tau, const T *ubar, T *u0, char *w, hipStream_t st) {
    const size_t sb = align_up_256((size_t)s.elems * s.tsize);
    T *XB = (T *)w, *X0 = (T *)(w + sb);
    double *part = (double *)(w + 2 * sb);
    int rc;
    if ((rc = forward<T>(s, ubar, XB, MUL_NONE, 0.0, st))) return rc;
    if ((rc = forward<T>(s, u0, X0, MUL_NONE, 0.0, st))) return rc;
    const int64_t per_field = s.nz * s.ny * s.nxh, nch = band_chunks(s);
    if (s.batch > 65535) return fail(GD_EINVAL, "batch too large for the band projection (at most 65535 fields)");
    hipLaunchKernelGGL(k_band_power<T>, dim3((unsigned)nch, (unsigned)s.batch), dim3(256), 0, st, XB, part, per_field,
                       nch, s);
    const unsigned mb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((per_field + 255) / 256, 1024));
    hipLaunchKernelGGL(k_band_mask<T>, dim3(mb, (unsigned)s.batch), dim3(256), 0, st, X0, XB, part, per_field, nch, s,
                       tau);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(GD_EHIP, "band projection launch: %s", hipGetErrorString(e));
    if ((rc = inverse<T>(s, X0, u0, MUL_NONE, 0.0, st))) return rc;
    const int64_t npts = s.batch * s.nx * s.ny * s.nz;
    hipLaunchKernelGGL(k_band_add<T>, dim3(stride_blocks(npts)), dim3(256), 0, st, u0, ubar, npts);
    e = hipGetLastError();
    return e == hipSuccess ? GD_OK : fail(GD_EHIP, "band projection launch: %s", hipGetErrorString(e));
}

__global__ void k_zero_i64(int64_t *p, int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = 0;
}


// PDF bin counts: LDS counters per workgroup (one field's chunk), then one
// global integer atomic per nonzero bin.
template <typename T>
__global__ __launch_bounds__(256) void k_pdf(const T *x, int64_t *counts, int64_t npts, int64_t chunk, int64_t nchunks,
                                             double lo, double hi, double scale, int nbins) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    unsigned *bins = reinterpret_cast<unsigned *>(lds_raw);
    for (int i = threadIdx.x; i < nbins; i += 256) bins[i] = 0u;
    __syncthreads();
    const int64_t b = blockIdx.x / nchunks, ch = blockIdx.x % nchunks;
    const int64_t i0 = ch * chunk, i1 = std::min(npts, i0 + chunk);
    const T *f = x + b * npts;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const double v = (double)f[i];
        if (v >= lo && v <= hi) {  // false for NaN
            int64_t k = (int64_t)floor((v - lo) * scale);
            if (k > nbins - 1) k = nbins - 1;
            atomicAdd(&bins[k], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += 256)
        if (bins[i]) atomicAdd(reinterpret_cast<unsigned long long *>(&counts[b * nbins + i]), (unsigned long long)bins[i]);
}

constexpr int kMaxPdfBins = 8192;

}  // namespace gdspec

using namespace gdspec;

extern "C" {

size_t germano_workspace_bytes(const gd_grid *g, int32_t solver) {
    if (validate_spec_grid(g)) return 0;
    const Spec s = spec_of(g);
    const size_t spec_bytes = align_up_256((size_t)s.elems * s.tsize);
    if (solver < 0) return spec_bytes;
    if (solver > GD_STEEPEST_DESCENT) return 0;
    const gd_grid v = spectral_grid(g, s);
    const size_t solve = deconvolve_workspace_bytes(&v, solver);
    return solve ? 2 * spec_bytes + solve : 0;
}

int germano_filter_apply(const gd_grid *g, double gamma, const void *x, void *y, void *work, size_t wb,
                         void *stream) {
    int rc = validate_spec_grid(g);
    if (rc) return rc;
    if (!(gamma > 0.0) || !std::isfinite(gamma)) return fail(GD_EINVAL, "gamma must be positive");
    if (!x || !y) return fail(GD_EINVAL, "x and y must be non-NULL");
    if (!work) return fail(GD_EWORKSPACE, "workspace is NULL");
    if ((uintptr_t)work % 256) return fail(GD_EALIGN, "workspace must be 256-byte aligned");
    const Spec s = spec_of(g);
    const size_t need = germano_workspace_bytes(g, -1);
    if (wb < need) return fail(GD_EWORKSPACE, "workspace too small: need %zu bytes, got %zu", need, wb);
    const size_t fb = (size_t)s.batch * s.nx * s.ny * s.nz * s.tsize;
    if (gd::ranges_overlap(x, fb, work, need) || gd::ranges_overlap(y, fb, work, need)) return fail(GD_EINVAL, "a field overlaps the workspace");
    const double ik = inv_kc2_of(g, gamma);
    hipStream_t st = (hipStream_t)stream;
    if (g->dtype == GD_F32) {
        if ((rc = forward<float>(s, (const float *)x, (float *)work, MUL_GHAT_N, ik, st))) return rc;
        return inverse<float>(s, (float *)work, (float *)y, MUL_NONE, ik, st);
    }
    if ((rc = forward<double>(s, (const double *)x, (double *)work, MUL_GHAT_N, ik, st))) return rc;
    return inverse<double>(s, (double *)work, (double *)y, MUL_NONE, ik, st);
}

int deconvolve_germano(int32_t solver, const gd_grid *g, double gamma, const void *ubar, void *u, const gd_opts *o,
                       void *work, size_t wb, gd_info *info, void *stream) {
    int rc = validate_spec_grid(g);
    if (rc) return rc;
    if ((rc = gd::validate_opts(o))) return rc;
    if (solver < GD_VANCITTERT || solver > GD_STEEPEST_DESCENT) return fail(GD_EINVAL, "bad solver %d", solver);
    if (!(gamma > 0.0) || !std::isfinite(gamma)) return fail(GD_EINVAL, "gamma must be positive");
    if (!ubar || !u || !info) return fail(GD_EINVAL, "ubar, u and info must be non-NULL");
    if (!work) return fail(GD_EWORKSPACE, "workspace is NULL");
    if ((uintptr_t)work % 256) return fail(GD_EALIGN, "workspace must be 256-byte aligned");
    const size_t need = germano_workspace_bytes(g, solver);
    if (wb < need) return fail(GD_EWORKSPACE, "workspace too small: need %zu bytes, got %zu", need, wb);
    const Spec s = spec_of(g);
    const size_t fb = (size_t)s.batch * s.nx * s.ny * s.nz * s.tsize;
    if (gd::ranges_overlap(ubar, fb, u, fb)) return fail(GD_EINVAL, "ubar and u overlap");
    if (gd::ranges_overlap(ubar, fb, work, need) || gd::ranges_overlap(u, fb, work, need))
        return fail(GD_EINVAL, "a field overlaps the workspace");
    const size_t sb = align_up_256((size_t)s.elems * s.tsize);
    char *w = (char *)work;
    void *UB = w, *U = w + sb;
    void *solve_work = w + 2 * sb;
    const double ik = inv_kc2_of(g, gamma);
    hipStream_t st = (hipStream_t)stream;
    const bool f32 = g->dtype == GD_F32;
    rc = f32 ? forward<float>(s, (const float *)ubar, (float *)UB, MUL_C, ik, st)
             : forward<double>(s, (const double *)ubar, (double *)UB, MUL_C, ik, st);
    if (rc) return rc;
    if (o->init == GD_INIT_GIVEN || o->init == GD_INIT_WARM) {
        rc = f32 ? forward<float>(s, (const float *)u, (float *)U, MUL_C, ik, st)
                 : forward<double>(s, (const double *)u, (double *)U, MUL_C, ik, st);
        if (rc) return rc;
    }
    if (o->init == GD_INIT_WARM) {  // band projection of the start (the partial sums use the solve's workspace)
        const int64_t per_field = s.nz * s.ny * s.nxh, nch = band_chunks(s);
        if (s.batch > 65535) return fail(GD_EINVAL, "batch too large for the band projection (at most 65535 fields)");
        double *part = (double *)(w + 2 * sb);
        const unsigned mb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((per_field + 255) / 256, 1024));
        if (f32) {
            hipLaunchKernelGGL((k_band_power<float, true>), dim3((unsigned)nch, (unsigned)s.batch), dim3(256), 0, st,
                               (const float *)UB, part, per_field, nch, s);
            hipLaunchKernelGGL(k_band_keep<float>, dim3(mb, (unsigned)s.batch), dim3(256), 0, st, (float *)U,
                               (const float *)UB, (const double *)part, per_field, nch, s, kWarmBandTau);
        } else {
            hipLaunchKernelGGL((k_band_power<double, true>), dim3((unsigned)nch, (unsigned)s.batch), dim3(256), 0, st,
                               (const double *)UB, part, per_field, nch, s);
            hipLaunchKernelGGL(k_band_keep<double>, dim3(mb, (unsigned)s.batch), dim3(256), 0, st, (double *)U,
                               (const double *)UB, (const double *)part, per_field, nch, s, kWarmBandTau);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(GD_EHIP, "band projection launch: %s", hipGetErrorString(e));
    }
    const gd_grid v = spectral_grid(g, s);
    const gd::SpecParams sp = spec_params(g, s, ik);
    rc = gd::solve_uniform(solver, &v, UB, U, o, solve_work, wb - 2 * sb, info, stream, nullptr, &sp);
    if (rc) return rc;
    return f32 ? inverse<float>(s, (float *)U, (float *)u, MUL_INV_CN, ik, st)
               : inverse<double>(s, (double *)U, (double *)u, MUL_INV_CN, ik, st);
}

int deconvolve_germano_autotune(int32_t solver, const gd_grid *g, double gamma, const void *ubar, void *u, void *work,
                                size_t wb, gd_info *info, void *stream, gd_tune_info *out) {
    int rc = validate_spec_grid(g);
    if (rc) return rc;
    if (solver < GD_VANCITTERT || solver > GD_STEEPEST_DESCENT) return fail(GD_EINVAL, "bad solver %d", solver);
    if (!(gamma > 0.0) || !std::isfinite(gamma)) return fail(GD_EINVAL, "gamma must be positive");
    if (!ubar || !u || !info) return fail(GD_EINVAL, "ubar, u and info must be non-NULL");
    if (!work || (uintptr_t)work % 256) return fail(GD_EALIGN, "workspace must be non-NULL and 256-byte aligned");
    const size_t need = germano_workspace_bytes(g, solver);
    if (wb < need) return fail(GD_EWORKSPACE, "workspace too small: need %zu bytes, got %zu", need, wb);
    const Spec s = spec_of(g);
    const size_t fb = (size_t)s.batch * s.nx * s.ny * s.nz * s.tsize;
    if (gd::ranges_overlap(ubar, fb, work, need)) return fail(GD_EINVAL, "ubar overlaps the workspace");
    const size_t sb = align_up_256((size_t)s.elems * s.tsize);
    char *w = (char *)work;
    const double ik = inv_kc2_of(g, gamma);
    hipStream_t st = (hipStream_t)stream;
    rc = g->dtype == GD_F32 ? forward<float>(s, (const float *)ubar, (float *)w, MUL_C, ik, st)
                            : forward<double>(s, (const double *)ubar, (double *)w, MUL_C, ik, st);
    if (rc) return rc;
    const gd_grid v = spectral_grid(g, s);
    const gd::SpecParams sp = spec_params(g, s, ik);
    return gd::tune_uniform(solver, &v, w, w + sb, w + 2 * sb, wb - 2 * sb, info, stream, out, &sp);
}

int32_t spectrum_shells(const gd_grid *g) {
    if (validate_spec_grid(g)) return 0;
    return (int32_t)num_shells(spec_of(g));
}

static int64_t spectrum_chunks(const Spec &s) {
    const int64_t rows = s.ny * s.nz;
    return std::max<int64_t>(1, std::min<int64_t>(rows / 8, std::max<int64_t>(1, 2048 / s.batch)));
}

size_t spectrum_workspace_bytes(const gd_grid *g) {
    if (validate_spec_grid(g)) return 0;
    const Spec s = spec_of(g);
    return align_up_256((size_t)s.elems * s.tsize) +
           align_up_256((size_t)s.batch * spectrum_chunks(s) * num_shells(s) * sizeof(double));
}

int energy_spectrum(const gd_grid *g, double kpow, const void *x, double *out, void *work, size_t wb, void *stream) {
    int rc = validate_spec_grid(g);
    if (rc) return rc;
    if (!std::isfinite(kpow)) return fail(GD_EINVAL, "kpow must be finite");
    if (!x || !out) return fail(GD_EINVAL, "x and out must be non-NULL");
    if (!work) return fail(GD_EWORKSPACE, "workspace is NULL");
    if ((uintptr_t)work % 256) return fail(GD_EALIGN, "workspace must be 256-byte aligned");
    const Spec s = spec_of(g);
    const size_t need = spectrum_workspace_bytes(g);
    if (wb < need) return fail(GD_EWORKSPACE, "workspace too small: need %zu bytes, got %zu", need, wb);
    const int64_t ns = num_shells(s), nch = spectrum_chunks(s);
    const size_t fb = (size_t)s.batch * s.nx * s.ny * s.nz * s.tsize;
    if (gd::ranges_overlap(x, fb, work, need) || gd::ranges_overlap(out, (size_t)s.batch * ns * 8, work, need))
        return fail(GD_EINVAL, "a buffer overlaps the workspace");
    if ((size_t)ns * sizeof(double) > kLdsBudget) return fail(GD_EINVAL, "too many shells");
    // waves per workgroup: up to four, each with its own bins within the LDS budget
    const int nw = (int)std::max<int64_t>(1, std::min<int64_t>(4, (int64_t)(kLdsBudget / ((size_t)ns * sizeof(double)))));
    const size_t lds = (size_t)nw * ns * sizeof(double);
    hipStream_t st = (hipStream_t)stream;
    double *part = (double *)((char *)work + align_up_256((size_t)s.elems * s.tsize));
    const double hp = 0.5 * kpow;
    const int ipow = (hp == std::floor(hp) && std::fabs(hp) <= 2.0 && hp != 0.0) ? (int)hp : kIpowNone;
    const int64_t rows = s.ny * s.nz, rpc = (rows + nch - 1) / nch;
    const dim3 grid((unsigned)(s.batch * nch));
    if (g->dtype == GD_F32) {
        if ((rc = forward<float>(s, (const float *)x, (float *)work, MUL_NONE, 0.0, st))) return rc;
        hipLaunchKernelGGL(k_spectrum_part<float>, grid, dim3(64 * nw), lds, st, (const float *)work, part, rows, rpc,
                           nch, ns, s, kpow, ipow);
    } else {
        if ((rc = forward<double>(s, (const double *)x, (double *)work, MUL_NONE, 0.0, st))) return rc;
        hipLaunchKernelGGL(k_spectrum_part<double>, grid, dim3(64 * nw), lds, st, (const double *)work, part, rows,
                           rpc, nch, ns, s, kpow, ipow);
    }
    const int64_t tot = s.batch * ns;
    hipLaunchKernelGGL(k_spectrum_reduce, dim3((unsigned)std::min<int64_t>(tot, 8192)), dim3(256), 0, st, part, out,
                       nch, ns, s.batch);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GD_OK : fail(GD_EHIP, "spectrum launch: %s", hipGetErrorString(e));
}

size_t band_project_workspace_bytes(const gd_grid *g) {
    if (validate_spec_grid(g)) return 0;
    const Spec s = spec_of(g);
    return 2 * align_up_256((size_t)s.elems * s.tsize) + align_up_256((size_t)s.batch * band_chunks(s) * sizeof(double));
}

int band_project(const gd_grid *g, double tau, const void *ubar, void *u0, void *work, size_t wb, void *stream) {
    int rc = validate_spec_grid(g);
    if (rc) return rc;
    if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(GD_EINVAL, "tau must be finite and >= 0");
    if (!ubar || !u0) return fail(GD_EINVAL, "ubar and u0 must be non-NULL");
    if (!work) return fail(GD_EWORKSPACE, "workspace is NULL");
    if ((uintptr_t)work % 256) return fail(GD_EALIGN, "workspace must be 256-byte aligned");
    const size_t need = band_project_workspace_bytes(g);
    if (wb < need) return fail(GD_EWORKSPACE, "workspace too small: need %zu bytes, got %zu", need, wb);
    const Spec s = spec_of(g);
    const size_t fb = (size_t)s.batch * s.nx * s.ny * s.nz * s.tsize;
    if (gd::ranges_overlap(ubar, fb, u0, fb)) return fail(GD_EINVAL, "ubar and u0 overlap");
    if (gd::ranges_overlap(ubar, fb, work, need) || gd::ranges_overlap(u0, fb, work, need))
        return fail(GD_EINVAL, "a field overlaps the workspace");
    hipStream_t st = (hipStream_t)stream;
    if (g->dtype == GD_F32)
        return band_project_run<float>(s, tau, (const float *)ubar, (float *)u0, (char *)work, st);
    return band_project_run<double>(s, tau, (const double *)ubar, (double *)u0, (char *)work, st);
}

int pdf_counts(const gd_grid *g, double lo, double hi, int32_t nbins, const void *x, int64_t *counts, void *stream) {
    int rc = gd::validate_grid(g);
    if (rc) return rc;
    if (!(lo < hi) || !std::isfinite(lo) || !std::isfinite(hi)) return fail(GD_EINVAL, "need finite lo < hi");
    if (nbins < 1 || nbins > kMaxPdfBins) return fail(GD_EINVAL, "nbins must be in [1, %d]", kMaxPdfBins);
    if (!x || !counts) return fail(GD_EINVAL, "x and counts must be non-NULL");
    const int64_t npts = g->n[0] * g->n[1] * (g->ndim == 3 ? g->n[2] : 1);
    const size_t tsize = g->dtype == GD_F32 ? 4 : 8;
    if (gd::ranges_overlap(x, (size_t)g->batch * npts * tsize, counts, (size_t)g->batch * nbins * 8))
        return fail(GD_EINVAL, "counts overlaps x");
    hipStream_t st = (hipStream_t)stream;
    const int64_t nc = g->batch * nbins;
    hipLaunchKernelGGL(k_zero_i64, dim3(stride_blocks(nc)), dim3(256), 0, st, counts, nc);
    const int64_t chunk = std::max<int64_t>(4096, (npts * g->batch + 2047) / 2048);
    const int64_t nch = (npts + chunk - 1) / chunk;
    const double scale = (double)nbins / (hi - lo);
    const dim3 grid((unsigned)(g->batch * nch));
    if (g->dtype == GD_F32)
        hipLaunchKernelGGL(k_pdf<float>, grid, dim3(256), nbins * sizeof(unsigned), st, (const float *)x, counts, npts,
                           chunk, nch, lo, hi, scale, nbins);
    else
        hipLaunchKernelGGL(k_pdf<double>, grid, dim3(256), nbins * sizeof(unsigned), st, (const double *)x, counts,
                           npts, chunk, nch, lo, hi, scale, nbins);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GD_OK : fail(GD_EHIP, "pdf launch: %s", hipGetErrorString(e));
}

}  // extern "C"
