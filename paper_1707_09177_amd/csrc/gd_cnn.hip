// gd_cnn.hip -- learned warm start for the deconvolution solve: a small
// periodic convolutional network u0 = ubar + s * f(ubar / s), trained on
// (ubar = G u, u) pairs, whose output starts a solver with GD_INIT_GIVEN.
//
// The paper starts every iteration from u0 = ubar (Algorithms 1-4); the
// network only replaces that starting point, the solve itself is unchanged.
//
// Network (2D): 6 layers of periodic 3x3 cross-correlation with bias,
// 1 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1 channels, ReLU after every layer but the
// last, then the deconvolution filter G itself, u0 = ubar + s * G z: the
// correction stays in the range of G like the paper's start u0 = ubar, so it
// adds nothing where G's transfer function vanishes (where the Krylov solvers
// are slowest); s is the per-sample RMS of ubar.  Weights of layer l are
// W[cout][tap][cin] (tap = 3 (dy + 1) + (dx + 1)) followed by bias[cout], all
// layers packed into one FP32 parameter vector.
//
// Data layout: activations are bfloat16, channels fastest (NHWC, 64 bytes per
// point).  The four 32 -> 32 layers run as implicit GEMMs on the matrix cores
// (v_mfma_f32_32x32x16_bf16: 32 points x 32 output channels per wave, K = 9
// taps x 32 input channels = 18 MFMA steps, FP32 accumulation); the input tile
// with its periodic halo sits in LDS and the layer's weights in registers.
// Their input gradients reuse the same kernel with transposed, tap-flipped
// weights.  The 1 -> 32 and 32 -> 1 layers (288 multiply-adds per point) and
// the weight gradients of the end layers use plain FP32 arithmetic; the
// 32 -> 32 weight gradients run on the matrix cores too.  Weight gradients are
// reduced deterministically (per-block partial sums added in a fixed order).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "gdecon.h"

namespace gd {
void set_error_text(const char *msg);
}

namespace gdcnn {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int C = 32;           // channels
constexpr int NL = 6;           // layers
constexpr int K = 9 * C;        // reduction length of a 32 -> 32 layer
constexpr int NMID = NL - 2;    // 32 -> 32 layers
constexpr int TY = 8, TX = 32;  // conv tile: 8 rows x 32 points (one MFMA M-tile per row)
constexpr int PSTR = 40;        // LDS stride of one point (32 channels + 8 pad) in bf16
constexpr int WGY = 8, WGX = 32;  // weight-gradient tile
constexpr int NW_MID = C * K + C;  // weights + biases of a 32 -> 32 layer
constexpr int NW_END = K + C;      // either end layer's weights (288) + up to 32 biases
constexpr int RMS_CHUNKS = 64;

struct Offsets {
    int64_t W[NL], b[NL], total;
};

Offsets offsets() {
    Offsets o;
    int64_t off = 0;
    for (int l = 0; l < NL; ++l) {
        const int ci = l == 0 ? 1 : C, co = l == NL - 1 ? 1 : C;
        o.W[l] = off;
        off += (int64_t)co * 9 * ci;
        o.b[l] = off;
        off += co;
    }
    o.total = off;
    return o;
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ---------------------------------------------------------------- small kernels

__global__ void k_cvt(const float *p, bf16 *q, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) q[i] = (bf16)p[i];
}

// Input-gradient weights of the 32 -> 32 layers: WT[m][cin][t][cout] =
// W[m][cout][8 - t][cin] (tap 8 - t is the mirrored offset of tap t).
__global__ void k_transpose(const bf16 *wbf, int64_t off_w1, int64_t layer_stride, bf16 *wT) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)NMID * C * K) return;
    const int m = (int)(i / (C * K));
    const int r = (int)(i % (C * K));
    const int cin = r / K, t = (r % K) / C, cout = r % C;
    wT[i] = wbf[off_w1 + m * layer_stride + ((int64_t)cout * 9 + (8 - t)) * C + cin];
}

template <typename T>
__global__ void k_rms_part(const T *ub, int64_t P, double *part) {
    __shared__ double red[256];
    const int b = blockIdx.y, chunk = blockIdx.x;
    const int64_t lo = P * chunk / RMS_CHUNKS, hi = P * (chunk + 1) / RMS_CHUNKS;
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const double v = (double)ub[(int64_t)b * P + i];
        acc += v * v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)b * RMS_CHUNKS + chunk] = red[0];
}

__global__ void k_rms_fin(const double *part, int B, int64_t P, double *s) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double acc = 0.0;
    for (int k = 0; k < RMS_CHUNKS; ++k) acc += part[(int64_t)b * RMS_CHUNKS + k];
    const double r = sqrt(acc / (double)P);
    s[b] = r > 0.0 ? r : 1.0;
}

// layer 1: one input channel (ubar / s, FP32) -> 32 channels, ReLU
template <typename T>
__global__ void k_conv_in(const T *ub, const double *s, const bf16 *w1, const float *b1, bf16 *out, int H, int W,
                          int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t HW = (int64_t)H * W;
    const int64_t b = p / HW;
    const int rem = (int)(p % HW), y = rem / W, x = rem % W;
    const float inv = (float)(1.0 / s[b]);
    float xv[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = wrap(y + t / 3 - 1, H), xx = wrap(x + t % 3 - 1, W);
        xv[t] = (float)ub[b * HW + (int64_t)yy * W + xx] * inv;
    }
    alignas(16) bf16 o[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float acc = b1[c];
#pragma unroll
        for (int t = 0; t < 9; ++t) acc += (float)w1[c * 9 + t] * xv[t];
        o[c] = (bf16)fmaxf(acc, 0.0f);
    }
    uint4 *dst = reinterpret_cast<uint4 *>(out + p * C);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = reinterpret_cast<const uint4 *>(o)[q];
}

// 32 -> 32 layer on the matrix cores.  Forward: out = relu(conv(in) + bias).
// Input gradient (BWD): out = conv'(in) * (mask > 0), where `in` holds the
// output gradient, `wmat` the transposed weights and `mask` the layer's input
// activation.  wmat: [cout][K] with K = tap * 32 + cin.
template <bool BWD>
__global__ __launch_bounds__(256) void k_conv_mid(const bf16 *in, const bf16 *wmat, const float *bias, const bf16 *mask,
                                                  bf16 *out, int H, int W, int tiles_x, int tiles_y) {
    __shared__ __attribute__((aligned(16))) bf16 tile[(TY + 2) * (TX + 2) * PSTR];
    const int blk = blockIdx.x;
    const int tx = blk % tiles_x, ty = (blk / tiles_x) % tiles_y;
    const int64_t b = blk / (tiles_x * tiles_y);
    const int x0 = tx * TX, y0 = ty * TY;
    const int64_t HW = (int64_t)H * W;
    const bf16 *inb = in + b * HW * C;
    const int tid = threadIdx.x;
    // tile with a one-point periodic halo, 16-byte chunks of 8 channels
    for (int q = tid; q < (TY + 2) * (TX + 2) * 4; q += 256) {
        const int pix = q >> 2, part = q & 3;
        const int r = pix / (TX + 2), c = pix % (TX + 2);
        const int gy = (int)((y0 + r - 1 + (int64_t)H) % H), gx = (int)((x0 + c - 1 + (int64_t)W) % W);
        *reinterpret_cast<uint4 *>(tile + pix * PSTR + part * 8) =
            *reinterpret_cast<const uint4 *>(inb + ((int64_t)gy * W + gx) * C + part * 8);
    }
    const int lane = tid & 63, wave = tid >> 6;
    const int j = lane & 31, kh = lane >> 5;
    bf16x8 Bf[K / 16];
#pragma unroll
    for (int ks = 0; ks < K / 16; ++ks) Bf[ks] = *reinterpret_cast<const bf16x8 *>(wmat + j * K + ks * 16 + kh * 8);
    float bj = 0.0f;
    if constexpr (!BWD) bj = bias[j];
    __syncthreads();
    for (int rr = wave; rr < TY; rr += 4) {
        f32x16 acc = {};
#pragma unroll
        for (int ks = 0; ks < K / 16; ++ks) {
            const int t = ks >> 1, dy = t / 3, dx = t % 3;
            const int pix = (rr + dy) * (TX + 2) + (j + dx);
            const bf16x8 A = *reinterpret_cast<const bf16x8 *>(tile + pix * PSTR + (ks & 1) * 16 + kh * 8);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, Bf[ks], acc, 0, 0, 0);
        }
        const int y = y0 + rr;
        if (y >= H) continue;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int i = 8 * (v >> 2) + 4 * kh + (v & 3);
            const int x = x0 + i;
            if (x >= W) continue;
            const int64_t idx = ((b * H + y) * (int64_t)W + x) * C + j;
            float val = acc[v];
            if constexpr (BWD) val = (float)mask[idx] > 0.0f ? val : 0.0f;
            else val = fmaxf(val + bj, 0.0f);
            out[idx] = (bf16)val;
        }
    }
}

// layer 6: 32 channels -> 1, no activation: z
__global__ void k_conv_out(const bf16 *a, const bf16 *w6, const float *b6, float *z, int H, int W, int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t HW = (int64_t)H * W;
    const int64_t b = p / HW;
    const int rem = (int)(p % HW), y = rem / W, x = rem % W;
    float acc = b6[0];
    for (int t = 0; t < 9; ++t) {
        const int yy = wrap(y + t / 3 - 1, H), xx = wrap(x + t % 3 - 1, W);
        const uint4 *src = reinterpret_cast<const uint4 *>(a + (b * HW + (int64_t)yy * W + xx) * C);
        alignas(16) bf16 v[C];
#pragma unroll
        for (int q = 0; q < 4; ++q) reinterpret_cast<uint4 *>(v)[q] = src[q];
#pragma unroll
        for (int c = 0; c < C; ++c) acc += (float)v[c] * (float)w6[t * C + c];
    }
    z[p] = acc;
}

// out = G in: the periodic trapezoidal filter (1/4, 1/2, 1/4) per axis
__device__ __forceinline__ float g_apply(const float *in, int64_t base, int y, int x, int H, int W) {
    const int ym = wrap(y - 1, H), yp = wrap(y + 1, H), xm = wrap(x - 1, W), xp = wrap(x + 1, W);
    auto row = [&](int yy) {
        const float *r = in + base + (int64_t)yy * W;
        return 0.5f * r[x] + 0.25f * (r[xm] + r[xp]);
    };
    return 0.5f * row(y) + 0.25f * (row(ym) + row(yp));
}

// y = G z; writes y (training) and/or u0 = ubar + s * y
template <typename T>
__global__ void k_gfin(const float *z, const T *ub, const double *s, float *y_out, T *u0, int H, int W, int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t HW = (int64_t)H * W;
    const int64_t b = p / HW;
    const int rem = (int)(p % HW), y = rem / W, x = rem % W;
    const float v = g_apply(z, b * HW, y, x, H, W);
    if (y_out) y_out[p] = v;
    if (u0) u0[p] = ub[p] + (T)(s[b] * (double)v);
}

// out = G in (the adjoint of the final filter: G is symmetric)
__global__ void k_gfilt(const float *in, float *out, int H, int W, int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t HW = (int64_t)H * W;
    const int64_t b = p / HW;
    const int rem = (int)(p % HW), y = rem / W, x = rem % W;
    out[p] = g_apply(in, b * HW, y, x, H, W);
}

// dL/dy = 2 (y - t) / N with t = (u - ubar) / s; per-block partial sums of (y - t)^2
template <typename T>
__global__ void k_loss(const float *yv, const T *ub, const T *u, const double *s, float *dy, double *part, int64_t HW,
                       int64_t N) {
    __shared__ double red[256];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double r2 = 0.0;
    if (p < N) {
        const int64_t b = p / HW;
        const double t = ((double)u[p] - (double)ub[p]) / s[b];
        const double r = (double)yv[p] - t;
        dy[p] = (float)(2.0 * r / (double)N);
        r2 = r * r;
    }
    red[threadIdx.x] = r2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_loss_fin(const double *part, int64_t nblk, int64_t N, double *loss) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < nblk; k += blockDim.x) acc += part[k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] / (double)N;
}

// input gradient of layer 6 through the ReLU of layer 5:
// dz5[p][c] = (sum_t W6[t][c] dy[p - off(t)]) * (a5[p][c] > 0)
__global__ void k_out_bwd(const float *dy, const bf16 *w6, const bf16 *a5, bf16 *dz, int H, int W, int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t HW = (int64_t)H * W;
    const int64_t b = p / HW;
    const int rem = (int)(p % HW), y = rem / W, x = rem % W;
    float g[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int yy = wrap(y - (t / 3 - 1), H), xx = wrap(x - (t % 3 - 1), W);
        g[t] = dy[b * HW + (int64_t)yy * W + xx];
    }
    alignas(16) bf16 m[C], o[C];
#pragma unroll
    for (int q = 0; q < 4; ++q) reinterpret_cast<uint4 *>(m)[q] = reinterpret_cast<const uint4 *>(a5 + p * C)[q];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float acc = 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) acc += (float)w6[t * C + c] * g[t];
        o[c] = (bf16)((float)m[c] > 0.0f ? acc : 0.0f);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) reinterpret_cast<uint4 *>(dz + p * C)[q] = reinterpret_cast<const uint4 *>(o)[q];
}

// Weight gradient of one layer over the points of this block's tiles:
// dW[o][t][c] = sum_p g[p][o] x[p + off(t)][c], db[o] = sum_p g[p][o].
// x: CI channels (32: bf16 activations; 1: ubar / s); g: CO channels
// (32: bf16 gradients; 1: FP32 dL/dy).  part[block][CO*9*CI + CO].
template <int CI, int CO, typename T>
__global__ __launch_bounds__(256) void k_wgrad(const bf16 *xa, const T *ub, const double *s, const bf16 *ga,
                                               const float *gf, float *part, int H, int W, int tiles_x, int tiles_y,
                                               int64_t ntiles) {
    constexpr int NWL = CO * 9 * CI + CO;
    constexpr int SLOTS = (NWL + 255) / 256;
    __shared__ float xs[(WGY + 2) * (WGX + 2) * CI];
    __shared__ float gs[WGY * WGX * CO];
    const int tid = threadIdx.x;
    float acc[SLOTS];
#pragma unroll
    for (int k = 0; k < SLOTS; ++k) acc[k] = 0.0f;
    const int64_t HW = (int64_t)H * W;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int tx = (int)(tile % tiles_x), ty = (int)((tile / tiles_x) % tiles_y);
        const int64_t b = tile / ((int64_t)tiles_x * tiles_y);
        const int x0 = tx * WGX, y0 = ty * WGY;
        for (int q = tid; q < (WGY + 2) * (WGX + 2) * CI; q += 256) {
            const int pix = q / CI, c = q % CI;
            const int r = pix / (WGX + 2), cc = pix % (WGX + 2);
            const int gy = (int)((y0 + r - 1 + (int64_t)H) % H), gx = (int)((x0 + cc - 1 + (int64_t)W) % W);
            const int64_t g = b * HW + (int64_t)gy * W + gx;
            float v;
            if constexpr (CI == 1) v = (float)ub[g] * (float)(1.0 / s[b]);
            else v = (float)xa[g * CI + c];
            xs[q] = v;
        }
        for (int q = tid; q < WGY * WGX * CO; q += 256) {
            const int pix = q / CO, o = q % CO;
            const int y = y0 + pix / WGX, x = x0 + pix % WGX;
            float v = 0.0f;  // points outside the field contribute nothing
            if (y < H && x < W) {
                const int64_t g = b * HW + (int64_t)y * W + x;
                if constexpr (CO == 1) v = gf[g];
                else v = (float)ga[g * CO + o];
            }
            gs[q] = v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SLOTS; ++k) {
            const int idx = tid + k * 256;
            if (idx < CO * 9 * CI) {
                const int o = idx / (9 * CI), t = (idx / CI) % 9, c = idx % CI;
                const int dy = t / 3, dx = t % 3;
                float a = 0.0f;
                for (int p = 0; p < WGY * WGX; ++p) {
                    const int py = p / WGX, px = p % WGX;
                    a += gs[p * CO + o] * xs[((py + dy) * (WGX + 2) + (px + dx)) * CI + c];
                }
                acc[k] += a;
            } else if (idx < NWL) {
                const int o = idx - CO * 9 * CI;
                float a = 0.0f;
                for (int p = 0; p < WGY * WGX; ++p) a += gs[p * CO + o];
                acc[k] += a;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < SLOTS; ++k) {
        const int idx = tid + k * 256;
        if (idx < NWL) part[(int64_t)blockIdx.x * NWL + idx] = acc[k];
    }
}

// Weight gradient of a 32 -> 32 layer on the matrix cores: for every tap t the
// 32 x 32 block dW[o][t][c] = sum_p g[p][o] x[p + off(t)][c] is a GEMM with
// K = points (16 per MFMA step).  LDS holds the tile's output gradient
// transposed, gT[o][p], and three transposed copies of the input tile with its
// halo, shifted by dx = 0, 1, 2 (xs[dx][c][row][j] = x[row][j + dx]), so every
// 8-point operand is one aligned 16-byte read.  Wave w owns taps w, w+4, w+8.
// Also the bias gradient db[o] = sum_p g[p][o].  part[block][32 * 288 + 32].
__global__ __launch_bounds__(256) void k_wgrad_mid(const bf16 *xa, const bf16 *ga, float *part, int H, int W,
                                                   int tiles_x, int tiles_y, int64_t ntiles) {
    constexpr int NP = WGY * WGX;        // points per tile
    constexpr int XR = WGY + 2;          // input rows with the halo
    constexpr int GST = NP + 8;          // padded row of gT (bf16)
    constexpr int XST = XR * WGX + 8;    // padded channel plane of an xs copy (bf16)
    constexpr int NWL = C * K + C;
    __shared__ __attribute__((aligned(16))) bf16 gT[C * GST];
    __shared__ __attribute__((aligned(16))) bf16 xs[3 * C * XST];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = lane & 31, kh = lane >> 5;
    f32x16 acc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) acc[q] = f32x16{};
    float db = 0.0f;
    const int64_t HW = (int64_t)H * W;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int tx = (int)(tile % tiles_x), ty = (int)((tile / tiles_x) % tiles_y);
        const int64_t b = tile / ((int64_t)tiles_x * tiles_y);
        const int x0 = tx * WGX, y0 = ty * WGY;
        for (int q = tid; q < NP * C; q += 256) {
            const int p = q / C, o = q % C;
            const int y = y0 + p / WGX, x = x0 + p % WGX;
            bf16 v = (bf16)0.0f;  // points outside the field contribute nothing
            if (y < H && x < W) v = ga[(b * HW + (int64_t)y * W + x) * C + o];
            gT[o * GST + p] = v;
        }
        for (int q = tid; q < XR * (WGX + 2) * C; q += 256) {
            const int pix = q / C, c = q % C;
            const int r = pix / (WGX + 2), col = pix % (WGX + 2);
            const int gy = (int)((y0 + r - 1 + (int64_t)H) % H), gx = (int)((x0 + col - 1 + (int64_t)W) % W);
            const bf16 v = xa[(b * HW + (int64_t)gy * W + gx) * C + c];
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int jc = col - dx;
                if (jc >= 0 && jc < WGX) xs[(dx * C + c) * XST + r * WGX + jc] = v;
            }
        }
        __syncthreads();
        if (tid < C)
            for (int p = 0; p < NP; ++p) db += (float)gT[tid * GST + p];
#pragma unroll 2
        for (int ks = 0; ks < NP / 16; ++ks) {
            const int p0 = ks * 16, py = p0 / WGX, px0 = p0 % WGX;
            const bf16x8 A = *reinterpret_cast<const bf16x8 *>(gT + j * GST + p0 + kh * 8);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int t = wave + 4 * q;
                if (t < 9) {
                    const int dy = t / 3, dx = t % 3;
                    const bf16x8 Bv =
                        *reinterpret_cast<const bf16x8 *>(xs + (dx * C + j) * XST + (py + dy) * WGX + px0 + kh * 8);
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, Bv, acc[q], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    float *pb = part + (int64_t)blockIdx.x * NWL;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int t = wave + 4 * q;
        if (t < 9)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int o = 8 * (v >> 2) + 4 * kh + (v & 3);
                pb[(o * 9 + t) * C + j] = acc[q][v];
            }
    }
    if (tid < C) pb[C * K + tid] = db;
}

// grad[w] = sum over blocks (in block order) of part[block][w]; the layer's
// weights and biases are consecutive in the parameter vector.
__global__ void k_reduce(const float *part, int nblk, int nw, float *grad) {
    // 32 weights per workgroup, 8 lanes per weight summing every 8th block,
    // then the 8 lane sums in lane order: a fixed order for every run
    __shared__ double red[8][32];
    const int wl = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int i = blockIdx.x * 32 + wl;
    double acc = 0.0;
    if (i < nw)
        for (int k = g; k < nblk; k += 8) acc += (double)part[(int64_t)k * nw + i];
    red[g][wl] = acc;
    __syncthreads();
    if (g == 0 && i < nw) {
        double t = 0.0;
        for (int q = 0; q < 8; ++q) t += red[q][wl];
        grad[i] = (float)t;
    }
}

__global__ void k_adam(float *p, float *m, float *v, const float *g, int64_t n, const int32_t *step, float lr, float b1,
                       float b2, float eps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = step[0] + 1;
    const float bc1 = (float)(1.0 - pow((double)b1, (double)t));
    const float bc2 = (float)(1.0 - pow((double)b2, (double)t));
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ void k_step_inc(int32_t *step) {
    if (blockIdx.x == 0 && threadIdx.x == 0) step[0] = step[0] + 1;
}

// ---------------------------------------------------------------- host side

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    gd::set_error_text(buf);
    return code;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Layout {
    size_t wbf, wT, s, rms, act, z, y, dy, dyz, dz, lpart, wpart, grad, total;
    int64_t N, nblk_pix;
    int nblk_w;
};

int64_t wgrad_tiles(const gd_grid *g) {
    return g->batch * ((g->n[1] + WGY - 1) / WGY) * ((g->n[0] + WGX - 1) / WGX);
}

Layout layout(const gd_grid *g, bool training, bool own_grad) {
    const Offsets off = offsets();
    Layout L;
    std::memset(&L, 0, sizeof L);
    L.N = g->batch * g->n[0] * g->n[1];
    L.nblk_pix = (L.N + 255) / 256;
    L.nblk_w = (int)std::min<int64_t>(wgrad_tiles(g), 512);
    size_t o = 0;
    L.wbf = o;
    o = align_up(o + (size_t)off.total * 2, 256);
    L.wT = o;
    if (training) o = align_up(o + (size_t)NMID * C * K * 2, 256);
    L.s = o;
    o = align_up(o + (size_t)g->batch * 8, 256);
    L.rms = o;
    o = align_up(o + (size_t)g->batch * RMS_CHUNKS * 8, 256);
    L.act = o;
    const size_t actb = align_up((size_t)L.N * C * 2, 256);
    o += (training ? NL - 1 : 2) * actb;
    L.z = o;
    o = align_up(o + (size_t)L.N * 4, 256);
    if (training) {
        L.y = o;
        o = align_up(o + (size_t)L.N * 4, 256);
        L.dy = o;
        o = align_up(o + (size_t)L.N * 4, 256);
        L.dyz = o;
        o = align_up(o + (size_t)L.N * 4, 256);
        L.dz = o;
        o += 2 * actb;
        L.lpart = o;
        o = align_up(o + (size_t)L.nblk_pix * 8, 256);
        L.wpart = o;
        o = align_up(o + (size_t)L.nblk_w * NW_MID * 4, 256);
        if (own_grad) {
            L.grad = o;
            o = align_up(o + (size_t)off.total * 4, 256);
        }
    }
    L.total = o;
    return L;
}

int check_net(const gd_cnn *net, bool training) {
    if (!net) return fail(GD_EINVAL, "network is NULL");
    if (net->ndim != 2) return fail(GD_EINVAL, "only the 2D network is built (ndim %d)", net->ndim);
    if (net->channels != C || net->layers != NL)
        return fail(GD_EINVAL, "the network has %d layers of %d channels", NL, C);
    if (!net->params) return fail(GD_EINVAL, "params is NULL");
    if (training && (!net->adam_m || !net->adam_v || !net->step))
        return fail(GD_EINVAL, "training needs adam_m, adam_v and step");
    return GD_OK;
}

int check_grid(const gd_grid *g) {
    if (!g) return fail(GD_EINVAL, "grid is NULL");
    if (g->ndim != 2) return fail(GD_EINVAL, "the warm start is built for 2D fields only");
    if (g->dtype != GD_F32 && g->dtype != GD_F64) return fail(GD_EINVAL, "dtype must be GD_F32 or GD_F64");
    if (g->n[0] < 1 || g->n[1] < 1 || g->batch < 1) return fail(GD_EINVAL, "sizes must be >= 1");
    if (g->n[0] * g->n[1] >= (int64_t(1) << 31) || g->n[0] * g->n[1] * g->batch > (int64_t(1) << 34) ||
        g->batch > 65535)
        return fail(GD_EINVAL, "field too large");
    return GD_OK;
}

#define GD_LAUNCH(...)                                                                   \
    do {                                                                                 \
        hipLaunchKernelGGL(__VA_ARGS__);                                                 \
        hipError_t e_ = hipGetLastError();                                               \
        if (e_ != hipSuccess) return fail(GD_EHIP, "launch: %s", hipGetErrorString(e_)); \
    } while (0)

// forward (train = false: u0 out; train = true: keep every activation and y)
template <typename T>
int run_forward(const gd_cnn *net, const gd_grid *g, const Layout &L, char *w, const T *ub, T *u0, bool train,
                hipStream_t st) {
    const Offsets off = offsets();
    const int H = (int)g->n[1], W = (int)g->n[0];
    const int64_t HW = (int64_t)H * W, N = L.N;
    bf16 *wbf = (bf16 *)(w + L.wbf);
    double *s = (double *)(w + L.s);
    const size_t actb = align_up((size_t)N * C * 2, 256);
    auto act = [&](int i) { return (bf16 *)(w + L.act + (size_t)i * actb); };
    const unsigned pblk = (unsigned)L.nblk_pix;
    GD_LAUNCH(k_cvt, dim3((unsigned)((off.total + 255) / 256)), dim3(256), 0, st, net->params, wbf, off.total);
    GD_LAUNCH(k_rms_part<T>, dim3(RMS_CHUNKS, (unsigned)g->batch), dim3(256), 0, st, ub, HW, (double *)(w + L.rms));
    GD_LAUNCH(k_rms_fin, dim3((unsigned)((g->batch + 63) / 64)), dim3(64), 0, st, (const double *)(w + L.rms),
              (int)g->batch, HW, s);
    GD_LAUNCH(k_conv_in<T>, dim3(pblk), dim3(256), 0, st, ub, s, wbf + off.W[0], net->params + off.b[0], act(0), H, W,
              N);
    const int tiles_x = (W + TX - 1) / TX, tiles_y = (H + TY - 1) / TY;
    const unsigned cblk = (unsigned)(g->batch * tiles_x * tiles_y);
    for (int m = 0; m < NMID; ++m) {
        const int l = m + 1;
        bf16 *src = train ? act(m) : act(m & 1);
        bf16 *dst = train ? act(m + 1) : act((m + 1) & 1);
        GD_LAUNCH(k_conv_mid<false>, dim3(cblk), dim3(256), 0, st, src, wbf + off.W[l], net->params + off.b[l],
                  (const bf16 *)nullptr, dst, H, W, tiles_x, tiles_y);
    }
    bf16 *last = train ? act(NL - 2) : act(NMID & 1);
    GD_LAUNCH(k_conv_out, dim3(pblk), dim3(256), 0, st, (const bf16 *)last, (const bf16 *)(wbf + off.W[NL - 1]),
              (const float *)(net->params + off.b[NL - 1]), (float *)(w + L.z), H, W, N);
    GD_LAUNCH(k_gfin<T>, dim3(pblk), dim3(256), 0, st, (const float *)(w + L.z), ub, (const double *)s,
              train ? (float *)(w + L.y) : (float *)nullptr, train ? (T *)nullptr : u0, H, W, N);
    return GD_OK;
}

template <int CI, int CO, typename T>
int wgrad_layer(const gd_grid *g, const Layout &L, char *w, const bf16 *xa, const T *ub, const double *s,
                const bf16 *ga, const float *gf, float *grad_layer, hipStream_t st) {
    constexpr int NWL = CO * 9 * CI + CO;
    const int H = (int)g->n[1], W = (int)g->n[0];
    const int tiles_x = (W + WGX - 1) / WGX, tiles_y = (H + WGY - 1) / WGY;
    const int64_t ntiles = wgrad_tiles(g);
    float *part = (float *)(w + L.wpart);
    if constexpr (CI == C && CO == C) {
        GD_LAUNCH(k_wgrad_mid, dim3((unsigned)L.nblk_w), dim3(256), 0, st, xa, ga, part, H, W, tiles_x, tiles_y,
                  ntiles);
    } else {
        auto kern = k_wgrad<CI, CO, T>;
        GD_LAUNCH(kern, dim3((unsigned)L.nblk_w), dim3(256), 0, st, xa, ub, s, ga, gf, part, H, W, tiles_x, tiles_y,
                  ntiles);
    }
    GD_LAUNCH(k_reduce, dim3((NWL + 31) / 32), dim3(256), 0, st, (const float *)part, L.nblk_w, NWL, grad_layer);
    return GD_OK;
}

template <typename T>
int run_train(const gd_cnn *net, const gd_grid *g, const Layout &L, char *w, const T *ub, const T *u, double *loss,
              hipStream_t st) {
    const Offsets off = offsets();
    int rc = run_forward<T>(net, g, L, w, ub, nullptr, true, st);
    if (rc) return rc;
    const int H = (int)g->n[1], W = (int)g->n[0];
    const int64_t HW = (int64_t)H * W, N = L.N;
    bf16 *wbf = (bf16 *)(w + L.wbf);
    bf16 *wT = (bf16 *)(w + L.wT);
    const double *s = (const double *)(w + L.s);
    const size_t actb = align_up((size_t)N * C * 2, 256);
    auto act = [&](int i) { return (bf16 *)(w + L.act + (size_t)i * actb); };
    auto dz = [&](int i) { return (bf16 *)(w + L.dz + (size_t)(i & 1) * actb); };
    float *grad = net->grad ? net->grad : (float *)(w + L.grad);
    float *dy = (float *)(w + L.dy);
    const unsigned pblk = (unsigned)L.nblk_pix;
    GD_LAUNCH(k_transpose, dim3((unsigned)((NMID * C * K + 255) / 256)), dim3(256), 0, st, (const bf16 *)wbf, off.W[1],
              off.W[2] - off.W[1], wT);
    GD_LAUNCH(k_loss<T>, dim3(pblk), dim3(256), 0, st, (const float *)(w + L.y), ub, u, s, dy,
              (double *)(w + L.lpart), HW, N);
    GD_LAUNCH(k_loss_fin, dim3(1), dim3(256), 0, st, (const double *)(w + L.lpart), L.nblk_pix, N, loss);
    // through the final filter: dL/dz = G dL/dy
    float *dyz = (float *)(w + L.dyz);
    GD_LAUNCH(k_gfilt, dim3(pblk), dim3(256), 0, st, (const float *)dy, dyz, H, W, N);
    // layer 6
    if ((rc = wgrad_layer<C, 1, T>(g, L, w, act(NL - 2), ub, s, nullptr, dyz, grad + off.W[NL - 1], st))) return rc;
    GD_LAUNCH(k_out_bwd, dim3(pblk), dim3(256), 0, st, (const float *)dyz, (const bf16 *)(wbf + off.W[NL - 1]),
              (const bf16 *)act(NL - 2), dz(0), H, W, N);
    // layers 5 .. 2: dz(k) holds the gradient at the output of layer l
    const int tiles_x = (W + TX - 1) / TX, tiles_y = (H + TY - 1) / TY;
    const unsigned cblk = (unsigned)(g->batch * tiles_x * tiles_y);
    int k = 0;
    for (int l = NL - 2; l >= 1; --l, ++k) {
        const bf16 *xin = act(l - 1);  // input activation of layer l
        if ((rc = wgrad_layer<C, C, T>(g, L, w, xin, ub, s, dz(k), nullptr, grad + off.W[l], st))) return rc;
        GD_LAUNCH(k_conv_mid<true>, dim3(cblk), dim3(256), 0, st, (const bf16 *)dz(k),
                  (const bf16 *)(wT + (size_t)(l - 1) * C * K), (const float *)nullptr, xin, dz(k + 1), H, W, tiles_x,
                  tiles_y);
    }
    // layer 1 (input x0 = ubar / s)
    if ((rc = wgrad_layer<1, C, T>(g, L, w, nullptr, ub, s, dz(k), nullptr, grad + off.W[0], st))) return rc;
    GD_LAUNCH(k_adam, dim3((unsigned)((off.total + 255) / 256)), dim3(256), 0, st, net->params, net->adam_m,
              net->adam_v, (const float *)grad, off.total, (const int32_t *)net->step, net->lr, net->beta1, net->beta2,
              net->eps);
    GD_LAUNCH(k_step_inc, dim3(1), dim3(64), 0, st, net->step);
    return GD_OK;
}

}  // namespace gdcnn

using namespace gdcnn;

extern "C" {

int64_t warmstart_param_count(const gd_cnn *net) {
    if (!net || net->ndim != 2 || net->channels != C || net->layers != NL) return 0;
    return offsets().total;
}

size_t warmstart_workspace_bytes(const gd_cnn *net, const gd_grid *g, int32_t training) {
    if (check_net(net, false) || check_grid(g)) return 0;
    return layout(g, training != 0, !net->grad).total;
}

int warmstart_forward(const gd_cnn *net, const gd_grid *g, const void *ubar, void *u0, void *work, size_t work_bytes,
                      void *stream) {
    int rc = check_net(net, false);
    if (rc) return rc;
    if ((rc = check_grid(g))) return rc;
    if (!ubar || !u0) return fail(GD_EINVAL, "ubar and u0 must be non-NULL");
    if (ubar == u0) return fail(GD_EINVAL, "ubar and u0 must differ");
    if (!work) return fail(GD_EWORKSPACE, "workspace is NULL");
    if ((uintptr_t)work % 256) return fail(GD_EALIGN, "workspace must be 256-byte aligned");
    const Layout L = layout(g, false, false);
    if (work_bytes < L.total) return fail(GD_EWORKSPACE, "workspace too small: need %zu bytes", L.total);
    hipStream_t st = (hipStream_t)stream;
    if (g->dtype == GD_F32)
        return run_forward<float>(net, g, L, (char *)work, (const float *)ubar, (float *)u0, false, st);
    return run_forward<double>(net, g, L, (char *)work, (const double *)ubar, (double *)u0, false, st);
}

int warmstart_train_step(const gd_cnn *net, const gd_grid *g, const void *ubar, const void *u, void *work,
                         size_t work_bytes, double *loss, void *stream) {
    int rc = check_net(net, true);
    if (rc) return rc;
    if ((rc = check_grid(g))) return rc;
    if (!ubar || !u || !loss) return fail(GD_EINVAL, "ubar, u and loss must be non-NULL");
    if (!work) return fail(GD_EWORKSPACE, "workspace is NULL");
    if ((uintptr_t)work % 256) return fail(GD_EALIGN, "workspace must be 256-byte aligned");
    const Layout L = layout(g, true, !net->grad);
    if (work_bytes < L.total) return fail(GD_EWORKSPACE, "workspace too small: need %zu bytes", L.total);
    hipStream_t st = (hipStream_t)stream;
    if (g->dtype == GD_F32)
        return run_train<float>(net, g, L, (char *)work, (const float *)ubar, (const float *)u, loss, st);
    return run_train<double>(net, g, L, (char *)work, (const double *)ubar, (const double *)u, loss, st);
}

}  // extern "C"
