// gd_cnn.hip -- learned warm start for the deconvolution solve: a small
// periodic convolutional network u0 = ubar + s * f(ubar / s), trained on
// (ubar = G u, u) pairs, whose output starts a solver with GD_INIT_GIVEN.
//
// The paper starts every iteration from u0 = ubar (Algorithms 1-4); the
// network only replaces that starting point, the solve itself is unchanged.
//
// Network: 6 layers of periodic 3x3 (2D) or 3x3x3 (3D) cross-correlation with
// bias, 1 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1 channels, ReLU after every layer
// but the last, then the deconvolution filter G itself, u0 = ubar + s * G z: the
// correction stays in the range of G like the paper's start u0 = ubar, so it
// adds nothing where G's transfer function vanishes (where the Krylov solvers
// are slowest); s is the per-sample RMS of ubar.  Weights of layer l are
// W[cout][tap][cin] (tap = 3 (dy + 1) + (dx + 1), in 3D 9 (dz + 1) + ...)
// followed by bias[cout], all layers packed into one FP32 parameter vector.
//
// A 3D field is a stack of nz planes and a 3D convolution is the sum of three
// 2D convolutions of the planes shifted by dz = -1, 0, +1, each with its own
// 3x3 slice of the weights: the 3D matrix-core kernel stages the three
// planes' tiles in LDS and runs the three 2D products one weight slice at a
// time into the same registers, then writes bf16 (bias and ReLU, or the ReLU
// mask) once.
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
int64_t checked_points(const int64_t *n, int ndim, int64_t cap);
}

namespace gdcnn {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int C = 32;           // channels
constexpr int K9 = 9 * C;       // reduction length of one 3x3 slice
constexpr int NL = 6;           // layers
constexpr int K = K9;           // reduction length of a 2D 32 -> 32 layer (one MFMA pass)
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

// parameter offsets for NT taps per layer (9 in 2D, 27 in 3D)
Offsets offsets(int NT) {
    Offsets o;
    int64_t off = 0;
    for (int l = 0; l < NL; ++l) {
        const int ci = l == 0 ? 1 : C, co = l == NL - 1 ? 1 : C;
        o.W[l] = off;
        off += (int64_t)co * NT * ci;
        o.b[l] = off;
        off += co;
    }
    o.total = off;
    return o;
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// plane pz = sample * nz + z shifted by dz planes within its sample (periodic)
__device__ __forceinline__ int64_t plane_shift(int64_t pz, int nz, int dz) {
    const int z = (int)(pz % nz);
    return pz - z + wrap(z + dz, nz);
}

// offsets of tap t of NT (9: 2D, 27: 3D)
template <int NT> __device__ __forceinline__ int tap_dz(int t) { return NT == 27 ? t / 9 - 1 : 0; }
__device__ __forceinline__ int tap_dy(int t) { return (t % 9) / 3 - 1; }
__device__ __forceinline__ int tap_dx(int t) { return t % 3 - 1; }

// ---------------------------------------------------------------- small kernels

__global__ void k_cvt(const float *p, bf16 *q, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) q[i] = (bf16)p[i];
}

// Per-dz 3x3 weight slices of the 32 -> 32 layers for the matrix-core kernel,
// out[m][dzi][row][t * 32 + col] (ndz = NT / 9 slices):
//   forward (BWD = false): row = cout, col = cin: W[m][cout][dzi * 9 + t][cin];
//   input gradient (BWD):  row = cin, col = cout: W[m][cout][NT - 1 - (dzi * 9 + t)][cin]
// (the mirrored tap: the input gradient correlates with the flipped kernel).
template <bool BWD>
__global__ void k_repack(const bf16 *wbf, int64_t off_w1, int64_t layer_stride, int NT, bf16 *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ndz = NT / 9;
    if (i >= (int64_t)NMID * ndz * C * K9) return;
    const int m = (int)(i / ((int64_t)ndz * C * K9));
    const int r = (int)(i % ((int64_t)ndz * C * K9));
    const int dzi = r / (C * K9), r2 = r % (C * K9);
    const int row = r2 / K9, t = (r2 % K9) / C, col = r2 % C;
    const int cout = BWD ? col : row, cin = BWD ? row : col;
    const int tap = BWD ? NT - 1 - (dzi * 9 + t) : dzi * 9 + t;
    out[i] = wbf[off_w1 + m * layer_stride + ((int64_t)cout * NT + tap) * C + cin];
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
template <typename T, int NT>
__global__ void k_conv_in(const T *ub, const double *s, const bf16 *w1, const float *b1, bf16 *out, int H, int W,
                          int nz, int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t HW = (int64_t)H * W;
    const int64_t pz = p / HW;
    const int rem = (int)(p % HW), y = rem / W, x = rem % W;
    const float inv = (float)(1.0 / s[pz / nz]);
    float xv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int yy = wrap(y + tap_dy(t), H), xx = wrap(x + tap_dx(t), W);
        xv[t] = (float)ub[plane_shift(pz, nz, tap_dz<NT>(t)) * HW + (int64_t)yy * W + xx] * inv;
    }
    alignas(16) bf16 o[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float acc = b1[c];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc += (float)w1[c * NT + t] * xv[t];
        o[c] = (bf16)fmaxf(acc, 0.0f);
    }
    uint4 *dst = reinterpret_cast<uint4 *>(out + p * C);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = reinterpret_cast<const uint4 *>(o)[q];
}

// 2D 32 -> 32 layer on the matrix cores.  wmat: [cout][K] with
// K = tap * 32 + cin.  MODE 0 (forward): out = relu(conv(in) + bias);
// MODE 1 (input gradient): out = conv'(in) * (mask > 0), with `in` the output
// gradient, `wmat` the transposed weights and `mask` the layer's input
// activation.
constexpr int kFwd = 0, kBwd = 1;
template <int MODE>
__global__ __launch_bounds__(256) void k_conv_mid(const bf16 *in, const bf16 *wmat, const float *bias, const bf16 *mask,
                                                  bf16 *out, int H, int W, int tiles_x, int tiles_y) {
    __shared__ __attribute__((aligned(16))) bf16 tile[(TY + 2) * (TX + 2) * PSTR];
    const int blk = blockIdx.x;
    const int tx = blk % tiles_x, ty = (blk / tiles_x) % tiles_y;
    const int64_t pz = blk / (tiles_x * tiles_y);  // output plane
    const int x0 = tx * TX, y0 = ty * TY;
    const int64_t HW = (int64_t)H * W;
    const bf16 *inb = in + pz * HW * C;
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
    if constexpr (MODE == kFwd) bj = bias[j];
    __syncthreads();
    for (int rr = wave; rr < TY; rr += 4) {
        f32x16 acc = {};
        bf16x8 Af[K / 16];  // every operand load issued before the first product
#pragma unroll
        for (int ks = 0; ks < K / 16; ++ks) {
            const int t = ks >> 1, dy = t / 3, dx = t % 3;
            const int pix = (rr + dy) * (TX + 2) + (j + dx);
            Af[ks] = *reinterpret_cast<const bf16x8 *>(tile + pix * PSTR + (ks & 1) * 16 + kh * 8);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ks = 0; ks < K / 16; ++ks) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Af[ks], Bf[ks], acc, 0, 0, 0);
        const int y = y0 + rr;
        if (y >= H) continue;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int i = 8 * (v >> 2) + 4 * kh + (v & 3);
            const int x = x0 + i;
            if (x >= W) continue;
            const int64_t idx = ((pz * H + y) * (int64_t)W + x) * C + j;
            float val = acc[v];
            if constexpr (MODE == kBwd) val = (float)mask[idx] > 0.0f ? val : 0.0f;
            else val = fmaxf(val + bj, 0.0f);
            out[idx] = (bf16)val;
        }
    }
}

// ---------------------------------------------------------------- fused 2D forward
//
// Inference in 2D runs all six layers in one kernel, so no activation goes
// through HBM.  A workgroup owns a strip of FV output columns and up to FY
// rows of one sample and marches down it.  Layer l keeps the rows of its
// input that its 3x3 taps need in an LDS ring (layers 2 .. 6; layer 1 reads
// ubar / s from a ring of its own); at step s layer l computes row
// ys + s - 2 (l - 1), two rows behind layer l - 1, so every input row a layer
// reads was written in an earlier step, and the row it writes goes to the
// fourth ring slot, which no layer reads in that step: one barrier per step.
// Columns: a frame of FW = 64 columns starting 5 left of the strip.  Layer l's
// row is needed on frame columns l - 1 .. FV + 10 - l, so with FV = 54 every
// layer computes the frame's 64 columns (two MFMA tiles for the 32 -> 32
// layers, one column per lane for layer 1) and layer 6 the strip's 54.
// A wave's work in a step has no branch (a layer outside its rows computes
// on stale ring rows and does not write), so the scheduler can interleave
// the matrix products with the vector work of layers 1 and 6.
constexpr int FW = 64, FV = FW - 10, FY = 256, FRC = FW + 2;  // frame, strip, rows per workgroup, ring columns
constexpr int FTHREADS = 512;
constexpr int RSL = 4;        // ring slots: three rows read, the fourth written in the same step
constexpr int RTR = RSL;      // a fifth slot per ring takes the rows of layers outside their rows
constexpr int URC = FRC;      // ubar ring columns: frame -1 .. FW
constexpr int URS = 64;       // ubar ring rows
constexpr int UBATCH = 16;    // ubar rows loaded together, every UBATCH steps
constexpr size_t kRingBytes = (size_t)(NL - 1) * (RSL + 1) * FRC * PSTR * sizeof(bf16);
constexpr size_t kFusedLds = kRingBytes + URS * URC * sizeof(float) + 2 * 8 * 64 * sizeof(float);
static_assert(kFusedLds <= 160 * 1024, "LDS of one CU");
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// max(x, 0) as one integer max on the bits (a negative float is a negative
// integer): fmaxf also quiets signalling NaNs, one more instruction per value
__device__ __forceinline__ float relu_bits(float x) {
    return __builtin_bit_cast(float, max(__builtin_bit_cast(int, x), 0));
}

// Workgroup barrier ordering LDS only: the fused kernel's threads share data
// through LDS alone, and a full barrier would also wait for the global loads
// it keeps in flight across steps.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename T>
__global__ __launch_bounds__(FTHREADS) void k_fwd2d_fused(const T *ub, const double *s, const bf16 *wbf,
                                                          const float *params, Offsets off, float *z, int H, int W) {
    extern __shared__ __attribute__((aligned(16))) unsigned char fused_lds[];
    bf16 *ring = reinterpret_cast<bf16 *>(fused_lds);                  // [layer 2..6][slot RSL][FRC][PSTR]
    float *uring = reinterpret_cast<float *>(fused_lds + kRingBytes);  // ubar / s: [row slot URS][URC]
    float *zpart = uring + URS * URC;  // layer 6 partial sums [step parity][wave][column]
    auto at = [&](int l, int slot, int col) { return ring + (((l - 2) * (RSL + 1) + slot) * FRC + col) * PSTR; };
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int b = blockIdx.z;
    const int x0 = blockIdx.x * FV, y0 = blockIdx.y * FY;
    const int rows = min(FY, H - y0);
    const int ys = y0 - 5;  // first row of layer 1's output
    const int64_t HW = (int64_t)H * W;
    const T *ubs = ub + (int64_t)b * HW;
    const float inv = (float)(1.0 / s[b]);
    // clear the rings once: ring columns 0 and FRC - 1 are never written and
    // feed only frame columns whose results are not needed
    for (int i = tid; i < (int)(kRingBytes / 16); i += FTHREADS) reinterpret_cast<uint4 *>(fused_lds)[i] = uint4{0, 0, 0, 0};

    // matrix-core role: wave w computes layer ML = 2 + w / 2, frame columns 32 (w % 2) ..
    const int ML = 2 + (wave >> 1), mh = wave & 1;
    const int j = lane & 31, kh = lane >> 5;
    bf16x8 Wf[K / 16];
    {
        const bf16 *wm = wbf + off.W[ML - 1];
#pragma unroll
        for (int ks = 0; ks < K / 16; ++ks) Wf[ks] = *reinterpret_cast<const bf16x8 *>(wm + j * K + ks * 16 + kh * 8);
    }
    f32x16 mb;  // biases of the output channels this lane holds: the accumulator's start
#pragma unroll
    for (int v = 0; v < 16; ++v) mb[v] = params[off.b[ML - 1] + 8 * (v >> 2) + 4 * kh + (v & 3)];
    // layers 1 and 6: wave w takes channels 4w .. 4w + 3, so their weights are
    // uniform across the wave
    const int q = __builtin_amdgcn_readfirstlane(wave);
    float w1r[4][9], b1r[4];
    bf16x2 w6p[9][2];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        b1r[k] = params[off.b[0] + 4 * q + k];
#pragma unroll
        for (int t = 0; t < 9; ++t) w1r[k][t] = (float)wbf[off.W[0] + (4 * q + k) * 9 + t];
    }
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int h = 0; h < 2; ++h) w6p[t][h] = *reinterpret_cast<const bf16x2 *>(wbf + off.W[NL - 1] + t * C + 4 * q + 2 * h);
    const float b6 = params[off.b[NL - 1]];

    // ubar / s enters a ring of URS rows (row ys - 1 + rho in slot rho % URS)
    // in batches of UBATCH rows, loaded a whole batch ahead: the loads of a
    // batch are waited for once, not once per step
    const int nu = rows + 12;  // rows rho = 0 .. rows + 11 feed layer 1
    auto urow = [&](int rho) { return (int64_t)((((ys - 1 + rho) % H) + H) % H) * W; };
    constexpr int UPT = (UBATCH * URC + FTHREADS - 1) / FTHREADS;  // loads per thread per batch
    T ubuf[UPT];
    auto ubatch_load = [&](int rho0) {  // rows rho0 .. rho0 + UBATCH - 1
#pragma unroll
        for (int k = 0; k < UPT; ++k) {
            const int e = tid + FTHREADS * k, rho = rho0 + e / URC, col = e % URC;
            ubuf[k] = (e < UBATCH * URC && rho < nu) ? ubs[urow(rho) + ((x0 - 6 + col) % W + W) % W] : T(0);
        }
    };
    auto ubatch_store = [&](int rho0) {
#pragma unroll
        for (int k = 0; k < UPT; ++k) {
            const int e = tid + FTHREADS * k, rho = rho0 + e / URC, col = e % URC;
            if (e < UBATCH * URC && rho < nu) uring[(rho % URS) * URC + col] = (float)ubuf[k] * inv;
        }
    };
    ubatch_load(0);
    ubatch_store(0);
    ubatch_load(UBATCH);
    ubatch_store(UBATCH);
    __syncthreads();

    const int nstep = rows + 15;  // layer 6 computes rows y0 .. y0 + rows - 1 at steps 15 .. rows + 14
    const int l6c = min(lane, FV - 1);  // layer 6: output frame column 5 + l6c
    // z of layer 6's row at step st2: the 8 waves' partial sums, in wave order
    auto zsum_out = [&](int st2) {
        if (st2 >= 15 && tid < FV) {
            const float *zp = zpart + (st2 & 1) * 8 * 64;
            float zsum = b6;
#pragma unroll
            for (int w = 0; w < 8; ++w) zsum += zp[w * 64 + tid];
            const int x = x0 + tid;
            if (x < W) z[(int64_t)b * HW + (int64_t)(ys + st2 - 10) * W + x] = zsum;
        }
    };
    for (int st = 0; st < nstep; ++st) {
        // ubar rows 2 UBATCH + st .. are loaded at the start of the step and
        // stored at its end (layer 1 reads rows st .. st + 2 of the ring)
        const bool ub_now = st % UBATCH == 0 && 2 * UBATCH + st < nu;
        if (ub_now) ubatch_load(2 * UBATCH + st);
        const int yM = ys + st - 2 * (ML - 1);
        const bool mact = st >= 3 * ML - 3 && st < 3 * ML - 3 + rows + 2 * (NL - ML);
        // ---- operand loads: layer ML's 18 fragments, layer 1's 9 ubar values,
        // layer 6's 9 channel quads.  Slots are row & (RSL - 1), also for the
        // (negative) rows of a layer before its first step; per input row one
        // base address, the taps' column offsets are immediates.
        const int rM = yM - 1 - ys;  // relative index of layer ML's first input row
        bf16x8 Af[K / 16];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const bf16 *rb = at(ML, (rM + dy) & (RSL - 1), 32 * mh + j) + kh * 8;
#pragma unroll
            for (int k = 0; k < 6; ++k)  // taps (dy, dx = k / 2), channel halves k % 2
                Af[6 * dy + k] = *reinterpret_cast<const bf16x8 *>(rb + (k >> 1) * PSTR + (k & 1) * 16);
        }
        float xv[9];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {  // ubar row ys + st + dy - 1 is rho = st + dy; frame column lane + dx - 1
            const float *ur = uring + ((st + dy) & (URS - 1)) * URC + lane;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) xv[3 * dy + dx] = ur[dx];
        }
        bf16x2 a6[9][2];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {  // layer 6 reads rows ys + st - 11 .. ys + st - 9
            const bf16 *rb = at(NL, (st - 11 + dy) & (RSL - 1), 5 + l6c) + 4 * q;  // frame column 5 + l6c + dx - 1
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                a6[3 * dy + dx][0] = *reinterpret_cast<const bf16x2 *>(rb + dx * PSTR);
                a6[3 * dy + dx][1] = *reinterpret_cast<const bf16x2 *>(rb + dx * PSTR + 2);
            }
        }
        __builtin_amdgcn_sched_barrier(0);  // every load above is issued before the first product
        // ---- products
        f32x16 acc = mb;
#pragma unroll
        for (int ks = 0; ks < K / 16; ++ks) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Wf[ks], Af[ks], acc, 0, 0, 0);
        alignas(8) bf16 v1[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float a = b1r[k];
#pragma unroll
            for (int t = 0; t < 9; ++t) a += w1r[k][t] * xv[t];
            v1[k] = (bf16)relu_bits(a);
        }
        float zp = 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int h = 0; h < 2; ++h) zp = __builtin_amdgcn_fdot2_f32_bf16(a6[t][h], w6p[t][h], zp, false);
        // interleave: one matrix product, then a share of the vector work
#pragma unroll
        for (int i = 0; i < K / 16; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);  // VALU
        }
        __builtin_amdgcn_sched_barrier(0);
        // ---- writes: rows for the next steps' readers, into this step's free
        // slots (a layer outside its rows writes to the spare slot: no branch)
        {
            bf16 *dst = at(ML + 1, mact ? (yM - ys) & (RSL - 1) : RTR, 32 * mh + j + 1);
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                alignas(8) bf16 v4[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) v4[k] = (bf16)relu_bits(acc[4 * g + k]);
                *reinterpret_cast<uint2 *>(dst + 8 * g + 4 * kh) = *reinterpret_cast<const uint2 *>(v4);
            }
        }
        *reinterpret_cast<uint2 *>(at(2, st < rows + 10 ? st & (RSL - 1) : RTR, lane + 1) + 4 * q) =
            *reinterpret_cast<const uint2 *>(v1);  // layer 1: frame column lane
        zpart[(st & 1) * 8 * 64 + q * 64 + lane] = zp;
        zsum_out(st - 1);  // the previous step's partial sums are complete (barrier below it)
        if (ub_now) ubatch_store(2 * UBATCH + st);
        lds_barrier();
    }
    zsum_out(nstep - 1);
}

// A whole 3D 32 -> 32 layer in one pass: the input tiles of planes z - 1, z,
// z + 1 (each with its periodic x-y halo) sit in LDS, and every output row
// accumulates its 3 x 18 MFMA steps in registers, one weight slice at a time
// (slices: [dz][cout][K], K = tap * 32 + cin), so no FP32 partial buffer goes
// through HBM.  MODE kFwd: out = relu(conv(in) + bias); kBwd: out =
// conv'(in) * (mask > 0) with the transposed, mirrored slices.
constexpr size_t kMid3Lds = (size_t)3 * (TY + 2) * (TX + 2) * PSTR * sizeof(bf16);
template <int MODE>
__global__ __launch_bounds__(256) void k_conv_mid3(const bf16 *in, const bf16 *slices, const float *bias,
                                                   const bf16 *mask, bf16 *out, int H, int W, int nz, int tiles_x,
                                                   int tiles_y) {
    extern __shared__ __attribute__((aligned(16))) unsigned char mid3_lds[];
    bf16 *tiles = reinterpret_cast<bf16 *>(mid3_lds);
    constexpr int TP = (TY + 2) * (TX + 2) * PSTR;  // one plane's tile
    const int blk = blockIdx.x;
    const int tx = blk % tiles_x, ty = (blk / tiles_x) % tiles_y;
    const int64_t pz = blk / (tiles_x * tiles_y);  // output plane
    const int x0 = tx * TX, y0 = ty * TY;
    const int64_t HW = (int64_t)H * W;
    const int tid = threadIdx.x;
    for (int dzi = 0; dzi < 3; ++dzi) {
        const bf16 *inb = in + plane_shift(pz, nz, dzi - 1) * HW * C;
        for (int q = tid; q < (TY + 2) * (TX + 2) * 4; q += 256) {
            const int pix = q >> 2, part = q & 3;
            const int r = pix / (TX + 2), c = pix % (TX + 2);
            const int gy = (int)((y0 + r - 1 + (int64_t)H) % H), gx = (int)((x0 + c - 1 + (int64_t)W) % W);
            *reinterpret_cast<uint4 *>(tiles + dzi * TP + pix * PSTR + part * 8) =
                *reinterpret_cast<const uint4 *>(inb + ((int64_t)gy * W + gx) * C + part * 8);
        }
    }
    const int lane = tid & 63, wave = tid >> 6;
    const int j = lane & 31, kh = lane >> 5;
    constexpr int RPW = TY / 4;  // output rows per wave
    f32x16 acc[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) acc[i] = f32x16{};
    __syncthreads();
    for (int dzi = 0; dzi < 3; ++dzi) {
        bf16x8 Bf[K / 16];
        const bf16 *wm = slices + (size_t)dzi * C * K9;
#pragma unroll
        for (int ks = 0; ks < K / 16; ++ks) Bf[ks] = *reinterpret_cast<const bf16x8 *>(wm + j * K + ks * 16 + kh * 8);
        const bf16 *tl = tiles + dzi * TP;
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int rr = wave + 4 * i;
            bf16x8 Af[K / 16];  // every operand load issued before the first product
#pragma unroll
            for (int ks = 0; ks < K / 16; ++ks) {
                const int t = ks >> 1, dy = t / 3, dx = t % 3;
                const int pix = (rr + dy) * (TX + 2) + (j + dx);
                Af[ks] = *reinterpret_cast<const bf16x8 *>(tl + pix * PSTR + (ks & 1) * 16 + kh * 8);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int ks = 0; ks < K / 16; ++ks) acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Af[ks], Bf[ks], acc[i], 0, 0, 0);
        }
    }
    float bj = 0.0f;
    if constexpr (MODE == kFwd) bj = bias[j];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        const int y = y0 + wave + 4 * i;
        if (y >= H) continue;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int xi = 8 * (v >> 2) + 4 * kh + (v & 3);
            const int x = x0 + xi;
            if (x >= W) continue;
            const int64_t idx = ((pz * H + y) * (int64_t)W + x) * C + j;
            float val = acc[i][v];
            if constexpr (MODE == kBwd) val = (float)mask[idx] > 0.0f ? val : 0.0f;
            else val = fmaxf(val + bj, 0.0f);
            out[idx] = (bf16)val;
        }
    }
}

// layer 6: 32 channels -> 1, no activation: z
template <int NT>
__global__ void k_conv_out(const bf16 *a, const bf16 *w6, const float *b6, float *z, int H, int W, int nz, int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t HW = (int64_t)H * W;
    const int64_t pz = p / HW;
    const int rem = (int)(p % HW), y = rem / W, x = rem % W;
    float acc = b6[0];
    for (int t = 0; t < NT; ++t) {
        const int yy = wrap(y + tap_dy(t), H), xx = wrap(x + tap_dx(t), W);
        const uint4 *src =
            reinterpret_cast<const uint4 *>(a + (plane_shift(pz, nz, tap_dz<NT>(t)) * HW + (int64_t)yy * W + xx) * C);
        alignas(16) bf16 v[C];
#pragma unroll
        for (int q = 0; q < 4; ++q) reinterpret_cast<uint4 *>(v)[q] = src[q];
#pragma unroll
        for (int c = 0; c < C; ++c) acc += (float)v[c] * (float)w6[t * C + c];
    }
    z[p] = acc;
}

// out = G in: the periodic trapezoidal filter (1/4, 1/2, 1/4) per axis (the
// z pass only when the field has several planes)
__device__ __forceinline__ float g_apply(const float *in, int64_t pz, int y, int x, int H, int W, int nz) {
    const int ym = wrap(y - 1, H), yp = wrap(y + 1, H), xm = wrap(x - 1, W), xp = wrap(x + 1, W);
    const int64_t HW = (int64_t)H * W;
    auto plane = [&](int64_t q) {
        auto row = [&](int yy) {
            const float *r = in + q * HW + (int64_t)yy * W;
            return 0.5f * r[x] + 0.25f * (r[xm] + r[xp]);
        };
        return 0.5f * row(y) + 0.25f * (row(ym) + row(yp));
    };
    if (nz == 1) return plane(pz);
    return 0.5f * plane(pz) + 0.25f * (plane(plane_shift(pz, nz, -1)) + plane(plane_shift(pz, nz, 1)));
}

// y = G z; writes y (training) and/or u0 = ubar + s * y
template <typename T>
__global__ void k_gfin(const float *z, const T *ub, const double *s, float *y_out, T *u0, int H, int W, int nz,
                       int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t HW = (int64_t)H * W;
    const int64_t pz = p / HW;
    const int rem = (int)(p % HW), y = rem / W, x = rem % W;
    const float v = g_apply(z, pz, y, x, H, W, nz);
    if (y_out) y_out[p] = v;
    if (u0) u0[p] = ub[p] + (T)(s[pz / nz] * (double)v);
}

// out = G in (the adjoint of the final filter: G is symmetric)
__global__ void k_gfilt(const float *in, float *out, int H, int W, int nz, int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t HW = (int64_t)H * W;
    const int64_t pz = p / HW;
    const int rem = (int)(p % HW), y = rem / W, x = rem % W;
    out[p] = g_apply(in, pz, y, x, H, W, nz);
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
template <int NT>
__global__ void k_out_bwd(const float *dy, const bf16 *w6, const bf16 *a5, bf16 *dz, int H, int W, int nz, int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int64_t HW = (int64_t)H * W;
    const int64_t pz = p / HW;
    const int rem = (int)(p % HW), y = rem / W, x = rem % W;
    float g[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int yy = wrap(y - tap_dy(t), H), xx = wrap(x - tap_dx(t), W);
        g[t] = dy[plane_shift(pz, nz, -tap_dz<NT>(t)) * HW + (int64_t)yy * W + xx];
    }
    alignas(16) bf16 m[C], o[C];
#pragma unroll
    for (int q = 0; q < 4; ++q) reinterpret_cast<uint4 *>(m)[q] = reinterpret_cast<const uint4 *>(a5 + p * C)[q];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float acc = 0.0f;
#pragma unroll
        for (int t = 0; t < NT; ++t) acc += (float)w6[t * C + c] * g[t];
        o[c] = (bf16)((float)m[c] > 0.0f ? acc : 0.0f);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) reinterpret_cast<uint4 *>(dz + p * C)[q] = reinterpret_cast<const uint4 *>(o)[q];
}

// Weight gradient of one layer (one 3x3 slice: the input x is read from the
// plane shifted by dzo) over the points of this block's tiles:
// dW[o][t][c] = sum_p g[p][o] x[p + off(t)][c], db[o] = sum_p g[p][o].
// x: CI channels (32: bf16 activations; 1: ubar / s); g: CO channels
// (32: bf16 gradients; 1: FP32 dL/dy).  part[block][CO*9*CI + CO].
template <int CI, int CO, typename T>
__global__ __launch_bounds__(256) void k_wgrad(const bf16 *xa, const T *ub, const double *s, const bf16 *ga,
                                               const float *gf, float *part, int H, int W, int nz, int dzo,
                                               int tiles_x, int tiles_y, int64_t ntiles) {
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
        const int64_t b = tile / ((int64_t)tiles_x * tiles_y);  // output plane
        const int64_t bx = plane_shift(b, nz, dzo);              // input plane
        const int x0 = tx * WGX, y0 = ty * WGY;
        for (int q = tid; q < (WGY + 2) * (WGX + 2) * CI; q += 256) {
            const int pix = q / CI, c = q % CI;
            const int r = pix / (WGX + 2), cc = pix % (WGX + 2);
            const int gy = (int)((y0 + r - 1 + (int64_t)H) % H), gx = (int)((x0 + cc - 1 + (int64_t)W) % W);
            const int64_t g = bx * HW + (int64_t)gy * W + gx;
            float v;
            if constexpr (CI == 1) v = (float)ub[g] * (float)(1.0 / s[bx / nz]);
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
// Also the bias gradient db[o] = sum_p g[p][o].  The input comes from the
// plane shifted by dzo (one 3x3 slice of a 3D layer).  part[block][32*288+32].
__global__ __launch_bounds__(256) void k_wgrad_mid(const bf16 *xa, const bf16 *ga, float *part, int H, int W, int nz,
                                                   int dzo, int tiles_x, int tiles_y, int64_t ntiles) {
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
            const bf16 v = xa[(plane_shift(b, nz, dzo) * HW + (int64_t)gy * W + gx) * C + c];
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

// grad = sum over blocks (in a fixed order) of part[block][w], where part
// holds one 3x3 slice [o][9][c] + biases; slice dzi of NT taps is scattered to
// W[o][dzi * 9 + t][c] (the identity in 2D) and the biases are written by the
// slice `bias_dzi` only.  grad points at the layer's first weight.
__global__ void k_reduce(const float *part, int nblk, int nw, float *grad, int NT, int dzi, int bias_dzi, int CI,
                         int CO) {
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
        const int nwt = CO * 9 * CI;
        if (i < nwt) {
            const int o = i / (9 * CI), tp = (i / CI) % 9, c = i % CI;
            grad[((int64_t)o * NT + dzi * 9 + tp) * CI + c] = (float)t;
        } else if (dzi == bias_dzi) {
            grad[(int64_t)CO * NT * CI + (i - nwt)] = (float)t;
        }
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
    size_t wbf, wT, wf, s, rms, act, z, zt, y, dy, dyz, dz, lpart, wpart, grad, total;
    int64_t N, nblk_pix;
    int nblk_w;
};

int taps_of(int ndim) { return ndim == 3 ? 27 : 9; }
int64_t planes_of(const gd_grid *g) { return g->batch * (g->ndim == 3 ? g->n[2] : 1); }

int64_t wgrad_tiles(const gd_grid *g) {
    return planes_of(g) * ((g->n[1] + WGY - 1) / WGY) * ((g->n[0] + WGX - 1) / WGX);
}

// applications of G to the network's output (the struct's 0 means 1)
int smooth_of(const gd_cnn *net) { return net->smooth > 0 ? net->smooth : 1; }
constexpr int kMaxSmooth = 8;

Layout layout(const gd_grid *g, bool training, bool own_grad, int smooth) {
    const int NT = taps_of(g->ndim), ndz = NT / 9;
    const Offsets off = offsets(NT);
    Layout L;
    std::memset(&L, 0, sizeof L);
    L.N = planes_of(g) * g->n[0] * g->n[1];
    L.nblk_pix = (L.N + 255) / 256;
    L.nblk_w = (int)std::min<int64_t>(wgrad_tiles(g), 512);
    const size_t slices = (size_t)NMID * ndz * C * K9 * 2;  // bf16 weight slices of the 32 -> 32 layers
    size_t o = 0;
    L.wbf = o;
    o = align_up(o + (size_t)off.total * 2, 256);
    L.wT = o;
    if (training) o = align_up(o + slices, 256);
    L.wf = o;
    if (ndz > 1) o = align_up(o + slices, 256);
    L.s = o;
    o = align_up(o + (size_t)g->batch * 8, 256);
    L.rms = o;
    o = align_up(o + (size_t)g->batch * RMS_CHUNKS * 8, 256);
    L.act = o;
    const size_t actb = align_up((size_t)L.N * C * 2, 256);
    o += (training ? NL - 1 : 2) * actb;
    L.z = o;
    o = align_up(o + (size_t)L.N * 4, 256);
    L.zt = o;  // the second buffer of G^m z (m > 1)
    if (smooth > 1) o = align_up(o + (size_t)L.N * 4, 256);
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
    if (net->ndim != 2 && net->ndim != 3) return fail(GD_EINVAL, "the network is 2D or 3D (ndim %d)", net->ndim);
    if (net->channels != C || net->layers != NL)
        return fail(GD_EINVAL, "the network has %d layers of %d channels", NL, C);
    if (!net->params) return fail(GD_EINVAL, "params is NULL");
    if (net->smooth < 0 || net->smooth > kMaxSmooth)
        return fail(GD_EINVAL, "smooth must be 0 .. %d (got %d)", kMaxSmooth, net->smooth);
    if (training && (!net->adam_m || !net->adam_v || !net->step))
        return fail(GD_EINVAL, "training needs adam_m, adam_v and step");
    return GD_OK;
}

int check_grid(const gd_cnn *net, const gd_grid *g) {
    if (!g) return fail(GD_EINVAL, "grid is NULL");
    if (g->ndim != net->ndim) return fail(GD_EINVAL, "a %dD network needs %dD fields", net->ndim, net->ndim);
    if (g->dtype != GD_F32 && g->dtype != GD_F64) return fail(GD_EINVAL, "dtype must be GD_F32 or GD_F64");
    if (g->n[0] < 1 || g->n[1] < 1 || g->batch < 1 || (g->ndim == 3 && g->n[2] < 1))
        return fail(GD_EINVAL, "sizes must be >= 1");
    // bound the factors before multiplying them
    if (g->batch > 65535 || (g->ndim == 3 && g->n[2] > (int64_t(1) << 24))) return fail(GD_EINVAL, "field too large");
    const int64_t planes = planes_of(g), n01 = gd::checked_points(g->n, 2, (int64_t(1) << 31) - 1);
    if (n01 < 0 || planes > (int64_t(1) << 24) || planes > (int64_t(1) << 34) / n01)
        return fail(GD_EINVAL, "field too large");
    return GD_OK;
}

#define GD_LAUNCH(...)                                                                   \
    do {                                                                                 \
        hipLaunchKernelGGL(__VA_ARGS__);                                                 \
        hipError_t e_ = hipGetLastError();                                               \
        if (e_ != hipSuccess) return fail(GD_EHIP, "launch: %s", hipGetErrorString(e_)); \
    } while (0)

// One 32 -> 32 layer (forward, or its input gradient with BWD) in one
// matrix-core pass: k_conv_mid in 2D, k_conv_mid3 (three plane-shifted
// products in registers) in 3D.
int mid_layer(bool bwd, const gd_grid *g, const Layout &L, char *w, const bf16 *in, const bf16 *slices,
              const float *bias, const bf16 *mask, bf16 *out, hipStream_t st) {
    const int NT = taps_of(g->ndim), ndz = NT / 9;
    const int H = (int)g->n[1], W = (int)g->n[0], nz = g->ndim == 3 ? (int)g->n[2] : 1;
    const int tiles_x = (W + TX - 1) / TX, tiles_y = (H + TY - 1) / TY;
    const unsigned cblk = (unsigned)(planes_of(g) * tiles_x * tiles_y);
    if (ndz == 1) {
        if (bwd)
            GD_LAUNCH(k_conv_mid<kBwd>, dim3(cblk), dim3(256), 0, st, in, slices, (const float *)nullptr, mask, out, H,
                      W, tiles_x, tiles_y);
        else
            GD_LAUNCH(k_conv_mid<kFwd>, dim3(cblk), dim3(256), 0, st, in, slices, bias, (const bf16 *)nullptr, out, H,
                      W, tiles_x, tiles_y);
        return GD_OK;
    }
    if (bwd)
        GD_LAUNCH(k_conv_mid3<kBwd>, dim3(cblk), dim3(256), kMid3Lds, st, in, slices, (const float *)nullptr, mask,
                  out, H, W, nz, tiles_x, tiles_y);
    else
        GD_LAUNCH(k_conv_mid3<kFwd>, dim3(cblk), dim3(256), kMid3Lds, st, in, slices, bias, (const bf16 *)nullptr,
                  out, H, W, nz, tiles_x, tiles_y);
    return GD_OK;
}

// y = G^m z: m - 1 filter passes ping-ponging between z and zt, then the last
// one fused with u0 = ubar + s y (inference) or writing y (training)
template <typename T>
int finish_forward(const gd_cnn *net, const Layout &L, char *w, const T *ub, T *u0, bool train, int H, int W, int nz,
                   hipStream_t st) {
    const int64_t N = L.N;
    const unsigned pblk = (unsigned)L.nblk_pix;
    const double *s = (const double *)(w + L.s);
    const float *zin = (const float *)(w + L.z);
    for (int k = 1; k < smooth_of(net); ++k) {
        float *zo = (k & 1) ? (float *)(w + L.zt) : (float *)(w + L.z);
        GD_LAUNCH(k_gfilt, dim3(pblk), dim3(256), 0, st, zin, zo, H, W, nz, N);
        zin = zo;
    }
    GD_LAUNCH(k_gfin<T>, dim3(pblk), dim3(256), 0, st, zin, ub, s, train ? (float *)(w + L.y) : (float *)nullptr,
              train ? (T *)nullptr : u0, H, W, nz, N);
    return GD_OK;
}

// forward (train = false: u0 out; train = true: keep every activation and y)
template <typename T>
int run_forward(const gd_cnn *net, const gd_grid *g, const Layout &L, char *w, const T *ub, T *u0, bool train,
                hipStream_t st) {
    const int NT = taps_of(g->ndim), ndz = NT / 9;
    const Offsets off = offsets(NT);
    const int H = (int)g->n[1], W = (int)g->n[0], nz = g->ndim == 3 ? (int)g->n[2] : 1;
    const int64_t P = (int64_t)H * W * nz, N = L.N;
    bf16 *wbf = (bf16 *)(w + L.wbf);
    double *s = (double *)(w + L.s);
    const size_t actb = align_up((size_t)N * C * 2, 256);
    auto act = [&](int i) { return (bf16 *)(w + L.act + (size_t)i * actb); };
    const unsigned pblk = (unsigned)L.nblk_pix;
    GD_LAUNCH(k_cvt, dim3((unsigned)((off.total + 255) / 256)), dim3(256), 0, st, net->params, wbf, off.total);
    bf16 *wf = (bf16 *)(w + L.wf);  // 3D: forward weight slices
    if (ndz > 1)
        GD_LAUNCH(k_repack<false>, dim3((unsigned)((NMID * ndz * C * K9 + 255) / 256)), dim3(256), 0, st,
                  (const bf16 *)wbf, off.W[1], off.W[2] - off.W[1], NT, wf);
    GD_LAUNCH(k_rms_part<T>, dim3(RMS_CHUNKS, (unsigned)g->batch), dim3(256), 0, st, ub, P, (double *)(w + L.rms));
    GD_LAUNCH(k_rms_fin, dim3((unsigned)((g->batch + 63) / 64)), dim3(64), 0, st, (const double *)(w + L.rms),
              (int)g->batch, P, s);
    if (NT == 9 && !train) {  // 2D inference: the six layers in one kernel
        const dim3 grid((unsigned)((W + FV - 1) / FV), (unsigned)((H + FY - 1) / FY), (unsigned)g->batch);
        GD_LAUNCH(k_fwd2d_fused<T>, grid, dim3(FTHREADS), kFusedLds, st, ub, (const double *)s, (const bf16 *)wbf,
                  (const float *)net->params, off, (float *)(w + L.z), H, W);
        return finish_forward<T>(net, L, w, ub, u0, false, H, W, nz, st);
    }
    if (NT == 9)
        GD_LAUNCH((k_conv_in<T, 9>), dim3(pblk), dim3(256), 0, st, ub, (const double *)s, (const bf16 *)(wbf + off.W[0]),
                  (const float *)(net->params + off.b[0]), act(0), H, W, nz, N);
    else
        GD_LAUNCH((k_conv_in<T, 27>), dim3(pblk), dim3(256), 0, st, ub, (const double *)s,
                  (const bf16 *)(wbf + off.W[0]), (const float *)(net->params + off.b[0]), act(0), H, W, nz, N);
    int rc;
    for (int m = 0; m < NMID; ++m) {
        const int l = m + 1;
        bf16 *src = train ? act(m) : act(m & 1);
        bf16 *dst = train ? act(m + 1) : act((m + 1) & 1);
        const bf16 *slices = ndz > 1 ? wf + (size_t)m * ndz * C * K9 : wbf + off.W[l];
        if ((rc = mid_layer(false, g, L, w, src, slices, net->params + off.b[l], nullptr, dst, st))) return rc;
    }
    bf16 *last = train ? act(NL - 2) : act(NMID & 1);
    if (NT == 9)
        GD_LAUNCH(k_conv_out<9>, dim3(pblk), dim3(256), 0, st, (const bf16 *)last, (const bf16 *)(wbf + off.W[NL - 1]),
                  (const float *)(net->params + off.b[NL - 1]), (float *)(w + L.z), H, W, nz, N);
    else
        GD_LAUNCH(k_conv_out<27>, dim3(pblk), dim3(256), 0, st, (const bf16 *)last, (const bf16 *)(wbf + off.W[NL - 1]),
                  (const float *)(net->params + off.b[NL - 1]), (float *)(w + L.z), H, W, nz, N);
    return finish_forward<T>(net, L, w, ub, u0, train, H, W, nz, st);
}

// Weight gradient of layer (CI -> CO) into grad_layer (its first weight): one
// pass per 3x3 slice (dz), each reduced and scattered into place.
template <int CI, int CO, typename T>
int wgrad_layer(const gd_grid *g, const Layout &L, char *w, const bf16 *xa, const T *ub, const double *s,
                const bf16 *ga, const float *gf, float *grad_layer, hipStream_t st) {
    constexpr int NWL = CO * 9 * CI + CO;
    const int NT = taps_of(g->ndim), ndz = NT / 9;
    const int H = (int)g->n[1], W = (int)g->n[0], nz = g->ndim == 3 ? (int)g->n[2] : 1;
    const int tiles_x = (W + WGX - 1) / WGX, tiles_y = (H + WGY - 1) / WGY;
    const int64_t ntiles = wgrad_tiles(g);
    float *part = (float *)(w + L.wpart);
    for (int dzi = 0; dzi < ndz; ++dzi) {
        const int dzo = ndz > 1 ? dzi - 1 : 0;
        if constexpr (CI == C && CO == C) {
            GD_LAUNCH(k_wgrad_mid, dim3((unsigned)L.nblk_w), dim3(256), 0, st, xa, ga, part, H, W, nz, dzo, tiles_x,
                      tiles_y, ntiles);
        } else {
            auto kern = k_wgrad<CI, CO, T>;
            GD_LAUNCH(kern, dim3((unsigned)L.nblk_w), dim3(256), 0, st, xa, ub, s, ga, gf, part, H, W, nz, dzo,
                      tiles_x, tiles_y, ntiles);
        }
        GD_LAUNCH(k_reduce, dim3((NWL + 31) / 32), dim3(256), 0, st, (const float *)part, L.nblk_w, NWL, grad_layer,
                  NT, dzi, (ndz - 1) / 2, CI, CO);
    }
    return GD_OK;
}

template <typename T>
int run_train(const gd_cnn *net, const gd_grid *g, const Layout &L, char *w, const T *ub, const T *u, double *loss,
              hipStream_t st) {
    const int NT = taps_of(g->ndim), ndz = NT / 9;
    const Offsets off = offsets(NT);
    int rc = run_forward<T>(net, g, L, w, ub, nullptr, true, st);
    if (rc) return rc;
    const int H = (int)g->n[1], W = (int)g->n[0], nz = g->ndim == 3 ? (int)g->n[2] : 1;
    const int64_t P = (int64_t)H * W * nz, N = L.N;
    bf16 *wbf = (bf16 *)(w + L.wbf);
    bf16 *wT = (bf16 *)(w + L.wT);
    const double *s = (const double *)(w + L.s);
    const size_t actb = align_up((size_t)N * C * 2, 256);
    auto act = [&](int i) { return (bf16 *)(w + L.act + (size_t)i * actb); };
    auto dz = [&](int i) { return (bf16 *)(w + L.dz + (size_t)(i & 1) * actb); };
    float *grad = net->grad ? net->grad : (float *)(w + L.grad);
    float *dy = (float *)(w + L.dy);
    const unsigned pblk = (unsigned)L.nblk_pix;
    GD_LAUNCH(k_repack<true>, dim3((unsigned)((NMID * ndz * C * K9 + 255) / 256)), dim3(256), 0, st, (const bf16 *)wbf,
              off.W[1], off.W[2] - off.W[1], NT, wT);
    GD_LAUNCH(k_loss<T>, dim3(pblk), dim3(256), 0, st, (const float *)(w + L.y), ub, u, s, dy,
              (double *)(w + L.lpart), P, N);
    GD_LAUNCH(k_loss_fin, dim3(1), dim3(256), 0, st, (const double *)(w + L.lpart), L.nblk_pix, N, loss);
    // through the final filters: dL/dz = G^m dL/dy (G is symmetric), m passes
    // ping-ponging between dyz and dy
    float *dyz = (float *)(w + L.dyz);
    {
        const float *gin = dy;
        for (int k = 0; k < smooth_of(net); ++k) {
            float *go = (k & 1) ? dy : (float *)(w + L.dyz);
            GD_LAUNCH(k_gfilt, dim3(pblk), dim3(256), 0, st, gin, go, H, W, nz, N);
            gin = go;
        }
        dyz = const_cast<float *>(gin);
    }
    // layer 6
    if ((rc = wgrad_layer<C, 1, T>(g, L, w, act(NL - 2), ub, s, nullptr, dyz, grad + off.W[NL - 1], st))) return rc;
    if (NT == 9)
        GD_LAUNCH(k_out_bwd<9>, dim3(pblk), dim3(256), 0, st, (const float *)dyz, (const bf16 *)(wbf + off.W[NL - 1]),
                  (const bf16 *)act(NL - 2), dz(0), H, W, nz, N);
    else
        GD_LAUNCH(k_out_bwd<27>, dim3(pblk), dim3(256), 0, st, (const float *)dyz, (const bf16 *)(wbf + off.W[NL - 1]),
                  (const bf16 *)act(NL - 2), dz(0), H, W, nz, N);
    // layers 5 .. 2: dz(k) holds the gradient at the output of layer l
    int k = 0;
    for (int l = NL - 2; l >= 1; --l, ++k) {
        const bf16 *xin = act(l - 1);  // input activation of layer l
        if ((rc = wgrad_layer<C, C, T>(g, L, w, xin, ub, s, dz(k), nullptr, grad + off.W[l], st))) return rc;
        if ((rc = mid_layer(true, g, L, w, dz(k), wT + (size_t)(l - 1) * ndz * C * K9, nullptr, xin, dz(k + 1), st)))
            return rc;
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
    if (!net || (net->ndim != 2 && net->ndim != 3) || net->channels != C || net->layers != NL) return 0;
    return offsets(taps_of(net->ndim)).total;
}

size_t warmstart_workspace_bytes(const gd_cnn *net, const gd_grid *g, int32_t training) {
    if (check_net(net, false) || check_grid(net, g)) return 0;
    return layout(g, training != 0, !net->grad, smooth_of(net)).total;
}

int warmstart_forward(const gd_cnn *net, const gd_grid *g, const void *ubar, void *u0, void *work, size_t work_bytes,
                      void *stream) {
    int rc = check_net(net, false);
    if (rc) return rc;
    if ((rc = check_grid(net, g))) return rc;
    if (!ubar || !u0) return fail(GD_EINVAL, "ubar and u0 must be non-NULL");
    if (ubar == u0) return fail(GD_EINVAL, "ubar and u0 must differ");
    if (!work) return fail(GD_EWORKSPACE, "workspace is NULL");
    if ((uintptr_t)work % 256) return fail(GD_EALIGN, "workspace must be 256-byte aligned");
    const Layout L = layout(g, false, false, smooth_of(net));
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
    if ((rc = check_grid(net, g))) return rc;
    if (!ubar || !u || !loss) return fail(GD_EINVAL, "ubar, u and loss must be non-NULL");
    if (!work) return fail(GD_EWORKSPACE, "workspace is NULL");
    if ((uintptr_t)work % 256) return fail(GD_EALIGN, "workspace must be 256-byte aligned");
    const Layout L = layout(g, true, !net->grad, smooth_of(net));
    if (work_bytes < L.total) return fail(GD_EWORKSPACE, "workspace too small: need %zu bytes", L.total);
    hipStream_t st = (hipStream_t)stream;
    if (g->dtype == GD_F32)
        return run_train<float>(net, g, L, (char *)work, (const float *)ubar, (const float *)u, loss, st);
    return run_train<double>(net, g, L, (char *)work, (const double *)ubar, (const double *)u, loss, st);
}

}  // extern "C"
