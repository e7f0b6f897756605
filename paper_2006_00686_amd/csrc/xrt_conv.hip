// 3x3 convolutions (stride 1, zero padding 1, no bias) of the learned preconditioner's
// small CNN, on gfx950: BF16 operands, FP32 accumulation.
//
// Tensors with one channel are float32 [B][H][W] (images); tensors with 32 channels are
// BF16 NHWC [B][H][W][32].  A layer with cin -> cout channels keeps its FP32 master
// weights as W[cout][3][3][cin]; kernels round them to BF16 when loading.
//   conv:        out[p][co] = sum_{t, ci} W[co][t][ci] * in[p + t][ci]
//   transposed:  out[p][ci] = sum_{t, co} W[co][t][ci] * in[p - t][co]
// (t runs over the 3x3 offsets).  The transposed convolution is the adjoint of the
// convolution and is computed by the same kernels reading the weights flipped and
// transposed.  Weight gradient: dW[co][t][ci] = sum_p dout[p][co] * in[p + t][ci].
//
// The 32 -> 32 layer is a dense contraction (implicit GEMM: M = pixels, N = 32 output
// channels, K = 9 x 32) on v_mfma_f32_32x32x16_bf16; its weight gradient (M = 32, N = 32
// per offset, K = pixels) also runs on MFMA after an LDS transpose.  The 1 -> 32 and
// 32 -> 1 layers (K = 9, or one output channel) run on the vector ALUs.
#include <hip/hip_runtime.h>

#include "xrt_internal.h"

namespace xrt {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// two floats rounded to BF16 (nearest even) and packed, low half first: one instruction
__device__ __forceinline__ uint32_t pk_bf16(float lo, float hi)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){lo, hi}, bf16x2));
}

constexpr int kCB = 256;

__device__ __forceinline__ float bf(float x) { return (float)(__bf16)x; }

// weight of the convolution read by a kernel running a (cin -> cout) convolution, from
// the stored weights of layer L: direct (L is cin -> cout) or transposed (L is
// cout -> cin, flipped).  t = 3*kh + kw of the running convolution.
__device__ __forceinline__ float wload(const float* W, bool tr, int co, int t, int ci, int cin, int cout)
{
    if (!tr) return W[(co * 9 + t) * cin + ci];
    // layer L: cin_L = cout, cout_L = cin; W_L[c_L][t_L][i_L] with c_L = ci, i_L = co, t_L = 8 - t
    return W[(ci * 9 + (8 - t)) * cout + co];
}

// ------------------------------------------------------------------ 1 -> 32 (VALU)
template <bool OUT_BF16>
__global__ __launch_bounds__(kCB) void k_conv_1to32(const float* __restrict__ x, const float* __restrict__ W, int tr,
                                                     void* __restrict__ out, int32_t B, int32_t H, int32_t Wd)
{
    const int64_t p = (int64_t)blockIdx.x * kCB + threadIdx.x;
    if (p >= (int64_t)B * H * Wd) return;
    const int32_t w = (int32_t)(p % Wd), h = (int32_t)((p / Wd) % H);
    const int64_t img = p - ((int64_t)h * Wd + w);
    float xin[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int32_t hh = h + t / 3 - 1, ww = w + t % 3 - 1;
        xin[t] = (hh >= 0 && hh < H && ww >= 0 && ww < Wd) ? bf(x[img + (int64_t)hh * Wd + ww]) : 0.0f;
    }
#pragma unroll
    for (int co = 0; co < 32; co += 2) {
        float a0 = 0.0f, a1 = 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            a0 = fmaf(bf(wload(W, tr, co, t, 0, 1, 32)), xin[t], a0);
            a1 = fmaf(bf(wload(W, tr, co + 1, t, 0, 1, 32)), xin[t], a1);
        }
        if constexpr (OUT_BF16) {
            __bf16* o = (__bf16*)out + p * 32 + co;
            o[0] = (__bf16)a0;
            o[1] = (__bf16)a1;
        } else {
            float* o = (float*)out + p * 32 + co;
            o[0] = a0;
            o[1] = a1;
        }
    }
}

// ------------------------------------------------------------------ 32 -> 1 (VALU)
// out[p] = residual[p] + sum (residual may be NULL)
__global__ __launch_bounds__(kCB) void k_conv_32to1(const __bf16* __restrict__ x, const float* __restrict__ W, int tr,
                                                     const float* __restrict__ residual, float* __restrict__ out,
                                                     int32_t B, int32_t H, int32_t Wd)
{
    const int64_t p = (int64_t)blockIdx.x * kCB + threadIdx.x;
    if (p >= (int64_t)B * H * Wd) return;
    const int32_t w = (int32_t)(p % Wd), h = (int32_t)((p / Wd) % H);
    const int64_t img = p - ((int64_t)h * Wd + w);
    float acc = 0.0f;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int32_t hh = h + t / 3 - 1, ww = w + t % 3 - 1;
        if (hh < 0 || hh >= H || ww < 0 || ww >= Wd) continue;
        const uint4* src = (const uint4*)(x + (img + (int64_t)hh * Wd + ww) * 32);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const uint4 q = src[v];
            const uint32_t words[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t bits = (words[e >> 1] >> ((e & 1) * 16)) << 16;
                const float a = __builtin_bit_cast(float, bits);
                acc = fmaf(bf(wload(W, tr, 0, t, v * 8 + e, 32, 1)), a, acc);
            }
        }
    }
    out[p] = (residual ? residual[p] : 0.0f) + acc;
}

// ------------------------------------------------------------------ 32 -> 32 (MFMA)
// One wavefront: 32 consecutive pixels of one image row x 32 output channels.
// K = 18 steps of 16 (offset t = s / 2, input channels (s % 2) * 16 .. + 16).
template <bool OUT_BF16>
__global__ __launch_bounds__(kCB) void k_conv_32to32(const __bf16* __restrict__ x, const float* __restrict__ W, int tr,
                                                      void* __restrict__ out, int32_t B, int32_t H, int32_t Wd)
{
    const int32_t lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * (kCB / 64) + (threadIdx.x >> 6);
    const int32_t wt = (Wd + 31) / 32;
    if (tile >= (int64_t)B * H * wt) return;
    const int32_t w0 = (int32_t)(tile % wt) * 32;
    const int64_t bh = tile / wt;
    const int32_t h = (int32_t)(bh % H);
    const int64_t img = (bh / H) * (int64_t)H * Wd;
    const int32_t m = lane & 31, kb = lane >> 5;

    f32x16 acc = {};
#pragma unroll
    for (int s = 0; s < 18; ++s) {
        const int t = s >> 1, ci0 = (s & 1) * 16 + kb * 8;
        // B operand: W[co = lane % 32][t][ci0 .. ci0 + 7]
        bf16x8 bw;
#pragma unroll
        for (int e = 0; e < 8; ++e) bw[e] = (__bf16)wload(W, tr, m, t, ci0 + e, 32, 32);
        // A operand: in[pixel (h + kh - 1, w0 + m + kw - 1)][ci0 .. ci0 + 7]
        const int32_t hh = h + t / 3 - 1, ww = w0 + m + t % 3 - 1;
        bf16x8 ax;
        if (hh >= 0 && hh < H && ww >= 0 && ww < Wd) {
            const uint4 q = *(const uint4*)(x + (img + (int64_t)hh * Wd + ww) * 32 + ci0);
            ax = __builtin_bit_cast(bf16x8, q);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) ax[e] = (__bf16)0.0f;
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ax, bw, acc, 0, 0, 0);
    }
    // D[i] of lane l: pixel 8 (i / 4) + 4 (l / 32) + i % 4, channel l % 32
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int32_t px = w0 + 8 * (i >> 2) + 4 * kb + (i & 3);
        if (px < Wd) {
            const int64_t o = (img + (int64_t)h * Wd + px) * 32 + m;
            if constexpr (OUT_BF16)
                ((__bf16*)out)[o] = (__bf16)acc[i];
            else
                ((float*)out)[o] = acc[i];
        }
    }
}

// ------------------------------------------------------------------ weight gradients
// Per-wave partial sums part[wave][cout][9][cin], reduced in a fixed order afterwards.

// 32 -> 32 on MFMA: per 32-pixel row tile, the tile of dout (32 px x 32 co) and three
// column-shifted copies of the input rows h-1..h+1 (32 px x 32 ci each) are staged in
// LDS channel-major, so both operands (8 consecutive pixels of one channel) are aligned
// 16-byte LDS reads.  D (per offset t) = dout^T (32 co x px) * in_shift (px x 32 ci).
constexpr int kWgWaves = 2;

__global__ __launch_bounds__(64 * kWgWaves) void k_wgrad_32x32(const __bf16* __restrict__ x,
                                                               const __bf16* __restrict__ dy, float* __restrict__ part,
                                                               int32_t B, int32_t H, int32_t Wd, int64_t ntiles)
{
    // per wave: dy [32 co][32 px] and x [3 kw][3 kh][32 ci][32 px]
    __shared__ __attribute__((aligned(16))) __bf16 sdy[kWgWaves][32][32];
    __shared__ __attribute__((aligned(16))) __bf16 sx[kWgWaves][9][32][32];
    const int32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t m = lane & 31, kb = lane >> 5;
    const int64_t gw = (int64_t)blockIdx.x * kWgWaves + wv, nw = (int64_t)gridDim.x * kWgWaves;
    const int32_t wt = (Wd + 31) / 32;
    f32x16 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x16{};
    for (int64_t tile = gw; tile < ntiles; tile += nw) {
        const int32_t w0 = (int32_t)(tile % wt) * 32;
        const int64_t bh = tile / wt;
        const int32_t h = (int32_t)(bh % H);
        const int64_t img = (bh / H) * (int64_t)H * Wd;
        // stage: lane = (pixel column lane % 32, channel half lane / 32); 16 channels as
        // two 16-byte loads, written channel-major into LDS
        {
            const int32_t px = lane & 31, half = lane >> 5;
            const int32_t ww = w0 + px;
            bf16x8 v0, v1;
            const bool okd = ww < Wd;
            if (okd) {
                const uint4* src = (const uint4*)(dy + (img + (int64_t)h * Wd + ww) * 32 + half * 16);
                v0 = __builtin_bit_cast(bf16x8, src[0]);
                v1 = __builtin_bit_cast(bf16x8, src[1]);
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                sdy[wv][half * 16 + e][px] = okd ? v0[e] : (__bf16)0.0f;
                sdy[wv][half * 16 + 8 + e][px] = okd ? v1[e] : (__bf16)0.0f;
            }
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int32_t hh = h + t / 3 - 1, wx = ww + t % 3 - 1;
                const bool ok = ww < Wd && hh >= 0 && hh < H && wx >= 0 && wx < Wd;
                if (ok) {
                    const uint4* src = (const uint4*)(x + (img + (int64_t)hh * Wd + wx) * 32 + half * 16);
                    v0 = __builtin_bit_cast(bf16x8, src[0]);
                    v1 = __builtin_bit_cast(bf16x8, src[1]);
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    sx[wv][t][half * 16 + e][px] = ok ? v0[e] : (__bf16)0.0f;
                    sx[wv][t][half * 16 + 8 + e][px] = ok ? v1[e] : (__bf16)0.0f;
                }
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        // two K-steps of 16 pixels
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int px0 = ks * 16 + kb * 8;
            const bf16x8 a = *(const bf16x8*)&sdy[wv][m][px0];   // A: dout^T [co = m][px]
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const bf16x8 b = *(const bf16x8*)&sx[wv][t][m][px0];   // B: in [px][ci = m]
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[t], 0, 0, 0);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    // D[i] of lane l: co = 8 (i / 4) + 4 (l / 32) + i % 4, ci = l % 32
    float* dst = part + gw * (32 * 9 * 32);
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int co = 8 * (i >> 2) + 4 * kb + (i & 3);
            dst[(co * 9 + t) * 32 + m] = acc[t][i];
        }
}

// thin layers on the vector ALUs: IN32 = (cin 32, cout 1), else (cin 1, cout 32).  A
// block is 32 channels (of the 32-channel side) x 8 pixel lanes; each thread keeps the 9
// offsets of its channel; the 8 lanes are summed through LDS in a fixed order.
template <bool IN32>
__global__ __launch_bounds__(kCB) void k_wgrad_thin(const void* __restrict__ xin, const void* __restrict__ dyin,
                                                     float* __restrict__ part, int32_t B, int32_t H, int32_t Wd)
{
    __shared__ float red[kCB / 32][32 * 9];
    const int32_t c = threadIdx.x & 31, jl = threadIdx.x >> 5;
    const int64_t n = (int64_t)B * H * Wd;
    float acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = 0.0f;
    for (int64_t p = (int64_t)blockIdx.x * (kCB / 32) + jl; p < n; p += (int64_t)gridDim.x * (kCB / 32)) {
        const int32_t w = (int32_t)(p % Wd), h = (int32_t)((p / Wd) % H);
        const int64_t img = p - ((int64_t)h * Wd + w);
        const float d = IN32 ? bf(((const float*)dyin)[p]) : (float)((const __bf16*)dyin)[p * 32 + c];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int32_t hh = h + t / 3 - 1, ww = w + t % 3 - 1;
            if (hh < 0 || hh >= H || ww < 0 || ww >= Wd) continue;
            const int64_t q = img + (int64_t)hh * Wd + ww;
            const float xv = IN32 ? (float)((const __bf16*)xin)[q * 32 + c] : bf(((const float*)xin)[q]);
            acc[t] = fmaf(d, xv, acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) red[jl][c * 9 + t] = acc[t];
    __syncthreads();
    for (int k = threadIdx.x; k < 32 * 9; k += kCB) {
        float sum = 0.0f;
        for (int q = 0; q < kCB / 32; ++q) sum += red[q][k];
        const int32_t cc = k / 9, t = k % 9;
        // dW[cout][t][cin]: (1 -> 32) index cc * 9 + t; (32 -> 1) index t * 32 + cc
        part[(int64_t)blockIdx.x * 288 + (IN32 ? t * 32 + cc : cc * 9 + t)] = sum;
    }
}

// out[k] = sum_j part[j][k]  (fixed order)
__global__ __launch_bounds__(kCB) void k_reduce_parts(const float* __restrict__ part, int64_t nparts, int32_t nw,
                                                       float* __restrict__ out)
{
    const int32_t k = (int32_t)(blockIdx.x * kCB + threadIdx.x);
    if (k >= nw) return;
    double s = 0.0;
    for (int64_t j = 0; j < nparts; ++j) s += (double)part[j * nw + k];
    out[k] = (float)s;
}

// ------------------------------------------------------------------ fused P and P^T
// y = x + C3 C2 C1 x (TR: y = x + C1^T C2^T C3^T x) for single-channel float32 images,
// with the hidden activations rounded to BF16 exactly as the layer-by-layer kernels
// round them, but never written to HBM: a block computes a kTH x kTW output tile, h2 on
// the tile plus a one-pixel ring (16 rows of 32 pixels: one MFMA column tile per row),
// h1 on a two-pixel ring (in LDS) and reads x on a three-pixel ring.
//   C1: D[co][px] = W1[co][t] * xpatch[t][px]       (K = 9 taps padded to 16)
//   C2: D[co][px] = W2[co][(t, ci)] * h1[(t, ci)][px] (K = 288, W2 held in registers)
//   C3: D[t][px]  = W3[t][c] * h2[c][px]              (K = 32; D of C2 is the B operand,
//       its channel order taken as the contraction order), then y = x + sum_t D[t][px + t].
constexpr int kTH = 14, kTW = 30;
constexpr int kH2R = kTH + 2, kH2C = kTW + 2;       // 16 x 32
constexpr int kH1R = kTH + 4, kH1C = kTW + 4;       // 18 x 34
constexpr int kXR = kTH + 6, kXC = kTW + 6;         // 20 x 36
constexpr int kH1N = kH1R * kH1C;                   // 612
constexpr int kH1Tiles = (kH1N + 31) / 32;          // 20
constexpr int kH1S = 40;                            // LDS stride of an h1 pixel (bf16; 80 B)
constexpr int kPB = 256;
static_assert(kH2C == 32 && kH2R == 4 * (kPB / 64), "one 32-pixel row per MFMA tile, four per wave");


template <bool TR>
__global__ __launch_bounds__(kPB) __attribute__((amdgpu_waves_per_eu(2))) void k_precond(const float* __restrict__ x, const float* __restrict__ Wa,
                                                  const float* __restrict__ Wb, const float* __restrict__ Wc,
                                                  float* __restrict__ y, int32_t H, int32_t Wd, uint32_t tiles_x,
                                                  uint32_t tiles_y, uint32_t ntiles)
{
    // x on the ring (FP32: also the residual), double-buffered: a tile's ring is stored
    // while other waves may still read the previous tile's; the tap partials have their
    // own buffer, so C3 need not wait for every wave's C2 reads of h1 (three barriers per
    // tile)
    __shared__ float sx2[2][kXR * kXC];
    __shared__ __attribute__((aligned(16))) __bf16 sh1[kH1N * kH1S];
    __shared__ float su[9 * kH2R * kH2C];   // tap partials [9][kH2R][kH2C]

    const int32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6, m = lane & 31, kb = lane >> 5;
    // weights as MFMA A operands (row m of lane l = l % 32, contraction index kb * 8 + e)
    bf16x8 a1, a2[18], a3[2];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int t = kb * 8 + e;
        a1[e] = (__bf16)(t < 9 ? wload(Wa, TR, m, t, 0, 1, 32) : 0.0f);
    }
#pragma unroll
    for (int st = 0; st < 18; ++st)
#pragma unroll
        for (int e = 0; e < 8; ++e) a2[st][e] = (__bf16)wload(Wb, TR, m, st >> 1, (st & 1) * 16 + kb * 8 + e, 32, 32);
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int j = st * 8 + e, c = 8 * (j >> 2) + 4 * kb + (j & 3);
            a3[st][e] = (__bf16)(m < 9 ? wload(Wc, TR, 0, m, c, 32, 1) : 0.0f);
        }

    // offsets in the x ring of the C1 taps of this lane (contraction index kb * 8 + e,
    // tap t = 3 dy + dx; indices past tap 8 read tap 8)
    int32_t tap_off[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int t = min(kb * 8 + e, 8);
        tap_off[e] = (t / 3) * kXC + t % 3;
    }

    // x on the three-pixel ring of a tile (zero outside the image), three values per
    // thread, loaded into registers one tile ahead so that the global loads of the next
    // tile are in flight while this one computes
    constexpr int kXPer = (kXR * kXC + kPB - 1) / kPB;
    float xr[kXPer];
    // tile index -> (column, row, image): 32-bit divisions of a wave-uniform value
    auto load_ring = [&](uint32_t t) {
        const uint32_t rest = t / tiles_x;
        const int32_t X0 = (int32_t)(t - rest * tiles_x) * kTW;
        const uint32_t bi = rest / tiles_y;
        const int32_t Y0 = (int32_t)(rest - bi * tiles_y) * kTH;
        const int64_t im = (int64_t)bi * H * Wd;
#pragma unroll
        for (int j = 0; j < kXPer; ++j) {
            const int k = threadIdx.x + j * kPB;
            const int32_t iy = Y0 - 3 + k / kXC, ix = X0 - 3 + k % kXC;
            const bool in = k < kXR * kXC && iy >= 0 && iy < H && ix >= 0 && ix < Wd;
            xr[j] = in ? x[im + (int64_t)iy * Wd + ix] : 0.0f;
        }
    };
    if (blockIdx.x < ntiles) load_ring(blockIdx.x);

    uint32_t parity = 0;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x, parity ^= 1u) {
        float* const sx = sx2[parity];
        const uint32_t rest = tile / tiles_x;
        const int32_t X0 = (int32_t)(tile - rest * tiles_x) * kTW;
        const uint32_t bi = rest / tiles_y;
        const int32_t Y0 = (int32_t)(rest - bi * tiles_y) * kTH;
        const int64_t img = (int64_t)bi * H * Wd;
        // the tile's x ring (3 pixels around it) lies inside the image: no edge masks
        const bool interior = X0 >= 3 && Y0 >= 3 && X0 + kTW + 3 <= Wd && Y0 + kTH + 3 <= H;
#pragma unroll
        for (int j = 0; j < kXPer; ++j) {
            const int k = threadIdx.x + j * kPB;
            if (k < kXR * kXC) sx[k] = xr[j];
        }
        __syncthreads();
        if (tile + gridDim.x < ntiles) load_ring(tile + gridDim.x);
        // C1 on the h1 region (pixels P = 32 T + m, row P / kH1C, column P % kH1C).  The 8
        // taps of a lane are read unconditionally from in-range addresses (a pixel past
        // the region reads pixel 0, a contraction index past the 9 taps reads tap 8) and
        // the unused ones are zeroed afterwards, so the reads are issued together
        for (int T = wv; T < kH1Tiles; T += kPB / 64) {
            const int32_t P = T * 32 + m;
            const bool valid = P < kH1N;
            const int32_t Pc = valid ? P : 0, pr = Pc / kH1C, pc = Pc - pr * kH1C;
            const float* const xp = &sx[pr * kXC + pc];
            float xv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) xv[e] = xp[tap_off[e]];
            // no masks: the weights of contraction indices past tap 8 are zero, and a
            // pixel past the region (which read pixel 0) is not stored
            u32x4 bxw;
#pragma unroll
            for (int e = 0; e < 4; ++e) bxw[e] = pk_bf16(xv[2 * e], xv[2 * e + 1]);
            const f32x16 d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, __builtin_bit_cast(bf16x8, bxw), f32x16{}, 0, 0, 0);
            if (valid) {
                // channels 8 g + 4 kb .. + 3 of pixel P (h1 is zero outside the image;
                // a tile whose x ring lies inside the image needs no mask)
                bool in = true;
                if (!interior) {
                    const int32_t iy = Y0 - 2 + pr, ix = X0 - 2 + pc;
                    in = iy >= 0 && iy < H && ix >= 0 && ix < Wd;
                }
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const uint32_t w0 = pk_bf16(d[4 * g], d[4 * g + 1]), w1 = pk_bf16(d[4 * g + 2], d[4 * g + 3]);
                    *reinterpret_cast<uint2*>(&sh1[P * kH1S + 8 * g + 4 * kb]) = make_uint2(in ? w0 : 0u, in ? w1 : 0u);
                }
            }
        }
        __syncthreads();
        // C2: h2 region rows R = wv + 4 j, column m; the four rows' accumulations are
        // interleaved (independent MFMA chains)
        f32x16 h2[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) h2[j] = f32x16{};
#pragma unroll
        for (int st = 0; st < 18; ++st) {
            const int t = st >> 1;
            bf16x8 b[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                b[j] = *(const bf16x8*)&sh1[((wv + 4 * j + t / 3) * kH1C + m + t % 3) * kH1S + (st & 1) * 16 + kb * 8];
#pragma unroll
            for (int j = 0; j < 4; ++j) h2[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2[st], b[j], h2[j], 0, 0, 0);
        }
        // C3 tap partials into LDS (h2 zero outside the image)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int32_t R = wv + 4 * j;
            bool in = true;
            if (!interior) {
                const int32_t iy = Y0 - 1 + R, ix = X0 - 1 + m;
                in = iy >= 0 && iy < H && ix >= 0 && ix < Wd;
            }
            u32x4 w0, w1;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t p0 = pk_bf16(h2[j][2 * e], h2[j][2 * e + 1]);
                const uint32_t p1 = pk_bf16(h2[j][8 + 2 * e], h2[j][8 + 2 * e + 1]);
                w0[e] = in ? p0 : 0u;
                w1[e] = in ? p1 : 0u;
            }
            f32x16 u = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a3[0], __builtin_bit_cast(bf16x8, w0), f32x16{}, 0, 0, 0);
            u = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a3[1], __builtin_bit_cast(bf16x8, w1), u, 0, 0, 0);
            // D[i] of lane l: tap 8 (i / 4) + 4 kb + i % 4 (taps 0..8 are used), pixel m
#pragma unroll
            for (int i = 0; i < 4; ++i) su[((4 * kb + i) * kH2R + R) * kH2C + m] = u[i];
            if (kb == 0) su[(8 * kH2R + R) * kH2C + m] = u[4];
        }
        __syncthreads();
        for (int k = threadIdx.x; k < kTH * kTW; k += kPB) {
            const int32_t r = k / kTW, c = k % kTW, iy = Y0 + r, ix = X0 + c;
            if (iy < H && ix < Wd) {
                float sum = 0.0f;
#pragma unroll
                for (int t = 0; t < 9; ++t) sum += su[(t * kH2R + r + t / 3) * kH2C + c + t % 3];
                y[img + (int64_t)iy * Wd + ix] = sx[(r + 3) * kXC + c + 3] + sum;
            }
        }
    }
}

bool shape_ok(int32_t cin, int32_t cout) { return (cin == 1 && cout == 32) || (cin == 32 && cout == 32) || (cin == 32 && cout == 1); }

}  // namespace
}  // namespace xrt

using namespace xrt;

extern "C" {

xrt_status xrt_conv3x3(int32_t cin, int32_t cout, int32_t transposed, int32_t batch, int32_t height, int32_t width,
                       const void* d_in, const float* d_weight, const float* d_residual, void* d_out,
                       int32_t out_bf16, void* stream)
{
    if (!shape_ok(cin, cout) || batch < 1 || height < 1 || width < 1 || !d_in || !d_weight || !d_out) {
        set_error("xrt_conv3x3: unsupported channels (1->32, 32->32, 32->1) or bad argument");
        return XRT_E_ARG;
    }
    const int tr = transposed ? 1 : 0;
    // channels of the convolution the kernels run: the layer's, or swapped for its adjoint
    const int32_t rin = tr ? cout : cin, rout = tr ? cin : cout;
    if (d_residual && rout != 1) {
        set_error("xrt_conv3x3: a residual is only added to single-channel outputs");
        return XRT_E_ARG;
    }
    const int64_t n = (int64_t)batch * height * width;
    hipStream_t s = (hipStream_t)stream;
    if (rin == 1) {
        const dim3 g((unsigned)((n + kCB - 1) / kCB));
        if (out_bf16)
            hipLaunchKernelGGL(k_conv_1to32<true>, g, dim3(kCB), 0, s, (const float*)d_in, d_weight, tr, d_out, batch,
                               height, width);
        else
            hipLaunchKernelGGL(k_conv_1to32<false>, g, dim3(kCB), 0, s, (const float*)d_in, d_weight, tr, d_out, batch,
                               height, width);
    } else if (rout == 1) {
        hipLaunchKernelGGL(k_conv_32to1, dim3((unsigned)((n + kCB - 1) / kCB)), dim3(kCB), 0, s, (const __bf16*)d_in,
                           d_weight, tr, d_residual, (float*)d_out, batch, height, width);
    } else {
        const int64_t tiles = (int64_t)batch * height * ((width + 31) / 32);
        const dim3 g((unsigned)((tiles + kCB / 64 - 1) / (kCB / 64)));
        if (out_bf16)
            hipLaunchKernelGGL(k_conv_32to32<true>, g, dim3(kCB), 0, s, (const __bf16*)d_in, d_weight, tr, d_out,
                               batch, height, width);
        else
            hipLaunchKernelGGL(k_conv_32to32<false>, g, dim3(kCB), 0, s, (const __bf16*)d_in, d_weight, tr, d_out,
                               batch, height, width);
    }
    return hip_fail(hipGetLastError(), "xrt_conv3x3 launch");
}

xrt_status xrt_precond_apply(int32_t transposed, int32_t batch, int32_t height, int32_t width, const float* d_x,
                             const float* d_w1, const float* d_w2, const float* d_w3, float* d_y, void* stream)
{
    if (batch < 1 || height < 1 || width < 1 || !d_x || !d_w1 || !d_w2 || !d_w3 || !d_y) {
        set_error("xrt_precond_apply: bad argument");
        return XRT_E_ARG;
    }
    const int64_t n = (int64_t)batch * height * width;
    const char *xb = (const char*)d_x, *yb = (const char*)d_y;
    if (xb < yb + n * 4 && yb < xb + n * 4) {
        set_error("xrt_precond_apply: output overlaps the input");
        return XRT_E_ARG;
    }
    const int32_t tiles_x = (width + kTW - 1) / kTW, tiles_y = (height + kTH - 1) / kTH;
    const int64_t ntiles = (int64_t)batch * tiles_x * tiles_y;
    if (ntiles >= ((int64_t)1 << 31)) {
        set_error("xrt_precond_apply: too many tiles (batch x height x width too large)");
        return XRT_E_SIZE;
    }
    // persistent workgroups, two per CU (the LDS and registers of one allow two)
    int cus = 256;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
        (void)hipGetLastError();
        cus = 256;
    }
    const int64_t want = 2 * (int64_t)cus;
    const unsigned grid = (unsigned)(ntiles < want ? ntiles : want);
    hipStream_t s = (hipStream_t)stream;
    if (transposed)
        hipLaunchKernelGGL(k_precond<true>, dim3(grid), dim3(kPB), 0, s, d_x, d_w3, d_w2, d_w1, d_y, height, width,
                           (uint32_t)tiles_x, (uint32_t)tiles_y, (uint32_t)ntiles);
    else
        hipLaunchKernelGGL(k_precond<false>, dim3(grid), dim3(kPB), 0, s, d_x, d_w1, d_w2, d_w3, d_y, height, width,
                           (uint32_t)tiles_x, (uint32_t)tiles_y, (uint32_t)ntiles);
    return hip_fail(hipGetLastError(), "xrt_precond_apply launch");
}

int64_t xrt_conv3x3_wgrad_workspace(int32_t cin, int32_t cout)
{
    if (!shape_ok(cin, cout)) return -1;
    return cin == 32 && cout == 32 ? (int64_t)1024 * kWgWaves * 32 * 9 * 32 : (int64_t)1024 * 288;
}

xrt_status xrt_conv3x3_wgrad(int32_t cin, int32_t cout, int32_t batch, int32_t height, int32_t width,
                             const void* d_in, const void* d_dout, float* d_work, int64_t work_floats,
                             float* d_dweight, void* stream)
{
    if (!shape_ok(cin, cout) || batch < 1 || height < 1 || width < 1 || !d_in || !d_dout || !d_work || !d_dweight ||
        work_floats < xrt_conv3x3_wgrad_workspace(cin, cout)) {
        set_error("xrt_conv3x3_wgrad: unsupported channels, bad argument or workspace too small");
        return XRT_E_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const int32_t nw = cout * 9 * cin;
    int64_t nparts;
    if (cin == 32 && cout == 32) {
        const int64_t tiles = (int64_t)batch * height * ((width + 31) / 32);
        int64_t blocks = (tiles + kWgWaves - 1) / kWgWaves;
        if (blocks > 1024) blocks = 1024;
        hipLaunchKernelGGL(k_wgrad_32x32, dim3((unsigned)blocks), dim3(64 * kWgWaves), 0, s, (const __bf16*)d_in,
                           (const __bf16*)d_dout, d_work, batch, height, width, tiles);
        nparts = blocks * kWgWaves;
    } else {
        const int64_t n = (int64_t)batch * height * width;
        int64_t blocks = (n + kCB / 32 - 1) / (kCB / 32);
        if (blocks > 1024) blocks = 1024;
        if (cin == 1)
            hipLaunchKernelGGL((k_wgrad_thin<false>), dim3((unsigned)blocks), dim3(kCB), 0, s, d_in, d_dout, d_work,
                               batch, height, width);
        else
            hipLaunchKernelGGL((k_wgrad_thin<true>), dim3((unsigned)blocks), dim3(kCB), 0, s, d_in, d_dout, d_work,
                               batch, height, width);
        nparts = blocks;
    }
    xrt_status st = hip_fail(hipGetLastError(), "xrt_conv3x3_wgrad launch");
    if (st != XRT_OK) return st;
    hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)((nw + kCB - 1) / kCB)), dim3(kCB), 0, s, (const float*)d_work,
                       nparts, nw, d_dweight);
    return hip_fail(hipGetLastError(), "xrt_conv3x3_wgrad reduce launch");
}

}  // extern "C"
