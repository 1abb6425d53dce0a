// Warm-start CNN for the multigrid solver: six 3x3 convolutions with zero
// "same" padding, channels 1 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, ReLU after the
// first five, residual output u = f + g(f), trained with MSE against multigrid
// solutions and Adam.
//
// Storage: activations and their gradients are bfloat16 NHWC with 32 channels;
// weights are FP32 masters with bfloat16 copies laid out for the matrix
// cores; every accumulation is FP32.  The four 32 -> 32 layers run on MFMA
// (v_mfma_f32_16x16x32_bf16): the forward pass and the input gradient are the
// same implicit GEMM (pixels x 32 outputs x 288 = 9 taps x 32 inputs), the
// input gradient using tap-flipped, transposed weights and a ReLU mask; the
// weight gradient is a second GEMM (288 x 32 x pixels) with the pixel tile
// transposed in LDS.  The 1 -> 32 and 32 -> 1 layers, the loss and Adam are
// VALU kernels.  All reductions write per-workgroup partials that a second
// kernel adds in a fixed order, so training is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mgcurv.h"

namespace mgc_cnn {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int C = 32;          // hidden channels
constexpr int NL = 6;          // layers
constexpr int TH = 8, TW = 32; // pixel tile of the 32 -> 32 weight gradient (rows x cols)
constexpr int CTH = 8;         // rows of the 32 -> 32 convolution's output tile (CTH x TW)
constexpr int RPW = CTH / 4;   // tile rows per wavefront (four wavefronts)
constexpr int PXS = 40;        // LDS pixel stride in bf16 (80 bytes: 8 lanes cover all banks)

// parameter offsets in the flat vector (W_l (3,3,ci,co) row-major, then b_l)
__host__ __device__ constexpr int cin_of(int l) { return l == 0 ? 1 : C; }
__host__ __device__ constexpr int cout_of(int l) { return l == NL - 1 ? 1 : C; }
__host__ __device__ constexpr int wsize(int l) { return 9 * cin_of(l) * cout_of(l); }
__host__ __device__ constexpr int woff(int l) { return l == 0 ? 0 : woff(l - 1) + wsize(l - 1) + cout_of(l - 1); }
__host__ __device__ constexpr int boff(int l) { return woff(l) + wsize(l); }
constexpr int NPARAM = boff(NL - 1) + 1;
static_assert(NPARAM == 37601, "parameter count");

// bfloat16 round to nearest even (explicit, so host tests can reproduce it bit for bit)
__device__ __forceinline__ bf16 to_bf16(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    unsigned short h = (unsigned short)(u >> 16);
    return __builtin_bit_cast(bf16, h);
}
__device__ __forceinline__ float from_bf16(bf16 x)
{
    unsigned short h = __builtin_bit_cast(unsigned short, x);
    return __uint_as_float(((unsigned)h) << 16);
}

// ---------------------------------------------------------------------------
// 32 -> 32 convolution on MFMA.  One workgroup (4 wavefronts) computes an
// CTH x 32 pixel tile for all 32 output channels; wave w owns the RPW = CTH/4
// rows from RPW*w, i.e. 2*RPW 16-pixel M tiles, times two 16-channel N tiles.
//   y[p][o] = sum_tap sum_i x[p + off(tap)][i] * Wt[tap][o][i]   (zero outside the image)
// FWD:   y = relu(acc + bias)               (Wt[tap][o][i] = W[ky][kx][i][o])
// DGRAD: y = acc * (mask[p][o] > 0)         (Wt[tap'][o][i] = W[2-ky][2-kx][o][i], x = dz of the next layer)
// ---------------------------------------------------------------------------
template <bool DGRAD>
__global__ __launch_bounds__(256) void conv32_kernel(const bf16* __restrict__ x, bf16* __restrict__ y,
                                                     const bf16* __restrict__ Wt, const float* __restrict__ bias,
                                                     const bf16* __restrict__ mask, int N, int H, int W)
{
    __shared__ __attribute__((aligned(16))) bf16 xs[(CTH + 2) * (TW + 2) * PXS];
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + CTH - 1) / CTH;
    const int tile = blockIdx.x;
    const int n = tile / (tiles_x * tiles_y);
    const int trem = tile - n * tiles_x * tiles_y;
    const int ty = trem / tiles_x, tx = trem - ty * tiles_x;
    const int r0 = ty * CTH, c0 = tx * TW;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // stage the input tile with a one-pixel halo (zeros outside the image)
    for (int q = tid; q < (CTH + 2) * (TW + 2) * 4; q += 256) {
        const int pix = q >> 2, part = q & 3;
        const int rr = pix / (TW + 2), cc = pix - rr * (TW + 2);
        const int gi = r0 - 1 + rr, gj = c0 - 1 + cc;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (gi >= 0 && gi < H && gj >= 0 && gj < W)
            v = *reinterpret_cast<const uint4*>(x + (((size_t)n * H + gi) * W + gj) * C + part * 8);
        *reinterpret_cast<uint4*>(xs + pix * PXS + part * 8) = v;
    }
    // weights (B operands): lane holds Wt[tap][nt*16 + lane%16][8*(lane/16) .. +7]
    bf16x8 wb[9][2];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
            wb[tap][nt] = *reinterpret_cast<const bf16x8*>(Wt + ((size_t)tap * C + nt * 16 + (lane & 15)) * C + 8 * (lane >> 4));
    __syncthreads();

    floatx4 acc[2 * RPW][2];
#pragma unroll
    for (int mt = 0; mt < 2 * RPW; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3, dx = tap % 3;
#pragma unroll
        for (int mt = 0; mt < 2 * RPW; ++mt) {
            const int rr = RPW * wave + (mt >> 1) + dy;       // halo-tile row
            const int cc = (mt & 1) * 16 + (lane & 15) + dx;   // halo-tile column
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(xs + (rr * (TW + 2) + cc) * PXS + 8 * (lane >> 4));
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wb[tap][nt], acc[mt][nt], 0, 0, 0);
        }
    }
    __syncthreads();  // xs is reused as the output staging tile
    // lane holds D[4*(lane/16) + i][lane%16] of each (mt, nt): pixel, channel
#pragma unroll
    for (int mt = 0; mt < 2 * RPW; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int prow = RPW * wave + (mt >> 1);
                const int pcol = (mt & 1) * 16 + 4 * (lane >> 4) + i;
                const int ch = nt * 16 + (lane & 15);
                float v = acc[mt][nt][i];
                if (!DGRAD) v = fmaxf(v + bias[ch], 0.0f);
                xs[(prow * TW + pcol) * PXS + ch] = to_bf16(v);
            }
    __syncthreads();
    for (int q = tid; q < CTH * TW * 4; q += 256) {
        const int pix = q >> 2, part = q & 3;
        const int rr = pix / TW, cc = pix - rr * TW;
        const int gi = r0 + rr, gj = c0 + cc;
        if (gi >= H || gj >= W) continue;
        const size_t g = (((size_t)n * H + gi) * W + gj) * C + part * 8;
        bf16x8 v = *reinterpret_cast<const bf16x8*>(xs + pix * PXS + part * 8);
        if (DGRAD) {
            const bf16x8 mk = *reinterpret_cast<const bf16x8*>(mask + g);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (!(from_bf16(mk[k]) > 0.0f)) v[k] = to_bf16(0.0f);
        }
        *reinterpret_cast<bf16x8*>(y + g) = v;
    }
}

// ---------------------------------------------------------------------------
// Weight gradient of a 32 -> 32 layer on MFMA:
//   dW[tap][i][o] = sum_p x[p + off(tap)][i] * dz[p][o],   db[o] = sum_p dz[p][o]
// GEMM with M = (tap, i) = 288, N = o = 32, K = pixels.  A workgroup walks a
// strided list of 8 x 32 pixel tiles; a K step of 32 pixels is one tile row.
// LDS holds the tile transposed (channel-major) in three copies shifted by
// dx = 0, 1, 2, so every operand read is an aligned 16-byte load.
// Wave w owns M tiles {w, w+4, ...} (tap-major: mt = tap*2 + i/16) for both N tiles.
// ---------------------------------------------------------------------------
constexpr int XCS = 456;   // bf16 per channel in the x copies (912 bytes: 8 lanes cover all banks)
constexpr int XRS = 40;    // bf16 per row
constexpr int DCS = 264;   // bf16 per channel of the dz tile (528 bytes)
constexpr int DRS = 32;

__global__ __launch_bounds__(256) void wgrad32_kernel(const bf16* __restrict__ x, const bf16* __restrict__ dz,
                                                      float* __restrict__ partials, int N, int H, int W)
{
    __shared__ __attribute__((aligned(16))) bf16 xs[3][C * XCS];
    __shared__ __attribute__((aligned(16))) bf16 ds[C * DCS];
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
    const int ntiles = N * tiles_x * tiles_y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    floatx4 acc[5][2];
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc[k][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.0f;   // thread (o = tid % 32, slice = tid / 32) partial bias gradient

    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int n = tile / (tiles_x * tiles_y);
        const int trem = tile - n * tiles_x * tiles_y;
        const int ty = trem / tiles_x, tx = trem - ty * tiles_x;
        const int r0 = ty * TH, c0 = tx * TW;
        __syncthreads();
        // x tile with halo, transposed and shifted: xs[dx][i][row][col] = x[r0 - 1 + row][c0 - 1 + col + dx][i]
        for (int q = tid; q < (TH + 2) * (TW + 2) * 4; q += 256) {
            const int pix = q >> 2, part = q & 3;
            const int rr = pix / (TW + 2), cc = pix - rr * (TW + 2);
            const int gi = r0 - 1 + rr, gj = c0 - 1 + cc;
            bf16x8 v;
            if (gi >= 0 && gi < H && gj >= 0 && gj < W)
                v = *reinterpret_cast<const bf16x8*>(x + (((size_t)n * H + gi) * W + gj) * C + part * 8);
            else
                for (int k = 0; k < 8; ++k) v[k] = to_bf16(0.0f);
#pragma unroll
            for (int dxs = 0; dxs < 3; ++dxs) {
                const int col = cc - dxs;
                if (col < 0 || col >= TW) continue;
#pragma unroll
                for (int k = 0; k < 8; ++k) xs[dxs][(part * 8 + k) * XCS + rr * XRS + col] = v[k];
            }
        }
        // dz tile transposed: ds[o][row][col]; pixels outside the image contribute zero
        for (int q = tid; q < TH * TW * 4; q += 256) {
            const int pix = q >> 2, part = q & 3;
            const int rr = pix / TW, cc = pix - rr * TW;
            const int gi = r0 + rr, gj = c0 + cc;
            bf16x8 v;
            if (gi < H && gj < W)
                v = *reinterpret_cast<const bf16x8*>(dz + (((size_t)n * H + gi) * W + gj) * C + part * 8);
            else
                for (int k = 0; k < 8; ++k) v[k] = to_bf16(0.0f);
#pragma unroll
            for (int k = 0; k < 8; ++k) ds[(part * 8 + k) * DCS + rr * DRS + cc] = v[k];
        }
        __syncthreads();
        // bias gradient: thread handles channel o = tid % 32 over rows slice = tid / 32
        {
            const int o = tid & 31, row = tid >> 5;   // 8 rows, one per slice
#pragma unroll 8
            for (int cc = 0; cc < TW; ++cc) bacc += from_bf16(ds[o * DCS + row * DRS + cc]);
        }
        // GEMM over the 8 K steps (tile rows)
        for (int kr = 0; kr < TH; ++kr) {
            bf16x8 b[2];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
                b[nt] = *reinterpret_cast<const bf16x8*>(ds + (nt * 16 + (lane & 15)) * DCS + kr * DRS + 8 * (lane >> 4));
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const int mt = wave + 4 * k;     // 0..17 valid
                if (mt >= 18) break;
                const int tap = mt >> 1, ib = (mt & 1) * 16;
                const int dy = tap / 3, dx = tap % 3;
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(
                    &xs[dx][(ib + (lane & 15)) * XCS + (kr + dy) * XRS + 8 * (lane >> 4)]);
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
                    acc[k][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[nt], acc[k][nt], 0, 0, 0);
            }
        }
    }
    // write this workgroup's partial: dW in (tap, i, o) order, then db
    float* out = partials + (size_t)blockIdx.x * (9 * C * C + C);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int mt = wave + 4 * k;
        if (mt >= 18) break;
        const int tap = mt >> 1, ib = (mt & 1) * 16;
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ci = ib + 4 * (lane >> 4) + i;
                const int co = nt * 16 + (lane & 15);
                out[(tap * C + ci) * C + co] = acc[k][nt][i];
            }
    }
    // bias: fixed-order combination of the 8 row slices
    __shared__ float bsl[8][C];
    bsl[tid >> 5][tid & 31] = bacc;
    __syncthreads();
    if (tid < C) {
        float s = 0.0f;
        for (int r = 0; r < 8; ++r) s += bsl[r][tid];
        out[9 * C * C + tid] = s;
    }
}

// ---------------------------------------------------------------------------
// Input layer 1 -> 32 (VALU): a1 = relu(conv(f, W0) + b0) as bfloat16 NHWC.
// W0q holds the bfloat16-rounded weights as floats, layout [tap][o].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void conv_in_kernel(const float* __restrict__ f, bf16* __restrict__ y,
                                                      const float* __restrict__ W0q, const float* __restrict__ b0,
                                                      int N, int H, int W)
{
    // the 288 weights and 32 biases in LDS (held in scalar registers they would spill)
    __shared__ float sw[9 * C], sb[C];
    for (int k = threadIdx.x; k < 9 * C; k += blockDim.x) sw[k] = W0q[k];
    if (threadIdx.x < C) sb[threadIdx.x] = b0[threadIdx.x];
    __syncthreads();
    const size_t total = (size_t)N * H * W;
    // 32-bit index arithmetic (a batch holds fewer than 2^31 pixels); 64-bit only for addresses
    const unsigned hw = (unsigned)H * (unsigned)W, tot = (unsigned)total;
    for (unsigned q = blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += gridDim.x * blockDim.x) {
        const size_t p = q;
        const unsigned n = q / hw;
        const unsigned rem = q - n * hw;
        const int i = (int)(rem / (unsigned)W), j = (int)(rem - (unsigned)i * (unsigned)W);
        float t[9];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int gi = i + tap / 3 - 1, gj = j + tap % 3 - 1;
            t[tap] = (gi >= 0 && gi < H && gj >= 0 && gj < W) ? f[((size_t)n * H + gi) * W + gj] : 0.0f;
        }
        // eight channels at a time; the group loop stays rolled so the weights are read from LDS
        // as they are needed instead of all being held in registers
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
            bf16x8 o8;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int o = 8 * k + e;
                float z = sb[o];
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) z = fmaf(t[tap], sw[tap * C + o], z);
                o8[e] = to_bf16(fmaxf(z, 0.0f));
            }
            *reinterpret_cast<bf16x8*>(y + p * C + 8 * k) = o8;
        }
    }
}

// ---------------------------------------------------------------------------
// Output layer 32 -> 1 (VALU) with the residual: u = f + conv(a5, W5) + b5.
// With a target: r = u - t, dz5 = 2 r / count (float), per-block sums of r^2.
// W5q: bfloat16-rounded weights as floats, layout [tap][i].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void conv_out_kernel(const bf16* __restrict__ a5, const float* __restrict__ f,
                                                       const float* __restrict__ W5q, const float* __restrict__ b5,
                                                       float* __restrict__ u, const float* __restrict__ target,
                                                       float* __restrict__ dz5, double* __restrict__ loss_part,
                                                       int N, int H, int W, double inv_count)
{
    __shared__ double lds[4];
    const size_t total = (size_t)N * H * W;
    double lsum = 0.0;
    // 32-bit index arithmetic (a batch holds fewer than 2^31 pixels); 64-bit only for addresses
    const unsigned hw = (unsigned)H * (unsigned)W, tot = (unsigned)total;
    for (unsigned q = blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += gridDim.x * blockDim.x) {
        const size_t p = q;
        const unsigned n = q / hw;
        const unsigned rem = q - n * hw;
        const int i = (int)(rem / (unsigned)W), j = (int)(rem - (unsigned)i * (unsigned)W);
        float z = b5[0];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int gi = i + tap / 3 - 1, gj = j + tap % 3 - 1;
            if (gi < 0 || gi >= H || gj < 0 || gj >= W) continue;
            const bf16* xp = a5 + (((size_t)n * H + gi) * W + gj) * C;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bf16x8 v = *reinterpret_cast<const bf16x8*>(xp + 8 * k);
#pragma unroll
                for (int e = 0; e < 8; ++e) z = fmaf(from_bf16(v[e]), W5q[tap * C + 8 * k + e], z);
            }
        }
        const float uu = f[p] + z;
        u[p] = uu;
        if (target) {
            const float r = uu - target[p];
            dz5[p] = (float)(2.0 * (double)r * inv_count);
            lsum += (double)r * (double)r;
        }
    }
    if (!target) return;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) lsum += __shfl_xor(lsum, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) loss_part[blockIdx.x] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

// Output-layer input gradient: dz4[p][i] = (sum_tap dz5[p - off(tap)] W5[tap][i]) * (a5[p][i] > 0)
__global__ __launch_bounds__(256) void out_dgrad_kernel(const float* __restrict__ dz5, const bf16* __restrict__ a5,
                                                        const float* __restrict__ W5q, bf16* __restrict__ dz4,
                                                        int N, int H, int W)
{
    __shared__ float sw[9 * C];   // the weights in LDS (held in scalar registers they would spill)
    for (int k = threadIdx.x; k < 9 * C; k += blockDim.x) sw[k] = W5q[k];
    __syncthreads();
    const size_t total = (size_t)N * H * W;
    // 32-bit index arithmetic (a batch holds fewer than 2^31 pixels); 64-bit only for addresses
    const unsigned hw = (unsigned)H * (unsigned)W, tot = (unsigned)total;
    for (unsigned q = blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += gridDim.x * blockDim.x) {
        const size_t p = q;
        const unsigned n = q / hw;
        const unsigned rem = q - n * hw;
        const int i = (int)(rem / (unsigned)W), j = (int)(rem - (unsigned)i * (unsigned)W);
        float d[9];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            // dz5 at p - off(tap) = (i - (ky - 1), j - (kx - 1))
            const int gi = i - (tap / 3 - 1), gj = j - (tap % 3 - 1);
            d[tap] = (gi >= 0 && gi < H && gj >= 0 && gj < W) ? dz5[((size_t)n * H + gi) * W + gj] : 0.0f;
        }
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {   // rolled: the weights are read from LDS as needed
            const bf16x8 m = *reinterpret_cast<const bf16x8*>(a5 + p * C + 8 * k);
            bf16x8 o;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                float s = 0.0f;
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) s = fmaf(d[tap], sw[tap * C + 8 * k + e], s);
                o[e] = to_bf16(from_bf16(m[e]) > 0.0f ? s : 0.0f);
            }
            *reinterpret_cast<bf16x8*>(dz4 + p * C + 8 * k) = o;
        }
    }
}

// Weight gradients of the two VALU layers, which pair a 32-channel bfloat16 field V with a
// scalar field S over the 3x3 taps:
//   output layer (32 -> 1): dW5[tap][i] = sum_q a5[q][i] dz5[q - off(tap)],  db5 = sum_p dz5[p]
//                           (V = a5, S = dz5, taps read S at q - off)
//   input layer (1 -> 32):  dW0[tap][o] = sum_p dz0[p][o] f[p + off(tap)],   db0[o] = sum_p dz0[p][o]
//                           (V = dz0, S = f, taps read S at p + off)
// with S zero outside the image.  A persistent grid of workgroups walks 8 x 64 pixel tiles; the
// tile's scalar field (with a one-pixel halo) is staged in LDS, and thread (channel ch = tid % 32,
// row slot = tid / 32) accumulates the nine taps and the bias for its channel over its row of
// every tile (one coalesced 64-byte read of V per pixel and warp of 32 lanes).  The eight row slots
// are then added in a fixed order and each workgroup writes its partial sums:
//   output layer: partials[wg * 289 + tap * 32 + i], bias at 288;
//   input layer:  partials[wg * 320 + tap * 32 + o], bias of o at 288 + o.
constexpr int SW_TH = 8, SW_TW = 64;
__global__ __launch_bounds__(256) void scalar_wgrad_kernel(const bf16* __restrict__ vfield,
                                                           const float* __restrict__ sfield,
                                                           float* __restrict__ partials, int N, int H, int W,
                                                           int input_layer)
{
    __shared__ float st[SW_TH + 2][SW_TW + 2];
    __shared__ float red[8][C][10];
    const int tid = threadIdx.x, ch = tid & 31, slot = tid >> 5;
    const int tiles_x = (W + SW_TW - 1) / SW_TW, tiles_y = (H + SW_TH - 1) / SW_TH;
    const int ntiles = N * tiles_x * tiles_y;
    const int sgn = input_layer ? 1 : -1;
    float acc[9], bacc = 0.0f;
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = 0.0f;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int n = tile / (tiles_x * tiles_y);
        const int trem = tile - n * tiles_x * tiles_y;
        const int ty = trem / tiles_x, tx = trem - ty * tiles_x;
        const int r0 = ty * SW_TH, c0 = tx * SW_TW;
        const float* sf = sfield + (size_t)n * H * W;
        __syncthreads();
        for (int q = tid; q < (SW_TH + 2) * (SW_TW + 2); q += 256) {
            const int rr = q / (SW_TW + 2), cc = q - rr * (SW_TW + 2);
            const int gi = r0 - 1 + rr, gj = c0 - 1 + cc;
            st[rr][cc] = (gi >= 0 && gi < H && gj >= 0 && gj < W) ? sf[(size_t)gi * W + gj] : 0.0f;
        }
        __syncthreads();
        const int gi = r0 + slot;
        if (gi < H) {
            const bf16* vrow = vfield + (((size_t)n * H + gi) * W) * C + ch;
            const int cend = min(SW_TW, W - c0);
            for (int cc = 0; cc < cend; ++cc) {
                const float v = from_bf16(vrow[(size_t)(c0 + cc) * C]);
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    const int dy = t / 3 - 1, dx = t % 3 - 1;
                    acc[t] = fmaf(v, st[1 + slot + sgn * dy][1 + cc + sgn * dx], acc[t]);
                }
                bacc += input_layer ? v : st[1 + slot][1 + cc];
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) red[slot][ch][t] = acc[t];
    red[slot][ch][9] = bacc;
    __syncthreads();
    const int stride = input_layer ? 320 : 289;
    float* out = partials + (size_t)blockIdx.x * stride;
    for (int k = tid; k < C * 10; k += 256) {
        const int c = k / 10, t = k - c * 10;
        float s = 0.0f;
        for (int r = 0; r < 8; ++r) s += red[r][c][t];
        if (t < 9) out[t * C + c] = s;
        else if (input_layer) out[288 + c] = s;
        else if (c == 0) out[288] = s;
    }
}

// grad[k] = sum over blocks b of partials[b * stride + k] in two fixed-order passes: slice y
// (blockIdx.y) adds the blocks [y chunk, (y + 1) chunk) in block order into part2[y * count + k],
// then sum_slices_f32 adds the slices in slice order.
constexpr int SUM_SLICES = 16;
__global__ void sum_partials_f32(const float* __restrict__ partials, int nblocks, int stride, int count,
                                 float* __restrict__ part2)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int chunk = (nblocks + SUM_SLICES - 1) / SUM_SLICES;
    const int b0 = blockIdx.y * chunk, b1 = min(b0 + chunk, nblocks);
    float s = 0.0f;
    for (int b = b0; b < b1; ++b) s += partials[(size_t)b * stride + k];
    part2[(size_t)blockIdx.y * count + k] = s;
}

__global__ void sum_slices_f32(const float* __restrict__ part2, int count, float* __restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    float s = 0.0f;
#pragma unroll
    for (int y = 0; y < SUM_SLICES; ++y) s += part2[(size_t)y * count + k];
    out[k] = s;
}

__global__ void sum_loss(const double* __restrict__ part, int n, double* __restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += part[k];
    out[0] = s;
}

// Scatter the gradient partial sums of each layer into the flat parameter layout.
// 32->32 layer partial order is (tap, i, o) + bias, the same as W (ky, kx, i, o) + b.
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float beta1, float beta2, float eps,
                            float bc1, float bc2)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = beta1 * m[k] + (1.0f - beta1) * gk;
    const float vk = beta2 * v[k] + (1.0f - beta2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float mhat = mk / bc1, vhat = vk / bc2;
    w[k] = w[k] - lr * mhat / (sqrtf(vhat) + eps);
}

// Refresh the bfloat16 / rounded copies of the weights from the FP32 masters.
//   W0q[tap][o], W5q[tap][i]: rounded floats;  Wf[l][tap][o][i] and Wb[l][tap'][o=i][i=o] for l = 1..4.
__global__ void refresh_weights_kernel(const float* __restrict__ w, float* __restrict__ W0q, float* __restrict__ W5q,
                                       bf16* __restrict__ Wf, bf16* __restrict__ Wb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < 9 * C) {
        W0q[k] = from_bf16(to_bf16(w[woff(0) + k]));                 // (ky, kx, 1, o) -> [tap][o]
        W5q[k] = from_bf16(to_bf16(w[woff(NL - 1) + k]));            // (ky, kx, i, 1) -> [tap][i]
    }
    if (k < 4 * 9 * C * C) {
        const int l = 1 + k / (9 * C * C);
        const int r = k % (9 * C * C);
        const int tap = r / (C * C), i = (r / C) % C, o = r % C;      // master order (tap, i, o)
        const bf16 q = to_bf16(w[woff(l) + r]);
        Wf[(size_t)(l - 1) * 9 * C * C + ((size_t)tap * C + o) * C + i] = q;
        Wb[(size_t)(l - 1) * 9 * C * C + ((size_t)(8 - tap) * C + i) * C + o] = q;
    }
}

}  // namespace mgc_cnn

using namespace mgc_cnn;

struct mg_cnn {
    int maxpix = 0;            // capacity in pixels (N * H * W)
    hipStream_t stream = nullptr;
    float* w = nullptr;        // FP32 masters
    float* g = nullptr;        // gradients
    float* m = nullptr;
    float* v = nullptr;
    float* W0q = nullptr;
    float* W5q = nullptr;
    bf16* Wf = nullptr;
    bf16* Wb = nullptr;
    bf16* act[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // a1..a5
    bf16* dzA = nullptr;
    bf16* dzB = nullptr;
    float* dz5 = nullptr;
    float* upred = nullptr;
    float* part = nullptr;     // weight-gradient partials
    float* part2 = nullptr;    // their per-slice sums (SUM_SLICES x count)
    size_t part_cap = 0;
    double* loss_part = nullptr;
    double* loss_dev = nullptr;
    double* loss_host = nullptr;
    int step = 0;
    std::string err;
};

namespace {

thread_local std::string g_cnn_error;
constexpr int WG32 = 512;       // workgroups of the MFMA weight-gradient kernel
constexpr int SW_WG = 256;      // workgroups of the scalar-field weight-gradient kernel
constexpr int LOSS_BLOCKS = 1024;

mg_status cfail(mg_cnn* c, mg_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf; else g_cnn_error = buf;
    return st;
}

mg_status chip(mg_cnn* c, hipError_t e, const char* what) { return cfail(c, MG_E_DEVICE, "%s: %s", what, hipGetErrorString(e)); }

mg_status check_shape(mg_cnn* c, int n, int H, int W)
{
    if (!c) return MG_E_INVALID;
    if (n < 1 || H < 1 || W < 1) return cfail(c, MG_E_SHAPE, "batch, height and width must be >= 1");
    if ((long long)n * H * W > c->maxpix) return cfail(c, MG_E_SHAPE, "batch of %lld pixels exceeds the capacity %d", (long long)n * H * W, c->maxpix);
    return MG_OK;
}

int grid_for(size_t total) { size_t g = (total + 255) / 256; return (int)(g < 8192 ? g : 8192); }

// out[k] = sum over the nblocks per-workgroup partials (stride apart) of element k, k < count.
void sum_partials(mg_cnn* c, const float* partials, int nblocks, int stride, int count, float* out)
{
    const unsigned gx = (unsigned)((count + 255) / 256);
    hipLaunchKernelGGL(sum_partials_f32, dim3(gx, SUM_SLICES), dim3(256), 0, c->stream, partials, nblocks, stride,
                       count, c->part2);
    hipLaunchKernelGGL(sum_slices_f32, dim3(gx), dim3(256), 0, c->stream, c->part2, count, out);
}

mg_status refresh(mg_cnn* c)
{
    hipLaunchKernelGGL(refresh_weights_kernel, dim3((4 * 9 * C * C + 255) / 256), dim3(256), 0, c->stream, c->w, c->W0q,
                       c->W5q, c->Wf, c->Wb);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MG_OK : chip(c, e, "weight refresh");
}

// Forward pass; keeps a1..a5.  With target: also dz5 and the loss partials.
mg_status forward(mg_cnn* c, const float* f, float* u, const float* target, int n, int H, int W)
{
    const size_t total = (size_t)n * H * W;
    hipLaunchKernelGGL(conv_in_kernel, dim3(grid_for(total)), dim3(256), 0, c->stream, f, c->act[0], c->W0q,
                       c->w + boff(0), n, H, W);
    const int tiles = n * ((H + CTH - 1) / CTH) * ((W + TW - 1) / TW);
    for (int l = 1; l <= 4; ++l)
        hipLaunchKernelGGL(conv32_kernel<false>, dim3(tiles), dim3(256), 0, c->stream, c->act[l - 1], c->act[l],
                           c->Wf + (size_t)(l - 1) * 9 * C * C, c->w + boff(l), (const bf16*)nullptr, n, H, W);
    hipLaunchKernelGGL(conv_out_kernel, dim3(target ? LOSS_BLOCKS : grid_for(total)), dim3(256), 0, c->stream, c->act[4],
                       f, c->W5q, c->w + boff(NL - 1), u, target, c->dz5, c->loss_part, n, H, W, 1.0 / (double)total);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MG_OK : chip(c, e, "forward");
}

// Backward pass into c->g (flat layout), after forward(..., target).  With trace_dz set (host,
// 5 x n H W x 32 bfloat16) the gradients dL/dz_l of the hidden layers' pre-activations
// (l = 0..4, ReLU mask applied) are copied out in layer order as they are produced, and
// with trace_dz5 set (host, n H W floats) dL/dz_5 of the output layer.
mg_status backward(mg_cnn* c, const float* f, int n, int H, int W, void* trace_dz = nullptr, float* trace_dz5 = nullptr)
{
    const size_t total = (size_t)n * H * W;
    hipError_t e;
    const int tiles = n * ((H + TH - 1) / TH) * ((W + TW - 1) / TW);      // weight-gradient tiles
    const int ctiles = n * ((H + CTH - 1) / CTH) * ((W + TW - 1) / TW);   // convolution tiles
    // output layer: weight gradient partials and dz4
    const int stiles = n * ((H + SW_TH - 1) / SW_TH) * ((W + SW_TW - 1) / SW_TW);
    const int nb_small = stiles < SW_WG ? stiles : SW_WG;
    hipLaunchKernelGGL(scalar_wgrad_kernel, dim3(nb_small), dim3(256), 0, c->stream, c->act[4], c->dz5, c->part,
                       n, H, W, 0);
    sum_partials(c, c->part, nb_small, 289, 289, c->g + woff(NL - 1));
    hipLaunchKernelGGL(out_dgrad_kernel, dim3(grid_for(total)), dim3(256), 0, c->stream, c->dz5, c->act[4], c->W5q,
                       c->dzA, n, H, W);
    auto trace = [&](const bf16* src, int layer) -> hipError_t {
        if (!trace_dz) return hipSuccess;
        return hipMemcpyAsync((bf16*)trace_dz + (size_t)layer * total * C, src, sizeof(bf16) * total * C,
                              hipMemcpyDeviceToHost, c->stream);
    };
    if (trace_dz5 && (e = hipMemcpyAsync(trace_dz5, c->dz5, sizeof(float) * total, hipMemcpyDeviceToHost,
                                         c->stream)) != hipSuccess)
        return chip(c, e, "trace copy");
    if ((e = trace(c->dzA, 4)) != hipSuccess) return chip(c, e, "trace copy");
    bf16* dz = c->dzA;
    bf16* other = c->dzB;
    for (int l = 4; l >= 1; --l) {
        // weight gradient of layer l: input a_l = act[l-1], output gradient dz
        const int nwg = tiles < WG32 ? tiles : WG32;
        hipLaunchKernelGGL(wgrad32_kernel, dim3(nwg), dim3(256), 0, c->stream, c->act[l - 1], dz, c->part, n, H, W);
        sum_partials(c, c->part, nwg, 9 * C * C + C, 9 * C * C + C, c->g + woff(l));
        // input gradient through layer l, masked by a_l > 0 (the ReLU of layer l - 1)
        hipLaunchKernelGGL(conv32_kernel<true>, dim3(ctiles), dim3(256), 0, c->stream, dz, other,
                           c->Wb + (size_t)(l - 1) * 9 * C * C, (const float*)nullptr, c->act[l - 1], n, H, W);
        if ((e = trace(other, l - 1)) != hipSuccess) return chip(c, e, "trace copy");
        bf16* t = dz; dz = other; other = t;
    }
    // input layer: weight gradient from f and dz0
    hipLaunchKernelGGL(scalar_wgrad_kernel, dim3(nb_small), dim3(256), 0, c->stream, dz, f, c->part, n, H, W, 1);
    sum_partials(c, c->part, nb_small, 320, 288, c->g + woff(0));
    sum_partials(c, c->part + 288, nb_small, 320, 32, c->g + boff(0));
    e = hipGetLastError();
    return e == hipSuccess ? MG_OK : chip(c, e, "backward");
}

mg_status read_loss(mg_cnn* c, double* loss)
{
    hipLaunchKernelGGL(sum_loss, dim3(1), dim3(64), 0, c->stream, c->loss_part, LOSS_BLOCKS, c->loss_dev);
    hipError_t e = hipMemcpyAsync(c->loss_host, c->loss_dev, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return chip(c, e, "loss copy");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return chip(c, e, "synchronize");
    *loss = *c->loss_host;
    return MG_OK;
}

}  // namespace

extern "C" {

int32_t mg_cnn_num_params(void) { return NPARAM; }

mg_status mg_cnn_init(int64_t max_pixels, void* hip_stream, mg_cnn** out)
{
    if (!out || max_pixels < 1) return cfail(nullptr, MG_E_INVALID, "out must be non-null and max_pixels >= 1");
    *out = nullptr;
    if (max_pixels > ((int64_t)1 << 31) - 1) return cfail(nullptr, MG_E_SHAPE, "max_pixels must be < 2^31");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return cfail(nullptr, MG_E_DEVICE, "no HIP device available");
    mg_cnn* c = new (std::nothrow) mg_cnn();
    if (!c) return cfail(nullptr, MG_E_NOMEM, "host allocation failed");
    c->maxpix = (int)max_pixels;
    c->stream = (hipStream_t)hip_stream;
    const size_t P = (size_t)max_pixels;
    c->part_cap = std::max<size_t>((size_t)WG32 * (9 * C * C + C), (size_t)SW_WG * 320);
    bool ok = true;
    auto al = [&](void** p, size_t bytes) { if (ok && hipMalloc(p, bytes ? bytes : 1) != hipSuccess) ok = false; };
    al((void**)&c->w, sizeof(float) * NPARAM);
    al((void**)&c->g, sizeof(float) * NPARAM);
    al((void**)&c->m, sizeof(float) * NPARAM);
    al((void**)&c->v, sizeof(float) * NPARAM);
    al((void**)&c->W0q, sizeof(float) * 9 * C);
    al((void**)&c->W5q, sizeof(float) * 9 * C);
    al((void**)&c->Wf, sizeof(bf16) * 4 * 9 * C * C);
    al((void**)&c->Wb, sizeof(bf16) * 4 * 9 * C * C);
    for (int k = 0; k < 5; ++k) al((void**)&c->act[k], sizeof(bf16) * C * P);
    al((void**)&c->dzA, sizeof(bf16) * C * P);
    al((void**)&c->dzB, sizeof(bf16) * C * P);
    al((void**)&c->dz5, sizeof(float) * P);
    al((void**)&c->upred, sizeof(float) * P);
    al((void**)&c->part, sizeof(float) * c->part_cap);
    al((void**)&c->part2, sizeof(float) * SUM_SLICES * (9 * C * C + C));
    al((void**)&c->loss_part, sizeof(double) * LOSS_BLOCKS);
    al((void**)&c->loss_dev, sizeof(double));
    if (ok && hipHostMalloc((void**)&c->loss_host, sizeof(double), hipHostMallocDefault) != hipSuccess) ok = false;
    if (!ok) {
        mg_cnn_destroy(c);
        (void)hipGetLastError();
        return cfail(nullptr, MG_E_NOMEM, "device allocation failed for %lld pixels", (long long)max_pixels);
    }
    *out = c;
    return MG_OK;
}

mg_status mg_cnn_set_params(mg_cnn* c, const float* host_params)
{
    if (!c || !host_params) return MG_E_INVALID;
    hipError_t e = hipMemcpyAsync(c->w, host_params, sizeof(float) * NPARAM, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return chip(c, e, "parameter copy");
    // zero the Adam moments with small fill kernels (graph-safe; no memset nodes)
    std::vector<float> zeros(NPARAM, 0.0f);
    if ((e = hipMemcpyAsync(c->m, zeros.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice, c->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(c->v, zeros.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice, c->stream)) != hipSuccess)
        return chip(c, e, "moment reset");
    c->step = 0;
    mg_status st = refresh(c);
    if (st != MG_OK) return st;
    e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? MG_OK : chip(c, e, "synchronize");
}

mg_status mg_cnn_get_params(mg_cnn* c, float* host_params)
{
    if (!c || !host_params) return MG_E_INVALID;
    hipError_t e = hipMemcpyAsync(host_params, c->w, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? MG_OK : chip(c, e, "parameter copy");
}

mg_status mg_cnn_get_state(mg_cnn* c, float* host_params, float* host_m, float* host_v, int32_t* step)
{
    if (!c || !host_params || !host_m || !host_v || !step) return MG_E_INVALID;
    hipError_t e = hipMemcpyAsync(host_params, c->w, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host_m, c->m, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(host_v, c->v, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return chip(c, e, "state copy");
    *step = c->step;
    return MG_OK;
}

mg_status mg_cnn_set_state(mg_cnn* c, const float* host_params, const float* host_m, const float* host_v, int32_t step)
{
    if (!c || !host_params || !host_m || !host_v) return MG_E_INVALID;
    if (step < 0) return cfail(c, MG_E_INVALID, "step must be >= 0");
    hipError_t e = hipMemcpyAsync(c->w, host_params, sizeof(float) * NPARAM, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->m, host_m, sizeof(float) * NPARAM, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->v, host_v, sizeof(float) * NPARAM, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return chip(c, e, "state copy");
    c->step = step;
    mg_status st = refresh(c);
    if (st != MG_OK) return st;
    e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? MG_OK : chip(c, e, "synchronize");
}

mg_status mg_cnn_forward(mg_cnn* c, const float* f, float* u, int32_t n, int32_t height, int32_t width)
{
    mg_status st = check_shape(c, n, height, width);
    if (st != MG_OK) return st;
    if (!f || !u) return cfail(c, MG_E_INVALID, "f and u must be non-null device pointers");
    return forward(c, f, u, nullptr, n, height, width);
}

mg_status mg_cnn_gradients(mg_cnn* c, const float* f, const float* target, int32_t n, int32_t height, int32_t width,
                           double* loss, float* host_grads)
{
    mg_status st = check_shape(c, n, height, width);
    if (st != MG_OK) return st;
    if (!f || !target) return cfail(c, MG_E_INVALID, "f and target must be non-null device pointers");
    if ((st = forward(c, f, c->upred, target, n, height, width)) != MG_OK) return st;
    if ((st = backward(c, f, n, height, width)) != MG_OK) return st;
    double l = 0.0;
    if ((st = read_loss(c, &l)) != MG_OK) return st;
    if (loss) *loss = l / ((double)n * height * width);
    if (host_grads) {
        hipError_t e = hipMemcpy(host_grads, c->g, sizeof(float) * NPARAM, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return chip(c, e, "gradient copy");
    }
    return MG_OK;
}

mg_status mg_cnn_gradient_trace(mg_cnn* c, const float* f, const float* target, int32_t n, int32_t height,
                                int32_t width, void* host_dz, float* host_dz5, float* host_grads)
{
    mg_status st = check_shape(c, n, height, width);
    if (st != MG_OK) return st;
    if (!f || !target || !host_dz || !host_dz5) return cfail(c, MG_E_INVALID, "f, target, host_dz and host_dz5 must be non-null");
    if ((st = forward(c, f, c->upred, target, n, height, width)) != MG_OK) return st;
    if ((st = backward(c, f, n, height, width, host_dz, host_dz5)) != MG_OK) return st;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return chip(c, e, "synchronize");
    if (host_grads && (e = hipMemcpy(host_grads, c->g, sizeof(float) * NPARAM, hipMemcpyDeviceToHost)) != hipSuccess)
        return chip(c, e, "gradient copy");
    return MG_OK;
}

mg_status mg_cnn_train_step(mg_cnn* c, const float* f, const float* target, int32_t n, int32_t height, int32_t width,
                            float lr, double* loss)
{
    mg_status st = check_shape(c, n, height, width);
    if (st != MG_OK) return st;
    if (!f || !target) return cfail(c, MG_E_INVALID, "f and target must be non-null device pointers");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return cfail(c, MG_E_INVALID, "lr must be finite and > 0");
    if ((st = forward(c, f, c->upred, target, n, height, width)) != MG_OK) return st;
    if ((st = backward(c, f, n, height, width)) != MG_OK) return st;
    c->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = 1.0f - std::pow(b1, (float)c->step), bc2 = 1.0f - std::pow(b2, (float)c->step);
    hipLaunchKernelGGL(adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, c->stream, c->w, c->g, c->m, c->v, NPARAM,
                       lr, b1, b2, 1e-8f, bc1, bc2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return chip(c, e, "adam");
    if ((st = refresh(c)) != MG_OK) return st;
    if (loss) {
        double l = 0.0;
        if ((st = read_loss(c, &l)) != MG_OK) return st;
        *loss = l / ((double)n * height * width);
    }
    return MG_OK;
}

mg_status mg_cnn_activation(mg_cnn* c, int32_t layer, void* host_out, int64_t count)
{
    if (!c || !host_out || layer < 1 || layer > 5 || count < 0 || count > (int64_t)c->maxpix * C) return MG_E_INVALID;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(host_out, c->act[layer - 1], sizeof(bf16) * count, hipMemcpyDeviceToHost);
    return e == hipSuccess ? MG_OK : chip(c, e, "activation copy");
}

void mg_cnn_destroy(mg_cnn* c)
{
    if (!c) return;
    if (c->stream || c->w) (void)hipStreamSynchronize(c->stream);
    void* ptrs[] = {c->w, c->g, c->m, c->v, c->W0q, c->W5q, c->Wf, c->Wb, c->act[0], c->act[1], c->act[2], c->act[3],
                    c->act[4], c->dzA, c->dzB, c->dz5, c->upred, c->part, c->part2, c->loss_part, c->loss_dev};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (c->loss_host) (void)hipHostFree(c->loss_host);
    delete c;
}

const char* mg_cnn_last_error(const mg_cnn* c) { return c ? c->err.c_str() : g_cnn_error.c_str(); }

}  // extern "C"
