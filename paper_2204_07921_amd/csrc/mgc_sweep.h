// Per-block and per-cell solvers shared by the single-image and the batched
// colour-sweep kernels (one code path, so both give bitwise equal results for
// the same lane-group shape).
#pragma once

#include "mgc_device.h"

namespace mgc {

// Pixel level (b = 1), two-phase: solve the pixel of the active colour in cell
// (cr, cc) of the colour pattern (NC x NC cells) from uin and write the cell
// into uout.
template <typename T, int KIND, int NC>
__device__ __forceinline__ void solve_cell(const T* __restrict__ uin, T* __restrict__ uout, const T* __restrict__ f,
                                           int H, int W, int colour, int cr, int cc, double alpha, int M, int G)
{
    const int i = NC * cr + colour / NC;
    const int j = NC * cc + colour % NC;
    double cval = 0.0;
    if (i < H && j < W) {
        Ring rg[9];
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx)
                make_ring(uin, H, W, i + dy, j + dx, i, i + 1, j, j + 1, rg[(dy + 1) * 3 + dx + 1]);
        const double fs = (double)f[(size_t)i * W + j] - (double)uin[(size_t)i * W + j];
        auto Kpart = [&](const auto& cs, auto& out) {
            constexpr int N = sizeof(out) / sizeof(double);
#pragma unroll
            for (int k = 0; k < N; ++k) out[k] = 0.0;
#pragma unroll
            for (int t = 0; t < 9; ++t)
#pragma unroll
                for (int k = 0; k < N; ++k) out[k] += abs_kappa<KIND>(rg[t], cs[k]);
        };
        auto Dpart = [&](double c) {
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < 9; ++t) acc += dabs_kappa<KIND>(rg[t], c);
            return acc;
        };
        cval = local_solve(Kpart, Dpart, NoSum(), fs, alpha, M, G);
    }
#pragma unroll
    for (int di = 0; di < NC; ++di) {
        const int ii = NC * cr + di;
        if (ii >= H) break;
#pragma unroll
        for (int dj = 0; dj < NC; ++dj) {
            const int jj = NC * cc + dj;
            if (jj >= W) break;
            const size_t idx = (size_t)ii * W + jj;
            T v = uin[idx];
            if (ii == i && jj == j) v = (T)((double)v + cval);
            uout[idx] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Ring candidates of block rows [r0, r1) x cols [c0, c1): the pixels of the box
// [r0 - 1, r1] x [c0 - 1, c1] at distance <= 1 from the block's boundary.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int band_count(int h, int w)
{
    if (h <= 2 || w <= 2) return (h + 2) * (w + 2);
    return 4 * (w + 2) + 4 * (h - 2);
}

__device__ __forceinline__ void band_pixel(int k, int r0, int r1, int c0, int c1, int& i, int& j)
{
    const int h = r1 - r0, w = c1 - c0, bw = w + 2;
    if (h <= 2 || w <= 2) { i = r0 - 1 + k / bw; j = c0 - 1 + k % bw; return; }
    const int top = 2 * bw, mid = 4 * (h - 2);
    if (k < top) { i = r0 - 1 + k / bw; j = c0 - 1 + k % bw; return; }
    k -= top;
    if (k < mid) {
        i = r0 + 1 + (k >> 2);
        const int m = k & 3;
        j = (m == 0) ? c0 - 1 : (m == 1) ? c0 : (m == 2) ? c1 - 1 : c1;
        return;
    }
    k -= mid;
    i = r1 - 1 + k / bw;
    j = c0 - 1 + k % bw;
}

// ---------------------------------------------------------------------------
// Block levels (b >= 2).  GROUP lanes per block; each lane keeps RPL ring
// records in registers (RPL = 0: records are rebuilt from memory at every
// evaluation, for blocks whose ring does not fit in registers).
//
// Fine block levels (LAZY = false) sum f - u over the block themselves and add
// c to the block in place.  Coarse levels (LAZY = true) read the block's sum
// from partial sums taken once at the start of the level (the other colours of
// a level never touch this block's pixels), see the corrections of the
// level's earlier colours through the pending array `cpend`, and store their
// own c there; one wide pass applies the level at its end.
// ---------------------------------------------------------------------------
struct CoarseArgs {
    const double* partials;  // per block: nchunk partial sums of f - u
    int nchunk;
    double* cpend;           // m_j x n_j pending corrections of this level
    int nj;
    int lb;                  // log2(b)
};

template <typename T, int KIND, int GROUP, int RPL, bool LAZY, class GSum>
__device__ __forceinline__ void solve_block(T* __restrict__ u, const T* __restrict__ f, int H, int W,
                                            int p, int q, int r0, int r1, int c0, int c1, int lane,
                                            double alpha, int M, int G, const GSum& gsum, const CoarseArgs& ca)
{
    const int h = r1 - r0, w = c1 - c0;
    double r = 0.0;
    if (LAZY) {
        const double* part = ca.partials + ((size_t)p * ca.nj + q) * ca.nchunk;
        for (int k = lane; k < ca.nchunk; k += GROUP) r += part[k];
    } else {
        for (int k = lane; k < h * w; k += GROUP) {
            const int i = r0 + k / w, j = c0 + k % w;
            const size_t idx = (size_t)i * W + j;
            r += (double)f[idx] - (double)u[idx];
        }
    }
    r = gsum(r);
    const double s = (double)h * (double)w;
    const double fs = r / s;
    const int ncand = band_count(h, w);

    double cval;
    if (RPL > 0) {
        Ring rg[RPL > 0 ? RPL : 1];
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const int k = lane + t * GROUP;
            if (k < ncand) {
                int i, j;
                band_pixel(k, r0, r1, c0, c1, i, j);
                make_ring<T, LAZY>(u, H, W, i, j, r0, r1, c0, c1, rg[t], ca.cpend, ca.nj, ca.lb);
            } else {
                zero_ring(rg[t]);
            }
        }
        auto Kpart = [&](const auto& cs, auto& out) {
            constexpr int N = sizeof(out) / sizeof(double);
#pragma unroll
            for (int k = 0; k < N; ++k) out[k] = 0.0;
#pragma unroll
            for (int t = 0; t < RPL; ++t)
#pragma unroll
                for (int k = 0; k < N; ++k) out[k] += abs_kappa<KIND>(rg[t], cs[k]);
        };
        auto Dpart = [&](double c) {
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < RPL; ++t) acc += dabs_kappa<KIND>(rg[t], c);
            return acc;
        };
        cval = local_solve(Kpart, Dpart, gsum, fs, alpha * s, M, G);
    } else {
        auto Kpart = [&](const auto& cs, auto& out) {
            constexpr int N = sizeof(out) / sizeof(double);
#pragma unroll
            for (int k = 0; k < N; ++k) out[k] = 0.0;
            for (int kk = lane; kk < ncand; kk += GROUP) {
                int i, j;
                Ring rr;
                band_pixel(kk, r0, r1, c0, c1, i, j);
                make_ring<T, LAZY>(u, H, W, i, j, r0, r1, c0, c1, rr, ca.cpend, ca.nj, ca.lb);
#pragma unroll
                for (int k = 0; k < N; ++k) out[k] += abs_kappa<KIND>(rr, cs[k]);
            }
        };
        auto Dpart = [&](double c) {
            double acc = 0.0;
            for (int kk = lane; kk < ncand; kk += GROUP) {
                int i, j;
                Ring rr;
                band_pixel(kk, r0, r1, c0, c1, i, j);
                make_ring<T, LAZY>(u, H, W, i, j, r0, r1, c0, c1, rr, ca.cpend, ca.nj, ca.lb);
                acc += dabs_kappa<KIND>(rr, c);
            }
            return acc;
        };
        cval = local_solve(Kpart, Dpart, gsum, fs, alpha * s, M, G);
    }
    if (LAZY) {
        if (lane == 0) ca.cpend[(size_t)p * ca.nj + q] = cval;
    } else if (cval != 0.0) {
        for (int k = lane; k < h * w; k += GROUP) {
            const int i = r0 + k / w, j = c0 + k % w;
            const size_t idx = (size_t)i * W + j;
            u[idx] = (T)((double)u[idx] + cval);
        }
    }
}

}  // namespace mgc
