// Per-block and per-cell solvers shared by the single-image and the batched
// colour-sweep kernels (one code path, so both give bitwise equal results for
// the same lane-group shape).
#pragma once

#include "mgc_device.h"

namespace mgc {

// Pixel level, pixel (i, j) not on the image border.  Exactly one tap of each
// ring pixel's stencil is (i, j) itself, so the slopes beta are constants of
// the ring position:  centre: u_xx, u_yy slope -2;  east/west neighbour: u_x
// slope -dx/2, u_xx slope 1;  north/south: u_y slope -dy/2, u_yy slope 1;
// diagonal (dy, dx): u_xy slope dy dx / 4.  For the centre and the diagonals
// q = 1 + |grad u|^2 does not move with c, so their curvature is
//   mean:      kappa(c) = (N0 + Nc c) q^{-3/2}            (linear in c)
//   Gaussian:  kappa(c) = det(c) / q^2, det quadratic in c.
// Only the four edge neighbours need the full rational evaluation.
template <int KIND>
struct PixelRing {
    double n0[5], nc[5], r[5];   // centre (0) and diagonals (1..4): mean N0, Nc, q^{-3/2};
                                 // Gaussian: centre n0 = u_xx, nc = u_yy, corners n0 = u_xx u_yy, nc = u_xy
    double m[5];                 // Gaussian: centre -u_xy^2; corners dy*dx
    double e[4][5];              // edge neighbours E, W, S, N: derivatives at c = 0
};

__device__ __forceinline__ void stencil_at(const double w[5][5], int r, int c, double d[5])
{
    d[0] = 0.5 * (w[r][c + 1] - w[r][c - 1]);
    d[1] = 0.5 * (w[r + 1][c] - w[r - 1][c]);
    d[2] = (w[r][c + 1] + w[r][c - 1]) - 2.0 * w[r][c];
    d[3] = (w[r + 1][c] + w[r - 1][c]) - 2.0 * w[r][c];
    d[4] = 0.25 * ((w[r + 1][c + 1] - w[r - 1][c + 1]) - (w[r + 1][c - 1] - w[r - 1][c - 1]));
}

// edge neighbour k (0 E, 1 W, 2 S, 3 N): derivatives moved by c with constant slopes
template <int K>
__device__ __forceinline__ void edge_derivs(const double a[5], double c, double d[5], double bd[5])
{
    constexpr double bx = K == 0 ? -0.5 : (K == 1 ? 0.5 : 0.0);
    constexpr double by = K == 2 ? -0.5 : (K == 3 ? 0.5 : 0.0);
    constexpr double bxx = K <= 1 ? 1.0 : 0.0;
    constexpr double byy = K >= 2 ? 1.0 : 0.0;
    d[0] = bx != 0.0 ? fma(bx, c, a[0]) : a[0];
    d[1] = by != 0.0 ? fma(by, c, a[1]) : a[1];
    d[2] = bxx != 0.0 ? a[2] + c : a[2];
    d[3] = byy != 0.0 ? a[3] + c : a[3];
    d[4] = a[4];
    bd[0] = bx; bd[1] = by; bd[2] = bxx; bd[3] = byy; bd[4] = 0.0;
}

template <int KIND, int K>
__device__ __forceinline__ double edge_abs(const double a[5], double c)
{
    double d[5], bd[5];
    edge_derivs<K>(a, c, d, bd);
    Ring r;
#pragma unroll
    for (int t = 0; t < 5; ++t) { r.a[t] = d[t]; r.b[t] = bd[t]; }
    return abs_kappa<KIND>(r, 0.0);
}

template <int KIND, int K>
__device__ __forceinline__ double edge_dabs(const double a[5], double c)
{
    double d[5], bd[5];
    edge_derivs<K>(a, c, d, bd);
    Ring r;
#pragma unroll
    for (int t = 0; t < 5; ++t) { r.a[t] = d[t]; r.b[t] = bd[t]; }
    return dabs_kappa<KIND>(r, 0.0);
}

template <int KIND>
__device__ __forceinline__ void make_pixel_ring(const double w[5][5], PixelRing<KIND>& R)
{
    const int dys[5] = {0, -1, -1, 1, 1}, dxs[5] = {0, -1, 1, -1, 1};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        double d[5];
        stencil_at(w, 2 + dys[k], 2 + dxs[k], d);
        const double q = fma(d[0], d[0], fma(d[1], d[1], 1.0));
        if (KIND == KIND_MEAN) {
            R.n0[k] = fma(fma(d[1], d[1], 1.0), d[2], fma(fma(d[0], d[0], 1.0), d[3], -2.0 * d[0] * d[1] * d[4]));
            R.nc[k] = k == 0 ? -2.0 * (1.0 + q) : -0.5 * (double)(dys[k] * dxs[k]) * d[0] * d[1];
            const double rq = rsqrt(q);
            R.r[k] = rq * rq * rq;
            R.m[k] = 0.0;
        } else {
            const double iq = 1.0 / q;
            R.r[k] = iq * iq;
            if (k == 0) { R.n0[k] = d[2]; R.nc[k] = d[3]; R.m[k] = -d[4] * d[4]; }
            else { R.n0[k] = d[2] * d[3]; R.nc[k] = d[4]; R.m[k] = (double)(dys[k] * dxs[k]); }
        }
    }
    stencil_at(w, 2, 3, R.e[0]);
    stencil_at(w, 2, 1, R.e[1]);
    stencil_at(w, 3, 2, R.e[2]);
    stencil_at(w, 1, 2, R.e[3]);
}

template <int KIND>
__device__ __forceinline__ double pixel_abs(const PixelRing<KIND>& R, double c)
{
    double s = 0.0;
    if (KIND == KIND_MEAN) {
#pragma unroll
        for (int k = 0; k < 5; ++k) s += fabs(fma(R.nc[k], c, R.n0[k])) * R.r[k];
    } else {
        s += fabs(fma(R.n0[0] - 2.0 * c, R.nc[0] - 2.0 * c, R.m[0])) * R.r[0];
#pragma unroll
        for (int k = 1; k < 5; ++k) {
            const double v = fma(0.25 * R.m[k], c, R.nc[k]);
            s += fabs(fma(-v, v, R.n0[k])) * R.r[k];
        }
    }
    s += edge_abs<KIND, 0>(R.e[0], c);
    s += edge_abs<KIND, 1>(R.e[1], c);
    s += edge_abs<KIND, 2>(R.e[2], c);
    s += edge_abs<KIND, 3>(R.e[3], c);
    return s;
}

template <int KIND>
__device__ __forceinline__ double pixel_dabs(const PixelRing<KIND>& R, double c)
{
    double s = 0.0;
    if (KIND == KIND_MEAN) {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const double n = fma(R.nc[k], c, R.n0[k]);
            const double sg = n > 0.0 ? 1.0 : (n < 0.0 ? -1.0 : 0.0);
            s += sg * R.nc[k] * R.r[k];
        }
    } else {
        {
            const double uxx = R.n0[0] - 2.0 * c, uyy = R.nc[0] - 2.0 * c;
            const double det = fma(uxx, uyy, R.m[0]);
            const double sg = det > 0.0 ? 1.0 : (det < 0.0 ? -1.0 : 0.0);
            s += sg * (-2.0 * (uxx + uyy)) * R.r[0];
        }
#pragma unroll
        for (int k = 1; k < 5; ++k) {
            const double v = fma(0.25 * R.m[k], c, R.nc[k]);
            const double det = fma(-v, v, R.n0[k]);
            const double sg = det > 0.0 ? 1.0 : (det < 0.0 ? -1.0 : 0.0);
            s += sg * (-0.5 * R.m[k] * v) * R.r[k];
        }
    }
    s += edge_dabs<KIND, 0>(R.e[0], c);
    s += edge_dabs<KIND, 1>(R.e[1], c);
    s += edge_dabs<KIND, 2>(R.e[2], c);
    s += edge_dabs<KIND, 3>(R.e[3], c);
    return s;
}

// Pixel level (b = 1), two-phase: solve the pixel of the active colour in cell
// (cr, cc) of the colour pattern (NC x NC cells) from uin and write the cell
// into uout.  Pixels on the image border use general ring records (clamped
// taps may alias the pixel itself); all others the constant-slope form above.
// MODE 0 decides per pixel; MODE 1 is for cells known to be interior (not in
// the first or last row or column of cells), MODE 2 always uses the general form.
template <typename T, int KIND, int NC, int MODE = 0>
__device__ __forceinline__ void solve_cell(const T* __restrict__ uin, T* __restrict__ uout, const T* __restrict__ f,
                                           int H, int W, int colour, int cr, int cc, double alpha, int M, int G)
{
    const int i = NC * cr + colour / NC;
    const int j = NC * cc + colour % NC;
    double cval = 0.0;
    if (MODE == 1 || (i < H && j < W)) {
        const double fs = (double)f[(size_t)i * W + j] - (double)uin[(size_t)i * W + j];
        if (MODE == 1 || (MODE == 0 && i >= 1 && i <= H - 2 && j >= 1 && j <= W - 2)) {
            double w[5][5];
#pragma unroll
            for (int dy = -2; dy <= 2; ++dy) {
                const int ci = clampi(i + dy, 0, H - 1);
#pragma unroll
                for (int dx = -2; dx <= 2; ++dx)
                    w[dy + 2][dx + 2] = (double)uin[(size_t)ci * W + clampi(j + dx, 0, W - 1)];
            }
            PixelRing<KIND> R;
            make_pixel_ring<KIND>(w, R);
            auto Kpart = [&](const auto& cs, auto& out) {
                constexpr int N = sizeof(out) / sizeof(double);
#pragma unroll
                for (int k = 0; k < N; ++k) out[k] = pixel_abs<KIND>(R, cs[k]);
            };
            auto Dpart = [&](double c) { return pixel_dabs<KIND>(R, c); };
            cval = local_solve(Kpart, Dpart, NoSum(), fs, alpha, M, G);
        } else {
            Ring rg[9];
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx)
                    make_ring(uin, H, W, i + dy, j + dx, i, i + 1, j, j + 1, rg[(dy + 1) * 3 + dx + 1]);
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
    }
#pragma unroll
    for (int di = 0; di < NC; ++di) {
        const int ii = NC * cr + di;
        if (MODE != 1 && ii >= H) break;
#pragma unroll
        for (int dj = 0; dj < NC; ++dj) {
            const int jj = NC * cc + dj;
            if (MODE != 1 && jj >= W) break;
            const size_t idx = (size_t)ii * W + jj;
            T v = uin[idx];
            if (ii == i && jj == j) v = (T)((double)v + cval);
            uout[idx] = v;
        }
    }
}

// Pixel level, a cell of the outer ring of cells (its pixel may sit on the
// image border, where clamped taps can alias the pixel itself): a 16-lane
// group per cell, lane t < 9 owning the ring record of neighbour
// (t / 3 - 1, t % 3 - 1), so each evaluation is one record plus a butterfly.
// Lanes t < NC * NC then write pixel t of the cell into uout.
__device__ __forceinline__ bool ring_cell(int k, int cells_r, int cells_c, int& cr, int& cc)
{
    if (cells_r <= 2 || cells_c <= 2) {   // every cell is on the ring
        if (k >= cells_r * cells_c) return false;
        cr = k / cells_c;
        cc = k % cells_c;
        return true;
    }
    if (k < cells_c) { cr = 0; cc = k; return true; }
    if ((k -= cells_c) < cells_c) { cr = cells_r - 1; cc = k; return true; }
    if ((k -= cells_c) < cells_r - 2) { cr = 1 + k; cc = 0; return true; }
    if ((k -= cells_r - 2) < cells_r - 2) { cr = 1 + k; cc = cells_c - 1; return true; }
    return false;
}

__host__ __device__ __forceinline__ int ring_cell_count(int cells_r, int cells_c)
{
    return (cells_r <= 2 || cells_c <= 2) ? cells_r * cells_c : 2 * cells_c + 2 * (cells_r - 2);
}

template <typename T, int KIND, int NC>
__device__ __forceinline__ void solve_ring_cell(const T* __restrict__ uin, T* __restrict__ uout,
                                                const T* __restrict__ f, int H, int W, int colour, int cr, int cc,
                                                int lane, double alpha, int M, int G)
{
    const int i = NC * cr + colour / NC;
    const int j = NC * cc + colour % NC;
    double cval = 0.0;
    if (i < H && j < W) {   // uniform within the group
        Ring rg;
        if (lane < 9)
            make_ring(uin, H, W, i + lane / 3 - 1, j + lane % 3 - 1, i, i + 1, j, j + 1, rg);
        else
            zero_ring(rg);
        const double fs = (double)f[(size_t)i * W + j] - (double)uin[(size_t)i * W + j];
        auto Kpart = [&](const auto& cs, auto& out) {
            constexpr int N = sizeof(out) / sizeof(double);
#pragma unroll
            for (int k = 0; k < N; ++k) out[k] = abs_kappa<KIND>(rg, cs[k]);
        };
        auto Dpart = [&](double c) { return dabs_kappa<KIND>(rg, c); };
        cval = local_solve(Kpart, Dpart, WaveSum<16>(), fs, alpha, M, G);
    }
    if (lane < NC * NC) {
        const int ii = NC * cr + lane / NC, jj = NC * cc + lane % NC;
        if (ii < H && jj < W) {
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
