// Per-block and per-cell solvers shared by the single-image and the batched
// colour-sweep kernels (one code path, so both give bitwise equal results for
// the same lane-group shape).
#pragma once

#include "mgc_device.h"

namespace mgc {

// Pixel level, pixel (i, j) not on the image border.  Exactly one tap of each
// ring pixel's stencil is (i, j) itself, so the slopes beta are constants of
// the ring position:  centre: u_xx, u_yy slope -2;  east/west neighbour: u_x
// slope -+1/2, u_xx slope 1;  south/north: u_y slope -+1/2, u_yy slope 1;
// diagonal (dy, dx): u_xy slope dy dx / 4.  For the centre and the diagonals
// q = 1 + |grad u|^2 does not move with c, so their curvature is a polynomial
// in c (mean: linear, Gaussian: quadratic) whose coefficients already carry the
// constant factor q^{-3/2} or q^{-2}.  For an edge neighbour let w be its
// moving first derivative (u_x for E/W, u_y for S/N), w = w0 + s c with
// s = -+1/2, and p = 1 + (the other first derivative)^2.  Then q = p + w^2 and
//   mean:     N = p c + P0 + w (A w + k),  A = the fixed second derivative
//             along w's axis' complement, k = -2 (other first derivative) u_xy;
//   Gaussian: D = D1 c + D0 (linear).
template <int KIND>
struct PixelRing {
    double g[5][KIND == KIND_MEAN ? 2 : 3];   // centre (0), diagonals (1..4): kappa = sum_m g[m] c^m
    double e[4][KIND == KIND_MEAN ? 5 : 4];   // E, W, S, N: mean {w0, p, P0, A, k}, Gaussian {w0, p, D0, D1}
};

// 3x3 central differences at (r, c) of a tap window with C columns
template <int C>
__device__ __forceinline__ void stencil_at(const double (*w)[C], int r, int c, double d[5])
{
    d[0] = 0.5 * (w[r][c + 1] - w[r][c - 1]);
    d[1] = 0.5 * (w[r + 1][c] - w[r - 1][c]);
    d[2] = (w[r][c + 1] + w[r][c - 1]) - 2.0 * w[r][c];
    d[3] = (w[r + 1][c] + w[r - 1][c]) - 2.0 * w[r][c];
    d[4] = 0.25 * ((w[r + 1][c + 1] - w[r - 1][c + 1]) - (w[r + 1][c - 1] - w[r - 1][c - 1]));
}

// edge neighbour K (0 E, 1 W, 2 S, 3 N): slope of its moving first derivative
template <int K>
struct EdgeSlope {
    static constexpr double s = (K == 0 || K == 2) ? -0.5 : 0.5;
};

template <int KIND, int K>
__device__ __forceinline__ void make_edge(const double d[5], double e[])
{
    constexpr bool X = K <= 1;   // u_x moves (E/W) or u_y moves (S/N)
    const double w0 = X ? d[0] : d[1];
    const double o = X ? d[1] : d[0];
    const double p = fma(o, o, 1.0);
    e[0] = w0;
    e[1] = p;
    if constexpr (KIND == KIND_MEAN) {
        // N = (1 + u_y^2) u_xx + (1 + u_x^2) u_yy - 2 u_x u_y u_xy with the moving
        // second derivative (u_xx for E/W) equal to its value + c
        const double mov2 = X ? d[2] : d[3], fix2 = X ? d[3] : d[2];
        e[2] = fma(p, mov2, fix2);
        e[3] = fix2;
        e[4] = -2.0 * o * d[4];
    } else {
        e[2] = fma(d[2], d[3], -d[4] * d[4]);
        e[3] = X ? d[3] : d[2];
    }
}

template <int KIND, int K>
__device__ __forceinline__ double edge_abs(const double e[], double c)
{
    const double w = fma(EdgeSlope<K>::s, c, e[0]);
    const double q = fma(w, w, e[1]);
    const double rq = rsqrt_pos(q);
    if (KIND == KIND_MEAN) {
        const double num = fma(w, fma(e[3], w, e[4]), fma(e[1], c, e[2]));
        return fabs(num) * (rq * rq * rq);
    } else {
        const double det = fma(e[3], c, e[2]);
        const double r2 = rq * rq;
        return fabs(det) * (r2 * r2);
    }
}

// dq/dc = 2 s w = -+w;  mean: N' = p + s (2 A w + k);  Gaussian: D' = D1
template <int KIND, int K>
__device__ __forceinline__ double edge_dabs(const double e[], double c)
{
    constexpr double s = EdgeSlope<K>::s;
    const double w = fma(s, c, e[0]);
    const double q = fma(w, w, e[1]);
    const double rq = rsqrt_pos(q);
    const double r2 = rq * rq;
    if (KIND == KIND_MEAN) {
        const double inner = fma(e[3], w, e[4]);
        const double num = fma(w, inner, fma(e[1], c, e[2]));
        const double dnum = fma(s, fma(e[3], w, inner), e[1]);
        const double t = fma(-3.0 * s * num, w, dnum * q);   // N' q - 3/2 N q'
        return signed_by(num, t * (r2 * r2 * rq));
    } else {
        const double det = fma(e[3], c, e[2]);
        const double t = fma(-4.0 * s * det, w, e[3] * q);   // D' q - 2 D q'
        return signed_by(det, t * (r2 * r2 * r2));
    }
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
        const double dd = (double)(dys[k] * dxs[k]);
        if constexpr (KIND == KIND_MEAN) {
            const double n0 = fma(fma(d[1], d[1], 1.0), d[2], fma(fma(d[0], d[0], 1.0), d[3], -2.0 * d[0] * d[1] * d[4]));
            const double nc = k == 0 ? -2.0 * (1.0 + q) : -0.5 * dd * d[0] * d[1];
            const double rq = rsqrt_pos(q);
            const double r = rq * rq * rq;
            R.g[k][0] = n0 * r;
            R.g[k][1] = nc * r;
        } else {
            const double rq = rsqrt_pos(q);
            const double r = (rq * rq) * (rq * rq);
            const double det0 = fma(d[2], d[3], -d[4] * d[4]);
            R.g[k][0] = det0 * r;
            if (k == 0) {   // (u_xx - 2c)(u_yy - 2c) - u_xy^2
                R.g[k][1] = -2.0 * (d[2] + d[3]) * r;
                R.g[k][2] = 4.0 * r;
            } else {        // u_xx u_yy - (u_xy + dy dx c / 4)^2
                R.g[k][1] = -0.5 * dd * d[4] * r;
                R.g[k][2] = -0.0625 * r;
            }
        }
    }
    double d[5];
    stencil_at(w, 2, 3, d);
    make_edge<KIND, 0>(d, R.e[0]);
    stencil_at(w, 2, 1, d);
    make_edge<KIND, 1>(d, R.e[1]);
    stencil_at(w, 3, 2, d);
    make_edge<KIND, 2>(d, R.e[2]);
    stencil_at(w, 1, 2, d);
    make_edge<KIND, 3>(d, R.e[3]);
}

template <int KIND>
__device__ __forceinline__ double pixel_abs(const PixelRing<KIND>& R, double c)
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        if constexpr (KIND == KIND_MEAN)
            s += fabs(fma(R.g[k][1], c, R.g[k][0]));
        else
            s += fabs(fma(fma(R.g[k][2], c, R.g[k][1]), c, R.g[k][0]));
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
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        if constexpr (KIND == KIND_MEAN) {
            s += signed_by(fma(R.g[k][1], c, R.g[k][0]), R.g[k][1]);
        } else {
            const double v = fma(fma(R.g[k][2], c, R.g[k][1]), c, R.g[k][0]);
            s += signed_by(v, fma(R.g[k][2], c + c, R.g[k][1]));
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
            PolyRing<KIND> rg[9];
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    Ring r;
                    make_ring(uin, H, W, i + dy, j + dx, i, i + 1, j, j + 1, r);
                    make_poly<KIND>(r, rg[(dy + 1) * 3 + dx + 1]);
                }
            auto Kpart = [&](const auto& cs, auto& out) {
                constexpr int N = sizeof(out) / sizeof(double);
#pragma unroll
                for (int k = 0; k < N; ++k) out[k] = 0.0;
#pragma unroll
                for (int t = 0; t < 9; ++t)
#pragma unroll
                    for (int k = 0; k < N; ++k) out[k] += abs_poly<KIND>(rg[t], cs[k]);
            };
            auto Dpart = [&](double c) {
                double acc = 0.0;
#pragma unroll
                for (int t = 0; t < 9; ++t) acc += dabs_poly<KIND>(rg[t], c);
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
        Ring r;
        if (lane < 9)
            make_ring(uin, H, W, i + lane / 3 - 1, j + lane % 3 - 1, i, i + 1, j, j + 1, r);
        else
            zero_ring(r);
        PolyRing<KIND> rg;
        make_poly<KIND>(r, rg);
        const double fs = (double)f[(size_t)i * W + j] - (double)uin[(size_t)i * W + j];
        auto Kpart = [&](const auto& cs, auto& out) {
            constexpr int N = sizeof(out) / sizeof(double);
#pragma unroll
            for (int k = 0; k < N; ++k) out[k] = abs_poly<KIND>(rg, cs[k]);
        };
        auto Dpart = [&](double c) { return dabs_poly<KIND>(rg, c); };
        cval = local_solve(Kpart, Dpart, WaveSum<16, 2>(), fs, alpha, M, G);
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
// Block level b = 2, blocks that touch no image border (1 <= p <= m_j - 2 and
// 1 <= q <= n_j - 2, so no clamped tap lands in the block).
//
// Mirroring the image across a block's horizontal or vertical centre line maps
// u_x, u_y, u_xy to exactly -u_x, -u_y or -u_xy (a difference of two taps
// reversed) and keeps u_xx, u_yy, q, the mean-curvature numerator and the
// Gaussian determinant; so every quadrant of the 4 x 4 ring, read in its own
// mirrored frame, is the top-left quadrant.  In that frame (block = {0, 1}^2)
// the quadrant holds four ring pixels with constant slopes:
//   corner (-1, -1): only u_xy moves (+c/4); q is constant, so kappa is a
//     polynomial in c (mean: linear, Gaussian: quadratic) with q folded in;
//   top edge (-1, 0): u_y moves (+c/2), u_yy (+c), u_xy (+c/4).  With w = u_y
//     and p = 1 + u_x^2, q = p + w^2 and, eliminating c = 2 (w - w0) from the
//     u_x w c/2 cross term, N = P0 + p c + w (A w + k) with P0 = u_xx + p u_yy,
//     A = u_xx - u_x, k = u_x (w0 - 2 u_xy); D = D0 + D1 c - c^2/16 with
//     D1 = u_xx - u_xy / 2;
//   left edge (0, -1): the same with x and y exchanged;
//   inside (0, 0): u_x, u_y move (+c/2), u_xx, u_yy (-c), u_xy (+c/4): the
//     general expansion in powers of c with these slopes.
// The lanes of a block split the quadrants (see solve_block2_interior).
// ---------------------------------------------------------------------------
template <int KIND>
struct QuadRing {
    double g[KIND == KIND_MEAN ? 2 : 3];     // corner: kappa = sum_m g[m] c^m
    double et[KIND == KIND_MEAN ? 5 : 4];    // top edge:  mean {w0, p, P0, A, k}, Gaussian {w0, p, D0, D1}
    double el[KIND == KIND_MEAN ? 5 : 4];    // left edge: the same
    PolyRing<KIND> in;                       // inside pixel
};

// Edge records of the quadrant: w = w0 + c/2 moves, q = p + w^2, dq/dc = w.
template <int KIND>
__device__ __forceinline__ void make_qedge(const double d[5], bool top, double e[])
{
    const double w0 = top ? d[1] : d[0];
    const double o = top ? d[0] : d[1];
    const double p = fma(o, o, 1.0);
    e[0] = w0;
    e[1] = p;
    const double mov2 = top ? d[3] : d[2], fix2 = top ? d[2] : d[3];
    if constexpr (KIND == KIND_MEAN) {
        e[2] = fma(p, mov2, fix2);
        e[3] = fix2 - o;
        e[4] = o * fma(-2.0, d[4], w0);
    } else {
        e[2] = fma(d[2], d[3], -d[4] * d[4]);
        e[3] = fma(-0.5, d[4], fix2);
    }
}

template <int KIND>
__device__ __forceinline__ double qedge_abs(const double e[], double c)
{
    const double w = fma(0.5, c, e[0]);
    const double q = fma(w, w, e[1]);
    const double rq = rsqrt_pos(q);
    if constexpr (KIND == KIND_MEAN) {
        const double num = fma(w, fma(e[3], w, e[4]), fma(e[1], c, e[2]));
        return fabs(num) * (rq * rq * rq);
    } else {
        const double det = fma(fma(-0.0625, c, e[3]), c, e[2]);
        const double r2 = rq * rq;
        return fabs(det) * (r2 * r2);
    }
}

// mean: N' = p + (2 A w + k) / 2, N' q - 3/2 N q';  Gaussian: D' = D1 - c/8, D' q - 2 D q'
template <int KIND>
__device__ __forceinline__ double qedge_dabs(const double e[], double c)
{
    const double w = fma(0.5, c, e[0]);
    const double q = fma(w, w, e[1]);
    const double rq = rsqrt_pos(q);
    const double r2 = rq * rq;
    if constexpr (KIND == KIND_MEAN) {
        const double inner = fma(e[3], w, e[4]);
        const double num = fma(w, inner, fma(e[1], c, e[2]));
        const double dnum = fma(0.5, fma(e[3], w, inner), e[1]);
        const double t = fma(-1.5 * num, w, dnum * q);
        return signed_by(num, t * (r2 * r2 * rq));
    } else {
        const double det = fma(fma(-0.0625, c, e[3]), c, e[2]);
        const double ddet = fma(-0.125, c, e[3]);
        const double t = fma(-2.0 * det, w, ddet * q);
        return signed_by(det, t * (r2 * r2 * r2));
    }
}

// wq[y + 2][x + 2] = tap at (y, x) of the quadrant's frame, y, x in -2..1
template <int KIND>
__device__ __forceinline__ void make_quad(const double (&wq)[4][4], QuadRing<KIND>& R)
{
    double d[5];
    stencil_at(wq, 1, 1, d);   // corner: u_xy slope +1/4
    {
        const double q = fma(d[0], d[0], fma(d[1], d[1], 1.0));
        const double rq = rsqrt_pos(q);
        if constexpr (KIND == KIND_MEAN) {
            const double n0 = fma(fma(d[1], d[1], 1.0), d[2], fma(fma(d[0], d[0], 1.0), d[3], -2.0 * d[0] * d[1] * d[4]));
            const double r = rq * rq * rq;
            R.g[0] = n0 * r;
            R.g[1] = (-0.5 * d[0] * d[1]) * r;
        } else {
            const double r = (rq * rq) * (rq * rq);
            R.g[0] = fma(d[2], d[3], -d[4] * d[4]) * r;
            R.g[1] = (-0.5 * d[4]) * r;
            R.g[2] = -0.0625 * r;
        }
    }
    stencil_at(wq, 1, 2, d);
    make_qedge<KIND>(d, true, R.et);
    stencil_at(wq, 2, 1, d);
    make_qedge<KIND>(d, false, R.el);
    Ring r;
    stencil_at(wq, 2, 2, r.a);
    r.b[0] = 0.5;
    r.b[1] = 0.5;
    r.b[2] = -1.0;
    r.b[3] = -1.0;
    r.b[4] = 0.25;
    make_poly<KIND>(r, R.in);
}

template <int KIND>
__device__ __forceinline__ double quad_abs(const QuadRing<KIND>& R, double c)
{
    double s;
    if constexpr (KIND == KIND_MEAN)
        s = fabs(fma(R.g[1], c, R.g[0]));
    else
        s = fabs(fma(fma(R.g[2], c, R.g[1]), c, R.g[0]));
    s += qedge_abs<KIND>(R.et, c);
    s += qedge_abs<KIND>(R.el, c);
    s += abs_poly<KIND>(R.in, c);
    return s;
}

template <int KIND>
__device__ __forceinline__ double quad_dabs(const QuadRing<KIND>& R, double c)
{
    double s;
    if constexpr (KIND == KIND_MEAN) {
        s = signed_by(fma(R.g[1], c, R.g[0]), R.g[1]);
    } else {
        const double v = fma(fma(R.g[2], c, R.g[1]), c, R.g[0]);
        s = signed_by(v, fma(R.g[2], c + c, R.g[1]));
    }
    s += qedge_dabs<KIND>(R.et, c);
    s += qedge_dabs<KIND>(R.el, c);
    s += dabs_poly<KIND>(R.in, c);
    return s;
}

// The 2 x 2 block at (r0, c0), off the image border, on a group of QL lanes:
// QL = 2: lane 0 the top two quadrants, lane 1 the bottom two (rows read in
// reverse), each lane reading a 4 x 6 window and mirroring its right quadrant in
// registers; QL = 4: one quadrant per lane (lane bit 1 mirrors rows, bit 0
// columns), a 4 x 4 window each.
template <typename T, int KIND, int QL>
__device__ __forceinline__ void solve_block2_interior(T* __restrict__ u, const T* __restrict__ f, int H, int W,
                                                      int r0, int c0, int lane, double alpha, int M, int G)
{
    static_assert(QL == 2 || QL == 4, "two or four lanes per block");
    constexpr int NQ = 4 / QL;        // quadrants per lane
    constexpr int WC = 2 + 2 * NQ;    // window columns
    const int ybit = QL == 2 ? lane : lane >> 1, xbit = QL == 2 ? 0 : lane & 1;
    const int sy = ybit ? -1 : 1, sx = xbit ? -1 : 1;
    const int Y = r0 + ybit, X = c0 + xbit;   // the frame's (0, 0) of the lane's first quadrant
    double win[4][WC];                        // rows Y + sy (a - 2), columns X + sx (b - 2)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const T* row = u + (size_t)clampi(Y + sy * (a - 2), 0, H - 1) * W;
#pragma unroll
        for (int b = 0; b < WC; ++b) win[a][b] = (double)row[clampi(X + sx * (b - 2), 0, W - 1)];
    }
    const size_t iy = (size_t)Y * W + X;
    double rsum = (double)f[iy] - win[2][2];
    if constexpr (NQ == 2) rsum += (double)f[iy + 1] - win[2][3];
    QuadRing<KIND> R[NQ];
#pragma unroll
    for (int h = 0; h < NQ; ++h) {   // h = 1: the right quadrant, mirrored
        double wq[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) wq[a][b] = h == 0 ? win[a][b] : win[a][5 - b];
        make_quad<KIND>(wq, R[h]);
    }
    const WaveSum<QL> gs;
    const double fs = gs(rsum) / 4.0;
    auto Kpart = [&](const auto& cs, auto& out) {
        constexpr int N = sizeof(out) / sizeof(double);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double v = quad_abs<KIND>(R[0], cs[k]);
            if constexpr (NQ == 2) v += quad_abs<KIND>(R[1], cs[k]);
            out[k] = v;
        }
    };
    auto Dpart = [&](double c) {
        double v = quad_dabs<KIND>(R[0], c);
        if constexpr (NQ == 2) v += quad_dabs<KIND>(R[1], c);
        return v;
    };
    const double cval = local_solve(Kpart, Dpart, gs, fs, alpha * 4.0, M, G);
    if (cval != 0.0) {
        u[iy] = (T)(win[2][2] + cval);
        if constexpr (NQ == 2) u[iy + 1] = (T)(win[2][3] + cval);
    }
}

// Grid-stride walk over the pixels of an H x W image: pixel p = t, t + stride, ... with its
// row and column advanced by the stride's quotient and remainder (no division per pixel).
struct PixelWalk {
    int i, j, si, sj, W;
    __device__ __forceinline__ PixelWalk(size_t p0, size_t stride, int W_) : W(W_)
    {
        i = (int)(p0 / (size_t)W_);
        j = (int)(p0 - (size_t)i * W_);
        si = (int)(stride / (size_t)W_);
        sj = (int)(stride - (size_t)si * W_);
    }
    __device__ __forceinline__ void next()
    {
        i += si;
        j += sj;
        if (j >= W) { j -= W; ++i; }
    }
};

// ---------------------------------------------------------------------------
// Bisection tree of the split coarse solve.  d successive bisection steps from
// the bracket [lo, hi] visit d of the 2^d - 1 midpoints of a binary tree: node 1
// is the bracket's midpoint, and node n's children 2n and 2n + 1 are the
// midpoints of the lower half of n's interval (taken when V' > 0 at n, as a step
// then sets hi = mid) and of its upper half.  tree_node_mid forms node n's
// midpoint from [lo, hi] along the path to n exactly as the steps would;
// tree_walk takes d steps along given signs, moving [lo, hi] as d sequential
// steps do.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ double tree_node_mid(int node, double lo, double hi)
{
    for (int k = 30 - __builtin_clz((unsigned)node); k >= 0; --k) {   // the path below the root
        const double mid = 0.5 * (lo + hi);
        if ((node >> k) & 1) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// pos(node, mid): whether V' > 0 at that node, whose midpoint is mid.
template <class Pos>
__host__ __device__ __forceinline__ void tree_walk(int d, double& lo, double& hi, Pos&& pos)
{
    int node = 1;
    for (int k = 0; k < d; ++k) {
        const double mid = 0.5 * (lo + hi);   // node's midpoint: [lo, hi] is its interval here
        if (pos(node, mid)) { hi = mid; node = 2 * node; }
        else { lo = mid; node = 2 * node + 1; }
    }
}

// Block index of pixel coordinate i for block side b (lb = log2(b), or -1 when b
// is not a power of two).
__host__ __device__ __forceinline__ int side_div(int i, int b, int lb) { return lb >= 0 ? i >> lb : i / b; }

// ---------------------------------------------------------------------------
// Ring candidates of block rows [r0, r1) x cols [c0, c1) of an H x W image: the
// pixels within distance 1 of a block side that does not lie on the image
// border, as strips two pixels wide.  A side on the border has nothing outside
// it, so its strip holds no ring pixel that the other strips miss.  The top and
// bottom strips span the block's columns widened by one on each side (clipped to
// the image), the left and right strips the rows between them.  For a block off
// the border that is the whole (h + 2) x (w + 2) box less its interior, 8b pixels
// for a b x b block; candidates whose taps all lie inside or all outside the
// block get the zero record.
// ---------------------------------------------------------------------------
struct RingBand {
    int r0, r1, c0, c1;
    int cl, wc;    // first column and width of the top and bottom strips
    int ra;        // first row of the left and right strips
    int nt, nb;    // pixels in the top and bottom strips (0 or 2 wc)
    int per;       // pixels per row of the left and right strips (0, 2 or 4)
    bool left;
    int n;         // candidates in all
};

__host__ __device__ __forceinline__ RingBand ring_band(int H, int W, int r0, int r1, int c0, int c1)
{
    RingBand B;
    B.r0 = r0; B.r1 = r1; B.c0 = c0; B.c1 = c1;
    const bool top = r0 > 0, bot = r1 < H, right = c1 < W;
    B.left = c0 > 0;
    B.cl = B.left ? c0 - 1 : c0;
    B.wc = (right ? c1 : c1 - 1) - B.cl + 1;
    B.ra = top ? r0 + 1 : r0;
    const int rb = bot ? r1 - 2 : r1 - 1;   // last row of the side strips
    const int hv = rb >= B.ra ? rb - B.ra + 1 : 0;
    B.nt = top ? 2 * B.wc : 0;
    B.nb = bot ? 2 * B.wc : 0;
    B.per = 2 * ((B.left ? 1 : 0) + (right ? 1 : 0));
    B.n = B.nt + B.nb + B.per * hv;
    return B;
}

__host__ __device__ __forceinline__ void band_at(const RingBand& B, int k, int& i, int& j)
{
    // the top and bottom strips are two rows of wc each
    if (k < B.nt) { const int r = k >= B.wc; i = B.r0 - 1 + r; j = B.cl + k - r * B.wc; return; }
    k -= B.nt;
    if (k < B.nb) { const int r = k >= B.wc; i = B.r1 - 1 + r; j = B.cl + k - r * B.wc; return; }
    k -= B.nb;
    const int m = k & (B.per - 1);
    i = B.ra + (B.per == 4 ? k >> 2 : k >> 1);
    j = (B.left && m < 2) ? B.c0 - 1 + m : B.c1 - 1 + (m & 1);
}

// Ring records built in chunks: a lane loads the taps of a chunk of its records
// (band positions k, k + GROUP, ...) before it forms any of them, so their
// memory round trips overlap instead of following one another.  A position at
// or past the band's end loads the taps of position 0 (clamped addresses, in
// bounds for any band) and gets the zero record.  The records are make_ring's,
// bit for bit.  A chunk is four records, fewer where registers are short: FP64
// taps take twice the registers, and 1,024-lane workgroups have 128 per lane.
template <typename T, int GROUP>
constexpr int ring_chunk()
{
    return (GROUP >= 1024 ? 2 : 4) / (sizeof(T) == 8 ? 2 : 1);
}

// Records read back from a region at every evaluation: f(record) for the lane's
// positions k = lane, lane + GROUP, ... in that order, with the loads of two
// records in flight at once (one at a time, each waited on its round trip).  The
// split solve's streamed kernel uses it; the one-workgroup streamed kernel has no
// registers to spare for the second record.
template <int KIND, int GROUP, class F>
__device__ __forceinline__ void for_region_records(const double* __restrict__ rec, int stride, int ncand, int lane,
                                                   F&& f)
{
    for (int k0 = lane; k0 < ncand; k0 += 2 * GROUP) {
        const int k1 = k0 + GROUP;
        PolyRing<KIND> p0, p1;
        load_poly<KIND>(rec, stride, k0, p0);
        load_poly<KIND>(rec, stride, k1 < ncand ? k1 : k0, p1);
        f(p0);
        if (k1 < ncand) f(p1);
    }
}

// Slot t of a lane's registers holds band position lane + t GROUP.  Each chunk
// sits under a branch on its first position: a chunk wholly past the band's end
// takes the zero records without loading, and the compiler cannot hoist a later
// chunk's loads above the branch, so no more than one chunk of taps is live.
template <typename T, int KIND, int GROUP, int RPL, bool LAZY, int CHUNK = ring_chunk<T, GROUP>()>
__device__ __forceinline__ void ring_to_regs(const T* __restrict__ u, int H, int W, const RingBand& band, int lane,
                                             const double* __restrict__ cpend, int nj, int pq,
                                             PolyRing<KIND> (&rg)[RPL])
{
    constexpr int CH = RPL < CHUNK ? RPL : CHUNK;
#pragma unroll
    for (int t0 = 0; t0 < RPL; t0 += CH) {
        if (lane + t0 * GROUP < band.n) {
            RingTaps<T, LAZY> tp[CH];
#pragma unroll
            for (int s = 0; s < CH; ++s) {
                if (t0 + s >= RPL) break;
                const int k = lane + (t0 + s) * GROUP;
                int i, j;
                band_at(band, k < band.n ? k : 0, i, j);
                load_taps<T, LAZY>(u, H, W, i, j, band.r0, band.r1, band.c0, band.c1, tp[s], cpend, nj, pq);
            }
#pragma unroll
            for (int s = 0; s < CH; ++s) {
                if (t0 + s >= RPL) break;
                Ring r;
                ring_from_taps<T, LAZY>(tp[s], r, lane + (t0 + s) * GROUP < band.n);
                make_poly<KIND>(r, rg[t0 + s]);
            }
        } else {
#pragma unroll
            for (int s = 0; s < CH; ++s) {
                if (t0 + s >= RPL) break;
                Ring r;
                zero_ring(r);
                make_poly<KIND>(r, rg[t0 + s]);
            }
        }
    }
}

// Rings larger than the registers hold: position k is expanded into column k of
// a region of rec_stride columns per coefficient, by lane k mod GROUP.
template <typename T, int KIND, int GROUP, bool LAZY, int CHUNK = ring_chunk<T, GROUP>()>
__device__ __forceinline__ void ring_to_region(const T* __restrict__ u, int H, int W, const RingBand& band, int lane,
                                               const double* __restrict__ cpend, int nj, int pq,
                                               double* __restrict__ rec, int rec_stride)
{
    constexpr int CH = CHUNK;
    for (int k0 = lane; k0 < band.n; k0 += CH * GROUP) {
        RingTaps<T, LAZY> tp[CH];
#pragma unroll
        for (int s = 0; s < CH; ++s) {
            const int k = k0 + s * GROUP;
            int i, j;
            band_at(band, k < band.n ? k : 0, i, j);
            load_taps<T, LAZY>(u, H, W, i, j, band.r0, band.r1, band.c0, band.c1, tp[s], cpend, nj, pq);
        }
#pragma unroll
        for (int s = 0; s < CH; ++s) {
            const int k = k0 + s * GROUP;
            if (k < band.n) {
                Ring r;
                PolyRing<KIND> pr;
                ring_from_taps<T, LAZY>(tp[s], r);
                make_poly<KIND>(r, pr);
                store_poly<KIND>(rec, rec_stride, k, pr);
            }
        }
    }
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
    double* rec;             // RPL = 0: this block's region for its expanded ring records, or null
    int rec_stride;          // records per coefficient row of a region (8b)
};

// Fine block levels walk their block's pixels (sum of f - u, then the update) in
// rounds of BLOCK_UNROLL elements per lane: block_walk gives the addresses of
// elements k0, k0 + GROUP, ... of a round (elements past n take element k0's
// address and are skipped by the caller) and advances the walk (i, j) by the
// round.
constexpr int BLOCK_UNROLL = 4;

template <int GROUP>
__device__ __forceinline__ void block_walk(int k0, int n, int& i, int& j, int si, int sj, int c1, int w, int W,
                                           size_t (&idx)[BLOCK_UNROLL])
{
#pragma unroll
    for (int m = 0; m < BLOCK_UNROLL; ++m) {
        idx[m] = (m == 0 || k0 + m * GROUP < n) ? (size_t)i * W + j : idx[0];
        i += si;
        j += sj;
        if (j >= c1) { j -= w; ++i; }
    }
}

template <typename T, int KIND, int GROUP, int RPL, bool LAZY, int CHUNK = ring_chunk<T, GROUP>(), class GSum>
__device__ __forceinline__ void solve_block(T* __restrict__ u, const T* __restrict__ f, int H, int W,
                                            int p, int q, int r0, int r1, int c0, int c1, int lane,
                                            double alpha, int M, int G, const GSum& gsum, const CoarseArgs& ca)
{
    const int h = r1 - r0, w = c1 - c0;
    double rsum = 0.0;   // this lane's part of the sum of f - u over the block
    if (LAZY) {
        const double* part = ca.partials + ((size_t)p * ca.nj + q) * ca.nchunk;
        for (int k = lane; k < ca.nchunk; k += GROUP) rsum += part[k];
    } else {
        // element k = lane + m GROUP is pixel (r0 + k / w, c0 + k % w), advanced incrementally;
        // BLOCK_UNROLL elements have their loads in flight together and are summed in order
        const int si = GROUP / w, sj = GROUP - si * w;
        int i = r0 + lane / w, j = c0 + lane % w;
        for (int k0 = lane; k0 < h * w; k0 += BLOCK_UNROLL * GROUP) {
            size_t idx[BLOCK_UNROLL];
            block_walk<GROUP>(k0, h * w, i, j, si, sj, c1, w, W, idx);
            double fv[BLOCK_UNROLL], uv[BLOCK_UNROLL];
#pragma unroll
            for (int m = 0; m < BLOCK_UNROLL; ++m) {
                fv[m] = (double)f[idx[m]];
                uv[m] = (double)u[idx[m]];
            }
#pragma unroll
            for (int m = 0; m < BLOCK_UNROLL; ++m) {
                if (k0 + m * GROUP >= h * w) break;
                rsum += fv[m] - uv[m];
            }
        }
    }
    // the group total of rsum (and with it f*) is taken after the ring records are built, so the
    // loads of both are in flight together
    const double s = (double)h * (double)w;
    const int pq = p * ca.nj + q;   // lazy levels: this block's pending correction
    const RingBand band = ring_band(H, W, r0, r1, c0, c1);
    const int ncand = band.n;

    double cval;
    if (RPL > 0) {
        PolyRing<KIND> rg[RPL > 0 ? RPL : 1];
        ring_to_regs<T, KIND, GROUP, (RPL > 0 ? RPL : 1), LAZY, CHUNK>(u, H, W, band, lane, ca.cpend, ca.nj, pq, rg);
        const double fs = gsum(rsum) / s;
        auto Kpart = [&](const auto& cs, auto& out) {
            constexpr int N = sizeof(out) / sizeof(double);
#pragma unroll
            for (int k = 0; k < N; ++k) out[k] = 0.0;
            // slots past the last candidate hold zero records and are skipped
            // (whole wavefronts at once on the coarse levels)
#pragma unroll
            for (int t = 0; t < RPL; ++t)
                if (lane + t * GROUP < ncand) {
#pragma unroll
                    for (int k = 0; k < N; ++k) out[k] += abs_poly<KIND>(rg[t], cs[k]);
                }
        };
        auto Dpart = [&](double c) {
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < RPL; ++t)
                if (lane + t * GROUP < ncand) acc += dabs_poly<KIND>(rg[t], c);
            return acc;
        };
        cval = local_solve(Kpart, Dpart, gsum, fs, alpha * s, M, G);
    } else if (ca.rec) {
        // rings larger than the registers hold: each lane expands its records once into the
        // block's region and reads them back (only its own) at every evaluation, in the same
        // order as the rebuilding loop below
        ring_to_region<T, KIND, GROUP, LAZY, CHUNK>(u, H, W, band, lane, ca.cpend, ca.nj, pq, ca.rec, ca.rec_stride);
        const double fs = gsum(rsum) / s;
        auto Kpart = [&](const auto& cs, auto& out) {
            constexpr int N = sizeof(out) / sizeof(double);
#pragma unroll
            for (int k = 0; k < N; ++k) out[k] = 0.0;
            for (int kk = lane; kk < ncand; kk += GROUP) {
                PolyRing<KIND> pr;
                load_poly<KIND>(ca.rec, ca.rec_stride, kk, pr);
#pragma unroll
                for (int k = 0; k < N; ++k) out[k] += abs_poly<KIND>(pr, cs[k]);
            }
        };
        auto Dpart = [&](double c) {
            double acc = 0.0;
            for (int kk = lane; kk < ncand; kk += GROUP) {
                PolyRing<KIND> pr;
                load_poly<KIND>(ca.rec, ca.rec_stride, kk, pr);
                acc += dabs_poly<KIND>(pr, c);
            }
            return acc;
        };
        cval = local_solve(Kpart, Dpart, gsum, fs, alpha * s, M, G);
    } else {
        const double fs = gsum(rsum) / s;
        auto Kpart = [&](const auto& cs, auto& out) {
            constexpr int N = sizeof(out) / sizeof(double);
#pragma unroll
            for (int k = 0; k < N; ++k) out[k] = 0.0;
            for (int kk = lane; kk < ncand; kk += GROUP) {
                int i, j;
                Ring rr;
                PolyRing<KIND> pr;
                band_at(band, kk, i, j);
                make_ring<T, LAZY>(u, H, W, i, j, r0, r1, c0, c1, rr, ca.cpend, ca.nj, pq);
                make_poly<KIND>(rr, pr);
#pragma unroll
                for (int k = 0; k < N; ++k) out[k] += abs_poly<KIND>(pr, cs[k]);
            }
        };
        auto Dpart = [&](double c) {
            double acc = 0.0;
            for (int kk = lane; kk < ncand; kk += GROUP) {
                int i, j;
                Ring rr;
                PolyRing<KIND> pr;
                band_at(band, kk, i, j);
                make_ring<T, LAZY>(u, H, W, i, j, r0, r1, c0, c1, rr, ca.cpend, ca.nj, pq);
                make_poly<KIND>(rr, pr);
                acc += dabs_poly<KIND>(pr, c);
            }
            return acc;
        };
        cval = local_solve(Kpart, Dpart, gsum, fs, alpha * s, M, G);
    }
    if (LAZY) {
        if (lane == 0) ca.cpend[(size_t)p * ca.nj + q] = cval;
    } else if (cval != 0.0) {
        const int si = GROUP / w, sj = GROUP - si * w;
        int i = r0 + lane / w, j = c0 + lane % w;
        for (int k0 = lane; k0 < h * w; k0 += BLOCK_UNROLL * GROUP) {
            size_t idx[BLOCK_UNROLL];
            block_walk<GROUP>(k0, h * w, i, j, si, sj, c1, w, W, idx);
            T uv[BLOCK_UNROLL];
#pragma unroll
            for (int m = 0; m < BLOCK_UNROLL; ++m) uv[m] = u[idx[m]];
#pragma unroll
            for (int m = 0; m < BLOCK_UNROLL; ++m) {
                if (k0 + m * GROUP >= h * w) break;
                u[idx[m]] = (T)((double)uv[m] + cval);
            }
        }
    }
}

// Blocks of one colour at b = 2: the colour's sub-grid is nbr x nbc, sub-block
// (bi, bj) being block (2 bi + pr, 2 bj + pc) of the m_j x n_j grid.  Its
// interior blocks (off the image border) form the rectangle [bi0, bi0 + nir) x
// [bj0, bj0 + nic); the border blocks (the rest) are numbered first, so they
// fill whole wavefronts of their own.
struct Split2 {
    int nbr, nbc, bi0, nir, bj0, nic, nborder;
};

__host__ __device__ __forceinline__ Split2 split2(int mj, int nj, int pr, int pc)
{
    Split2 S;
    S.nbr = (mj - pr + 1) / 2;
    S.nbc = (nj - pc + 1) / 2;
    S.bi0 = pr == 0 ? 1 : 0;   // p = 0 is on the border
    S.bj0 = pc == 0 ? 1 : 0;
    const int ri = mj - 2 - pr, ci = nj - 2 - pc;   // p <= m_j - 2  <=>  bi <= (m_j - 2 - pr) / 2
    S.nir = ri >= 0 ? ri / 2 - S.bi0 + 1 : 0;
    S.nic = ci >= 0 ? ci / 2 - S.bj0 + 1 : 0;
    if (S.nir < 0) S.nir = 0;
    if (S.nic < 0) S.nic = 0;
    if (S.nir == 0 || S.nic == 0) S.nir = S.nic = 0;
    S.nborder = S.nbr * S.nbc - S.nir * S.nic;
    return S;
}

__host__ __device__ __forceinline__ bool split2_at(const Split2& S, int k, int& bi, int& bj)
{
    if (k >= S.nborder) {
        k -= S.nborder;
        bi = S.bi0 + k / S.nic;
        bj = S.bj0 + k % S.nic;
        return true;
    }
    if (S.nir == 0) {   // no interior: every block is a border block
        bi = k / S.nbc;
        bj = k % S.nbc;
        return false;
    }
    const int top = S.bi0 * S.nbc;
    if (k < top) { bi = k / S.nbc; bj = k % S.nbc; return false; }
    k -= top;
    const int bot0 = S.bi0 + S.nir, bot = (S.nbr - bot0) * S.nbc;
    if (k < bot) { bi = bot0 + k / S.nbc; bj = k % S.nbc; return false; }
    k -= bot;
    const int side = S.nbc - S.nic;   // border blocks per middle row (left, then right)
    const int m = k % side;
    bi = S.bi0 + k / side;
    bj = m < S.bj0 ? m : S.nic + m;
    return false;
}

// One lane of the QL-lane group solving sub-block k of a b = 2 colour.
template <typename T, int KIND, int QL>
__device__ __forceinline__ void solve_b2_item(T* __restrict__ u, const T* __restrict__ f, int H, int W, int pr, int pc,
                                              const Split2& S, int k, int lane, double alpha, int M, int G)
{
    int bi, bj;
    const bool interior = split2_at(S, k, bi, bj);
    const int p = 2 * bi + pr, q = 2 * bj + pc;
    const int r0 = 2 * p, c0 = 2 * q;
    if (interior) {
        solve_block2_interior<T, KIND, QL>(u, f, H, W, r0, c0, lane, alpha, M, G);
    } else {
        // one record at a time: the few border blocks must not raise the registers of the kernel
        const CoarseArgs ca{nullptr, 0, nullptr, 0, nullptr, 16};
        solve_block<T, KIND, QL, 16 / QL, false, 1>(u, f, H, W, p, q, r0, min(r0 + 2, H), c0, min(c0 + 2, W), lane,
                                                    alpha, M, G, WaveSum<QL>(), ca);
    }
}

}  // namespace mgc
