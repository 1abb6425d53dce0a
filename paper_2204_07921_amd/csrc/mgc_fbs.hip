// The paper's own local step on gfx950: forward-backward splitting (Algorithm 2)
// with the tangent-plane estimates of Proposition 1 (mean curvature, eq. (c-sol1))
// and Proposition 2 (Gaussian curvature), backward step eq. (c-sol2) in its patch
// form (Section 2.2), on patches of side b_j = 2^j - 1 with the four-colour order
// of Section 2.3.  Host runtime and the mg_fbs_* entry points of include/mgcurv.h.
//
// Tangent planes.  On ring r = 1 .. 2^(j-1) around a patch centre O the eight
// pixels at offsets r (di, dj) form four chords through O (W-E, N-S, NW-SE,
// NE-SW); each chord with either ring pixel perpendicular to it spans a plane.
// With l the half chord length in the image plane (r on axis chords, r sqrt 2 on
// diagonal ones, which is also the distance of the third vertex from the chord),
// h = (u_a + u_b) / 2 and e = (u_b - u_a) / 2, the plane rises by e / l along the
// chord and by (u_t - h) / l across it, so the signed distance from (O, u_O) to it
// is l (h - u_O) / sqrt(l^2 + e^2 + (u_t - h)^2) (positive when the plane is above
// the point; on the finest level this is eq. (distance to tri)), and the half
// chord's squared 3-D length is ds^2 = l^2 + e^2.  Positions outside the image
// take the value of the nearest image pixel (the prolonged domain).
//
// Data flow per V-cycle (state dtype T = float or double, local math in FP64):
//   level 1 (b = 1): one launch; a workgroup loads a 64 x 64 tile (32 x 64 for
//     double) of u with a 4-pixel halo into LDS (16-byte vectors when the box
//     lies inside the image) and runs the four colour sweeps there, shrinking
//     the region it trusts by one pixel per colour (each sweep reads one pixel
//     around the updated pixel) and reading f at the pixels it solves, then
//     writes the tile to the other buffer.  Every pixel is read once and
//     written once per level.
//   levels with patch side 3 and 7: one launch each, the same scheme with a
//     tile of patches and a halo of 4 patches (corrections kept in LDS); the
//     sums of f over their patches come from one pass over f per V-cycle.
//   larger patches: (1) per patch and row chunk, FP64 partial sums of f - u over
//     the patch (the patch's own pixels do not change before its colour);
//     (2) four colour launches, a lane group per patch holding the rings,
//     reading tap values as u + the correction of the tap's patch (rounded to T)
//     when that patch's colour came earlier in the level; (3) u <- u + c_patch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/mgcurv.h"
#include "mgc_internal.h"

#include "mgc_fbs_device.h"

namespace fbs {

// ---------------------------------------------------------------------------
// Level 1 (b = 1): the four colours of the level in one launch.
// ---------------------------------------------------------------------------
constexpr int PHALO = 4;

// FBS correction of pixel (i, j) from its clamped 3x3 neighbourhood `at(ii, jj)`.
template <int KIND, class At>
__device__ __forceinline__ double pixel_correction(const At& at, int i, int j, int H, int W, double fs, double alpha,
                                                   int steps)
{
    double v[8];
    bool self[8];
    const double uo = at(i, j);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int ii = clampi(i + ring_di(k), 0, H - 1), jj = clampi(j + ring_dj(k), 0, W - 1);
        v[k] = at(ii, jj);
        self[k] = ii == i && jj == j;
    }
    double c = 0.0, eta = 1.0;
    for (int t = 0; t < steps; ++t) {
        double w8[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) w8[k] = self[k] ? v[k] + c : v[k];
        double sum = 0.0;
        GcAcc g = gc_empty();
        ring_accumulate<KIND>(uo + c, w8, 1.0, 0, sum, g);
        const double est = KIND == 0 ? sum * 0.125 : gc_choice(g);
        c = backward(c, c + est, eta * alpha, fs);
        if (t + 1 < steps) eta = 1.0 / sqrt(1.0 + (double)t);
    }
    return c;
}

// The same correction for a pixel off the image border: no tap is clamped, so
// none is the pixel itself, and the eight ring values are read from LDS at fixed
// offsets of the centre (W, E, N, S, NW, SE, NE, SW for a row stride LW).
template <int KIND, int LW, typename T>
__device__ __forceinline__ double interior_correction(const T* __restrict__ cp, double uo, double fs, double alpha,
                                                      int steps)
{
    const double v[8] = {(double)cp[-1],      (double)cp[1],      (double)cp[-LW],     (double)cp[LW],
                         (double)cp[-LW - 1], (double)cp[LW + 1], (double)cp[-LW + 1], (double)cp[LW - 1]};
    double c = 0.0, eta = 1.0;
    for (int t = 0; t < steps; ++t) {
        double sum = 0.0;
        GcAcc g = gc_empty();
        ring_accumulate<KIND>(uo + c, v, 1.0, 0, sum, g);
        const double est = KIND == 0 ? sum * 0.125 : gc_choice(g);
        c = backward(c, c + est, eta * alpha, fs);
        if (t + 1 < steps) eta = 1.0 / sqrt(1.0 + (double)t);
    }
    return c;
}

template <typename T, int KIND, int TH, int TW, int NT>
__global__ __launch_bounds__(NT) void fbs_pixel_level_kernel(const T* __restrict__ uin, T* __restrict__ uout,
                                                             const T* __restrict__ f, int H, int W, double alpha,
                                                             int steps, int vec16)
{
    constexpr int LW = TW + 2 * PHALO;
    __shared__ __attribute__((aligned(16))) T su[(TH + 2 * PHALO) * LW];
    const int y0 = blockIdx.y * TH, x0 = blockIdx.x * TW;
    const int ly = y0 - PHALO, lx = x0 - PHALO;
    const int r_lo = max(0, ly), r_hi = min(H, y0 + TH + PHALO);
    const int c_lo = max(0, lx), c_hi = min(W, x0 + TW + PHALO);
    const int nr = r_hi - r_lo, nc = c_hi - c_lo;
    // a tile whose loaded box lies inside the image moves whole 16-byte vectors (vec16: the
    // buffers and the row length allow it); the others take the general copy
    const bool box = vec16 && ly >= 0 && lx >= 0 && y0 + TH + PHALO <= H && x0 + TW + PHALO <= W;
    // with a margin on every side (no loaded edge is an image edge) every pixel the tile solves
    // lies off the image border, at least one pixel inside the loaded box: the whole workgroup
    // takes the unclamped form
    const bool inner = ly > 0 && lx > 0 && y0 + TH + PHALO < H && x0 + TW + PHALO < W;
    // u of the loaded region; f is read from memory at the pixel solved (once per colour that
    // solves it), which halves the workgroup's LDS and lets more workgroups share a CU
    if (box)
        box_copy16<NT, TH + 2 * PHALO, LW>(uin + (size_t)ly * W + lx, (long)W, su, LW);
    else
        tile_copy<NT, 12>(nr, nc, uin + (size_t)r_lo * W + c_lo, (long)W, su + (r_lo - ly) * LW + (c_lo - lx), LW);
    __syncthreads();
    auto at = [&](int ii, int jj) { return (double)su[(ii - ly) * LW + (jj - lx)]; };
    for (int k = 0; k < 4; ++k) {
        // region still exact after sweep k: k + 1 pixels inside every tile edge that is not an image edge
        const int vr0 = r_lo == 0 ? 0 : r_lo + k + 1, vr1 = r_hi == H ? H : r_hi - k - 1;
        const int vc0 = c_lo == 0 ? 0 : c_lo + k + 1, vc1 = c_hi == W ? W : c_hi - k - 1;
        const int i0 = vr0 + ((vr0 & 1) != (k >> 1)), j0 = vc0 + ((vc0 & 1) != (k & 1));
        const int ni = i0 < vr1 ? (vr1 - i0 + 1) / 2 : 0, nj = j0 < vc1 ? (vc1 - j0 + 1) / 2 : 0;
        if (ni > 0 && nj > 0)
        for (GridWalk w(threadIdx.x, NT, nj); w.a < ni; w.next()) {
            const int i = i0 + 2 * w.a, j = j0 + 2 * w.b;
            const int o = (i - ly) * LW + (j - lx);
            const double fv = (double)f[(size_t)i * W + j];
            const double uo = (double)su[o];
            const double fs = fv - uo;
            const double c = inner ? interior_correction<KIND, LW>(su + o, uo, fs, alpha, steps)
                                   : pixel_correction<KIND>(at, i, j, H, W, fs, alpha, steps);
            // pixels of one colour read only other colours (or themselves), so the write is safe
            su[o] = (T)(uo + c);
        }
        __syncthreads();
    }
    const int onr = min(H, y0 + TH) - y0, onc = min(W, x0 + TW) - x0;
    if (box)
        box_copy16<NT, TH, TW>(su + PHALO * LW + PHALO, LW, uout + (size_t)y0 * W + x0, (long)W);
    else
        tile_copy<NT, 8>(onr, onc, su + (y0 - ly) * LW + (x0 - lx), LW, uout + (size_t)y0 * W + x0, (long)W);
}

// Tile of the pixel level per state type: (rows, columns, threads).
template <typename T> struct PixelTile { static constexpr int TH = 64, TW = 64, NT = 512; };
template <> struct PixelTile<double> { static constexpr int TH = 32, TW = 64, NT = 512; };

// One colour of level 1, in place (for single-sweep inspection).
template <typename T, int KIND>
__global__ __launch_bounds__(256) void fbs_pixel_colour_kernel(T* __restrict__ u, const T* __restrict__ f, int H,
                                                               int W, int colour, double alpha, int steps)
{
    const int pr = colour >> 1, pc = colour & 1;
    const int ni = (H - pr + 1) / 2, nj = (W - pc + 1) / 2;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)ni * nj) return;
    const int i = pr + 2 * (int)(t / nj), j = pc + 2 * (int)(t % nj);
    auto at = [&](int ii, int jj) { return (double)u[(size_t)ii * W + jj]; };
    const double uo = at(i, j);
    const double c = pixel_correction<KIND>(at, i, j, H, W, (double)f[(size_t)i * W + j] - uo, alpha, steps);
    u[(size_t)i * W + j] = (T)(uo + c);
}

// ---------------------------------------------------------------------------
// Levels j >= 2.
// ---------------------------------------------------------------------------

// A whole coarse level with small patches (side B) in one launch.  A workgroup
// owns TP x TP patches and loads them with a halo of HALO patches into LDS;
// colour k is solved for the patches at least k + 1 patches inside every
// loaded edge that is not an image edge (a patch reads at most one pixel of
// its neighbours and their corrections of earlier colours), so after the four
// colours the owned patches are exact.  A group of G = (B + 1) / 2 lanes
// solves one patch (lane l holds ring l + 1).  Corrections live in LDS; the
// owned pixels are written to the other buffer with their patch's correction.
template <typename T, int KIND, int B, int TP, int NT>
__global__ __launch_bounds__(NT) void fbs_patch_level_kernel(const T* __restrict__ uin, T* __restrict__ uout,
                                                             const double* __restrict__ fsum, int H, int W, int mj,
                                                             int nj, double alpha, int steps)
{
    constexpr int HALO = 4, LP = TP + 2 * HALO, LPX = LP * B, R = (B + 1) / 2, G = R;
    __shared__ T su[LPX * LPX];
    __shared__ double sc[LP * LP];    // corrections of the loaded patches
    __shared__ double ss[LP * LP];    // sums of f - u over the loaded patches
    const int P0 = blockIdx.y * TP, Q0 = blockIdx.x * TP;
    const int lp0 = P0 - HALO, lq0 = Q0 - HALO;
    const int pa = max(0, lp0), pb = min(mj, P0 + TP + HALO);
    const int qa = max(0, lq0), qb = min(nj, Q0 + TP + HALO);
    const int ly = lp0 * B, lx = lq0 * B;
    const int ra = pa * B, rb = min(H, pb * B), ca = qa * B, cb = min(W, qb * B);
    tile_copy<NT, 16>(rb - ra, cb - ca, uin + (size_t)ra * W + ca, (long)W, su + (ra - ly) * LPX + (ca - lx), LPX);
    for (int t = threadIdx.x; t < LP * LP; t += NT) sc[t] = 0.0;
    __syncthreads();
    // sum of f - u over each patch as (sum of f) - (sum of u): the sums of f come
    // from fbs_fsums_kernel, the patch's pixels do not change before its colour
    for (int t = threadIdx.x; t < LP * LP; t += NT) {
        const int pl = t / LP, ql = t - pl * LP, p = lp0 + pl, q = lq0 + ql;
        if (p < pa || p >= pb || q < qa || q >= qb) continue;
        double su_sum = 0.0;
        for (int i = p * B; i < min(p * B + B, H); ++i)
            for (int j = q * B; j < min(q * B + B, W); ++j) su_sum += (double)su[(i - ly) * LPX + (j - lx)];
        ss[t] = fsum[(size_t)p * nj + q] - su_sum;
    }
    __syncthreads();
    const int lane = threadIdx.x % G;
    for (int k = 0; k < 4; ++k) {
        const int vp0 = pa == 0 ? 0 : pa + k + 1, vp1 = pb == mj ? mj : pb - k - 1;
        const int vq0 = qa == 0 ? 0 : qa + k + 1, vq1 = qb == nj ? nj : qb - k - 1;
        const int p0 = vp0 + ((vp0 & 1) != (k >> 1)), q0 = vq0 + ((vq0 & 1) != (k & 1));
        const int np = p0 < vp1 ? (vp1 - p0 + 1) / 2 : 0, nq = q0 < vq1 ? (vq1 - q0 + 1) / 2 : 0;
        if (np > 0 && nq > 0)
        for (GridWalk w(threadIdx.x / G, NT / G, nq); w.a < np; w.next()) {
            const int p = p0 + 2 * w.a, q = q0 + 2 * w.b;
            const int r0 = p * B, r1 = min(r0 + B, H), c0 = q * B, c1 = min(c0 + B, W);
            const double s = (double)((r1 - r0) * (c1 - c0)), fs = ss[(p - lp0) * LP + (q - lq0)] / s;
            const int oi = r0 + R - 1, oj = c0 + R - 1;
            auto value = [&](int i, int j, double shift) {
                const int ci = clampi(i, 0, H - 1), cj = clampi(j, 0, W - 1);
                const double x = (double)su[(ci - ly) * LPX + (cj - lx)];
                const int tp = ci / B, tq = cj / B;
                if (tp == p && tq == q) return x + shift;
                const double cp = sc[(tp - lp0) * LP + (tq - lq0)];
                return cp != 0.0 ? (double)(T)(x + cp) : x;
            };
            // patches whose taps stay inside the image: ring r < R lies in the patch,
            // ring R in the neighbour (p + di, q + dj); same values as `value`
            const bool interior = r0 >= 1 && c0 >= 1 && r0 + B < H && c0 + B < W;
            const int r = lane + 1;
            auto ring_value = [&](int m, double shift) {
                const int di = ring_di(m), dj = ring_dj(m);
                if (!interior) return value(oi + r * di, oj + r * dj, shift);
                const double x = (double)su[(oi + r * di - ly) * LPX + (oj + r * dj - lx)];
                if (r < R) return x + shift;
                const double cp = sc[(p + di - lp0) * LP + (q + dj - lq0)];
                return cp != 0.0 ? (double)(T)(x + cp) : x;
            };
            double c = 0.0, eta = 1.0;
            for (int t = 0; t < steps; ++t) {
                double sum = 0.0;
                GcAcc acc = gc_empty();
                const double uo = value(oi, oj, c);
                double v[8];
#pragma unroll
                for (int m = 0; m < 8; ++m) v[m] = ring_value(m, c);
                ring_accumulate<KIND>(uo, v, (double)r, 8 * (r - 1), sum, acc);
                double est;
                if constexpr (KIND == 0) {
                    est = group_sum<G>(sum) / (double)(8 * R);
                } else {
                    group_extremes<G>(acc);
                    est = gc_choice(acc);
                }
                c = backward(c, c + est, eta * alpha * s, fs);
                eta = 1.0 / sqrt(1.0 + (double)t);
            }
            if (lane == 0) sc[(p - lp0) * LP + (q - lq0)] = c;
        }
        __syncthreads();
    }
    // owned pixels with their patch's correction: one row segment of a patch per step
    const int o_r0 = P0 * B, onr = min(H, (P0 + TP) * B) - o_r0, ntq = min(nj, Q0 + TP) - Q0;
    if (onr > 0 && ntq > 0)
        for (GridWalk w(threadIdx.x, NT, ntq); w.a < onr; w.next()) {
            const int i = o_r0 + w.a, q = Q0 + w.b;
            const double c = sc[(i / B - lp0) * LP + (q - lq0)];
            const T* srow = su + (i - ly) * LPX - lx;
            T* drow = uout + (size_t)i * W;
#pragma unroll
            for (int m = 0; m < B; ++m) {
                const int j = q * B + m;
                if (j < W) drow[j] = c != 0.0 ? (T)((double)srow[j] + c) : srow[j];
            }
        }
}

// Sums of f over the patches of side 3 and of side 7 (row-major within a patch):
// a workgroup loads a 42 x 42 tile of f, which holds 14 x 14 and 6 x 6 whole patches.
template <typename T>
__global__ __launch_bounds__(256) void fbs_fsums_kernel(const T* __restrict__ f, int H, int W, double* __restrict__ fsum3,
                                                        double* __restrict__ fsum7)
{
    constexpr int TS = 42;
    __shared__ T sf[TS * TS];
    const int y0 = blockIdx.y * TS, x0 = blockIdx.x * TS;
    const int nr = min(TS, H - y0), nc = min(TS, W - x0);
    tile_copy<256, 7>(nr, nc, f + (size_t)y0 * W + x0, (long)W, sf, TS);
    __syncthreads();
    const int n3 = (W + 2) / 3, n7 = (W + 6) / 7;
    for (int t = threadIdx.x; t < 14 * 14 + 6 * 6; t += 256) {
        const int B = t < 196 ? 3 : 7, k = t < 196 ? t : t - 196, per = TS / B;
        const int pl = k / per, ql = k - pl * per;
        if (pl * B >= nr || ql * B >= nc) continue;
        double S = 0.0;
        for (int r = pl * B; r < min(pl * B + B, nr); ++r)
            for (int c = ql * B; c < min(ql * B + B, nc); ++c) S += (double)sf[r * TS + c];
        const int p = y0 / B + pl, q = x0 / B + ql;
        if (B == 3) fsum3[(size_t)p * n3 + q] = S;
        else fsum7[(size_t)p * n7 + q] = S;
    }
}

// Partial sums of f - u per (patch, row chunk), L lanes per group (patches too
// large for the colour kernel's own groups to sum).
template <typename T, int L>
__global__ __launch_bounds__(256) void fbs_sums_kernel(const T* __restrict__ u, const T* __restrict__ f, int H, int W,
                                                       int b, int nj, int ngroups, int nchunk, int rows_per,
                                                       double* __restrict__ psums)
{
    __shared__ double lds[4];
    const int g = (int)((blockIdx.x * blockDim.x + threadIdx.x) / L);
    const int lane = threadIdx.x % L;
    const bool live = g < ngroups;
    double acc = 0.0;
    if (live) {
        const int patch = g / nchunk, k = g - patch * nchunk;
        const int p = patch / nj, q = patch - p * nj;
        const int r0 = p * b + k * rows_per, r1 = min(min(r0 + rows_per, p * b + b), H);
        const int c0 = q * b, c1 = min(c0 + b, W), w = c1 - c0;
        const int n = (r1 > r0 ? r1 - r0 : 0) * w;
        for (int t = lane; t < n; t += L) {
            const size_t idx = (size_t)(r0 + t / w) * W + (c0 + t % w);
            acc += (double)f[idx] - (double)u[idx];
        }
    }
    if constexpr (L <= 64) {
#pragma unroll
        for (int off = 1; off < L; off <<= 1) acc += __shfl_xor(acc, off, 64);
    } else {
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
        if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
        __syncthreads();
        acc = (lds[0] + lds[1]) + (lds[2] + lds[3]);
    }
    if (live && lane == 0) psums[g] = acc;
}

// One colour of a coarse level: a group of G lanes per patch, lane l taking rings
// l + 1, l + 1 + G, ...; the patch's correction goes to cpend.  A neighbour's
// entry in cpend counts only if its colour was solved earlier in this pass
// (solved_from <= colour' < colour); other entries are stale and read as 0.
// With nchunk == 0 the group sums f - u over the patch itself, else it adds
// the row-chunk partials of fbs_sums_kernel.
template <typename T, int KIND, int G>
__global__ __launch_bounds__(256) void fbs_patch_kernel(const T* __restrict__ u, const T* __restrict__ f, int H, int W,
                                                        int b, int mj, int nj, int colour, int solved_from, int nchunk,
                                                        const double* __restrict__ psums, double* __restrict__ cpend,
                                                        double alpha, int steps)
{
    const int R = (b + 1) / 2;
    const int pr = colour >> 1, pc = colour & 1;
    const int na = (mj - pr + 1) / 2, nb = (nj - pc + 1) / 2;
    const int gid = (int)((blockIdx.x * blockDim.x + threadIdx.x) / G), lane = threadIdx.x % G;
    const bool live = gid < na * nb;
    const int p = live ? 2 * (gid / nb) + pr : 0, q = live ? 2 * (gid % nb) + pc : 0;
    const int r0 = p * b, r1 = min(r0 + b, H), c0 = q * b, c1 = min(c0 + b, W);
    const int oi = r0 + R - 1, oj = c0 + R - 1;
    const int patch = p * nj + q;
    double S = 0.0;
    if (nchunk == 0) {
        const int w = c1 - c0, n = live ? (r1 - r0) * w : 0;
        for (int t = lane; t < n; t += G) {
            const size_t idx = (size_t)(r0 + t / w) * W + (c0 + t % w);
            S += (double)f[idx] - (double)u[idx];
        }
#pragma unroll
        for (int off = 1; off < G; off <<= 1) S += __shfl_xor(S, off, 64);
    } else if (live) {
        for (int k = 0; k < nchunk; ++k) S += psums[(size_t)patch * nchunk + k];
    }
    const double s = (double)((r1 - r0) * (c1 - c0));
    const double fs = S / s;
    // state value at a clamped position: u + pending correction of its patch (own patch: + shift)
    auto value = [&](int i, int j, double shift) {
        const int ci = clampi(i, 0, H - 1), cj = clampi(j, 0, W - 1);
        const double x = (double)u[(size_t)ci * W + cj];
        const int dp = ci < r0 ? -1 : (ci >= r1 ? 1 : 0), dq = cj < c0 ? -1 : (cj >= c1 ? 1 : 0);
        if (dp == 0 && dq == 0) return x + shift;
        const int np = p + dp, nq = q + dq;
        const int ncol = 2 * (np & 1) + (nq & 1);
        if (ncol < solved_from || ncol >= colour) return x;
        const double cp = cpend[(size_t)np * nj + nq];
        return cp != 0.0 ? (double)(T)(x + cp) : x;
    };
    double c = 0.0, eta = 1.0;
    for (int t = 0; t < steps; ++t) {
        double sum = 0.0;
        GcAcc g = gc_empty();
        if (live) {
            const double uo = value(oi, oj, c);
            for (int r = lane + 1; r <= R; r += G) {
                double v[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) v[k] = value(oi + r * ring_di(k), oj + r * ring_dj(k), c);
                ring_accumulate<KIND>(uo, v, (double)r, 8 * (r - 1), sum, g);
            }
        }
        double est;
        if constexpr (KIND == 0) {
#pragma unroll
            for (int off = 1; off < G; off <<= 1) sum += __shfl_xor(sum, off, 64);
            est = sum / (double)(8 * R);
        } else {
#pragma unroll
            for (int off = 1; off < G; off <<= 1) {
                const double ok = __shfl_xor(g.kmin, off, 64), od = __shfl_xor(g.dmin, off, 64);
                const int oid = __shfl_xor(g.imin, off, 64);
                if (ok < g.kmin || (ok == g.kmin && oid < g.imin)) { g.kmin = ok; g.dmin = od; g.imin = oid; }
                const double xk = __shfl_xor(g.kmax, off, 64), xd = __shfl_xor(g.dmax, off, 64);
                const int xid = __shfl_xor(g.imax, off, 64);
                if (xk > g.kmax || (xk == g.kmax && xid < g.imax)) { g.kmax = xk; g.dmax = xd; g.imax = xid; }
            }
            est = gc_choice(g);
        }
        c = backward(c, c + est, eta * alpha * s, fs);
        eta = 1.0 / sqrt(1.0 + (double)t);
    }
    if (live && lane == 0) cpend[patch] = c;
}

// dst <- src + c of the pixel's patch (rounded to T) for patches whose colour
// lies in [cmin, cmax].  In place (src == dst) only pixels with a nonzero
// correction are written.
template <typename T>
__global__ __launch_bounds__(256) void fbs_apply_kernel(const T* src, T* dst, int H, int W, int b, int nj,
                                                        const double* __restrict__ cpend, int in_place, int cmin,
                                                        int cmax)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= W) return;
    const int q = j / b;
    for (int i = blockIdx.y; i < H; i += gridDim.y) {
        const int p = i / b, col = 2 * (p & 1) + (q & 1);
        const double c = (col >= cmin && col <= cmax) ? cpend[(size_t)p * nj + q] : 0.0;
        const size_t idx = (size_t)i * W + j;
        if (in_place) {
            if (c != 0.0) dst[idx] = (T)((double)src[idx] + c);
        } else {
            dst[idx] = c != 0.0 ? (T)((double)src[idx] + c) : src[idx];
        }
    }
}

// relErr(u) (Section 4): partial sums of (u - prev)^2 and u^2, then one
// workgroup adds the partials in a fixed order.
constexpr int NORM_BLOCKS = 1024;

template <typename T>
__global__ __launch_bounds__(256) void fbs_norms_kernel(const T* __restrict__ u, const T* __restrict__ prev, size_t n,
                                                        double* __restrict__ part)
{
    __shared__ double lds[8];
    double a = 0.0, b = 0.0;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const double x = (double)u[t], d = x - (double)prev[t];
        a += d * d;
        b += x * x;
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        lds[threadIdx.x >> 6] = a;
        lds[4 + (threadIdx.x >> 6)] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
        part[2 * blockIdx.x + 1] = (lds[4] + lds[5]) + (lds[6] + lds[7]);
    }
}

__global__ __launch_bounds__(256) void fbs_norms_final_kernel(const double* __restrict__ part, int np,
                                                              double* __restrict__ out)
{
    __shared__ double lds[8];
    double a = 0.0, b = 0.0;
    for (int t = threadIdx.x; t < np; t += blockDim.x) {
        a += part[2 * t];
        b += part[2 * t + 1];
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        lds[threadIdx.x >> 6] = a;
        lds[4 + (threadIdx.x >> 6)] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
        out[1] = (lds[4] + lds[5]) + (lds[6] + lds[7]);
    }
}

// Row chunks of the partial sums: about 16k pixels each.
void patch_geometry(int H, int W, int b, int* mj, int* nj, int* nchunk, int* rows_per)
{
    *mj = (H + b - 1) / b;
    *nj = (W + b - 1) / b;
    int rp = 16384 / b;
    if (rp < 1) rp = 1;
    if (rp > b) rp = b;
    *rows_per = rp;
    *nchunk = (b + rp - 1) / rp;
}

}  // namespace fbs

// ---------------------------------------------------------------------------
// Host runtime
// ---------------------------------------------------------------------------
namespace {

// A captured V-cycle for one (u, f) pair.  what: 0 = V-cycle only; 1 = then
// F(u) and a copy to the host mirror; 2 = copy of u to prev first, then the
// V-cycle, F(u), the relErr(u) norms and the host copy.
struct FbsGraph {
    const void* u = nullptr;
    const void* f = nullptr;
    int what = -1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

constexpr int NGRAPHS = 4;

}  // namespace

struct mg_fbs_ctx {
    mg_fbs_params P;
    int device;
    hipStream_t stream;    // caller's stream: every launch and graph replay goes here
    hipStream_t gstream;   // own stream, used only to capture graphs (default priority)
    void* scratch[2];      // two H x W state images for the one-launch levels
    void* prev;            // H x W state image (relErr(u) stop rule)
    double* psums;         // patch partial sums, max over the levels that use them
    double* cpend;         // corrections of the current level, max patches over coarse levels
    double* fsum3;         // sums of f over the patches of side 3 and 7 (fused levels)
    double* fsum7;
    double* epart;         // energy partials
    double* npart;         // norm partials (2 * NORM_BLOCKS)
    double* dev3;          // energy, ||u - prev||^2, ||u||^2
    double* host3;         // pinned copy of dev3
    FbsGraph graphs[NGRAPHS];
    int next_graph;
    std::string err;
};

namespace {

thread_local std::string g_fbs_init_error;

// Patches up to this side are summed by the colour kernel's own lane groups.
constexpr int INLINE_SUM_MAX_SIDE = 15;

mg_status ffail(mg_fbs_ctx* ctx, mg_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf; else g_fbs_init_error = buf;
    return st;
}

mg_status fhip(mg_fbs_ctx* ctx, hipError_t e, const char* what)
{
    return ffail(ctx, MG_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool is64(const mg_fbs_ctx* c) { return c->P.state_dtype == MG_F64; }
size_t fbytes(const mg_fbs_ctx* c) { return (size_t)c->P.height * c->P.width * (is64(c) ? 8 : 4); }

mg_status fcheck(mg_fbs_ctx* ctx, const void* u, const void* f)
{
    if (!ctx) return MG_E_INVALID;
    if (!u || !f) return ffail(ctx, MG_E_INVALID, "u and f must be non-null device pointers");
    const size_t n = fbytes(ctx);
    const char* a = (const char*)u;
    const char* b = (const char*)f;
    if (a < b + n && b < a + n) return ffail(ctx, MG_E_INVALID, "u must not overlap f");
    return MG_OK;
}

template <typename T>
hipError_t launch_pixel_level(const mg_fbs_ctx* c, hipStream_t st, const void* uin, void* uout, const void* f)
{
    const int H = c->P.height, W = c->P.width;
    using Tile = fbs::PixelTile<T>;
    dim3 grid((W + Tile::TW - 1) / Tile::TW, (H + Tile::TH - 1) / Tile::TH), block(Tile::NT);
    // 16-byte accesses need 16-byte aligned buffers and rows of whole vectors
    const int vec16 = ((((uintptr_t)uin | (uintptr_t)uout | (uintptr_t)f) & 15) == 0) && W % (16 / (int)sizeof(T)) == 0;
    if (c->P.curvature == MG_CURV_MEAN)
        hipLaunchKernelGGL((fbs::fbs_pixel_level_kernel<T, 0, Tile::TH, Tile::TW, Tile::NT>), grid, block, 0, st,
                           (const T*)uin, (T*)uout, (const T*)f, H, W, c->P.alpha, c->P.steps, vec16);
    else
        hipLaunchKernelGGL((fbs::fbs_pixel_level_kernel<T, 1, Tile::TH, Tile::TW, Tile::NT>), grid, block, 0, st,
                           (const T*)uin, (T*)uout, (const T*)f, H, W, c->P.alpha, c->P.steps, vec16);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pixel_colour(const mg_fbs_ctx* c, hipStream_t st, void* u, const void* f, int colour)
{
    const int H = c->P.height, W = c->P.width;
    const size_t n = (size_t)((H - (colour >> 1) + 1) / 2) * ((W - (colour & 1) + 1) / 2);
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (c->P.curvature == MG_CURV_MEAN)
        hipLaunchKernelGGL((fbs::fbs_pixel_colour_kernel<T, 0>), grid, block, 0, st, (T*)u, (const T*)f, H, W,
                           colour, c->P.alpha, c->P.steps);
    else
        hipLaunchKernelGGL((fbs::fbs_pixel_colour_kernel<T, 1>), grid, block, 0, st, (T*)u, (const T*)f, H, W,
                           colour, c->P.alpha, c->P.steps);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sums(const mg_fbs_ctx* c, hipStream_t st, const void* u, const void* f, int b)
{
    const int H = c->P.height, W = c->P.width;
    int mj, nj, nchunk, rows_per;
    fbs::patch_geometry(H, W, b, &mj, &nj, &nchunk, &rows_per);
    const int ngroups = mj * nj * nchunk;
    const long pix = (long)b * (b < rows_per ? b : rows_per);   // pixels per group
    auto grid_for = [&](int L) { return dim3((unsigned)(((size_t)ngroups * L + 255) / 256)); };
#define FBS_SUMS(L)                                                                                                 \
    hipLaunchKernelGGL((fbs::fbs_sums_kernel<T, L>), grid_for(L), dim3(256), 0, st, (const T*)u, (const T*)f, H, W, \
                       b, nj, ngroups, nchunk, rows_per, c->psums)
    if (pix <= 1024) FBS_SUMS(64);
    else FBS_SUMS(256);
#undef FBS_SUMS
    return hipGetLastError();
}

template <typename T, int KIND>
hipError_t launch_patch_kind(const mg_fbs_ctx* c, hipStream_t st, const void* u, const void* f, int b, int colour,
                             int solved_from)
{
    const int H = c->P.height, W = c->P.width;
    int mj, nj, nchunk, rows_per;
    fbs::patch_geometry(H, W, b, &mj, &nj, &nchunk, &rows_per);
    if (b <= INLINE_SUM_MAX_SIDE) nchunk = 0;
    const int pr = colour >> 1, pc = colour & 1;
    const int npatch = ((mj - pr + 1) / 2) * ((nj - pc + 1) / 2);
    if (npatch <= 0) return hipSuccess;
    const int R = (b + 1) / 2;
    const int G = R < 64 ? R : 64;
    dim3 grid((unsigned)(((size_t)npatch * G + 255) / 256)), block(256);
#define FBS_PATCH(GG)                                                                                               \
    hipLaunchKernelGGL((fbs::fbs_patch_kernel<T, KIND, GG>), grid, block, 0, st, (const T*)u, (const T*)f, H, W, b, \
                       mj, nj, colour, solved_from, nchunk, (const double*)c->psums, c->cpend, c->P.alpha,           \
                       c->P.steps)
    switch (G) {
    case 2: FBS_PATCH(2); break;
    case 4: FBS_PATCH(4); break;
    case 8: FBS_PATCH(8); break;
    case 16: FBS_PATCH(16); break;
    case 32: FBS_PATCH(32); break;
    default: FBS_PATCH(64); break;
    }
#undef FBS_PATCH
    return hipGetLastError();
}

template <typename T>
hipError_t launch_patch(const mg_fbs_ctx* c, hipStream_t st, const void* u, const void* f, int b, int colour,
                        int solved_from)
{
    return c->P.curvature == MG_CURV_MEAN ? launch_patch_kind<T, 0>(c, st, u, f, b, colour, solved_from)
                                          : launch_patch_kind<T, 1>(c, st, u, f, b, colour, solved_from);
}

template <typename T>
hipError_t launch_apply(const mg_fbs_ctx* c, hipStream_t st, const void* src, void* dst, int b, int cmin, int cmax)
{
    const int H = c->P.height, W = c->P.width;
    const int nj = (W + b - 1) / b;
    const int gy = H < 1024 ? H : 1024;
    dim3 grid((W + 255) / 256, gy), block(256);
    hipLaunchKernelGGL(fbs::fbs_apply_kernel<T>, grid, block, 0, st, (const T*)src, (T*)dst, H, W, b, nj,
                       (const double*)c->cpend, src == dst ? 1 : 0, cmin, cmax);
    return hipGetLastError();
}

// Patch sides whose whole level runs as one fused launch, and its tile in patches.
template <typename T, int KIND, int B, int TP>
hipError_t launch_patch_level_kind(const mg_fbs_ctx* c, hipStream_t st, const void* src, void* dst)
{
    constexpr int NT = 256;
    const int H = c->P.height, W = c->P.width;
    const int mj = (H + B - 1) / B, nj = (W + B - 1) / B;
    dim3 grid((nj + TP - 1) / TP, (mj + TP - 1) / TP), block(NT);
    hipLaunchKernelGGL((fbs::fbs_patch_level_kernel<T, KIND, B, TP, NT>), grid, block, 0, st, (const T*)src, (T*)dst,
                       (const double*)(B == 3 ? c->fsum3 : c->fsum7), H, W, mj, nj, c->P.alpha, c->P.steps);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fsums(const mg_fbs_ctx* c, hipStream_t st, const void* f)
{
    const int H = c->P.height, W = c->P.width;
    dim3 grid((W + 41) / 42, (H + 41) / 42), block(256);
    hipLaunchKernelGGL(fbs::fbs_fsums_kernel<T>, grid, block, 0, st, (const T*)f, H, W, c->fsum3, c->fsum7);
    return hipGetLastError();
}

bool has_fused_level(int b) { return b == 3 || b == 7; }

template <typename T>
hipError_t launch_patch_level(const mg_fbs_ctx* c, hipStream_t st, const void* src, void* dst, int b)
{
    const bool mc = c->P.curvature == MG_CURV_MEAN;
    // tiles of (16 + 8) * 3 and (8 + 8) * 7 pixels square
    constexpr int TP7 = 8;
    if (b == 3) return mc ? launch_patch_level_kind<T, 0, 3, 16>(c, st, src, dst)
                          : launch_patch_level_kind<T, 1, 3, 16>(c, st, src, dst);
    return mc ? launch_patch_level_kind<T, 0, 7, TP7>(c, st, src, dst)
              : launch_patch_level_kind<T, 1, 7, TP7>(c, st, src, dst);
}

// Coarse level j >= 2 on the state in `src`; the result lands in `dst`.
// only_colour < 0 runs the four colours, else that colour alone.
template <typename T>
mg_status coarse_level(mg_fbs_ctx* c, hipStream_t st, const void* src, void* dst, const void* f, int level,
                       int only_colour)
{
    const int b = (1 << level) - 1;
    hipError_t e;
    if (b > INLINE_SUM_MAX_SIDE && (e = launch_sums<T>(c, st, src, f, b)) != hipSuccess)
        return fhip(c, e, "patch sums launch");
    const int first = only_colour < 0 ? 0 : only_colour, last = only_colour < 0 ? 3 : only_colour;
    for (int colour = first; colour <= last; ++colour) {
        e = launch_patch<T>(c, st, src, f, b, colour, first);
        if (e != hipSuccess) return fhip(c, e, "patch colour launch");
    }
    e = launch_apply<T>(c, st, src, dst, b, first, last);
    if (e != hipSuccess) return fhip(c, e, "apply launch");
    return MG_OK;
}

// The levels of one V-cycle in order: 1..J, then J-1..1 for the full cycle.
// Levels run as one launch (the pixel level and patch sides 3 and 7) read one
// buffer and write another; the others may write in place.  Buffers are
// assigned from the last level back so that the last level writes u: only a
// lone one-launch level needs a final copy.  The sums of f for the one-launch
// coarse levels are computed first, in the same stream (a forked branch costs
// more in cross-queue waits than it overlaps).
template <typename T>
mg_status run_levels(mg_fbs_ctx* c, hipStream_t st, void* u, const void* f, const int* levels, int nlevels)
{
    auto one_launch = [&](int level) { return level == 1 || has_fused_level((1 << level) - 1); };
    void* dst[64];
    dst[nlevels - 1] = u;
    for (int n = nlevels - 2; n >= 0; --n)
        dst[n] = one_launch(levels[n + 1]) ? (dst[n + 1] == c->scratch[0] ? c->scratch[1] : c->scratch[0]) : dst[n + 1];
    // the first level reads u; if it is a one-launch level it cannot also write u:
    // then it writes scratch[0], and either the next level (which may write to
    // another buffer) or a final copy brings the result to u
    if (one_launch(levels[0]) && dst[0] == u) dst[0] = c->scratch[0];
    bool need_fsums = false;
    for (int n = 0; n < nlevels; ++n) need_fsums = need_fsums || (levels[n] > 1 && one_launch(levels[n]));
    hipError_t e;
    if (need_fsums && (e = launch_fsums<T>(c, st, f)) != hipSuccess) return fhip(c, e, "patch sums of f launch");
    const void* cur = u;
    for (int n = 0; n < nlevels; ++n) {
        const int level = levels[n];
        const int b = (1 << level) - 1;
        if (level == 1) {
            e = launch_pixel_level<T>(c, st, cur, dst[n], f);
            if (e != hipSuccess) return fhip(c, e, "pixel level launch");
        } else if (has_fused_level(b)) {
            e = launch_patch_level<T>(c, st, cur, dst[n], b);
            if (e != hipSuccess) return fhip(c, e, "patch level launch");
        } else {
            mg_status r = coarse_level<T>(c, st, cur, dst[n], f, level, -1);
            if (r != MG_OK) return r;
        }
        cur = dst[n];
    }
    if (cur != u) {
        e = hipMemcpyAsync(u, cur, fbytes(c), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return fhip(c, e, "state copy");
    }
    return MG_OK;
}

mg_status vcycle_enqueue(mg_fbs_ctx* c, hipStream_t st, void* u, const void* f)
{
    int lv[64], n = 0;
    for (int j = 1; j <= c->P.levels; ++j) lv[n++] = j;
    if (c->P.cycle == 1)
        for (int j = c->P.levels - 1; j >= 1; --j) lv[n++] = j;
    return is64(c) ? run_levels<double>(c, st, u, f, lv, n) : run_levels<float>(c, st, u, f, lv, n);
}

mgc::LaunchCtx energy_ctx(const mg_fbs_ctx* c, hipStream_t st)
{
    mgc::LaunchCtx L;
    L.stream = st;
    L.H = c->P.height;
    L.W = c->P.width;
    L.alpha = c->P.alpha;
    L.kind = c->P.curvature;
    L.f64 = is64(c);
    L.M = 0;
    L.G = 0;
    return L;
}

// F(u) into dev3[0] and, if `norms`, ||u - prev||^2 and ||u||^2 into
// dev3[1..2], then a copy to the pinned host mirror (enqueued only).
mg_status measure_enqueue(mg_fbs_ctx* c, hipStream_t st, const void* u, const void* f, bool norms)
{
    hipError_t e = mgc::launch_energy(energy_ctx(c, st), u, f, c->epart, c->dev3);
    if (e != hipSuccess) return fhip(c, e, "energy launch");
    if (norms) {
        const size_t n = (size_t)c->P.height * c->P.width;
        if (is64(c))
            hipLaunchKernelGGL(fbs::fbs_norms_kernel<double>, dim3(fbs::NORM_BLOCKS), dim3(256), 0, st,
                               (const double*)u, (const double*)c->prev, n, c->npart);
        else
            hipLaunchKernelGGL(fbs::fbs_norms_kernel<float>, dim3(fbs::NORM_BLOCKS), dim3(256), 0, st,
                               (const float*)u, (const float*)c->prev, n, c->npart);
        hipLaunchKernelGGL(fbs::fbs_norms_final_kernel, dim3(1), dim3(256), 0, st, (const double*)c->npart,
                           fbs::NORM_BLOCKS, c->dev3 + 1);
        if ((e = hipGetLastError()) != hipSuccess) return fhip(c, e, "norm launch");
    }
    e = hipMemcpyAsync(c->host3, c->dev3, 3 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return fhip(c, e, "result copy");
    return MG_OK;
}

void drop_graph(FbsGraph& g)
{
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = FbsGraph();
}

// The captured graph for (u, f, what), capturing it on the own stream first if needed.
mg_status get_graph(mg_fbs_ctx* c, void* u, const void* f, int what, hipGraphExec_t* out)
{
    for (auto& g : c->graphs)
        if (g.exec && g.u == u && g.f == f && g.what == what) {
            *out = g.exec;
            return MG_OK;
        }
    FbsGraph& g = c->graphs[c->next_graph];
    c->next_graph = (c->next_graph + 1) % NGRAPHS;
    drop_graph(g);
    hipStream_t st = c->gstream;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fhip(c, e, "begin capture");
    mg_status r = MG_OK;
    if (what == 2) {
        e = hipMemcpyAsync(c->prev, u, fbytes(c), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) r = fhip(c, e, "state copy");
    }
    if (r == MG_OK) r = vcycle_enqueue(c, st, u, f);
    if (r == MG_OK && what >= 1) r = measure_enqueue(c, st, u, f, what == 2);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(st, &graph);
    if (r != MG_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
    }
    if (e != hipSuccess) return fhip(c, e, "end capture");
    g.graph = graph;
    if ((e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0)) != hipSuccess) {
        drop_graph(g);
        return fhip(c, e, "graph instantiate");
    }
    g.u = u;
    g.f = f;
    g.what = what;
    *out = g.exec;
    return MG_OK;
}

// Launch graph `what` for (u, f) into the caller's stream (captured once on the
// own stream); wait: also block until it is done.
mg_status replay(mg_fbs_ctx* c, void* u, const void* f, int what, bool wait)
{
    hipGraphExec_t exec;
    mg_status r = get_graph(c, u, f, what, &exec);
    if (r != MG_OK) return r;
    hipError_t e;
    if ((e = hipGraphLaunch(exec, c->stream)) != hipSuccess) return fhip(c, e, "graph launch");
    if (wait && (e = hipStreamSynchronize(c->stream)) != hipSuccess) return fhip(c, e, "stream synchronize");
    return MG_OK;
}

mg_status measure_now(mg_fbs_ctx* c, const void* u, const void* f)
{
    mg_status r = measure_enqueue(c, c->stream, u, f, false);
    if (r != MG_OK) return r;
    hipError_t e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? MG_OK : fhip(c, e, "stream synchronize");
}

}  // namespace

extern "C" {

void mg_fbs_default_params(mg_fbs_params* p, int32_t height, int32_t width)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->height = height;
    p->width = width;
    p->alpha = 20.0;
    p->curvature = MG_CURV_MEAN;
    p->levels = 3;
    p->state_dtype = MG_F32;
    p->steps = 1;
    p->cycle = 0;
}

mg_status mg_fbs_init(const mg_fbs_params* params, void* hip_stream, mg_fbs_ctx** out)
{
    if (!params || !out) return ffail(nullptr, MG_E_INVALID, "params and out must be non-null");
    *out = nullptr;
    const mg_fbs_params& p = *params;
    if (p.height < 2 || p.width < 2) return ffail(nullptr, MG_E_SHAPE, "height and width must be >= 2 (got %d x %d)", p.height, p.width);
    if ((int64_t)p.height * p.width > ((int64_t)1 << 31) - 1)
        return ffail(nullptr, MG_E_SHAPE, "image larger than 2^31 - 1 pixels");
    if (!(p.alpha >= 0.0) || !std::isfinite(p.alpha)) return ffail(nullptr, MG_E_INVALID, "alpha must be finite and >= 0");
    if (p.curvature != MG_CURV_MEAN && p.curvature != MG_CURV_GAUSS) return ffail(nullptr, MG_E_INVALID, "curvature must be 0 (mean) or 1 (Gaussian)");
    if (p.state_dtype != MG_F32 && p.state_dtype != MG_F64) return ffail(nullptr, MG_E_DTYPE, "state_dtype must be MG_F32 or MG_F64");
    if (p.levels < 1 || p.levels > 16) return ffail(nullptr, MG_E_INVALID, "levels must be in [1, 16]");
    if (p.steps < 1 || p.steps > 64) return ffail(nullptr, MG_E_INVALID, "steps must be in [1, 64]");
    if (p.cycle != 0 && p.cycle != 1) return ffail(nullptr, MG_E_INVALID, "cycle must be 0 (fine to coarse) or 1 (and back)");
    if (p.reserved != 0) return ffail(nullptr, MG_E_INVALID, "reserved must be 0");

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) return ffail(nullptr, MG_E_DEVICE, "no HIP device available");
    mg_fbs_ctx* c = new (std::nothrow) mg_fbs_ctx();
    if (!c) return ffail(nullptr, MG_E_NOMEM, "host allocation failed");
    c->P = p;
    c->stream = (hipStream_t)hip_stream;
    c->gstream = nullptr;
    c->scratch[0] = c->scratch[1] = c->prev = nullptr;
    c->psums = c->cpend = c->epart = c->npart = c->dev3 = c->host3 = nullptr;
    c->fsum3 = c->fsum7 = nullptr;
    c->next_graph = 0;
    (void)hipGetDevice(&c->device);
    size_t n_ps = 1, n_cp = 1;
    for (int level = 2; level <= p.levels; ++level) {
        int mj, nj, nchunk, rows_per;
        fbs::patch_geometry(p.height, p.width, (1 << level) - 1, &mj, &nj, &nchunk, &rows_per);
        if ((size_t)mj * nj * nchunk > n_ps) n_ps = (size_t)mj * nj * nchunk;
        if ((size_t)mj * nj > n_cp) n_cp = (size_t)mj * nj;
    }
    const size_t nb = fbytes(c);
    const int ne = mgc::energy_partials_count(p.height, p.width);
    if (hipMalloc(&c->scratch[0], nb) != hipSuccess || hipMalloc(&c->scratch[1], nb) != hipSuccess ||
        hipMalloc(&c->prev, nb) != hipSuccess ||
        hipMalloc((void**)&c->psums, sizeof(double) * n_ps) != hipSuccess ||
        hipMalloc((void**)&c->cpend, sizeof(double) * n_cp) != hipSuccess ||
        hipMalloc((void**)&c->fsum3, sizeof(double) * ((p.height + 2) / 3) * ((p.width + 2) / 3)) != hipSuccess ||
        hipMalloc((void**)&c->fsum7, sizeof(double) * ((p.height + 6) / 7) * ((p.width + 6) / 7)) != hipSuccess ||
        hipMalloc((void**)&c->epart, sizeof(double) * ne) != hipSuccess ||
        hipMalloc((void**)&c->npart, sizeof(double) * 2 * fbs::NORM_BLOCKS) != hipSuccess ||
        hipMalloc((void**)&c->dev3, 3 * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void**)&c->host3, 3 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        mg_fbs_destroy(c);
        (void)hipGetLastError();
        return ffail(nullptr, MG_E_NOMEM, "device allocation of 2 x %zu bytes failed", nb);
    }
    if (hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess) {
        mg_fbs_destroy(c);
        (void)hipGetLastError();
        return ffail(nullptr, MG_E_DEVICE, "stream creation failed");
    }
    *out = c;
    return MG_OK;
}

mg_status mg_fbs_vcycle(mg_fbs_ctx* ctx, void* u, const void* f, double* energy_after)
{
    mg_status st = fcheck(ctx, u, f);
    if (st != MG_OK) return st;
    if ((st = replay(ctx, u, f, energy_after ? 1 : 0, energy_after != nullptr)) != MG_OK) return st;
    if (energy_after) *energy_after = ctx->host3[0];
    return MG_OK;
}

mg_status mg_fbs_level(mg_fbs_ctx* ctx, void* u, const void* f, int32_t level)
{
    mg_status st = fcheck(ctx, u, f);
    if (st != MG_OK) return st;
    if (level < 1 || level > ctx->P.levels) return ffail(ctx, MG_E_INVALID, "level must be in [1, %d]", ctx->P.levels);
    int lv[1] = {level};
    return is64(ctx) ? run_levels<double>(ctx, ctx->stream, u, f, lv, 1)
                     : run_levels<float>(ctx, ctx->stream, u, f, lv, 1);
}

mg_status mg_fbs_sweep(mg_fbs_ctx* ctx, void* u, const void* f, int32_t level, int32_t colour)
{
    mg_status st = fcheck(ctx, u, f);
    if (st != MG_OK) return st;
    if (level < 1 || level > ctx->P.levels) return ffail(ctx, MG_E_INVALID, "level must be in [1, %d]", ctx->P.levels);
    if (colour < 0 || colour > 3) return ffail(ctx, MG_E_INVALID, "colour must be in [0, 4)");
    if (level == 1) {
        hipError_t e = is64(ctx) ? launch_pixel_colour<double>(ctx, ctx->stream, u, f, colour)
                                 : launch_pixel_colour<float>(ctx, ctx->stream, u, f, colour);
        return e == hipSuccess ? MG_OK : fhip(ctx, e, "pixel colour launch");
    }
    return is64(ctx) ? coarse_level<double>(ctx, ctx->stream, u, u, f, level, colour)
                     : coarse_level<float>(ctx, ctx->stream, u, u, f, level, colour);
}

mg_status mg_fbs_energy(mg_fbs_ctx* ctx, const void* u, const void* f, double* energy)
{
    mg_status st = fcheck(ctx, u, f);
    if (st != MG_OK) return st;
    if (!energy) return ffail(ctx, MG_E_INVALID, "energy output must be non-null");
    if ((st = measure_now(ctx, u, f)) != MG_OK) return st;
    *energy = ctx->host3[0];
    return MG_OK;
}

mg_status mg_fbs_solve(mg_fbs_ctx* ctx, void* u, const void* f, double tol, int32_t max_vcycles, int32_t stop,
                       int32_t* vcycles_done, double* final_energy, double* energy_trace)
{
    mg_status st = fcheck(ctx, u, f);
    if (st != MG_OK) return st;
    if (max_vcycles < 0) return ffail(ctx, MG_E_INVALID, "max_vcycles must be >= 0");
    if (!std::isfinite(tol)) return ffail(ctx, MG_E_INVALID, "tol must be finite");
    if (stop != MG_STOP_ENERGY && stop != MG_STOP_RELERR_U) return ffail(ctx, MG_E_INVALID, "stop must be MG_STOP_ENERGY or MG_STOP_RELERR_U");
    if ((st = measure_now(ctx, u, f)) != MG_OK) return st;
    double e_prev = ctx->host3[0];
    if (!std::isfinite(e_prev)) return ffail(ctx, MG_E_NONFINITE, "energy of the initial state is not finite");
    if (energy_trace) energy_trace[0] = e_prev;
    int done = 0;
    bool converged = false;
    double e = e_prev;
    const bool relerr = stop == MG_STOP_RELERR_U;
    while (done < max_vcycles) {
        if ((st = replay(ctx, u, f, relerr ? 2 : 1, true)) != MG_OK) return st;
        ++done;
        e = ctx->host3[0];
        if (energy_trace) energy_trace[done] = e;
        if (!std::isfinite(e)) return ffail(ctx, MG_E_NONFINITE, "energy became non-finite after V-cycle %d", done);
        if (tol > 0.0) {
            const bool hit = relerr ? std::sqrt(ctx->host3[1]) < tol * std::sqrt(ctx->host3[2])
                                    : (e == e_prev || std::fabs(e - e_prev) < tol * std::fabs(e));
            if (hit) { converged = true; break; }
        }
        e_prev = e;
    }
    if (vcycles_done) *vcycles_done = done;
    if (final_energy) *final_energy = e;
    return (tol > 0.0 && !converged) ? MG_NOT_CONVERGED : MG_OK;
}

void mg_fbs_destroy(mg_fbs_ctx* ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->gstream) (void)hipStreamSynchronize(ctx->gstream);
    for (auto& g : ctx->graphs) drop_graph(g);
    if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);

    if (ctx->scratch[0]) (void)hipFree(ctx->scratch[0]);
    if (ctx->scratch[1]) (void)hipFree(ctx->scratch[1]);
    if (ctx->prev) (void)hipFree(ctx->prev);
    if (ctx->psums) (void)hipFree(ctx->psums);
    if (ctx->cpend) (void)hipFree(ctx->cpend);
    if (ctx->fsum3) (void)hipFree(ctx->fsum3);
    if (ctx->fsum7) (void)hipFree(ctx->fsum7);
    if (ctx->epart) (void)hipFree(ctx->epart);
    if (ctx->npart) (void)hipFree(ctx->npart);
    if (ctx->dev3) (void)hipFree(ctx->dev3);
    if (ctx->host3) (void)hipHostFree(ctx->host3);
    delete ctx;
}

const char* mg_fbs_last_error(const mg_fbs_ctx* ctx)
{
    if (ctx) return ctx->err.c_str();
    return g_fbs_init_error.c_str();
}

}  // extern "C"
