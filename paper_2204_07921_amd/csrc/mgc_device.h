// Device-side building blocks of the multigrid curvature sweep (gfx950).
//
// A "ring record" describes one pixel p whose curvature changes when a block B
// is shifted by c: the five finite-difference derivatives of u at p (3x3
// central differences of Table 1's curvatures, replicated ghost pixels) and
// their slopes in c.  Because every derivative is a linear combination of
// taps and exactly the taps inside B move by c, each derivative is affine in
// c: d(c) = a + beta * c, with beta the same stencil applied to the 0/1 mask
// of taps inside B.  Evaluating the local energy at a new c then needs no
// memory traffic at all.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mgc {

enum { KIND_MEAN = 0, KIND_GAUSS = 1 };

struct Ring {
    // derivative order: u_x, u_y, u_xx, u_yy, u_xy
    double a[5];
    double b[5];
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ void zero_ring(Ring& r)
{
#pragma unroll
    for (int k = 0; k < 5; ++k) { r.a[k] = 0.0; r.b[k] = 0.0; }
}

// 3x3 central differences of a tap window t[row][col] (row 0 = i - 1, col 0 = j - 1).
__device__ __forceinline__ void stencil5(const double t[3][3], double d[5])
{
    d[0] = 0.5 * (t[1][2] - t[1][0]);
    d[1] = 0.5 * (t[2][1] - t[0][1]);
    d[2] = (t[1][2] + t[1][0]) - 2.0 * t[1][1];
    d[3] = (t[2][1] + t[0][1]) - 2.0 * t[1][1];
    d[4] = 0.25 * ((t[2][2] - t[0][2]) - (t[2][0] - t[0][0]));
}

// Index in the m_j x n_j pending corrections of the block holding tap (ci, cj)
// (clamped into the image) of a ring pixel of block B = rows [r0, r1) x cols
// [c0, c1), pq = p nj + q.  A ring pixel lies within one pixel of B and a tap
// within one pixel of it, so for b >= 2 a tap above (below, left of, right of) B
// lies in the neighbouring block on that side: comparisons give the index for
// any block side, powers of two or not.
// Side of v against [lo, hi) (lo < hi): -1 below, +1 at or above hi, 0 inside; and
// 1 inside, 0 outside.  Taken from sign bits, so a lane computes them without
// compare masks (which, for the nine taps of several records, outgrow the scalar
// registers).
__host__ __device__ __forceinline__ int side_of(int v, int lo, int hi)
{
    return ((v - lo) >> 31) - ((hi - 1 - v) >> 31);
}
__host__ __device__ __forceinline__ int inside_of(int v, int lo, int hi)
{
    return 1 + ((v - lo) >> 31) + ((hi - 1 - v) >> 31);
}

__host__ __device__ __forceinline__ int tap_block(int pq, int nj, int ci, int cj, int r0, int r1, int c0, int c1)
{
    return pq + side_of(ci, r0, r1) * nj + side_of(cj, c0, c1);
}

// The nine clamped taps of pixel (i, j) as loaded from memory (and, LAZY, the
// pending correction of the block each lies in): the first half of a ring
// record.  Kept apart from the arithmetic so that a lane can put the loads of
// several records in flight before it uses any of them.  mask: bit 3 (dy + 1) +
// (dx + 1) is set when tap (dy, dx) lies inside B, bit 9 when (i, j) lies inside
// the image.
template <typename T, bool LAZY>
struct RingTaps {
    T v[3][3];
    double cp[LAZY ? 3 : 1][LAZY ? 3 : 1];
    int mask;
};

// Loads the taps of pixel (i, j) for block rows [r0, r1) x cols [c0, c1).  Every
// address is clamped into the image, so any (i, j) may be passed.
template <typename T, bool LAZY>
__device__ __forceinline__ void load_taps(const T* __restrict__ u, int H, int W, int i, int j, int r0, int r1,
                                          int c0, int c1, RingTaps<T, LAZY>& tp,
                                          const double* __restrict__ cpend, int nj, int pq)
{
    int mask = (inside_of(i, 0, H) & inside_of(j, 0, W)) << 9;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        const int ci = clampi(i + dy, 0, H - 1);
        const int rin = inside_of(ci, r0, r1);
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int cj = clampi(j + dx, 0, W - 1);
            tp.v[dy + 1][dx + 1] = u[(size_t)ci * W + cj];
            if constexpr (LAZY) tp.cp[dy + 1][dx + 1] = cpend[tap_block(pq, nj, ci, cj, r0, r1, c0, c1)];
            mask |= (rin & inside_of(cj, c0, c1)) << (3 * (dy + 1) + (dx + 1));
        }
    }
    tp.mask = mask;
}

// The ring record from loaded taps.  With pending corrections (coarse levels
// apply a level's corrections lazily) a tap's value is u + c_pending of its
// block, rounded to the state type exactly as an eager update would have stored
// it.  Pixels outside the image, pixels whose nine clamped taps lie all inside
// or all outside B (their curvature does not depend on c), and any pixel with
// use = false get the zero record, which contributes exactly 0 to every sum
// below.  The slopes are the stencil of the 0/1 mask of taps inside B, formed
// in integers (the same small exact values as the FP64 stencil of the mask);
// the zero record is selected at the end rather than branched to, so the build
// takes no divergent paths.
template <typename T, bool LAZY>
__device__ __forceinline__ void ring_from_taps(const RingTaps<T, LAZY>& tp, Ring& r, bool use = true)
{
    double t[3][3];
    int m[3][3];
#pragma unroll
    for (int y = 0; y < 3; ++y)
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            const double v = (double)tp.v[y][x];
            if constexpr (LAZY) t[y][x] = (double)(T)(v + tp.cp[y][x]);
            else t[y][x] = v;
            m[y][x] = (tp.mask >> (3 * y + x)) & 1;
        }
    const int n = __builtin_popcount(tp.mask & 511);
    const bool keep = use && (tp.mask >> 9) != 0 && n != 0 && n != 9;
    double a[5], bs[5];
    stencil5(t, a);
    bs[0] = 0.5 * (double)(m[1][2] - m[1][0]);
    bs[1] = 0.5 * (double)(m[2][1] - m[0][1]);
    bs[2] = (double)(m[1][2] + m[1][0] - 2 * m[1][1]);
    bs[3] = (double)(m[2][1] + m[0][1] - 2 * m[1][1]);
    bs[4] = 0.25 * (double)((m[2][2] - m[0][2]) - (m[2][0] - m[0][0]));
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        r.a[k] = keep ? a[k] : 0.0;
        r.b[k] = keep ? bs[k] : 0.0;
    }
}

// Build the ring record of pixel (i, j) for block rows [r0, r1) x cols [c0, c1).
// LAZY: pq = p nj + q (see tap_block).
template <typename T, bool LAZY = false>
__device__ __forceinline__ void make_ring(const T* __restrict__ u, int H, int W, int i, int j,
                                          int r0, int r1, int c0, int c1, Ring& r,
                                          const double* __restrict__ cpend = nullptr, int nj = 0, int pq = 0)
{
    if (i < 0 || i >= H || j < 0 || j >= W) { zero_ring(r); return; }
    RingTaps<T, LAZY> tp;
    load_taps<T, LAZY>(u, H, W, i, j, r0, r1, c0, c1, tp, cpend, nj, pq);
    ring_from_taps<T, LAZY>(tp, r);
}

// |kappa| of a ring record at shift c.
template <int KIND>
__device__ __forceinline__ double abs_kappa(const Ring& r, double c)
{
    const double ux = fma(r.b[0], c, r.a[0]);
    const double uy = fma(r.b[1], c, r.a[1]);
    const double uxx = fma(r.b[2], c, r.a[2]);
    const double uyy = fma(r.b[3], c, r.a[3]);
    const double uxy = fma(r.b[4], c, r.a[4]);
    const double q = fma(ux, ux, fma(uy, uy, 1.0));
    if (KIND == KIND_MEAN) {
        // div(grad u / sqrt(1 + |grad u|^2)) expanded: numerator / q^{3/2}
        const double num = fma(fma(uy, uy, 1.0), uxx, fma(fma(ux, ux, 1.0), uyy, -2.0 * ux * uy * uxy));
        const double rq = rsqrt(q);
        return fabs(num) * (rq * rq * rq);
    } else {
        const double det = fma(uxx, uyy, -uxy * uxy);
        const double iq = 1.0 / q;
        return fabs(det) * (iq * iq);
    }
}

// 1/sqrt(q) for finite q > 0: the hardware estimate, then one step of the
// series 1/sqrt(q) = y (1 - e)^{-1/2} = y (1 + e/2 + 3e^2/8 + ...), e = 1 - q y^2,
// which takes the estimate to full double precision.
__device__ __forceinline__ double rsqrt_pos(double q)
{
    const double y = __builtin_amdgcn_rsq(q);
    const double e = fma(-q * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// sign(n) * v with sign(0) = 0 (the one-sided derivative convention of |kappa|).
__device__ __forceinline__ double signed_by(double n, double v)
{
    const double sg = n > 0.0 ? 1.0 : (n < 0.0 ? -1.0 : 0.0);
    return sg * v;
}

// A ring record expanded in powers of c.  With every derivative affine in c,
//   q(c) = 1 + u_x^2 + u_y^2                                   quadratic,
//   mean:     N(c) = (1 + u_y^2) u_xx + (1 + u_x^2) u_yy - 2 u_x u_y u_xy   cubic,   kappa = N q^{-3/2},
//   Gaussian: D(c) = u_xx u_yy - u_xy^2                        quadratic, kappa = D q^{-2}.
// The expansion is done once per record; an evaluation is then a few Horner
// steps, and the record holds 7 (mean) or 6 (Gaussian) doubles instead of 10.
template <int KIND>
struct PolyRing {
    static constexpr int NN = KIND == KIND_MEAN ? 4 : 3;
    static constexpr int NCOEF = 3 + NN;
    double q0, q1, q2;
    double n[NN];
};

// Records kept in memory, coefficient-major: coefficient m of record k at reg[m * stride + k].
template <int KIND>
__device__ __forceinline__ void store_poly(double* __restrict__ reg, int stride, int k, const PolyRing<KIND>& p)
{
    reg[k] = p.q0;
    reg[stride + k] = p.q1;
    reg[2 * stride + k] = p.q2;
#pragma unroll
    for (int m = 0; m < PolyRing<KIND>::NN; ++m) reg[(3 + m) * stride + k] = p.n[m];
}

template <int KIND>
__device__ __forceinline__ void load_poly(const double* __restrict__ reg, int stride, int k, PolyRing<KIND>& p)
{
    p.q0 = reg[k];
    p.q1 = reg[stride + k];
    p.q2 = reg[2 * stride + k];
#pragma unroll
    for (int m = 0; m < PolyRing<KIND>::NN; ++m) p.n[m] = reg[(3 + m) * stride + k];
}

template <int KIND>
__device__ __forceinline__ void make_poly(const Ring& r, PolyRing<KIND>& p)
{
    const double a0 = r.a[0], a1 = r.a[1], a2 = r.a[2], a3 = r.a[3], a4 = r.a[4];
    const double b0 = r.b[0], b1 = r.b[1], b2 = r.b[2], b3 = r.b[3], b4 = r.b[4];
    p.q0 = fma(a0, a0, fma(a1, a1, 1.0));
    p.q1 = 2.0 * fma(a0, b0, a1 * b1);
    p.q2 = fma(b0, b0, b1 * b1);
    if constexpr (KIND == KIND_MEAN) {
        // 1 + u_y^2, 1 + u_x^2 and u_x u_y as quadratics in c
        const double py0 = fma(a1, a1, 1.0), py1 = 2.0 * a1 * b1, py2 = b1 * b1;
        const double px0 = fma(a0, a0, 1.0), px1 = 2.0 * a0 * b0, px2 = b0 * b0;
        const double m0 = a0 * a1, m1 = fma(a0, b1, b0 * a1), m2 = b0 * b1;
        p.n[0] = fma(py0, a2, px0 * a3) - 2.0 * (m0 * a4);
        p.n[1] = (fma(py0, b2, py1 * a2) + fma(px0, b3, px1 * a3)) - 2.0 * fma(m0, b4, m1 * a4);
        p.n[2] = (fma(py1, b2, py2 * a2) + fma(px1, b3, px2 * a3)) - 2.0 * fma(m1, b4, m2 * a4);
        p.n[3] = fma(py2, b2, px2 * b3) - 2.0 * (m2 * b4);
    } else {
        p.n[0] = fma(a2, a3, -a4 * a4);
        p.n[1] = fma(a2, b3, b2 * a3) - 2.0 * (a4 * b4);
        p.n[2] = fma(b2, b3, -b4 * b4);
    }
}

// |kappa| of an expanded record at shift c.
template <int KIND>
__device__ __forceinline__ double abs_poly(const PolyRing<KIND>& p, double c)
{
    const double q = fma(fma(p.q2, c, p.q1), c, p.q0);
    const double rq = rsqrt_pos(q);
    if constexpr (KIND == KIND_MEAN) {
        const double num = fma(fma(fma(p.n[3], c, p.n[2]), c, p.n[1]), c, p.n[0]);
        return fabs(num) * (rq * rq * rq);
    } else {
        const double det = fma(fma(p.n[2], c, p.n[1]), c, p.n[0]);
        const double r2 = rq * rq;
        return fabs(det) * (r2 * r2);
    }
}

// d|kappa|/dc = sign(kappa) dkappa/dc at shift c (sign(0) = 0):
//   mean:     (N' q - 3/2 N q') q^{-5/2},   Gaussian: (D' q - 2 D q') q^{-3}.
template <int KIND>
__device__ __forceinline__ double dabs_poly(const PolyRing<KIND>& p, double c)
{
    const double c2 = c + c;
    const double q = fma(fma(p.q2, c, p.q1), c, p.q0);
    const double dq = fma(p.q2, c2, p.q1);
    const double rq = rsqrt_pos(q);
    const double r2 = rq * rq;
    if constexpr (KIND == KIND_MEAN) {
        const double num = fma(fma(fma(p.n[3], c, p.n[2]), c, p.n[1]), c, p.n[0]);
        const double dnum = fma(p.n[2], c2, fma(p.n[3], 3.0 * (c * c), p.n[1]));
        const double t = fma(-1.5 * num, dq, dnum * q);
        return signed_by(num, t * (r2 * r2 * rq));
    } else {
        const double det = fma(fma(p.n[2], c, p.n[1]), c, p.n[0]);
        const double ddet = fma(p.n[2], c2, p.n[1]);
        const double t = fma(-2.0 * det, dq, ddet * q);
        return signed_by(det, t * (r2 * r2 * r2));
    }
}

// The 3x3 clamped window of u around (i, j), loaded (kept apart from the
// arithmetic so that a loop can have the loads of several windows in flight).
template <typename T>
__device__ __forceinline__ void load_window(const T* __restrict__ u, int H, int W, int i, int j, T (&v)[3][3])
{
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        const int ci = clampi(i + dy, 0, H - 1);
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) v[dy + 1][dx + 1] = u[(size_t)ci * W + clampi(j + dx, 0, W - 1)];
    }
}

// |kappa| of the window's centre pixel.
template <int KIND, typename T>
__device__ __forceinline__ double abs_kappa_window(const T (&v)[3][3])
{
    double t[3][3];
#pragma unroll
    for (int y = 0; y < 3; ++y)
#pragma unroll
        for (int x = 0; x < 3; ++x) t[y][x] = (double)v[y][x];
    Ring r;
    stencil5(t, r.a);
#pragma unroll
    for (int k = 0; k < 5; ++k) r.b[k] = 0.0;
    return abs_kappa<KIND>(r, 0.0);
}

// |kappa| at pixel (i, j) of the unshifted image (energy kernel).
template <int KIND, typename T>
__device__ __forceinline__ double abs_kappa_at(const T* __restrict__ u, int H, int W, int i, int j)
{
    T v[3][3];
    load_window(u, H, W, i, j, v);
    return abs_kappa_window<KIND>(v);
}

// ---------------------------------------------------------------------------
// Group sums.  Every lane of the group receives the bitwise identical total
// (butterfly; IEEE addition is commutative), so all lanes of a group take
// identical branches in the local solver.  sum(x) reduces one value,
// sum_n<N>(x) reduces N values with one synchronisation.
//
// Butterfly step OFF adds the value of a partner lane in the other half of an
// aligned 2*OFF-lane group.  Inside a row of 16 lanes the partner value comes
// through a DPP lane permutation (no LDS round trip): quad permutations for 1
// and 2; for 4 and 8 the mirror inside 8 or 16 lanes, which pairs each lane with
// one of the other half, and after the earlier steps every lane of a half holds
// the same value, so the sum is the one xor 4 / xor 8 would give.  Across rows
// (16, 32) the row-swap permutes exchange whole rows or half-waves.
// ---------------------------------------------------------------------------
template <int OFF>
__device__ __forceinline__ double butterfly_step(double x)
{
    const long long v = __double_as_longlong(x);
    const int lo = (int)(unsigned)(v & 0xffffffffll), hi = (int)(v >> 32);
    if constexpr (OFF < 16) {
        constexpr int ctrl = OFF == 1 ? 0xB1 : OFF == 2 ? 0x4E : OFF == 4 ? 0x141 : 0x140;
        const int plo = __builtin_amdgcn_update_dpp(0, lo, ctrl, 0xF, 0xF, false);
        const int phi = __builtin_amdgcn_update_dpp(0, hi, ctrl, 0xF, 0xF, false);
        return x + __hiloint2double(phi, plo);
    } else {
        // each swap returns the lane's own row (or half) and its partner's, in some order
        auto sl = OFF == 16 ? __builtin_amdgcn_permlane16_swap((unsigned)lo, (unsigned)lo, false, false)
                            : __builtin_amdgcn_permlane32_swap((unsigned)lo, (unsigned)lo, false, false);
        auto sh = OFF == 16 ? __builtin_amdgcn_permlane16_swap((unsigned)hi, (unsigned)hi, false, false)
                            : __builtin_amdgcn_permlane32_swap((unsigned)hi, (unsigned)hi, false, false);
        return __hiloint2double((int)sh[0], (int)sl[0]) + __hiloint2double((int)sh[1], (int)sl[1]);
    }
}

template <int GROUP>
__device__ __forceinline__ double butterfly(double x)
{
    if constexpr (GROUP > 1) x = butterfly_step<1>(x);
    if constexpr (GROUP > 2) x = butterfly_step<2>(x);
    if constexpr (GROUP > 4) x = butterfly_step<4>(x);
    if constexpr (GROUP > 8) x = butterfly_step<8>(x);
    if constexpr (GROUP > 16) x = butterfly_step<16>(x);
    if constexpr (GROUP > 32) x = butterfly_step<32>(x);
    return x;
}
template <int GROUP, int CHUNK_ = 8>
struct WaveSum {
    static constexpr int CHUNK = CHUNK_;   // samples per fused reduction in local_solve
    __device__ __forceinline__ double operator()(double x) const
    {
        return butterfly<GROUP>(x);
    }
    template <int N>
    __device__ __forceinline__ void sum_n(double (&x)[N]) const
    {
#pragma unroll
        for (int k = 0; k < N; ++k) x[k] = (*this)(x[k]);
    }
};

// GROUP = a multiple of 64 equal to blockDim.x: wave butterfly, then the wave
// totals through LDS in fixed order.  Two LDS halves alternate so one barrier
// per reduction suffices.
template <int GROUP>
struct BlockSum {
    static constexpr int NW = GROUP / 64;
    static constexpr int NMAX = 8;   // values per sum_n
    static constexpr int CHUNK = 8;
    double* lds;   // 2 * NW * NMAX doubles
    mutable int parity;
    __device__ __forceinline__ double operator()(double x) const
    {
        double v[1] = {x};
        sum_n<1>(v);
        return v[0];
    }
    template <int N>
    __device__ __forceinline__ void sum_n(double (&x)[N]) const
    {
        static_assert(N <= NMAX, "too many values");
        const int wave = threadIdx.x >> 6;
        double* slot = lds + parity * NW * NMAX;
#pragma unroll
        for (int k = 0; k < N; ++k) x[k] = butterfly<64>(x[k]);
        if ((threadIdx.x & 63) == 0) {
#pragma unroll
            for (int k = 0; k < N; ++k) slot[k * NW + wave] = x[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < N; ++k) {
            double s = slot[k * NW];
#pragma unroll
            for (int w = 1; w < NW; ++w) s += slot[k * NW + w];
            x[k] = s;
        }
        parity ^= 1;
    }
};

// Single lane (pixel level): nothing to reduce.
struct NoSum {
    static constexpr int CHUNK = 1;   // nothing to fuse; fewer live registers
    __device__ __forceinline__ double operator()(double x) const { return x; }
    template <int N>
    __device__ __forceinline__ void sum_n(double (&)[N]) const {}
};

// ---------------------------------------------------------------------------
// The local solver (one block).
//   s = |B|, fs = f* = mean of (f - u) over B, as = alpha * s
//   K(c)  = group total of |kappa| over the ring at shift c
//   V(c)  = K(c) + as/2 (c - fs)^2,   V'(c) = K'(c) + as (c - fs)
// Every global minimiser of V lies in [fs - rho, fs + rho], rho = sqrt(2 K(fs) / as),
// since V(c*) <= V(fs) forces as/2 (c* - fs)^2 <= K(fs).
// `Kpart<N>(cs, out)` writes this lane's partial |kappa| sums at N shifts,
// `Dpart(c)` this lane's partial d|kappa|/dc; `gs` reduces over the group.
// Evaluation order and values are those of the scalar definition: samples
// c_i = fs + rho (2 i - M) / M, i* = first arg min of V(c_i), G bisection
// steps on the sign of V' in [c_{i*-1}, c_{i*+1}], the bisection point wins
// unless the best sample is lower by more than eta = 1e-12 (1 + V(0)), and the
// result is kept only if it lowers the local energy by more than eta (c = 0 is
// always a candidate of the arg min and wins the ties rounding cannot resolve,
// so an applied block update lowers the energy).
// ---------------------------------------------------------------------------
template <class KP, class DP, class GS>
__device__ __forceinline__ double local_solve(KP&& Kpart, DP&& Dpart, const GS& gs, double fs, double as, int M, int G)
{
    constexpr int CH = GS::CHUNK;  // samples per fused reduction
    double k2[2];
    {
        const double c2[2] = {0.0, fs};
        Kpart(c2, k2);
        gs.template sum_n<2>(k2);
    }
    const double K0 = k2[0];
    const double Kf = k2[1];
    const double rho = sqrt(2.0 * Kf / as);
    const double V0 = K0 + 0.5 * as * fs * fs;
    const double eta = 1e-12 * (1.0 + V0);
    double ct, Kt;
    if (rho == 0.0) {
        ct = fs;
        Kt = Kf;
    } else {
        // samples i = 0..M except M/2 (= f*, already known), CH per fused reduction,
        // scanned in increasing i so that ties keep the first index.  The sample
        // offsets (2i - M) / M are the rounded quotients; for M a power of two the
        // product with the exact 1/M is the same number, so that case (the usual
        // one) gets its own copy of the loops without the division.
        auto scan = [&](auto pow2) {
            constexpr bool P2 = decltype(pow2)::value;
            const double invm = 1.0 / (double)M;
            auto frac = [&](int i) {
                const double n = (double)(2 * i - M);
                return P2 ? n * invm : n / (double)M;
            };
            double vbest = 0.0, kbest = 0.0;
            int istar = -1;
            auto consider = [&](int i, double ci, double ki) {
                const double vi = ki + 0.5 * as * (ci - fs) * (ci - fs);
                if (istar < 0 || vi < vbest) { vbest = vi; kbest = ki; istar = i; }
            };
            for (int t0 = 0; t0 < M; t0 += CH) {
                double cs[CH], ks[CH];
#pragma unroll
                for (int t = 0; t < CH; ++t) {
                    const int tt = t0 + t < M ? t0 + t : M - 1;
                    const int i = tt < M / 2 ? tt : tt + 1;
                    cs[t] = fs + rho * frac(i);
                }
                Kpart(cs, ks);
                gs.template sum_n<CH>(ks);
#pragma unroll
                for (int t = 0; t < CH; ++t) {
                    const int tt = t0 + t;
                    if (tt >= M) break;
                    const int i = tt < M / 2 ? tt : tt + 1;
                    if (i == M / 2 + 1) consider(M / 2, fs, Kf);
                    consider(i, cs[t], ks[t]);
                }
            }
            const double cbest = fs + rho * frac(istar);
            const int ilo = istar > 0 ? istar - 1 : 0;
            const int ihi = istar < M ? istar + 1 : M;
            double lo = fs + rho * frac(ilo);
            double hi = fs + rho * frac(ihi);
            for (int g = 0; g < G; ++g) {
                const double mid = 0.5 * (lo + hi);
                const double d = gs(Dpart(mid)) + as * (mid - fs);
                if (d > 0.0) hi = mid; else lo = mid;
            }
            const double cbis = 0.5 * (lo + hi);
            double kb[1];
            {
                const double cb[1] = {cbis};
                Kpart(cb, kb);
                gs.template sum_n<1>(kb);
            }
            const double vbis = kb[0] + 0.5 * as * (cbis - fs) * (cbis - fs);
            if (vbest < vbis - eta) { ct = cbest; Kt = kbest; }
            else { ct = cbis; Kt = kb[0]; }
        };
        if ((M & (M - 1)) == 0) scan(std::true_type());
        else scan(std::false_type());
    }
    const double delta = (Kt - K0) + 0.5 * as * ct * (ct - 2.0 * fs);
    return delta < -eta ? ct : 0.0;
}

}  // namespace mgc
