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

// Value of tap (i, j) (already clamped) as the sweep sees it.  With pending
// corrections (coarse levels apply a level's corrections lazily) the value is
// u + c_pending of the tap's block, rounded to the state type exactly as an
// eager update would have stored it.
template <typename T, bool LAZY>
__device__ __forceinline__ double tap_value(const T* __restrict__ u, int W, int i, int j,
                                            const double* __restrict__ cpend, int nj, int lb)
{
    const double v = (double)u[(size_t)i * W + j];
    if (!LAZY) return v;
    const double c = cpend[(size_t)(i >> lb) * nj + (j >> lb)];
    return (double)(T)(v + c);
}

// Build the ring record of pixel (i, j) for block rows [r0, r1) x cols [c0, c1).
// Pixels outside the image, and pixels whose nine clamped taps lie all inside or
// all outside B (their curvature does not depend on c), get the zero record,
// which contributes exactly 0 to every sum below.
template <typename T, bool LAZY = false>
__device__ __forceinline__ void make_ring(const T* __restrict__ u, int H, int W, int i, int j,
                                          int r0, int r1, int c0, int c1, Ring& r,
                                          const double* __restrict__ cpend = nullptr, int nj = 0, int lb = 0)
{
    if (i < 0 || i >= H || j < 0 || j >= W) { zero_ring(r); return; }
    double t[3][3], m[3][3];
    int n = 0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        const int ci = clampi(i + dy, 0, H - 1);
        const bool rin = ci >= r0 && ci < r1;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int cj = clampi(j + dx, 0, W - 1);
            const bool in = rin && cj >= c0 && cj < c1;
            t[dy + 1][dx + 1] = tap_value<T, LAZY>(u, W, ci, cj, cpend, nj, lb);
            m[dy + 1][dx + 1] = in ? 1.0 : 0.0;
            n += in ? 1 : 0;
        }
    }
    if (n == 0 || n == 9) { zero_ring(r); return; }
    stencil5(t, r.a);
    stencil5(m, r.b);
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

// d|kappa|/dc = sign(kappa) dkappa/dc at shift c (sign(0) = 0).
template <int KIND>
__device__ __forceinline__ double dabs_kappa(const Ring& r, double c)
{
    const double bx = r.b[0], by = r.b[1], bxx = r.b[2], byy = r.b[3], bxy = r.b[4];
    const double ux = fma(bx, c, r.a[0]);
    const double uy = fma(by, c, r.a[1]);
    const double uxx = fma(bxx, c, r.a[2]);
    const double uyy = fma(byy, c, r.a[3]);
    const double uxy = fma(bxy, c, r.a[4]);
    const double q = fma(ux, ux, fma(uy, uy, 1.0));
    const double dq = 2.0 * fma(ux, bx, uy * by);
    if (KIND == KIND_MEAN) {
        const double px = fma(ux, ux, 1.0), py = fma(uy, uy, 1.0);
        const double num = fma(py, uxx, fma(px, uyy, -2.0 * ux * uy * uxy));
        const double dnum = 2.0 * uy * by * uxx + py * bxx
                          - 2.0 * (bx * uy * uxy + ux * by * uxy + ux * uy * bxy)
                          + 2.0 * ux * bx * uyy + px * byy;
        const double rq = rsqrt(q);
        const double r2 = rq * rq;
        const double dk = fma(-1.5 * num * dq, r2, dnum) * (r2 * rq);
        const double s = (num > 0.0) ? 1.0 : ((num < 0.0) ? -1.0 : 0.0);
        return s * dk;
    } else {
        const double det = fma(uxx, uyy, -uxy * uxy);
        const double ddet = bxx * uyy + uxx * byy - 2.0 * uxy * bxy;
        const double iq = 1.0 / q;
        const double dk = fma(-2.0 * det * dq, iq, ddet) * (iq * iq);
        const double s = (det > 0.0) ? 1.0 : ((det < 0.0) ? -1.0 : 0.0);
        return s * dk;
    }
}

// |kappa| at pixel (i, j) of the unshifted image (energy kernel).
template <int KIND, typename T>
__device__ __forceinline__ double abs_kappa_at(const T* __restrict__ u, int H, int W, int i, int j)
{
    double t[3][3];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        const int ci = clampi(i + dy, 0, H - 1);
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx)
            t[dy + 1][dx + 1] = (double)u[(size_t)ci * W + clampi(j + dx, 0, W - 1)];
    }
    Ring r;
    stencil5(t, r.a);
#pragma unroll
    for (int k = 0; k < 5; ++k) r.b[k] = 0.0;
    return abs_kappa<KIND>(r, 0.0);
}

// ---------------------------------------------------------------------------
// Group sums.  Every lane of the group receives the bitwise identical total
// (xor butterfly; IEEE addition is commutative), so all lanes of a group take
// identical branches in the local solver.  sum(x) reduces one value,
// sum_n<N>(x) reduces N values with one synchronisation.
// ---------------------------------------------------------------------------
template <int GROUP>
struct WaveSum {
    __device__ __forceinline__ double operator()(double x) const
    {
#pragma unroll
        for (int off = 1; off < GROUP; off <<= 1) x += __shfl_xor(x, off, 64);
        return x;
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
        for (int k = 0; k < N; ++k) {
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) x[k] += __shfl_xor(x[k], off, 64);
        }
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
// result is kept only if the local energy change is below eta.
// ---------------------------------------------------------------------------
template <class KP, class DP, class GS>
__device__ __forceinline__ double local_solve(KP&& Kpart, DP&& Dpart, const GS& gs, double fs, double as, int M, int G)
{
    constexpr int CH = 8;  // samples per fused reduction
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
        // scanned in increasing i so that ties keep the first index
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
                cs[t] = fs + rho * ((double)(2 * i - M) / (double)M);
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
        const double cbest = fs + rho * ((double)(2 * istar - M) / (double)M);
        const int ilo = istar > 0 ? istar - 1 : 0;
        const int ihi = istar < M ? istar + 1 : M;
        double lo = fs + rho * ((double)(2 * ilo - M) / (double)M);
        double hi = fs + rho * ((double)(2 * ihi - M) / (double)M);
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
    }
    const double delta = (Kt - K0) + 0.5 * as * ct * (ct - 2.0 * fs);
    return delta < eta ? ct : 0.0;
}

}  // namespace mgc
