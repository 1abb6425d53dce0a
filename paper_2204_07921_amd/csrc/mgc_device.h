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

// Build the ring record of pixel (i, j) for block rows [r0, r1) x cols [c0, c1).
// Pixels outside the image, and pixels whose nine clamped taps lie all inside or
// all outside B (their curvature does not depend on c), get the zero record,
// which contributes exactly 0 to every sum below.
template <typename T>
__device__ __forceinline__ void make_ring(const T* __restrict__ u, int H, int W, int i, int j,
                                          int r0, int r1, int c0, int c1, Ring& r)
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
            t[dy + 1][dx + 1] = (double)u[(size_t)ci * W + cj];
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
// identical branches in the local solver.
// ---------------------------------------------------------------------------
template <int GROUP>
struct WaveSum {
    __device__ __forceinline__ double operator()(double x) const
    {
#pragma unroll
        for (int off = 1; off < GROUP; off <<= 1) x += __shfl_xor(x, off, 64);
        return x;
    }
};

// GROUP = a multiple of 64 equal to blockDim.x: wave butterfly, then the wave
// totals through LDS in fixed order.  Two LDS halves alternate so one barrier
// per reduction suffices.
template <int GROUP>
struct BlockSum {
    static constexpr int NW = GROUP / 64;
    double* lds;   // 2 * NW doubles
    mutable int parity;
    __device__ __forceinline__ double operator()(double x) const
    {
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) x += __shfl_xor(x, off, 64);
        const int wave = threadIdx.x >> 6;
        double* slot = lds + parity * NW;
        if ((threadIdx.x & 63) == 0) slot[wave] = x;
        __syncthreads();
        double s = slot[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) s += slot[w];
        parity ^= 1;
        return s;
    }
};

// ---------------------------------------------------------------------------
// The local solver (one block).  `Keval(c)` returns the group total of |kappa|
// over the ring at shift c, `Deval(c)` the group total of d|kappa|/dc.
//   s = |B|, fs = f* = mean of (f - u) over B, as = alpha * s
//   V(c) = K(c) + as/2 (c - fs)^2,   V'(c) = K'(c) + as (c - fs)
// Every global minimiser of V lies in [fs - rho, fs + rho], rho = sqrt(2 K(fs) / as),
// since V(c*) <= V(fs) forces as/2 (c* - fs)^2 <= K(fs).
// ---------------------------------------------------------------------------
template <class KF, class DF>
__device__ __forceinline__ double local_solve(KF&& Keval, DF&& Deval, double fs, double as, int M, int G)
{
    const double K0 = Keval(0.0);
    const double Kf = Keval(fs);
    const double rho = sqrt(2.0 * Kf / as);
    const double V0 = K0 + 0.5 * as * fs * fs;
    const double eta = 1e-12 * (1.0 + V0);
    double ct, Kt;
    if (rho == 0.0) {
        ct = fs;
        Kt = Kf;
    } else {
        double vbest = 0.0, kbest = 0.0;
        int istar = 0;
        for (int i = 0; i <= M; ++i) {
            const double ci = fs + rho * ((double)(2 * i - M) / (double)M);
            const double ki = (2 * i == M) ? Kf : Keval(ci);
            const double vi = ki + 0.5 * as * (ci - fs) * (ci - fs);
            if (i == 0 || vi < vbest) { vbest = vi; kbest = ki; istar = i; }
        }
        const double cbest = fs + rho * ((double)(2 * istar - M) / (double)M);
        const int ilo = istar > 0 ? istar - 1 : 0;
        const int ihi = istar < M ? istar + 1 : M;
        double lo = fs + rho * ((double)(2 * ilo - M) / (double)M);
        double hi = fs + rho * ((double)(2 * ihi - M) / (double)M);
        for (int g = 0; g < G; ++g) {
            const double mid = 0.5 * (lo + hi);
            const double d = Deval(mid) + as * (mid - fs);
            if (d > 0.0) hi = mid; else lo = mid;
        }
        const double cbis = 0.5 * (lo + hi);
        const double kbis = Keval(cbis);
        const double vbis = kbis + 0.5 * as * (cbis - fs) * (cbis - fs);
        if (vbest < vbis - eta) { ct = cbest; Kt = kbest; }
        else { ct = cbis; Kt = kbis; }
    }
    const double delta = (Kt - K0) + 0.5 * as * ct * (ct - 2.0 * fs);
    return delta < eta ? ct : 0.0;
}

}  // namespace mgc
