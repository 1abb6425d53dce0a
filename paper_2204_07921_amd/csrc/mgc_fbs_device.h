// Device building blocks of the paper's own local step (tangent-plane distances,
// Propositions 1-2, eq. (c-sol2)) shared by the FBS path and the reconstruction path.
#pragma once

#include <hip/hip_runtime.h>

#include "mgc_device.h"

namespace fbs {

constexpr double SQRT2 = 1.4142135623730951;

using mgc::rsqrt_pos;   // refined hardware 1/sqrt; the arguments here are >= l^2 >= 1

// The value of lane (l xor OFF): a DPP quad permutation for OFF = 1 and 2 (no LDS
// round trip), the LDS permute otherwise.
template <int OFF>
__device__ __forceinline__ int xlane_i(int x)
{
    if constexpr (OFF == 1) return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);
    else if constexpr (OFF == 2) return __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);
    else return __shfl_xor(x, OFF, 64);
}

template <int OFF>
__device__ __forceinline__ double xlane(double x)
{
    const long long v = __double_as_longlong(x);
    const int lo = xlane_i<OFF>((int)(unsigned)(v & 0xffffffffll)), hi = xlane_i<OFF>((int)(v >> 32));
    return __hiloint2double(hi, lo);
}

// Sum over an aligned group of G lanes (xor butterfly, every lane gets the same total).
template <int G, int OFF = 1>
__device__ __forceinline__ double group_sum(double x)
{
    if constexpr (OFF >= G) return x;
    else return group_sum<G, 2 * OFF>(x + xlane<OFF>(x));
}

// Extremes of the normal curvatures d / ds^2 with the first plane index on ties.
struct GcAcc {
    double kmin, dmin, kmax, dmax;
    int imin, imax;
};

// Two planes sharing the chord a-b, third vertices t0 and t1.
__device__ __forceinline__ void chord(double ua, double ub, double l, double l2, double uo, double t0, double t1,
                                      double& d0, double& d1, double& ds2)
{
    const double h = 0.5 * (ua + ub), e = 0.5 * (ub - ua);
    const double s = l2 + e * e;
    const double num = l * (h - uo);
    const double g0 = t0 - h, g1 = t1 - h;
    d0 = num * rsqrt_pos(s + g0 * g0);
    d1 = num * rsqrt_pos(s + g1 * g1);
    ds2 = s;
}

// v = ring values in the order W, E, N, S, NW, SE, NE, SW; planes in the order
// (W-E | N), (W-E | S), (N-S | W), (N-S | E), (NW-SE | NE), (NW-SE | SW),
// (NE-SW | NW), (NE-SW | SE); global plane index base + k.
template <int KIND>
__device__ __forceinline__ void ring_accumulate(double uo, const double (&v)[8], double r, int base, double& sum,
                                                GcAcc& g)
{
    double d[8], s[4];
    const double la = r, la2 = r * r, ld = r * SQRT2, ld2 = 2.0 * r * r;
    chord(v[0], v[1], la, la2, uo, v[2], v[3], d[0], d[1], s[0]);
    chord(v[2], v[3], la, la2, uo, v[0], v[1], d[2], d[3], s[1]);
    chord(v[4], v[5], ld, ld2, uo, v[6], v[7], d[4], d[5], s[2]);
    chord(v[6], v[7], ld, ld2, uo, v[4], v[5], d[6], d[7], s[3]);
    if constexpr (KIND == 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) sum += d[k];
    } else {
        double inv[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) inv[m] = 1.0 / s[m];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double kap = d[k] * inv[k >> 1];
            const int idx = base + k;
            if (kap < g.kmin || (kap == g.kmin && idx < g.imin)) { g.kmin = kap; g.dmin = d[k]; g.imin = idx; }
            if (kap > g.kmax || (kap == g.kmax && idx < g.imax)) { g.kmax = kap; g.dmax = d[k]; g.imax = idx; }
        }
    }
}

// Combine the extremes over an aligned group of G lanes (same rule as ring_accumulate).
template <int G, int OFF = 1>
__device__ __forceinline__ void group_extremes(GcAcc& acc)
{
    if constexpr (OFF < G) {
        const double ok = xlane<OFF>(acc.kmin), od = xlane<OFF>(acc.dmin);
        const int oid = xlane_i<OFF>(acc.imin);
        if (ok < acc.kmin || (ok == acc.kmin && oid < acc.imin)) { acc.kmin = ok; acc.dmin = od; acc.imin = oid; }
        const double xk = xlane<OFF>(acc.kmax), xd = xlane<OFF>(acc.dmax);
        const int xid = xlane_i<OFF>(acc.imax);
        if (xk > acc.kmax || (xk == acc.kmax && xid < acc.imax)) { acc.kmax = xk; acc.dmax = xd; acc.imax = xid; }
        group_extremes<G, 2 * OFF>(acc);
    }
}

__device__ __forceinline__ GcAcc gc_empty()
{
    GcAcc g;
    g.kmin = INFINITY;
    g.kmax = -INFINITY;
    g.dmin = g.dmax = 0.0;
    g.imin = g.imax = 0x7fffffff;
    return g;
}

__device__ __forceinline__ double gc_choice(const GcAcc& g) { return fabs(g.kmin) <= fabs(g.kmax) ? g.dmin : g.dmax; }

// Backward step (eq. (c-sol2), patch form): weight w = eta_t alpha s.
__device__ __forceinline__ double backward(double c, double half, double w, double fs)
{
    return (c + half + w * fs) / (2.0 + w);
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Offsets of the ring values, in the order ring_accumulate expects.
__device__ __forceinline__ constexpr int ring_di(int k) { return k < 2 ? 0 : (k < 4 ? (k == 2 ? -1 : 1) : ((k & 1) ? 1 : -1)); }
__device__ __forceinline__ constexpr int ring_dj(int k)
{
    return k < 2 ? (k == 0 ? -1 : 1) : (k < 4 ? 0 : (k == 4 ? -1 : (k == 5 ? 1 : (k == 6 ? 1 : -1))));
}

// Row-major positions (a, b) in a grid with nb columns of the elements t0,
// t0 + S, t0 + 2 S, ...: one division at the start, then a fixed step with a
// carry (the index arithmetic of strided loops otherwise dominates these
// kernels' instruction counts).
struct GridWalk {
    int a, b, da, db, nb;
    __device__ __forceinline__ GridWalk(int t0, int S, int nb_) : nb(nb_)
    {
        a = t0 / nb;
        b = t0 - a * nb;
        da = S / nb;
        db = S - da * nb;
    }
    __device__ __forceinline__ bool next()
    {
        a += da;
        b += db;
        const bool carry = b >= nb;
        if (carry) {
            b -= nb;
            ++a;
        }
        return carry;
    }
};

// dst[r * dstride + c] = src[r * sstride + c] for an nr x nc region, thread t
// taking the elements t, t + NT, ... in row-major order with K loads in flight
// before the first store; offsets advance by a fixed step.
template <int NT, int K, class T, class SS, class DS>
__device__ __forceinline__ void tile_copy(int nr, int nc, const T* __restrict__ src, SS sstride, T* __restrict__ dst,
                                          DS dstride)
{
    if (nr <= 0 || nc <= 0) return;
    const int n = nr * nc;
    GridWalk w(threadIdx.x, NT, nc);
    SS so = (SS)w.a * sstride + w.b;
    DS dof = (DS)w.a * dstride + w.b;
    const SS sstep = (SS)w.da * sstride + w.db, scarry = sstride - nc;
    const DS dstep = (DS)w.da * dstride + w.db, dcarry = dstride - nc;
    for (int base = threadIdx.x; base < n; base += NT * K) {
        T tmp[K];
        {
            GridWalk v = w;
            SS o = so;
#pragma unroll
            for (int m = 0; m < K; ++m) {
                if (base + m * NT < n) tmp[m] = src[o];
                o += sstep;
                if (v.next()) o += scarry;
            }
        }
#pragma unroll
        for (int m = 0; m < K; ++m) {
            if (base + m * NT < n) dst[dof] = tmp[m];
            so += sstep;
            dof += dstep;
            if (w.next()) {
                so += scarry;
                dof += dcarry;
            }
        }
    }
}

// dst[r * dstride + c] = src[r * sstride + c] for an NR x NC box in 16-byte
// accesses (src, dst and both strides 16-byte aligned, NC whole vectors); each
// thread issues all of its loads before its stores.  Loads past the box read its
// last vector again, so none is conditional and all stay in registers (a
// conditionally loaded vector array is kept in scratch memory, one load at a
// time); only the stores are guarded.
template <int NT, int NR, int NC, class T, class SS, class DS>
__device__ __forceinline__ void box_copy16(const T* __restrict__ src, SS sstride, T* __restrict__ dst, DS dstride)
{
    constexpr int V = 16 / (int)sizeof(T), NV = NC / V, N = NR * NV, K = (N + NT - 1) / NT;
    static_assert(NC % V == 0, "rows must be whole 16-byte vectors");
    uint4 x[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        const int q = min((int)threadIdx.x + m * NT, N - 1);
        const int r = q / NV, cv = q - r * NV;
        x[m] = *reinterpret_cast<const uint4*>(src + (SS)r * sstride + cv * V);
    }
#pragma unroll
    for (int m = 0; m < K; ++m) {
        const int q = (int)threadIdx.x + m * NT;
        if (q < N) {
            const int r = q / NV, cv = q - r * NV;
            *reinterpret_cast<uint4*>(dst + (DS)r * dstride + cv * V) = x[m];
        }
    }
}

}  // namespace fbs
