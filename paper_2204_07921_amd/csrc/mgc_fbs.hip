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
//   level 1 (b = 1): one launch; a workgroup loads a 32 x 64 tile of u with a
//     4-pixel halo into LDS and runs the four colour sweeps there, shrinking the
//     region it trusts by one pixel per colour (each sweep reads one pixel
//     around the updated pixel), then writes the tile to the other buffer.
//     Every pixel is read once and written once per level.
//   level j >= 2: (1) per patch and row chunk, FP64 partial sums of f - u over
//     the patch (the patch's own pixels do not change before its colour) and
//     zeroed pending corrections; (2) four colour launches, a lane group per
//     patch holding the rings, reading tap values as u + the pending correction
//     of the tap's patch (rounded to T); (3) u <- u + c_patch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/mgcurv.h"
#include "mgc_internal.h"

namespace fbs {

constexpr double SQRT2 = 1.4142135623730951;

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
    d0 = num / sqrt(s + g0 * g0);
    d1 = num / sqrt(s + g1 * g1);
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
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double kap = d[k] / s[k >> 1];
            const int idx = base + k;
            if (kap < g.kmin || (kap == g.kmin && idx < g.imin)) { g.kmin = kap; g.dmin = d[k]; g.imin = idx; }
            if (kap > g.kmax || (kap == g.kmax && idx < g.imax)) { g.kmax = kap; g.dmax = d[k]; g.imax = idx; }
        }
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

// ---------------------------------------------------------------------------
// Level 1 (b = 1): the four colours of the level in one launch.
// ---------------------------------------------------------------------------
constexpr int PT_H = 32, PT_W = 64, PHALO = 4;
constexpr int PL_H = PT_H + 2 * PHALO, PL_W = PT_W + 2 * PHALO;

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
        eta = 1.0 / sqrt(1.0 + (double)t);
    }
    return c;
}

template <typename T, int KIND>
__global__ __launch_bounds__(256) void fbs_pixel_level_kernel(const T* __restrict__ uin, T* __restrict__ uout,
                                                              const T* __restrict__ f, int H, int W, double alpha,
                                                              int steps)
{
    __shared__ T su[PL_H * PL_W];
    const int y0 = blockIdx.y * PT_H, x0 = blockIdx.x * PT_W;
    const int ly = y0 - PHALO, lx = x0 - PHALO;
    const int r_lo = max(0, ly), r_hi = min(H, y0 + PT_H + PHALO);
    const int c_lo = max(0, lx), c_hi = min(W, x0 + PT_W + PHALO);
    const int nr = r_hi - r_lo, nc = c_hi - c_lo;
    for (int t = threadIdx.x; t < nr * nc; t += blockDim.x) {
        const int i = r_lo + t / nc, j = c_lo + t % nc;
        su[(i - ly) * PL_W + (j - lx)] = uin[(size_t)i * W + j];
    }
    __syncthreads();
    auto at = [&](int ii, int jj) { return (double)su[(ii - ly) * PL_W + (jj - lx)]; };
    for (int k = 0; k < 4; ++k) {
        // region still exact after sweep k: k + 1 pixels inside every tile edge that is not an image edge
        const int vr0 = r_lo == 0 ? 0 : r_lo + k + 1, vr1 = r_hi == H ? H : r_hi - k - 1;
        const int vc0 = c_lo == 0 ? 0 : c_lo + k + 1, vc1 = c_hi == W ? W : c_hi - k - 1;
        const int i0 = vr0 + ((vr0 & 1) != (k >> 1)), j0 = vc0 + ((vc0 & 1) != (k & 1));
        const int ni = i0 < vr1 ? (vr1 - i0 + 1) / 2 : 0, nj = j0 < vc1 ? (vc1 - j0 + 1) / 2 : 0;
        for (int t = threadIdx.x; t < ni * nj; t += blockDim.x) {
            const int i = i0 + 2 * (t / nj), j = j0 + 2 * (t % nj);
            const double uo = at(i, j);
            const double fs = (double)f[(size_t)i * W + j] - uo;
            const double c = pixel_correction<KIND>(at, i, j, H, W, fs, alpha, steps);
            // pixels of one colour read only other colours (or themselves), so the write is safe
            su[(i - ly) * PL_W + (j - lx)] = (T)(uo + c);
        }
        __syncthreads();
    }
    const int o_r1 = min(H, y0 + PT_H), o_c1 = min(W, x0 + PT_W);
    for (int t = threadIdx.x; t < PT_H * PT_W; t += blockDim.x) {
        const int i = y0 + t / PT_W, j = x0 + t % PT_W;
        if (i < o_r1 && j < o_c1) uout[(size_t)i * W + j] = su[(i - ly) * PL_W + (j - lx)];
    }
}

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

// Partial sums of f - u per (patch, row chunk), L lanes per group; chunk 0 of
// every patch also zeroes the patch's pending correction.
template <typename T, int L>
__global__ __launch_bounds__(256) void fbs_sums_kernel(const T* __restrict__ u, const T* __restrict__ f, int H, int W,
                                                       int b, int nj, int ngroups, int nchunk, int rows_per,
                                                       double* __restrict__ psums, double* __restrict__ cpend)
{
    __shared__ double lds[4];
    const int g = (int)((blockIdx.x * blockDim.x + threadIdx.x) / L);
    const int lane = threadIdx.x % L;
    const bool live = g < ngroups;
    double acc = 0.0;
    int patch = 0, k = 0;
    if (live) {
        patch = g / nchunk;
        k = g - patch * nchunk;
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
    if (live && lane == 0) {
        psums[g] = acc;
        if (k == 0) cpend[patch] = 0.0;
    }
}

// One colour of a coarse level: a group of G lanes per patch, lane l taking rings
// l + 1, l + 1 + G, ...; the patch's correction goes to cpend.
template <typename T, int KIND, int G>
__global__ __launch_bounds__(256) void fbs_patch_kernel(const T* __restrict__ u, int H, int W, int b, int mj, int nj,
                                                        int colour, int nchunk, const double* __restrict__ psums,
                                                        double* __restrict__ cpend, double alpha, int steps)
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
    if (live)
        for (int k = 0; k < nchunk; ++k) S += psums[(size_t)patch * nchunk + k];
    const double s = (double)((r1 - r0) * (c1 - c0));
    const double fs = S / s;
    // state value at a clamped position: u + pending correction of its patch (own patch: + shift)
    auto value = [&](int i, int j, double shift) {
        const int ci = clampi(i, 0, H - 1), cj = clampi(j, 0, W - 1);
        const double x = (double)u[(size_t)ci * W + cj];
        const int dp = ci < r0 ? -1 : (ci >= r1 ? 1 : 0), dq = cj < c0 ? -1 : (cj >= c1 ? 1 : 0);
        if (dp == 0 && dq == 0) return x + shift;
        const double cp = cpend[(size_t)(p + dp) * nj + (q + dq)];
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

// dst <- src + c of the pixel's patch (rounded to T).  In place (src == dst)
// only pixels with a nonzero correction are written.
template <typename T>
__global__ __launch_bounds__(256) void fbs_apply_kernel(const T* src, T* dst, int H, int W, int b, int nj,
                                                        const double* __restrict__ cpend, int in_place)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= W) return;
    const int q = j / b;
    for (int i = blockIdx.y; i < H; i += gridDim.y) {
        const double c = cpend[(size_t)(i / b) * nj + q];
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
struct mg_fbs_ctx {
    mg_fbs_params P;
    int device;
    hipStream_t stream;
    void* ping;        // H x W state image (level 1 writes here)
    void* prev;        // H x W state image (relErr(u) stop rule)
    double* psums;     // patch partial sums, max over coarse levels
    double* cpend;     // pending corrections, max patches over coarse levels
    double* epart;     // energy partials
    double* npart;     // norm partials (2 * NORM_BLOCKS)
    double* dev3;      // energy, ||u - prev||^2, ||u||^2
    double* host3;     // pinned copy of dev3
    std::string err;
};

namespace {

thread_local std::string g_fbs_init_error;

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
hipError_t launch_pixel_level(const mg_fbs_ctx* c, const void* uin, void* uout, const void* f)
{
    const int H = c->P.height, W = c->P.width;
    dim3 grid((W + fbs::PT_W - 1) / fbs::PT_W, (H + fbs::PT_H - 1) / fbs::PT_H), block(256);
    if (c->P.curvature == MG_CURV_MEAN)
        hipLaunchKernelGGL((fbs::fbs_pixel_level_kernel<T, 0>), grid, block, 0, c->stream, (const T*)uin, (T*)uout,
                           (const T*)f, H, W, c->P.alpha, c->P.steps);
    else
        hipLaunchKernelGGL((fbs::fbs_pixel_level_kernel<T, 1>), grid, block, 0, c->stream, (const T*)uin, (T*)uout,
                           (const T*)f, H, W, c->P.alpha, c->P.steps);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pixel_colour(const mg_fbs_ctx* c, void* u, const void* f, int colour)
{
    const int H = c->P.height, W = c->P.width;
    const size_t n = (size_t)((H - (colour >> 1) + 1) / 2) * ((W - (colour & 1) + 1) / 2);
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (c->P.curvature == MG_CURV_MEAN)
        hipLaunchKernelGGL((fbs::fbs_pixel_colour_kernel<T, 0>), grid, block, 0, c->stream, (T*)u, (const T*)f, H, W,
                           colour, c->P.alpha, c->P.steps);
    else
        hipLaunchKernelGGL((fbs::fbs_pixel_colour_kernel<T, 1>), grid, block, 0, c->stream, (T*)u, (const T*)f, H, W,
                           colour, c->P.alpha, c->P.steps);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sums(const mg_fbs_ctx* c, const void* u, const void* f, int b)
{
    const int H = c->P.height, W = c->P.width;
    int mj, nj, nchunk, rows_per;
    fbs::patch_geometry(H, W, b, &mj, &nj, &nchunk, &rows_per);
    const int ngroups = mj * nj * nchunk;
    const long pix = (long)b * (b < rows_per ? b : rows_per);   // pixels per group
    auto grid_for = [&](int L) { return dim3((unsigned)(((size_t)ngroups * L + 255) / 256)); };
#define FBS_SUMS(L)                                                                                                   \
    hipLaunchKernelGGL((fbs::fbs_sums_kernel<T, L>), grid_for(L), dim3(256), 0, c->stream, (const T*)u, (const T*)f, \
                       H, W, b, nj, ngroups, nchunk, rows_per, c->psums, c->cpend)
    if (pix <= 16) FBS_SUMS(1);
    else if (pix <= 128) FBS_SUMS(8);
    else if (pix <= 1024) FBS_SUMS(64);
    else FBS_SUMS(256);
#undef FBS_SUMS
    return hipGetLastError();
}

template <typename T, int KIND>
hipError_t launch_patch_kind(const mg_fbs_ctx* c, const void* u, int b, int colour)
{
    const int H = c->P.height, W = c->P.width;
    int mj, nj, nchunk, rows_per;
    fbs::patch_geometry(H, W, b, &mj, &nj, &nchunk, &rows_per);
    const int pr = colour >> 1, pc = colour & 1;
    const int npatch = ((mj - pr + 1) / 2) * ((nj - pc + 1) / 2);
    if (npatch <= 0) return hipSuccess;
    const int R = (b + 1) / 2;
    const int G = R < 64 ? R : 64;
    dim3 grid((unsigned)(((size_t)npatch * G + 255) / 256)), block(256);
#define FBS_PATCH(GG)                                                                                                  \
    hipLaunchKernelGGL((fbs::fbs_patch_kernel<T, KIND, GG>), grid, block, 0, c->stream, (const T*)u, H, W, b, mj, nj, \
                       colour, nchunk, (const double*)c->psums, c->cpend, c->P.alpha, c->P.steps)
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
hipError_t launch_patch(const mg_fbs_ctx* c, const void* u, int b, int colour)
{
    return c->P.curvature == MG_CURV_MEAN ? launch_patch_kind<T, 0>(c, u, b, colour)
                                          : launch_patch_kind<T, 1>(c, u, b, colour);
}

template <typename T>
hipError_t launch_apply(const mg_fbs_ctx* c, const void* src, void* dst, int b)
{
    const int H = c->P.height, W = c->P.width;
    const int nj = (W + b - 1) / b;
    const int gy = H < 1024 ? H : 1024;
    dim3 grid((W + 255) / 256, gy), block(256);
    hipLaunchKernelGGL(fbs::fbs_apply_kernel<T>, grid, block, 0, c->stream, (const T*)src, (T*)dst, H, W, b, nj,
                       (const double*)c->cpend, src == dst ? 1 : 0);
    return hipGetLastError();
}

// Coarse level j >= 2 on the state in `src`; the result lands in `dst`.
template <typename T>
mg_status coarse_level(mg_fbs_ctx* c, const void* src, void* dst, const void* f, int level, int only_colour)
{
    const int b = (1 << level) - 1;
    hipError_t e = launch_sums<T>(c, src, f, b);
    if (e != hipSuccess) return fhip(c, e, "patch sums launch");
    for (int colour = 0; colour < 4; ++colour) {
        if (only_colour >= 0 && colour != only_colour) continue;
        e = launch_patch<T>(c, src, b, colour);
        if (e != hipSuccess) return fhip(c, e, "patch colour launch");
    }
    e = launch_apply<T>(c, src, dst, b);
    if (e != hipSuccess) return fhip(c, e, "apply launch");
    return MG_OK;
}

// The levels of one V-cycle in order: 1..J, then J-1..1 for the full cycle.
template <typename T>
mg_status run_levels(mg_fbs_ctx* c, void* u, const void* f, const int* levels, int nlevels)
{
    void* cur = u;
    for (int n = 0; n < nlevels; ++n) {
        const int level = levels[n];
        if (level == 1) {
            void* other = cur == u ? c->ping : u;
            hipError_t e = launch_pixel_level<T>(c, cur, other, f);
            if (e != hipSuccess) return fhip(c, e, "pixel level launch");
            cur = other;
        } else {
            mg_status st = coarse_level<T>(c, cur, u, f, level, -1);
            if (st != MG_OK) return st;
            cur = u;
        }
    }
    if (cur != u) {
        hipError_t e = hipMemcpyAsync(u, cur, fbytes(c), hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return fhip(c, e, "state copy");
    }
    return MG_OK;
}

mg_status vcycle(mg_fbs_ctx* c, void* u, const void* f)
{
    int lv[64], n = 0;
    for (int j = 1; j <= c->P.levels; ++j) lv[n++] = j;
    if (c->P.cycle == 1)
        for (int j = c->P.levels - 1; j >= 1; --j) lv[n++] = j;
    return is64(c) ? run_levels<double>(c, u, f, lv, n) : run_levels<float>(c, u, f, lv, n);
}

mg_status level_only(mg_fbs_ctx* c, void* u, const void* f, int level)
{
    int lv[1] = {level};
    return is64(c) ? run_levels<double>(c, u, f, lv, 1) : run_levels<float>(c, u, f, lv, 1);
}

mg_status sweep_only(mg_fbs_ctx* c, void* u, const void* f, int level, int colour)
{
    if (level == 1) {
        hipError_t e = is64(c) ? launch_pixel_colour<double>(c, u, f, colour) : launch_pixel_colour<float>(c, u, f, colour);
        return e == hipSuccess ? MG_OK : fhip(c, e, "pixel colour launch");
    }
    return is64(c) ? coarse_level<double>(c, u, u, f, level, colour) : coarse_level<float>(c, u, u, f, level, colour);
}

mgc::LaunchCtx energy_ctx(const mg_fbs_ctx* c)
{
    mgc::LaunchCtx L;
    L.stream = c->stream;
    L.H = c->P.height;
    L.W = c->P.width;
    L.alpha = c->P.alpha;
    L.kind = c->P.curvature;
    L.f64 = is64(c);
    L.M = 0;
    L.G = 0;
    return L;
}

// Enqueue F(u) into dev3[0] and, if `norms`, ||u - prev||^2 and ||u||^2 into
// dev3[1..2]; copy to the pinned host mirror and wait.
mg_status measure(mg_fbs_ctx* c, const void* u, const void* f, bool norms)
{
    hipError_t e = mgc::launch_energy(energy_ctx(c), u, f, c->epart, c->dev3);
    if (e != hipSuccess) return fhip(c, e, "energy launch");
    if (norms) {
        const size_t n = (size_t)c->P.height * c->P.width;
        if (is64(c))
            hipLaunchKernelGGL(fbs::fbs_norms_kernel<double>, dim3(fbs::NORM_BLOCKS), dim3(256), 0, c->stream,
                               (const double*)u, (const double*)c->prev, n, c->npart);
        else
            hipLaunchKernelGGL(fbs::fbs_norms_kernel<float>, dim3(fbs::NORM_BLOCKS), dim3(256), 0, c->stream,
                               (const float*)u, (const float*)c->prev, n, c->npart);
        hipLaunchKernelGGL(fbs::fbs_norms_final_kernel, dim3(1), dim3(256), 0, c->stream, (const double*)c->npart,
                           fbs::NORM_BLOCKS, c->dev3 + 1);
        if ((e = hipGetLastError()) != hipSuccess) return fhip(c, e, "norm launch");
    }
    e = hipMemcpyAsync(c->host3, c->dev3, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return fhip(c, e, "result copy");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fhip(c, e, "stream synchronize");
    return MG_OK;
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
    c->ping = c->prev = nullptr;
    c->psums = c->cpend = c->epart = c->npart = c->dev3 = c->host3 = nullptr;
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
    if (hipMalloc(&c->ping, nb) != hipSuccess || hipMalloc(&c->prev, nb) != hipSuccess ||
        hipMalloc((void**)&c->psums, sizeof(double) * n_ps) != hipSuccess ||
        hipMalloc((void**)&c->cpend, sizeof(double) * n_cp) != hipSuccess ||
        hipMalloc((void**)&c->epart, sizeof(double) * ne) != hipSuccess ||
        hipMalloc((void**)&c->npart, sizeof(double) * 2 * fbs::NORM_BLOCKS) != hipSuccess ||
        hipMalloc((void**)&c->dev3, 3 * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void**)&c->host3, 3 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        mg_fbs_destroy(c);
        (void)hipGetLastError();
        return ffail(nullptr, MG_E_NOMEM, "device allocation of 2 x %zu bytes failed", nb);
    }
    *out = c;
    return MG_OK;
}

mg_status mg_fbs_vcycle(mg_fbs_ctx* ctx, void* u, const void* f, double* energy_after)
{
    mg_status st = fcheck(ctx, u, f);
    if (st != MG_OK) return st;
    if ((st = vcycle(ctx, u, f)) != MG_OK || !energy_after) return st;
    if ((st = measure(ctx, u, f, false)) != MG_OK) return st;
    *energy_after = ctx->host3[0];
    return MG_OK;
}

mg_status mg_fbs_level(mg_fbs_ctx* ctx, void* u, const void* f, int32_t level)
{
    mg_status st = fcheck(ctx, u, f);
    if (st != MG_OK) return st;
    if (level < 1 || level > ctx->P.levels) return ffail(ctx, MG_E_INVALID, "level must be in [1, %d]", ctx->P.levels);
    return level_only(ctx, u, f, level);
}

mg_status mg_fbs_sweep(mg_fbs_ctx* ctx, void* u, const void* f, int32_t level, int32_t colour)
{
    mg_status st = fcheck(ctx, u, f);
    if (st != MG_OK) return st;
    if (level < 1 || level > ctx->P.levels) return ffail(ctx, MG_E_INVALID, "level must be in [1, %d]", ctx->P.levels);
    if (colour < 0 || colour > 3) return ffail(ctx, MG_E_INVALID, "colour must be in [0, 4)");
    return sweep_only(ctx, u, f, level, colour);
}

mg_status mg_fbs_energy(mg_fbs_ctx* ctx, const void* u, const void* f, double* energy)
{
    mg_status st = fcheck(ctx, u, f);
    if (st != MG_OK) return st;
    if (!energy) return ffail(ctx, MG_E_INVALID, "energy output must be non-null");
    if ((st = measure(ctx, u, f, false)) != MG_OK) return st;
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
    if ((st = measure(ctx, u, f, false)) != MG_OK) return st;
    double e_prev = ctx->host3[0];
    if (!std::isfinite(e_prev)) return ffail(ctx, MG_E_NONFINITE, "energy of the initial state is not finite");
    if (energy_trace) energy_trace[0] = e_prev;
    int done = 0;
    bool converged = false;
    double e = e_prev;
    const bool relerr = stop == MG_STOP_RELERR_U;
    while (done < max_vcycles) {
        if (relerr) {
            hipError_t he = hipMemcpyAsync(ctx->prev, u, fbytes(ctx), hipMemcpyDeviceToDevice, ctx->stream);
            if (he != hipSuccess) return fhip(ctx, he, "state copy");
        }
        if ((st = vcycle(ctx, u, f)) != MG_OK) return st;
        if ((st = measure(ctx, u, f, relerr)) != MG_OK) return st;
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
    if (ctx->ping) (void)hipFree(ctx->ping);
    if (ctx->prev) (void)hipFree(ctx->prev);
    if (ctx->psums) (void)hipFree(ctx->psums);
    if (ctx->cpend) (void)hipFree(ctx->cpend);
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
