// Multigrid reconstruction (Section 5) on gfx950: recover u from b = A u + noise by
// minimising 1/2 ||A u - b||^2 + alpha sum |H(u)|.  A is a 5 x 5 blur with a zero
// boundary (its weights are a parameter of the context).  On patches of side 2^j - 1
// (Section 2.2) and for each colour k (Section 2.3), the corrections c of all patches
// of the colour solve the coupled system of Section 5,
//     (G + 2 alpha I) c = r,  G_il = <A phi_i, A phi_l>,  r_i = <b - A u, A phi_i> + 2 alpha d_i,
// with d_i the tangent-plane estimate of Proposition 1 for patch i; the system is
// solved matrix-free by conjugate gradients in FP64 with a fixed number of
// iterations from c = 0, and u <- u + sum c_i phi_i.
//
// Per colour: t = b - A u (FP64 image); d_i (lane group per patch, rings of the
// patch); r_i = sum over the patch of (A^T t) + 2 alpha d_i; then per CG iteration
// v = sum p_i phi_i (image), w = A v, q_i = sum over the patch of (A^T w) + 2 alpha p_i,
// and the vector updates.  Dot products: per-workgroup partials in a fixed order; every
// workgroup of the next kernel adds the partials itself in the same order, so all see
// the bitwise identical total.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/mgcurv.h"
#include "mgc_device.h"
#include "mgc_fbs_device.h"

namespace rec {

constexpr int RB = 2;              // blur radius (5 x 5)
constexpr int NW = (2 * RB + 1) * (2 * RB + 1);

struct Blur {
    double w[NW];   // w[(dy + 2) * 5 + dx + 2]: (A u)(p) = sum w[o] u(p + o)
    double g[5];    // 1-D factor: the normalised Gaussian is g[dy + 2] g[dx + 2]
};

// Patches of colour k of a level with side b: index g -> patch (p, q).
struct ColourGrid {
    int b, mj, nj, pr, pc, na, nb;
    __host__ __device__ int count() const { return na * nb; }
};

inline ColourGrid colour_grid(int H, int W, int b, int colour)
{
    ColourGrid g;
    g.b = b;
    g.mj = (H + b - 1) / b;
    g.nj = (W + b - 1) / b;
    g.pr = colour >> 1;
    g.pc = colour & 1;
    g.na = (g.mj - g.pr + 1) / 2;
    g.nb = (g.nj - g.pc + 1) / 2;
    if (g.na < 0) g.na = 0;
    if (g.nb < 0) g.nb = 0;
    return g;
}

// Sum of NT values of a workgroup in a fixed order (wave butterfly, then the waves
// in order through LDS); every thread receives the total.
template <int NT>
__device__ __forceinline__ double block_total(double x, double* lds)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) x += __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = x;
    __syncthreads();
    double s = lds[0];
#pragma unroll
    for (int k = 1; k < NT / 64; ++k) s += lds[k];
    __syncthreads();
    return s;
}

// Every workgroup adds the same n partials in the same order.
template <int NT>
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int n, double* lds)
{
    double x = 0.0;
    for (int t = threadIdx.x; t < n; t += NT) x += part[t];
    return block_total<NT>(x, lds);
}

// Pixel kernels run on a 2-D grid: x over columns, y over rows (row-strided), so
// no pixel index is ever divided.
#define REC_PIXELS                                                          \
    const int j = blockIdx.x * blockDim.x + threadIdx.x;                     \
    if (j >= W) return;                                                      \
    for (int i = blockIdx.y; i < H; i += gridDim.y)

// t = b - A u
template <typename T>
__global__ __launch_bounds__(256) void residual_kernel(const T* __restrict__ u, const T* __restrict__ b, int H, int W,
                                                       Blur bl, double* __restrict__ t)
{
    REC_PIXELS {
        double acc = 0.0;
#pragma unroll
        for (int dy = -RB; dy <= RB; ++dy) {
            const int ii = i + dy;
            if (ii < 0 || ii >= H) continue;
#pragma unroll
            for (int dx = -RB; dx <= RB; ++dx) {
                const int jj = j + dx;
                if (jj < 0 || jj >= W) continue;
                acc += bl.w[(dy + RB) * 5 + dx + RB] * (double)u[(size_t)ii * W + jj];
            }
        }
        const size_t k = (size_t)i * W + j;
        t[k] = (double)b[k] - acc;
    }
}

// One factor of <A phi_i, A phi_l> (the Gaussian is separable, so the inner product of two
// blurred patch indicators is a product of a row and a column factor): the overlap, over the n
// rows of the image, of the blurred indicators of rows [a1, e1) and [a2, e2).
__host__ __device__ inline double blur_overlap(const Blur& bl, int a1, int e1, int a2, int e2, int n)
{
    const int lo = max(0, max(a1, a2) - RB), hi = min(n, min(e1, e2) + RB);   // both nonzero only here
    double s = 0.0;
    for (int i = lo; i < hi; ++i) {
        double r1 = 0.0, r2 = 0.0;
#pragma unroll
        for (int d = -RB; d <= RB; ++d) {
            if (i + d >= a1 && i + d < e1) r1 += bl.g[d + RB];
            if (i + d >= a2 && i + d < e2) r2 += bl.g[d + RB];
        }
        s += r1 * r2;
    }
    return s;
}

// Squared norm of the blurred indicator of rows [a, e): the diagonal factor.
__host__ __device__ inline double blur_factor(const Blur& bl, int a, int e, int n)
{
    return blur_overlap(bl, a, e, a, e, n);
}

// Patch (p, q) of a colour-grid index.
__device__ __forceinline__ void patch_of(const ColourGrid& cg, int g, int& p, int& q)
{
    p = 2 * (g / cg.nb) + cg.pr;
    q = 2 * (g % cg.nb) + cg.pc;
}

// S_i = sum over the pixels of patch i of (A^T img) (G lanes per patch, fixed order).
template <int G>
__device__ __forceinline__ double patch_adjoint_sum(const double* __restrict__ img, int H, int W, const Blur& bl,
                                                    int r0, int r1, int c0, int c1, int lane)
{
    const int w = c1 - c0, n = (r1 - r0) * w;
    double acc = 0.0;
    for (int t = lane; t < n; t += G) {
        const int i = r0 + t / w, j = c0 + t % w;
        double a = 0.0;
#pragma unroll
        for (int dy = -RB; dy <= RB; ++dy) {
            const int ii = i - dy;
            if (ii < 0 || ii >= H) continue;
#pragma unroll
            for (int dx = -RB; dx <= RB; ++dx) {
                const int jj = j - dx;
                if (jj < 0 || jj >= W) continue;
                a += bl.w[(dy + RB) * 5 + dx + RB] * img[(size_t)ii * W + jj];
            }
        }
        acc += a;
    }
#pragma unroll
    for (int off = 1; off < G; off <<= 1) acc += __shfl_xor(acc, off, 64);
    return acc;
}

// d_i (Proposition 1 on the patch's rings), r_i = sum_patch A^T t + 2 alpha d_i,
// x_i = 0, p_i = r_i, and per-workgroup partials of r . r.
// With `diagonal` (patch side >= 5: the blurred indicators of two patches of one
// colour, each reaching 2 pixels beyond its patch, are separated by a gap of b >= 5
// pixels and never overlap, so G is diagonal) the kernel solves directly:
// x_i = r_i / (<A phi_i, A phi_i> + 2 alpha).
template <typename T, int G>
__global__ __launch_bounds__(256) void rhs_kernel(const T* __restrict__ u, const double* __restrict__ t, int H, int W,
                                                  Blur bl, ColourGrid cg, double alpha, int diagonal,
                                                  double* __restrict__ x, double* __restrict__ r,
                                                  double* __restrict__ pv, double* __restrict__ part_rr)
{
    __shared__ double lds[4];
    const int gid = (int)((blockIdx.x * blockDim.x + threadIdx.x) / G), lane = threadIdx.x % G;
    const bool live = gid < cg.count();
    double rr = 0.0;
    if (live) {
        int p, q;
        patch_of(cg, gid, p, q);
        const int b = cg.b, R = (b + 1) / 2;
        const int r0 = p * b, r1 = min(r0 + b, H), c0 = q * b, c1 = min(c0 + b, W);
        const int oi = r0 + R - 1, oj = c0 + R - 1;
        auto value = [&](int i, int j) {
            return (double)u[(size_t)fbs::clampi(i, 0, H - 1) * W + fbs::clampi(j, 0, W - 1)];
        };
        const double uo = value(oi, oj);
        double sum = 0.0;
        fbs::GcAcc unused = fbs::gc_empty();
        for (int rr_ = lane + 1; rr_ <= R; rr_ += G) {
            double v[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) v[m] = value(oi + rr_ * fbs::ring_di(m), oj + rr_ * fbs::ring_dj(m));
            fbs::ring_accumulate<0>(uo, v, (double)rr_, 8 * (rr_ - 1), sum, unused);
        }
#pragma unroll
        for (int off = 1; off < G; off <<= 1) sum += __shfl_xor(sum, off, 64);
        const double d = sum / (double)(8 * R);
        const double ri = patch_adjoint_sum<G>(t, H, W, bl, r0, r1, c0, c1, lane) + 2.0 * alpha * d;
        const size_t id = (size_t)gid;   // patch vectors are stored in colour-grid order
        if (lane == 0) {
            if (diagonal) {
                const double gii = blur_factor(bl, r0, r1, H) * blur_factor(bl, c0, c1, W);
                x[id] = ri / (gii + 2.0 * alpha);
            } else {
                x[id] = 0.0;
                r[id] = ri;
                pv[id] = ri;
                rr = ri * ri;
            }
        }
    } else {
        // keep the group's shuffles complete for lanes of a dead group
        double z = 0.0;
#pragma unroll
        for (int off = 1; off < G; off <<= 1) z += __shfl_xor(z, off, 64);
#pragma unroll
        for (int off = 1; off < G; off <<= 1) z += __shfl_xor(z, off, 64);
    }
    const double tot = block_total<256>(rr, lds);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = tot;
}

// scal[k] = sum of the partials (one workgroup)
__global__ __launch_bounds__(256) void scalar_kernel(const double* __restrict__ part, int n, double* __restrict__ scal, int k)
{
    __shared__ double lds[4];
    const double s = sum_partials<256>(part, n, lds);
    if (threadIdx.x == 0) scal[k] = s;
}

// Row (or column) factors of one colour's Gram matrix G_il = <A phi_i, A phi_l>:
// tab[k * (2 DH + 1) + d + DH] = blur_overlap of the colour's patch row k and patch row k + d
// (rows p = 2k + par of the level's m patch rows of side b in an image of n rows; 0 where row
// k + d does not exist).  Two patches of one colour interact only if their blurred indicators
// (each reaching RB pixels beyond the patch) overlap: |2d| b < b + 2 RB.
__global__ __launch_bounds__(256) void overlap_table_kernel(Blur bl, int b, int n, int m, int par, int cnt, int DH,
                                                            double* __restrict__ tab)
{
    const int ND = 2 * DH + 1;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < cnt * ND; t += gridDim.x * blockDim.x) {
        const int k = t / ND, d = t - k * ND - DH;
        const int p = 2 * k + par, p2 = p + 2 * d;
        double v = 0.0;
        if (p2 >= 0 && p2 < m) v = blur_overlap(bl, p * b, min(p * b + b, n), p2 * b, min(p2 * b + b, n), n);
        tab[t] = v;
    }
}

// q = (G + 2 alpha I) p on one colour, G_il = row factor x column factor, and partials of p . q.
template <int DH>
__global__ __launch_bounds__(256) void gram_stencil_kernel(const double* __restrict__ pv, ColourGrid cg,
                                                           const double* __restrict__ tab_r,
                                                           const double* __restrict__ tab_c, double alpha,
                                                           double* __restrict__ qv, double* __restrict__ part_pq)
{
    __shared__ double lds[4];
    constexpr int ND = 2 * DH + 1;
    double pq = 0.0;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < cg.count(); g += gridDim.x * blockDim.x) {
        const int a = g / cg.nb, c = g - a * cg.nb;
        double acc = 0.0;
#pragma unroll
        for (int da = -DH; da <= DH; ++da) {
            const int a2 = a + da;
            if (a2 < 0 || a2 >= cg.na) continue;
            const double* prow = pv + (size_t)a2 * cg.nb;
            double row = 0.0;
#pragma unroll
            for (int dc = -DH; dc <= DH; ++dc) {
                const int c2 = c + dc;
                if (c2 < 0 || c2 >= cg.nb) continue;
                row += tab_c[c * ND + dc + DH] * prow[c2];
            }
            acc += tab_r[a * ND + da + DH] * row;
        }
        const size_t id = (size_t)g;
        const double qi = fma(2.0 * alpha, pv[id], acc);
        qv[id] = qi;
        pq += pv[id] * qi;
    }
    const double tot = block_total<256>(pq, lds);
    if (threadIdx.x == 0) part_pq[blockIdx.x] = tot;
}

// a = rr / pq; x += a p; r -= a q; partials of the new r . r
__global__ __launch_bounds__(256) void update_xr_kernel(ColourGrid cg, const double* __restrict__ part_pq, int npart,
                                                        const double* __restrict__ scal, int k_rr,
                                                        double* __restrict__ x, double* __restrict__ r,
                                                        const double* __restrict__ pv, const double* __restrict__ qv,
                                                        double* __restrict__ part_rr)
{
    __shared__ double lds[4];
    const double pq = sum_partials<256>(part_pq, npart, lds);
    const double rr = scal[k_rr];
    const double a = pq > 0.0 ? rr / pq : 0.0;
    double acc = 0.0;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < cg.count(); g += gridDim.x * blockDim.x) {
        const size_t id = (size_t)g;
        x[id] += a * pv[id];
        const double rn = r[id] - a * qv[id];
        r[id] = rn;
        acc += rn * rn;
    }
    const double tot = block_total<256>(acc, lds);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = tot;
}

// rr_new = sum of the partials; beta = rr_new / rr; p = r + beta p; scal[k_new] = rr_new
__global__ __launch_bounds__(256) void update_p_kernel(ColourGrid cg, const double* __restrict__ part_rr, int npart,
                                                       double* __restrict__ scal, int k_old, int k_new,
                                                       const double* __restrict__ r, double* __restrict__ pv)
{
    __shared__ double lds[4];
    const double rn = sum_partials<256>(part_rr, npart, lds);
    const double ro = scal[k_old];
    const double beta = ro > 0.0 ? rn / ro : 0.0;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < cg.count(); g += gridDim.x * blockDim.x) {
        const size_t id = (size_t)g;
        pv[id] = r[id] + beta * pv[id];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[k_new] = rn;
}

// u <- u + x_i on the pixels of colour-k patches (rounded to T)
template <typename T>
__global__ __launch_bounds__(256) void apply_kernel(T* __restrict__ u, int H, int W, ColourGrid cg,
                                                    const double* __restrict__ x)
{
    REC_PIXELS {
        const int p = i / cg.b, q = j / cg.b;
        if ((p & 1) == cg.pr && (q & 1) == cg.pc) {
            const double c = x[(size_t)(p >> 1) * cg.nb + (q >> 1)];   // colour-grid order
            const size_t k = (size_t)i * W + j;
            if (c != 0.0) u[k] = (T)((double)u[k] + c);
        }
    }
}

// Energy partials: 1/2 (A u - b)^2 + alpha |kappa_MC(u)|, one partial per workgroup
template <typename T>
__global__ __launch_bounds__(256) void energy_kernel(const T* __restrict__ u, const T* __restrict__ b, int H, int W,
                                                     Blur bl, double alpha, double* __restrict__ part)
{
    __shared__ double lds[4];
    double acc = 0.0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < W; j += gridDim.x * blockDim.x) {
        for (int i = blockIdx.y; i < H; i += gridDim.y) {
            double a = 0.0;
#pragma unroll
            for (int dy = -RB; dy <= RB; ++dy) {
                const int ii = i + dy;
                if (ii < 0 || ii >= H) continue;
#pragma unroll
                for (int dx = -RB; dx <= RB; ++dx) {
                    const int jj = j + dx;
                    if (jj < 0 || jj >= W) continue;
                    a += bl.w[(dy + RB) * 5 + dx + RB] * (double)u[(size_t)ii * W + jj];
                }
            }
            const double res = a - (double)b[(size_t)i * W + j];
            acc += 0.5 * res * res + alpha * mgc::abs_kappa_at<0>(u, H, W, i, j);
        }
    }
    const double tot = block_total<256>(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = tot;
}

constexpr int GRID_PIX = 2048;   // partial sums of the energy and of the norms

inline dim3 pixel_grid(int H, int W) { return dim3((W + 255) / 256, H < 1024 ? H : 1024); }

}  // namespace rec

// ---------------------------------------------------------------------------
// Host runtime
// ---------------------------------------------------------------------------
struct mg_recon_ctx {
    mg_recon_params P;
    int device;
    hipStream_t stream;
    hipStream_t gstream;     // own stream, only for capturing graphs (default priority)
    rec::Blur blur;
    double* t;               // H x W FP64: b - A u
    double* tab;             // Gram row and column factors of one colour: 5 (H + W) doubles
    double* x;               // patch vectors of one colour, in colour-grid order (a * nb + c)
    double* r;
    double* pv;
    double* qv;
    double* part_a;          // workgroup partials
    double* part_b;
    double* scal;            // CG scalars (two r . r slots) and the energy
    double* host1;           // pinned energy
    void* prev;              // previous iterate for relErr(u)
    double* norms_part;      // relErr(u) partials
    hipGraph_t graph;
    hipGraphExec_t exec;
    const void* g_u;
    const void* g_b;
    std::string err;
};

namespace {

thread_local std::string g_recon_init_error;

mg_status rfail(mg_recon_ctx* ctx, mg_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf; else g_recon_init_error = buf;
    return st;
}

mg_status rhip(mg_recon_ctx* ctx, hipError_t e, const char* what)
{
    return rfail(ctx, MG_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool r64(const mg_recon_ctx* c) { return c->P.state_dtype == MG_F64; }
size_t rbytes(const mg_recon_ctx* c) { return (size_t)c->P.height * c->P.width * (r64(c) ? 8 : 4); }

mg_status rcheck(mg_recon_ctx* ctx, const void* u, const void* b)
{
    if (!ctx) return MG_E_INVALID;
    if (!u || !b) return rfail(ctx, MG_E_INVALID, "u and b must be non-null device pointers");
    const size_t n = rbytes(ctx);
    const char* a = (const char*)u;
    const char* bb = (const char*)b;
    if (a < bb + n && bb < a + n) return rfail(ctx, MG_E_INVALID, "u must not overlap b");
    return MG_OK;
}

// lanes per patch for the patch-wise sums
int lanes_for(int b) { return b == 1 ? 1 : (b <= 3 ? 8 : (b <= 7 ? 64 : 256)); }

int groups_grid(int count, int G) { return (int)(((size_t)count * G + 255) / 256); }

template <typename T>
mg_status colour_sweep(mg_recon_ctx* c, hipStream_t st, void* u, const void* b, int level, int colour)
{
    const int H = c->P.height, W = c->P.width;
    const int bs = (1 << level) - 1;
    const rec::ColourGrid cg = rec::colour_grid(H, W, bs, colour);
    const int n = cg.count();
    if (n == 0) return MG_OK;
    const int G = lanes_for(bs);
    const int ng = groups_grid(n, G);        // workgroups of the patch-wise kernels
    const int nv = (n + 255) / 256;          // workgroups of the vector kernels
    const dim3 blk(256), gp = rec::pixel_grid(H, W);
    const int diagonal = bs >= 5;
    hipLaunchKernelGGL(rec::residual_kernel<T>, gp, blk, 0, st, (const T*)u, (const T*)b, H, W, c->blur, c->t);
    switch (G) {
    case 1: hipLaunchKernelGGL((rec::rhs_kernel<T, 1>), dim3(ng), blk, 0, st, (const T*)u, (const double*)c->t, H, W, c->blur, cg, c->P.alpha, diagonal, c->x, c->r, c->pv, c->part_b); break;
    case 8: hipLaunchKernelGGL((rec::rhs_kernel<T, 8>), dim3(ng), blk, 0, st, (const T*)u, (const double*)c->t, H, W, c->blur, cg, c->P.alpha, diagonal, c->x, c->r, c->pv, c->part_b); break;
    case 64: hipLaunchKernelGGL((rec::rhs_kernel<T, 64>), dim3(ng), blk, 0, st, (const T*)u, (const double*)c->t, H, W, c->blur, cg, c->P.alpha, diagonal, c->x, c->r, c->pv, c->part_b); break;
    default: hipLaunchKernelGGL((rec::rhs_kernel<T, 256>), dim3(ng), blk, 0, st, (const T*)u, (const double*)c->t, H, W, c->blur, cg, c->P.alpha, diagonal, c->x, c->r, c->pv, c->part_b); break;
    }
    if (!diagonal) hipLaunchKernelGGL(rec::scalar_kernel, dim3(1), blk, 0, st, (const double*)c->part_b, ng, c->scal, 0);
    // the colour's Gram factors (the operator depends only on the geometry and A)
    const int dh = (2 * rec::RB + bs) / (2 * bs);   // largest |d| with |2d| b < b + 2 RB
    double* tab_r = c->tab;
    double* tab_c = c->tab + (size_t)cg.na * (2 * dh + 1);
    if (!diagonal) {
        const int nr = cg.na * (2 * dh + 1), nc = cg.nb * (2 * dh + 1);
        hipLaunchKernelGGL(rec::overlap_table_kernel, dim3((nr + 255) / 256), blk, 0, st, c->blur, bs, H, cg.mj, cg.pr,
                           cg.na, dh, tab_r);
        hipLaunchKernelGGL(rec::overlap_table_kernel, dim3((nc + 255) / 256), blk, 0, st, c->blur, bs, W, cg.nj, cg.pc,
                           cg.nb, dh, tab_c);
    }
    for (int it = 0; it < (diagonal ? 0 : c->P.cg_iters); ++it) {
        const int k_old = it & 1, k_new = k_old ^ 1;
        if (dh == 2)
            hipLaunchKernelGGL(rec::gram_stencil_kernel<2>, dim3(nv), blk, 0, st, (const double*)c->pv, cg,
                               (const double*)tab_r, (const double*)tab_c, c->P.alpha, c->qv, c->part_a);
        else
            hipLaunchKernelGGL(rec::gram_stencil_kernel<1>, dim3(nv), blk, 0, st, (const double*)c->pv, cg,
                               (const double*)tab_r, (const double*)tab_c, c->P.alpha, c->qv, c->part_a);
        hipLaunchKernelGGL(rec::update_xr_kernel, dim3(nv), blk, 0, st, cg, (const double*)c->part_a, nv,
                           (const double*)c->scal, k_old, c->x, c->r, (const double*)c->pv, (const double*)c->qv, c->part_b);
        hipLaunchKernelGGL(rec::update_p_kernel, dim3(nv), blk, 0, st, cg, (const double*)c->part_b, nv, c->scal, k_old,
                           k_new, (const double*)c->r, c->pv);
    }
    hipLaunchKernelGGL(rec::apply_kernel<T>, gp, blk, 0, st, (T*)u, H, W, cg, (const double*)c->x);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? MG_OK : rhip(c, e, "reconstruction sweep launch");
}

template <typename T>
mg_status vcycle_t(mg_recon_ctx* c, hipStream_t st, void* u, const void* b)
{
    for (int level = 1; level <= c->P.levels; ++level)
        for (int colour = 0; colour < 4; ++colour) {
            mg_status s = colour_sweep<T>(c, st, u, b, level, colour);
            if (s != MG_OK) return s;
        }
    return MG_OK;
}

mg_status vcycle_enqueue(mg_recon_ctx* c, hipStream_t st, void* u, const void* b)
{
    return r64(c) ? vcycle_t<double>(c, st, u, b) : vcycle_t<float>(c, st, u, b);
}

template <typename T>
mg_status energy_enqueue_t(mg_recon_ctx* c, hipStream_t st, const void* u, const void* b)
{
    // at most GRID_PIX workgroups (hence partials): columns first, the rest over rows
    int ex = (c->P.width + 255) / 256;
    if (ex > rec::GRID_PIX) ex = rec::GRID_PIX;
    int ey = rec::GRID_PIX / ex;
    if (ey > c->P.height) ey = c->P.height;
    const dim3 eg(ex, ey);
    hipLaunchKernelGGL(rec::energy_kernel<T>, eg, dim3(256), 0, st, (const T*)u, (const T*)b,
                       c->P.height, c->P.width, c->blur, c->P.alpha, c->part_a);
    hipLaunchKernelGGL(rec::scalar_kernel, dim3(1), dim3(256), 0, st, (const double*)c->part_a, (int)(eg.x * eg.y),
                       c->scal, 2);
    hipError_t e = hipMemcpyAsync(c->host1, c->scal + 2, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? MG_OK : rhip(c, e, "energy launch");
}

mg_status energy_now(mg_recon_ctx* c, const void* u, const void* b, double* out)
{
    mg_status s = r64(c) ? energy_enqueue_t<double>(c, c->stream, u, b) : energy_enqueue_t<float>(c, c->stream, u, b);
    if (s != MG_OK) return s;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return rhip(c, e, "stream synchronize");
    *out = *c->host1;
    return MG_OK;
}

void drop_graph(mg_recon_ctx* c)
{
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->exec = nullptr;
    c->graph = nullptr;
    c->g_u = c->g_b = nullptr;
}

// One V-cycle as a graph captured once per (u, b), replayed into the caller's stream.
mg_status replay_vcycle(mg_recon_ctx* c, void* u, const void* b)
{
    if (!c->exec || c->g_u != u || c->g_b != b) {
        drop_graph(c);
        hipError_t e = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return rhip(c, e, "begin capture");
        mg_status s = vcycle_enqueue(c, c->gstream, u, b);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(c->gstream, &g);
        if (s != MG_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return rhip(c, e, "end capture");
        c->graph = g;
        if ((e = hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0)) != hipSuccess) {
            drop_graph(c);
            return rhip(c, e, "graph instantiate");
        }
        c->g_u = u;
        c->g_b = b;
    }
    hipError_t e = hipGraphLaunch(c->exec, c->stream);
    return e == hipSuccess ? MG_OK : rhip(c, e, "graph launch");
}

template <typename T>
__global__ __launch_bounds__(256) void norms_kernel(const T* __restrict__ u, const T* __restrict__ prev, size_t n,
                                                    double* __restrict__ part)
{
    __shared__ double lds[4];
    double a = 0.0, bb = 0.0;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
        const double x = (double)u[k], d = x - (double)prev[k];
        a += d * d;
        bb += x * x;
    }
    const double ta = rec::block_total<256>(a, lds);
    const double tb = rec::block_total<256>(bb, lds);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = ta;
        part[rec::GRID_PIX + blockIdx.x] = tb;
    }
}

}  // namespace

extern "C" {

void mg_recon_default_params(mg_recon_params* p, int32_t height, int32_t width)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->height = height;
    p->width = width;
    p->alpha = 0.01;
    p->blur_sigma = 1.0;
    p->levels = 3;
    p->state_dtype = MG_F32;
    p->cg_iters = 20;
}

mg_status mg_recon_init(const mg_recon_params* params, void* hip_stream, mg_recon_ctx** out)
{
    if (!params || !out) return rfail(nullptr, MG_E_INVALID, "params and out must be non-null");
    *out = nullptr;
    const mg_recon_params& p = *params;
    if (p.height < 2 || p.width < 2) return rfail(nullptr, MG_E_SHAPE, "height and width must be >= 2 (got %d x %d)", p.height, p.width);
    if ((int64_t)p.height * p.width > ((int64_t)1 << 31) - 1)
        return rfail(nullptr, MG_E_SHAPE, "image larger than 2^31 - 1 pixels");
    if (!(p.alpha >= 0.0) || !std::isfinite(p.alpha)) return rfail(nullptr, MG_E_INVALID, "alpha must be finite and >= 0");
    if (!(p.blur_sigma > 0.0) || !std::isfinite(p.blur_sigma)) return rfail(nullptr, MG_E_INVALID, "blur_sigma must be finite and > 0");
    if (p.state_dtype != MG_F32 && p.state_dtype != MG_F64) return rfail(nullptr, MG_E_DTYPE, "state_dtype must be MG_F32 or MG_F64");
    if (p.levels < 1 || p.levels > 16) return rfail(nullptr, MG_E_INVALID, "levels must be in [1, 16]");
    if (p.cg_iters < 1 || p.cg_iters > 1000) return rfail(nullptr, MG_E_INVALID, "cg_iters must be in [1, 1000]");
    if (p.reserved != 0) return rfail(nullptr, MG_E_INVALID, "reserved must be 0");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) return rfail(nullptr, MG_E_DEVICE, "no HIP device available");
    mg_recon_ctx* c = new (std::nothrow) mg_recon_ctx();
    if (!c) return rfail(nullptr, MG_E_NOMEM, "host allocation failed");
    c->P = p;
    c->stream = (hipStream_t)hip_stream;
    c->gstream = nullptr;
    c->t = c->tab = c->x = c->r = c->pv = c->qv = c->part_a = c->part_b = c->scal = c->host1 = nullptr;
    c->norms_part = nullptr;
    c->prev = nullptr;
    c->graph = nullptr;
    c->exec = nullptr;
    c->g_u = c->g_b = nullptr;
    (void)hipGetDevice(&c->device);
    // the 5 x 5 normalised Gaussian of A
    double tot = 0.0;
    for (int dy = -rec::RB; dy <= rec::RB; ++dy)
        for (int dx = -rec::RB; dx <= rec::RB; ++dx) {
            const double v = std::exp(-(dx * dx + dy * dy) / (2.0 * p.blur_sigma * p.blur_sigma));
            c->blur.w[(dy + rec::RB) * 5 + dx + rec::RB] = v;
            tot += v;
        }
    for (int k = 0; k < rec::NW; ++k) c->blur.w[k] /= tot;
    double g1 = 0.0;
    for (int d = -rec::RB; d <= rec::RB; ++d) g1 += std::exp(-(d * d) / (2.0 * p.blur_sigma * p.blur_sigma));
    for (int d = -rec::RB; d <= rec::RB; ++d)
        c->blur.g[d + rec::RB] = std::exp(-(d * d) / (2.0 * p.blur_sigma * p.blur_sigma)) / g1;
    size_t npatch = 1;
    int maxgroups = 1;
    for (int level = 1; level <= p.levels; ++level) {
        const int b = (1 << level) - 1;
        const size_t m = (size_t)((p.height + b - 1) / b) * ((p.width + b - 1) / b);
        if (m > npatch) npatch = m;
        for (int colour = 0; colour < 4; ++colour) {
            const rec::ColourGrid cg = rec::colour_grid(p.height, p.width, b, colour);
            const int ng = groups_grid(cg.count(), lanes_for(b));
            if (ng > maxgroups) maxgroups = ng;
        }
    }
    const size_t img = (size_t)p.height * p.width;
    const size_t npart = (size_t)(maxgroups > rec::GRID_PIX ? maxgroups : rec::GRID_PIX);
    if (hipMalloc((void**)&c->t, img * 8) != hipSuccess ||
        hipMalloc((void**)&c->tab, (size_t)5 * (p.height + p.width) * 8) != hipSuccess ||
        hipMalloc((void**)&c->x, npatch * 8) != hipSuccess ||
        hipMalloc((void**)&c->r, npatch * 8) != hipSuccess || hipMalloc((void**)&c->pv, npatch * 8) != hipSuccess ||
        hipMalloc((void**)&c->qv, npatch * 8) != hipSuccess || hipMalloc((void**)&c->part_a, npart * 8) != hipSuccess ||
        hipMalloc((void**)&c->part_b, npart * 8) != hipSuccess || hipMalloc((void**)&c->scal, 8 * 8) != hipSuccess ||
        hipMalloc(&c->prev, rbytes(c)) != hipSuccess ||
        hipMalloc((void**)&c->norms_part, 2 * rec::GRID_PIX * 8) != hipSuccess ||
        hipHostMalloc((void**)&c->host1, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess) {
        mg_recon_destroy(c);
        (void)hipGetLastError();
        return rfail(nullptr, MG_E_NOMEM, "device allocation failed (image of %zu pixels)", img);
    }
    *out = c;
    return MG_OK;
}

mg_status mg_recon_sweep(mg_recon_ctx* ctx, void* u, const void* b, int32_t level, int32_t colour)
{
    mg_status st = rcheck(ctx, u, b);
    if (st != MG_OK) return st;
    if (level < 1 || level > ctx->P.levels) return rfail(ctx, MG_E_INVALID, "level must be in [1, %d]", ctx->P.levels);
    if (colour < 0 || colour > 3) return rfail(ctx, MG_E_INVALID, "colour must be in [0, 4)");
    return r64(ctx) ? colour_sweep<double>(ctx, ctx->stream, u, b, level, colour)
                    : colour_sweep<float>(ctx, ctx->stream, u, b, level, colour);
}

mg_status mg_recon_vcycle(mg_recon_ctx* ctx, void* u, const void* b, double* energy_after)
{
    mg_status st = rcheck(ctx, u, b);
    if (st != MG_OK) return st;
    if ((st = replay_vcycle(ctx, u, b)) != MG_OK) return st;
    if (!energy_after) return MG_OK;
    return energy_now(ctx, u, b, energy_after);
}

mg_status mg_recon_energy(mg_recon_ctx* ctx, const void* u, const void* b, double* energy)
{
    mg_status st = rcheck(ctx, u, b);
    if (st != MG_OK) return st;
    if (!energy) return rfail(ctx, MG_E_INVALID, "energy output must be non-null");
    return energy_now(ctx, u, b, energy);
}

mg_status mg_recon_solve(mg_recon_ctx* ctx, void* u, const void* b, double tol, int32_t max_vcycles,
                         int32_t* vcycles_done, double* final_energy)
{
    mg_status st = rcheck(ctx, u, b);
    if (st != MG_OK) return st;
    if (max_vcycles < 0 || !std::isfinite(tol)) return rfail(ctx, MG_E_INVALID, "bad tol or max_vcycles");
    double e;
    if ((st = energy_now(ctx, u, b, &e)) != MG_OK) return st;
    if (!std::isfinite(e)) return rfail(ctx, MG_E_NONFINITE, "energy of the initial state is not finite");
    const size_t n = (size_t)ctx->P.height * ctx->P.width;
    int done = 0;
    bool conv = false;
    while (done < max_vcycles) {
        hipError_t he = hipMemcpyAsync(ctx->prev, u, rbytes(ctx), hipMemcpyDeviceToDevice, ctx->stream);
        if (he != hipSuccess) return rhip(ctx, he, "state copy");
        if ((st = replay_vcycle(ctx, u, b)) != MG_OK) return st;
        if (r64(ctx))
            hipLaunchKernelGGL(norms_kernel<double>, dim3(rec::GRID_PIX), dim3(256), 0, ctx->stream, (const double*)u,
                               (const double*)ctx->prev, n, ctx->norms_part);
        else
            hipLaunchKernelGGL(norms_kernel<float>, dim3(rec::GRID_PIX), dim3(256), 0, ctx->stream, (const float*)u,
                               (const float*)ctx->prev, n, ctx->norms_part);
        hipLaunchKernelGGL(rec::scalar_kernel, dim3(1), dim3(256), 0, ctx->stream, (const double*)ctx->norms_part,
                           rec::GRID_PIX, ctx->scal, 3);
        hipLaunchKernelGGL(rec::scalar_kernel, dim3(1), dim3(256), 0, ctx->stream,
                           (const double*)ctx->norms_part + rec::GRID_PIX, rec::GRID_PIX, ctx->scal, 4);
        he = hipMemcpyAsync(ctx->host1 + 1, ctx->scal + 3, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
        if (he != hipSuccess) return rhip(ctx, he, "norm copy");
        if ((st = energy_now(ctx, u, b, &e)) != MG_OK) return st;
        ++done;
        if (!std::isfinite(e)) return rfail(ctx, MG_E_NONFINITE, "energy became non-finite after V-cycle %d", done);
        if (tol > 0.0 && std::sqrt(ctx->host1[1]) < tol * std::sqrt(ctx->host1[2])) {
            conv = true;
            break;
        }
    }
    if (vcycles_done) *vcycles_done = done;
    if (final_energy) *final_energy = e;
    return (tol > 0.0 && !conv) ? MG_NOT_CONVERGED : MG_OK;
}

void mg_recon_destroy(mg_recon_ctx* ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->gstream) (void)hipStreamSynchronize(ctx->gstream);
    drop_graph(ctx);
    if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
    for (double* q : {ctx->t, ctx->tab, ctx->x, ctx->r, ctx->pv, ctx->qv, ctx->part_a, ctx->part_b, ctx->scal,
                      ctx->norms_part})
        if (q) (void)hipFree(q);
    if (ctx->prev) (void)hipFree(ctx->prev);
    if (ctx->host1) (void)hipHostFree(ctx->host1);
    delete ctx;
}

const char* mg_recon_last_error(const mg_recon_ctx* ctx)
{
    if (ctx) return ctx->err.c_str();
    return g_recon_init_error.c_str();
}

}  // extern "C"
