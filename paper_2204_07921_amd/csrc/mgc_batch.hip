// Batched multigrid curvature minimisation: many images of different sizes,
// alphas and curvature kinds in one packed buffer, float32 state.
//
// Every (level, colour) is ONE persistent kernel over the concatenated work
// list of all images (cells at the pixel level, same-colour blocks above it).
// Images are visited in curvature-kind order (mean first, then Gaussian), so
// neighbouring lane groups almost always run the same kind.  A work item finds
// its image by binary search over cumulative item counts.  Converged images
// drop out through a per-image active flag; the lists are never rebuilt.
// One V-cycle, the per-image FP64 energies and their copy to the host are
// captured once in a hipGraph and replayed.  Lane-group shapes per level and
// the persistent grid size are chosen by a small timing autotuner.
//
// The per-block and per-cell solvers are the same device code as the
// single-image path (mgc_sweep.h), so a batch reproduces single-image runs
// bit for bit when the same group shapes are used.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mgcurv.h"
#include "mgc_internal.h"
#include "mgc_sweep.h"

namespace mgc {

struct BatchImg {
    long long off;  // element offset in the packed buffers
    int H, W;
    double alpha;
    int kind;
    int J;
};

__device__ __forceinline__ int find_slot(const int* __restrict__ cum, int n, int t)
{
    // largest k in [0, n) with cum[k] <= t (cum[0] = 0, cum[n] = total)
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cum[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// Pixel level, four colours, two-phase (uin -> uout).  Inactive images are
// skipped in every pass, so after the four passes their data is still in uin = u.
// Interior cells (cum_in) take one thread each (constant-slope form); the outer
// ring of cells of every image (cum_ring) takes a 16-lane group per cell.
__global__ __launch_bounds__(256) void batch_pixels_kernel(const float* __restrict__ uin, float* __restrict__ uout,
                                                           const float* __restrict__ f, const BatchImg* __restrict__ imgs,
                                                           const int* __restrict__ order, const int* __restrict__ cum,
                                                           int n, int total, const int* __restrict__ active, int colour,
                                                           int M, int G)
{
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
        const int k = find_slot(cum, n, t);
        const int img = order[k];
        if (!active[img]) continue;
        const BatchImg im = imgs[img];
        const int ic = (im.W + 1) / 2 - 2;
        const int cell = t - cum[k];
        const int cr = 1 + cell / ic, cc = 1 + cell % ic;
        if (im.kind == 0)
            solve_cell<float, 0, 2, 1>(uin + im.off, uout + im.off, f + im.off, im.H, im.W, colour, cr, cc, im.alpha, M, G);
        else
            solve_cell<float, 1, 2, 1>(uin + im.off, uout + im.off, f + im.off, im.H, im.W, colour, cr, cc, im.alpha, M, G);
    }
}

__global__ __launch_bounds__(256) void batch_ring_cells_kernel(const float* __restrict__ uin, float* __restrict__ uout,
                                                               const float* __restrict__ f,
                                                               const BatchImg* __restrict__ imgs,
                                                               const int* __restrict__ order, const int* __restrict__ cum,
                                                               int n, int total, const int* __restrict__ active,
                                                               int colour, int M, int G)
{
    const int ngroups = gridDim.x * (blockDim.x / 16);
    const int lane = threadIdx.x & 15;
    for (int t = (blockIdx.x * blockDim.x + threadIdx.x) >> 4; t < total; t += ngroups) {
        const int k = find_slot(cum, n, t);
        const int img = order[k];
        if (!active[img]) continue;   // uniform within the group
        const BatchImg im = imgs[img];
        int cr, cc;
        ring_cell(t - cum[k], (im.H + 1) / 2, (im.W + 1) / 2, cr, cc);
        if (im.kind == 0)
            solve_ring_cell<float, 0, 2>(uin + im.off, uout + im.off, f + im.off, im.H, im.W, colour, cr, cc, lane,
                                         im.alpha, M, G);
        else
            solve_ring_cell<float, 1, 2>(uin + im.off, uout + im.off, f + im.off, im.H, im.W, colour, cr, cc, lane,
                                         im.alpha, M, G);
    }
}

struct BatchLevelArgs {
    int b, lb, pr, pc;            // lb = log2(b), or -1 when b is not a power of two
    const double* partials;       // coarse: block partial sums
    const long long* part_off;    // per image offset into partials
    int nchunk;
    double* cpend;                // coarse: pending corrections
    const long long* pend_off;    // per image offset into cpend
};

template <int GROUP, int RPL, bool LAZY, class GSum>
__device__ __forceinline__ void batch_block_item(float* __restrict__ u, const float* __restrict__ f,
                                                 const BatchImg& im, int img, int local, int lane,
                                                 const BatchLevelArgs& a, int M, int G, const GSum& gs)
{
    const int mj = side_div(im.H + a.b - 1, a.b, a.lb), nj = side_div(im.W + a.b - 1, a.b, a.lb);
    if constexpr (RPL < 0) {   // b = 2, mirrored form off the image border (GROUP = 2 or 4)
        const Split2 S = split2(mj, nj, a.pr, a.pc);
        if (im.kind == 0)
            solve_b2_item<float, 0, GROUP>(u + im.off, f + im.off, im.H, im.W, a.pr, a.pc, S, local, lane, im.alpha,
                                           M, G);
        else
            solve_b2_item<float, 1, GROUP>(u + im.off, f + im.off, im.H, im.W, a.pr, a.pc, S, local, lane, im.alpha,
                                           M, G);
    } else {
        const int nbc = (nj - a.pc + 1) / 2;
        const int bi = local / nbc, bj = local - bi * nbc;
        const int p = 2 * bi + a.pr, q = 2 * bj + a.pc;
        const int r0 = p * a.b, c0 = q * a.b;
        const int r1 = min(r0 + a.b, im.H), c1 = min(c0 + a.b, im.W);
        CoarseArgs ca{LAZY ? a.partials + a.part_off[img] : nullptr, a.nchunk, LAZY ? a.cpend + a.pend_off[img] : nullptr,
                      nj, nullptr, 8 * a.b};
        // both curvatures share this kernel's registers: the widest shapes build their rings in
        // smaller chunks
        constexpr int CH = GROUP >= 1024 ? 1 : (RPL >= 8 ? 2 : ring_chunk<float, GROUP>());
        if (im.kind == 0)
            solve_block<float, 0, GROUP, RPL, LAZY, CH>(u + im.off, f + im.off, im.H, im.W, p, q, r0, r1, c0, c1, lane,
                                                        im.alpha, M, G, gs, ca);
        else
            solve_block<float, 1, GROUP, RPL, LAZY, CH>(u + im.off, f + im.off, im.H, im.W, p, q, r0, r1, c0, c1, lane,
                                                        im.alpha, M, G, gs, ca);
    }
}

template <int GROUP, int RPL, bool LAZY>
__global__ __launch_bounds__(GROUP > 64 ? GROUP : 256) void batch_blocks_kernel(
    float* __restrict__ u, const float* __restrict__ f, const BatchImg* __restrict__ imgs,
    const int* __restrict__ order, const int* __restrict__ cum, int n, int total, const int* __restrict__ active,
    BatchLevelArgs a, int M, int G)
{
    if constexpr (GROUP <= 64) {
        const int ngroups = gridDim.x * (blockDim.x / GROUP);
        const int lane = threadIdx.x & (GROUP - 1);
        for (int t = (blockIdx.x * blockDim.x + threadIdx.x) / GROUP; t < total; t += ngroups) {
            const int k = find_slot(cum, n, t);
            const int img = order[k];
            if (!active[img]) continue;  // uniform within the group
            const BatchImg im = imgs[img];
            batch_block_item<GROUP, RPL, LAZY>(u, f, im, img, t - cum[k], lane, a, M, G, WaveSum<GROUP>());
        }
    } else {
        __shared__ double lds[2 * (GROUP / 64) * BlockSum<GROUP>::NMAX];
        for (int t = blockIdx.x; t < total; t += gridDim.x) {
            const int k = find_slot(cum, n, t);
            const int img = order[k];
            if (!active[img]) continue;  // uniform within the workgroup
            const BatchImg im = imgs[img];
            BlockSum<GROUP> gs{lds, 0};
            batch_block_item<GROUP, RPL, LAZY>(u, f, im, img, t - cum[k], threadIdx.x, a, M, G, gs);
            __syncthreads();  // LDS reuse by the next item
        }
    }
}

// Coarse level begin: partial sums of f - u per (image, block, chunk).  Grid: x = block*chunk slot, y = image.
__global__ __launch_bounds__(256) void batch_block_sums_kernel(const float* __restrict__ u, const float* __restrict__ f,
                                                               const BatchImg* __restrict__ imgs,
                                                               const int* __restrict__ active, int b, int lb,
                                                               int nchunk, int rows_per, double* __restrict__ partials,
                                                               const long long* __restrict__ part_off)
{
    __shared__ double lds[4];
    const int img = blockIdx.y;
    if (!active[img]) return;
    const BatchImg im = imgs[img];
    const int mj = side_div(im.H + b - 1, b, lb), nj = side_div(im.W + b - 1, b, lb);
    for (int slot = blockIdx.x; slot < mj * nj * nchunk; slot += gridDim.x) {
        const int blk = slot / nchunk, k = slot - blk * nchunk;
        const int p = blk / nj, q = blk - p * nj;
        const int c0 = q * b, c1 = min(c0 + b, im.W), w = c1 - c0;
        const int ra = p * b + k * rows_per;
        const int rb = min(min(ra + rows_per, (p + 1) * b), im.H);
        const int cnt = (rb > ra ? rb - ra : 0) * w;
        double acc = 0.0;
        // U elements per round have their loads in flight together; they are summed in the
        // order of t (elements past the chunk's end take element t0's address and are skipped)
        constexpr int U = 8;
        const int B = (int)blockDim.x;
        for (int t0 = threadIdx.x; t0 < cnt; t0 += U * B) {
            double fv[U], uv[U];
#pragma unroll
            for (int m = 0; m < U; ++m) {
                const int t = (m == 0 || t0 + m * B < cnt) ? t0 + m * B : t0;
                const int i = ra + t / w, j = c0 + t % w;
                const size_t idx = (size_t)im.off + (size_t)i * im.W + j;
                fv[m] = (double)f[idx];
                uv[m] = (double)u[idx];
            }
#pragma unroll
            for (int m = 0; m < U; ++m) {
                if (t0 + m * B >= cnt) break;
                acc += fv[m] - uv[m];
            }
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
        if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) partials[part_off[img] + slot] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void batch_fill_kernel(double* __restrict__ x, size_t n, double v)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) x[t] = v;
}

// Coarse level end: u += pending correction of the pixel's block.  Grid: x strides pixels, y = image.
__global__ __launch_bounds__(256) void batch_apply_kernel(float* __restrict__ u, const BatchImg* __restrict__ imgs,
                                                          const int* __restrict__ active, int b, int lb,
                                                          const double* __restrict__ cpend,
                                                          const long long* __restrict__ pend_off)
{
    const int img = blockIdx.y;
    if (!active[img]) return;
    const BatchImg im = imgs[img];
    const int nj = side_div(im.W + b - 1, b, lb);
    const size_t n = (size_t)im.H * im.W;
    const double* cp = cpend + pend_off[img];
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    if (t0 >= n) return;
    // U pixels per round have their loads in flight together (past n: pixel t0's address, skipped)
    constexpr int U = 4;
    PixelWalk pw(t0, stride, im.W);
    for (size_t t = t0; t < n; t += U * stride) {
        size_t px[U];
        double c[U];
        float uv[U];
        const int i0 = pw.i, j0 = pw.j;
#pragma unroll
        for (int m = 0; m < U; ++m) {
            const bool ok = m == 0 || t + m * stride < n;
            const int i = ok ? pw.i : i0, j = ok ? pw.j : j0;
            px[m] = im.off + (ok ? t + m * stride : t);
            c[m] = cp[(size_t)side_div(i, b, lb) * nj + side_div(j, b, lb)];
            uv[m] = u[px[m]];
            pw.next();
        }
#pragma unroll
        for (int m = 0; m < U; ++m) {
            if (t + m * stride >= n) break;
            if (c[m] != 0.0) u[px[m]] = (float)((double)uv[m] + c[m]);
        }
    }
}

// Per-image FP64 energies: grid x = ECH chunks, y = image; then one thread per image adds its chunks in order.
constexpr int ECH = 64;

__global__ __launch_bounds__(256) void batch_energy_partial_kernel(const float* __restrict__ u,
                                                                   const float* __restrict__ f,
                                                                   const BatchImg* __restrict__ imgs,
                                                                   double* __restrict__ partials)
{
    __shared__ double lds[4];
    const int img = blockIdx.y;
    const BatchImg im = imgs[img];
    const size_t n = (size_t)im.H * im.W;
    const float* uu = u + im.off;
    const float* ff = f + im.off;
    double acc = 0.0;
    const size_t p0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    if (p0 < n) {
        // U pixels per round have their loads in flight together and are summed in the order of
        // p; a pixel past n repeats pixel p's window and adds 0.0 (every term is >= 0, so the sum
        // is bitwise the one without it), which keeps the loads out of a branch
        constexpr int U = 2;
        PixelWalk pw(p0, stride, im.W);
        for (size_t p = p0; p < n; p += U * stride) {
            float v[U][3][3], fv[U];
            const int i0 = pw.i, j0 = pw.j;
#pragma unroll
            for (int m = 0; m < U; ++m) {
                const bool ok = m == 0 || p + m * stride < n;
                const int i = ok ? pw.i : i0, j = ok ? pw.j : j0;
                load_window(uu, im.H, im.W, i, j, v[m]);
                fv[m] = ff[(size_t)i * im.W + j];
                pw.next();
            }
#pragma unroll
            for (int m = 0; m < U; ++m) {
                const double d = (double)v[m][1][1] - (double)fv[m];
                const double k = im.kind == 0 ? abs_kappa_window<0>(v[m]) : abs_kappa_window<1>(v[m]);
                const double e = k + 0.5 * im.alpha * d * d;
                acc += (m == 0 || p + m * stride < n) ? e : 0.0;
            }
        }
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[(size_t)img * gridDim.x + blockIdx.x] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

__global__ void batch_energy_final_kernel(const double* __restrict__ partials, int n, int nch, double* __restrict__ out)
{
    const int img = blockIdx.x * blockDim.x + threadIdx.x;
    if (img >= n) return;
    double s = 0.0;
    for (int k = 0; k < nch; ++k) s += partials[(size_t)img * nch + k];
    out[img] = s;
}

// ---------------------------------------------------------------------------
// Group-shape candidates per block level (the autotuner picks one per level).
// ---------------------------------------------------------------------------
struct BlockCfg {
    int group, rpl;
};

static std::vector<BlockCfg> block_candidates(int b)
{
    // the first entry is the single-image path's shape for this block side
    switch (b) {
    case 2: return {{4, -1}, {2, -1}, {2, 8}, {4, 4}, {16, 1}, {8, 2}};   // -1: mirrored form off the border
    case 4: return {{8, 4}, {32, 1}, {16, 2}, {4, 8}};
    case 8: return {{32, 2}, {16, 4}, {64, 1}, {8, 8}};
    case 16: return {{64, 2}, {32, 4}, {16, 8}};
    case 32: return {{256, 1}, {64, 4}, {32, 8}, {128, 2}};
    case 64: return {{256, 2}, {128, 4}, {64, 8}, {512, 1}};
    case 128: return {{256, 4}, {512, 2}};
    case 256: return {{512, 4}, {1024, 2}};
    case 512: return {{512, 8}, {1024, 4}};
    default: return {{1024, 0}};
    }
}

template <int GROUP, int RPL, bool LAZY>
static hipError_t launch_bb(hipStream_t s, int grid, float* u, const float* f, const BatchImg* imgs, const int* order,
                            const int* cum, int n, int total, const int* active, const BatchLevelArgs& a, int M, int G)
{
    if (total == 0) return hipSuccess;
    const int block = GROUP > 64 ? GROUP : 256;  // one workgroup per item above one wavefront
    hipLaunchKernelGGL((batch_blocks_kernel<GROUP, RPL, LAZY>), dim3(grid), dim3(block), 0, s, u, f, imgs, order, cum,
                       n, total, active, a, M, G);
    return hipGetLastError();
}

static hipError_t launch_batch_blocks(hipStream_t s, BlockCfg cfg, int grid, float* u, const float* f,
                                      const BatchImg* imgs, const int* order, const int* cum, int n, int total,
                                      const int* active, const BatchLevelArgs& a, int M, int G)
{
    const bool lazy = level_is_lazy(a.b);
#define MGC_CASE(GR, RP, LZ)                                                                                     \
    if (cfg.group == GR && cfg.rpl == RP && lazy == LZ)                                                          \
        return launch_bb<GR, RP, LZ>(s, grid, u, f, imgs, order, cum, n, total, active, a, M, G);
    MGC_CASE(2, -1, false) MGC_CASE(4, -1, false)
    MGC_CASE(16, 1, false) MGC_CASE(8, 2, false) MGC_CASE(4, 4, false) MGC_CASE(2, 8, false)
    MGC_CASE(32, 1, false) MGC_CASE(16, 2, false) MGC_CASE(8, 4, false) MGC_CASE(4, 8, false)
    MGC_CASE(64, 1, false) MGC_CASE(32, 2, false) MGC_CASE(16, 4, false) MGC_CASE(8, 8, false)
    MGC_CASE(64, 2, false) MGC_CASE(32, 4, false) MGC_CASE(16, 8, false)
    MGC_CASE(64, 4, false) MGC_CASE(32, 8, false) MGC_CASE(128, 2, false) MGC_CASE(256, 1, false)
    MGC_CASE(256, 2, true) MGC_CASE(128, 4, true) MGC_CASE(64, 8, true) MGC_CASE(512, 1, true)
    MGC_CASE(256, 4, true) MGC_CASE(512, 2, true)
    MGC_CASE(512, 4, true) MGC_CASE(1024, 2, true)
    MGC_CASE(512, 8, true) MGC_CASE(1024, 4, true)
    MGC_CASE(1024, 0, true)
#undef MGC_CASE
    return hipErrorInvalidValue;
}

}  // namespace mgc

using mgc::BatchImg;

struct mg_curv_batch {
    int n = 0;
    int M = 16, G = 32;
    int sched = 0;                            // block_schedule, equal across the batch
    int Jmax = 0;
    hipStream_t user_stream = nullptr;
    hipStream_t gstream = nullptr;            // own stream for graph capture and replay
    std::vector<mg_curv_params> P;
    std::vector<BatchImg> h_imgs;
    std::vector<int> h_order;                 // images in curvature-kind order
    std::vector<int> h_active;
    long long total_elems = 0;
    BatchImg* d_imgs = nullptr;
    int* d_order = nullptr;
    int* d_active = nullptr;
    float* pingpong = nullptr;
    // pixel level: cumulative interior-cell and ring-cell counts in kind order
    int* d_cells_cum = nullptr;
    int cells_total = 0;
    int* d_ring_cum = nullptr;
    int ring_total = 0;
    // block levels: [level][colour] cumulative same-colour block counts
    std::vector<int*> d_blk_cum;              // index (level - 2) * 4 + colour
    std::vector<int> blk_total;
    // coarse levels: per-image offsets into the partial sums and pending arrays
    std::vector<long long*> d_part_off, d_pend_off;   // index level - 2
    std::vector<int> nchunk, rows_per;
    double* partials = nullptr;
    double* cpend = nullptr;
    // energies
    double* e_partials = nullptr;
    double* e_dev = nullptr;
    double* e_host = nullptr;                 // pinned, n doubles
    // tuning
    std::vector<mgc::BlockCfg> cfg;           // per level (index level - 2)
    std::vector<int> grid;                    // persistent grid per level (index level - 1)
    // graph of one V-cycle + energies + copy to the host
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::string err;
    std::vector<void*> owned;                 // device allocations to free
};

namespace {

thread_local std::string g_batch_init_error;

mg_status bfail(mg_curv_batch* b, mg_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf; else g_batch_init_error = buf;
    return st;
}

mg_status bhip(mg_curv_batch* b, hipError_t e, const char* what)
{
    return bfail(b, MG_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int side_of(const mg_curv_batch* b, int level) { return mgc::block_side(level, b->sched); }

// log2(bs) for a power of two, -1 otherwise
int lbits(int bs)
{
    int l = 0;
    while ((1 << l) < bs) ++l;
    return (1 << l) == bs ? l : -1;
}

// lane-group shapes of a level: those of the power-of-two side that holds its ring
std::vector<mgc::BlockCfg> candidates_of(const mg_curv_batch* b, int level)
{
    const int bs = side_of(b, level);
    return mgc::block_candidates(bs == 2 ? 2 : mgc::shape_side(bs));
}

int levels_for(int H, int W)
{
    int m = H > W ? H : W, J = 0;
    while ((1 << J) < m) ++J;
    return J < 1 ? 1 : J;
}

template <typename X>
bool dalloc(mg_curv_batch* b, X** p, size_t count)
{
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(X) * (count ? count : 1)) != hipSuccess) return false;
    b->owned.push_back(q);
    *p = (X*)q;
    return true;
}

template <typename X>
bool upload(mg_curv_batch* b, X** p, const std::vector<X>& v)
{
    if (!dalloc(b, p, v.size())) return false;
    return v.empty() || hipMemcpy(*p, v.data(), sizeof(X) * v.size(), hipMemcpyHostToDevice) == hipSuccess;
}

int default_grid(int level)
{
    (void)level;
    return 2048;  // persistent workgroups (8 per CU)
}

mg_status check_ptrs(mg_curv_batch* b, const void* u, const void* f)
{
    if (!b) return MG_E_INVALID;
    if (!u || !f) return bfail(b, MG_E_INVALID, "u and f must be non-null device pointers");
    const size_t n = (size_t)b->total_elems * sizeof(float);
    const char* a = (const char*)u;
    const char* c = (const char*)f;
    if (a < c + n && c < a + n) return bfail(b, MG_E_INVALID, "u must not overlap f");
    return MG_OK;
}

// Enqueue one colour sweep of one level on stream s.
mg_status batch_sweep(mg_curv_batch* b, hipStream_t s, float* u, const float* f, int level, int colour)
{
    hipError_t e;
    if (level == 1) return bfail(b, MG_E_INVALID, "the pixel level runs all colours together");
    const int bs = side_of(b, level);
    const int li = level - 2;
    const int total = b->blk_total[li * 4 + colour];
    mgc::BatchLevelArgs a{bs, lbits(bs), colour >> 1, colour & 1, b->partials, b->d_part_off[li], b->nchunk[li],
                          b->cpend, b->d_pend_off[li]};
    const mgc::BlockCfg cfg = b->cfg[li];
    const int grid = cfg.group > 64 ? std::min(total, 2048) : b->grid[level - 1];
    e = mgc::launch_batch_blocks(s, cfg, grid > 0 ? grid : 1, u, f, b->d_imgs, b->d_order, b->d_blk_cum[li * 4 + colour],
                                 b->n, total, b->d_active, a, b->M, b->G);
    if (e != hipSuccess) return bhip(b, e, "batched block sweep launch");
    return MG_OK;
}

mg_status batch_level_begin(mg_curv_batch* b, hipStream_t s, const float* u, const float* f, int level)
{
    const int bs = side_of(b, level), li = level - 2;
    int maxslots = 1;
    for (int i = 0; i < b->n; ++i) {
        const int mj = (b->h_imgs[i].H + bs - 1) / bs, nj = (b->h_imgs[i].W + bs - 1) / bs;
        maxslots = std::max(maxslots, mj * nj * b->nchunk[li]);
    }
    hipLaunchKernelGGL(mgc::batch_block_sums_kernel, dim3(std::min(maxslots, 1024), b->n), dim3(256), 0, s, u, f,
                       b->d_imgs, b->d_active, bs, lbits(bs), b->nchunk[li], b->rows_per[li], b->partials,
                       b->d_part_off[li]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bhip(b, e, "batched block sums");
    // every image's pending array of this level starts at zero
    size_t npend = 0;
    for (int i = 0; i < b->n; ++i)
        npend += (size_t)((b->h_imgs[i].H + bs - 1) / bs) * ((b->h_imgs[i].W + bs - 1) / bs);
    hipLaunchKernelGGL(mgc::batch_fill_kernel, dim3((unsigned)std::min<size_t>((npend + 255) / 256, 4096)), dim3(256),
                       0, s, b->cpend, npend, 0.0);
    e = hipGetLastError();
    if (e != hipSuccess) return bhip(b, e, "batched pending fill");
    return MG_OK;
}

mg_status batch_level_end(mg_curv_batch* b, hipStream_t s, float* u, int level)
{
    const int bs = side_of(b, level);
    hipLaunchKernelGGL(mgc::batch_apply_kernel, dim3(64, b->n), dim3(256), 0, s, u, b->d_imgs, b->d_active, bs,
                       lbits(bs), b->cpend, b->d_pend_off[level - 2]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bhip(b, e, "batched apply");
    return MG_OK;
}

mg_status batch_level(mg_curv_batch* b, hipStream_t s, float* u, const float* f, int level)
{
    hipError_t e;
    if (level == 1) {
        const float* cur = u;
        float* nxt = b->pingpong;
        for (int colour = 0; colour < 4; ++colour) {
            if (b->ring_total > 0)
                hipLaunchKernelGGL(mgc::batch_ring_cells_kernel, dim3(std::min((b->ring_total * 16 + 255) / 256, 4096)),
                                   dim3(256), 0, s, cur, nxt, f, b->d_imgs, b->d_order, b->d_ring_cum, b->n,
                                   b->ring_total, b->d_active, colour, b->M, b->G);
            if (b->cells_total > 0)
                hipLaunchKernelGGL(mgc::batch_pixels_kernel, dim3(b->grid[0]), dim3(256), 0, s, cur, nxt, f, b->d_imgs,
                                   b->d_order, b->d_cells_cum, b->n, b->cells_total, b->d_active, colour, b->M, b->G);
            e = hipGetLastError();
            if (e != hipSuccess) return bhip(b, e, "batched pixel sweep");
            float* t = (float*)cur;
            cur = nxt;
            nxt = t;
        }
        return MG_OK;
    }
    const bool lazy = mgc::level_is_lazy(side_of(b, level));
    mg_status st;
    if (lazy && (st = batch_level_begin(b, s, u, f, level)) != MG_OK) return st;
    for (int colour = 0; colour < 4; ++colour)
        if ((st = batch_sweep(b, s, u, f, level, colour)) != MG_OK) return st;
    if (lazy && (st = batch_level_end(b, s, u, level)) != MG_OK) return st;
    return MG_OK;
}

mg_status batch_vcycle_enqueue(mg_curv_batch* b, hipStream_t s, float* u, const float* f)
{
    for (int level = 1; level <= b->Jmax; ++level) {
        mg_status st = batch_level(b, s, u, f, level);
        if (st != MG_OK) return st;
    }
    return MG_OK;
}

mg_status batch_energy_enqueue(mg_curv_batch* b, hipStream_t s, const float* u, const float* f)
{
    hipLaunchKernelGGL(mgc::batch_energy_partial_kernel, dim3(mgc::ECH, b->n), dim3(256), 0, s, u, f, b->d_imgs,
                       b->e_partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bhip(b, e, "batched energy");
    hipLaunchKernelGGL(mgc::batch_energy_final_kernel, dim3((b->n + 63) / 64), dim3(64), 0, s, b->e_partials, b->n,
                       mgc::ECH, b->e_dev);
    e = hipGetLastError();
    if (e != hipSuccess) return bhip(b, e, "batched energy final");
    e = hipMemcpyAsync(b->e_host, b->e_dev, sizeof(double) * b->n, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return bhip(b, e, "energy copy");
    return MG_OK;
}

void drop_graph(mg_curv_batch* b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
}

mg_status set_all_active(mg_curv_batch* b, hipStream_t s, int v)
{
    std::fill(b->h_active.begin(), b->h_active.end(), v);
    hipError_t e = hipMemcpyAsync(b->d_active, b->h_active.data(), sizeof(int) * b->n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return bhip(b, e, "active flags");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bhip(b, e, "active flags sync");
    return MG_OK;
}

}  // namespace

extern "C" {

mg_status mg_curv_batch_init(const mg_curv_params* params, int32_t n, void* hip_stream, mg_curv_batch** out)
{
    if (!params || !out || n < 1) return bfail(nullptr, MG_E_INVALID, "params, out must be non-null and n >= 1");
    *out = nullptr;
    const mg_curv_params& p0 = params[0];
    for (int i = 0; i < n; ++i) {
        const mg_curv_params& p = params[i];
        if (p.height < 2 || p.width < 2) return bfail(nullptr, MG_E_SHAPE, "image %d: height and width must be >= 2", i);
        if (!(p.alpha > 0.0) || !std::isfinite(p.alpha)) return bfail(nullptr, MG_E_INVALID, "image %d: alpha must be finite and > 0", i);
        if (p.curvature != MG_CURV_MEAN && p.curvature != MG_CURV_GAUSS) return bfail(nullptr, MG_E_INVALID, "image %d: bad curvature", i);
        if (p.state_dtype != MG_F32) return bfail(nullptr, MG_E_DTYPE, "batched images use float32 state");
        if (p.fine_colours != 4) return bfail(nullptr, MG_E_INVALID, "batched images use four fine colours");
        if (p.cycle != 0) return bfail(nullptr, MG_E_INVALID, "batched images use the half V-cycle");
        if (p.block_schedule != 0 && p.block_schedule != 1)
            return bfail(nullptr, MG_E_INVALID, "image %d: block_schedule must be 0 or 1", i);
        if (p.block_schedule != p0.block_schedule)
            return bfail(nullptr, MG_E_INVALID, "block_schedule must be equal across the batch");
        if (p.samples != p0.samples || p.bisections != p0.bisections)
            return bfail(nullptr, MG_E_INVALID, "samples and bisections must be equal across the batch");
        if (p.samples < 2 || p.samples > 256 || (p.samples & 1)) return bfail(nullptr, MG_E_INVALID, "samples must be even and in [2, 256]");
        if (p.bisections < 0 || p.bisections > 64) return bfail(nullptr, MG_E_INVALID, "bisections must be in [0, 64]");
        const int Ja = levels_for(p.height, p.width);
        if (p.levels < 0 || p.levels > Ja + 1) return bfail(nullptr, MG_E_INVALID, "image %d: levels out of range", i);
        const int Ji = p.levels > 0 ? p.levels : Ja;
        if (Ji > 27 || mgc::block_side(Ji, p.block_schedule) > (1 << 26))
            return bfail(nullptr, MG_E_INVALID, "image %d: the block side at level %d exceeds 2^26 pixels", i, Ji);
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return bfail(nullptr, MG_E_DEVICE, "no HIP device available");
    mg_curv_batch* b = new (std::nothrow) mg_curv_batch();
    if (!b) return bfail(nullptr, MG_E_NOMEM, "host allocation failed");
    b->n = n;
    b->M = p0.samples;
    b->G = p0.bisections;
    b->sched = p0.block_schedule;
    b->user_stream = (hipStream_t)hip_stream;
    b->P.assign(params, params + n);
    long long off = 0;
    for (int i = 0; i < n; ++i) {
        const mg_curv_params& p = params[i];
        BatchImg im;
        im.off = off;
        im.H = p.height;
        im.W = p.width;
        im.alpha = p.alpha;
        im.kind = p.curvature;
        im.J = p.levels > 0 ? p.levels : levels_for(p.height, p.width);
        b->Jmax = std::max(b->Jmax, im.J);
        b->h_imgs.push_back(im);
        off += (long long)p.height * p.width;
    }
    b->total_elems = off;
    for (int kind = 0; kind < 2; ++kind)
        for (int i = 0; i < n; ++i)
            if (b->h_imgs[i].kind == kind) b->h_order.push_back(i);
    b->h_active.assign(n, 1);

    bool ok = hipStreamCreate(&b->gstream) == hipSuccess;
    ok = ok && upload(b, &b->d_imgs, b->h_imgs) && upload(b, &b->d_order, b->h_order) && upload(b, &b->d_active, b->h_active);
    ok = ok && dalloc(b, &b->pingpong, (size_t)b->total_elems);
    // pixel level
    std::vector<int> cum(1, 0), rcum(1, 0);
    for (int k = 0; k < n; ++k) {
        const BatchImg& im = b->h_imgs[b->h_order[k]];
        const int cr = (im.H + 1) / 2, cc = (im.W + 1) / 2;
        const int inner = (cr > 2 && cc > 2) ? (cr - 2) * (cc - 2) : 0;
        cum.push_back(cum.back() + inner);
        rcum.push_back(rcum.back() + mgc::ring_cell_count(cr, cc));
    }
    b->cells_total = cum.back();
    b->ring_total = rcum.back();
    ok = ok && upload(b, &b->d_cells_cum, cum) && upload(b, &b->d_ring_cum, rcum);
    // block levels
    size_t max_part = 1, max_pend = 1;
    for (int level = 2; level <= b->Jmax; ++level) {
        const int bs = side_of(b, level);
        for (int colour = 0; colour < 4; ++colour) {
            std::vector<int> c(1, 0);
            for (int k = 0; k < n; ++k) {
                const BatchImg& im = b->h_imgs[b->h_order[k]];
                int cnt = 0;
                if (level <= im.J) {
                    const int mj = (im.H + bs - 1) / bs, nj = (im.W + bs - 1) / bs;
                    cnt = ((mj - (colour >> 1) + 1) / 2) * ((nj - (colour & 1) + 1) / 2);
                }
                c.push_back(c.back() + cnt);
            }
            int* d = nullptr;
            ok = ok && upload(b, &d, c);
            b->d_blk_cum.push_back(d);
            b->blk_total.push_back(c.back());
        }
        int nblk, nch, rp;
        mgc::coarse_geometry(2, 2, bs, &nblk, &nch, &rp);
        b->nchunk.push_back(nch);
        b->rows_per.push_back(rp);
        std::vector<long long> po(n), pe(n);
        size_t tp = 0, te = 0;
        for (int i = 0; i < n; ++i) {
            const BatchImg& im = b->h_imgs[i];
            const size_t nb = (size_t)((im.H + bs - 1) / bs) * ((im.W + bs - 1) / bs);
            po[i] = (long long)tp;
            pe[i] = (long long)te;
            tp += nb * nch;
            te += nb;
        }
        max_part = std::max(max_part, tp);
        max_pend = std::max(max_pend, te);
        long long *dpo = nullptr, *dpe = nullptr;
        ok = ok && upload(b, &dpo, po) && upload(b, &dpe, pe);
        b->d_part_off.push_back(dpo);
        b->d_pend_off.push_back(dpe);
        b->cfg.push_back(candidates_of(b, level)[0]);
    }
    for (int level = 1; level <= b->Jmax; ++level) b->grid.push_back(default_grid(level));
    ok = ok && dalloc(b, &b->partials, max_part) && dalloc(b, &b->cpend, max_pend);
    ok = ok && dalloc(b, &b->e_partials, (size_t)n * mgc::ECH) && dalloc(b, &b->e_dev, (size_t)n);
    ok = ok && hipHostMalloc((void**)&b->e_host, sizeof(double) * n, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        mg_curv_batch_destroy(b);
        (void)hipGetLastError();
        return bfail(nullptr, MG_E_NOMEM, "device allocation failed for a batch of %lld pixels", off);
    }
    *out = b;
    return MG_OK;
}

int64_t mg_curv_batch_offset(const mg_curv_batch* b, int32_t i)
{
    if (!b || i < 0 || i > b->n) return -1;
    return i == b->n ? b->total_elems : b->h_imgs[i].off;
}

mg_status mg_curv_batch_vcycle(mg_curv_batch* b, void* u, const void* f, double* energies)
{
    mg_status st = check_ptrs(b, u, f);
    if (st != MG_OK) return st;
    st = batch_vcycle_enqueue(b, b->user_stream, (float*)u, (const float*)f);
    if (st != MG_OK || !energies) return st;
    st = batch_energy_enqueue(b, b->user_stream, (const float*)u, (const float*)f);
    if (st != MG_OK) return st;
    hipError_t e = hipStreamSynchronize(b->user_stream);
    if (e != hipSuccess) return bhip(b, e, "stream synchronize");
    std::memcpy(energies, b->e_host, sizeof(double) * b->n);
    return MG_OK;
}

mg_status mg_curv_batch_sweep(mg_curv_batch* b, void* u, const void* f, int32_t level, int32_t colour)
{
    mg_status st = check_ptrs(b, u, f);
    if (st != MG_OK) return st;
    if (level < 2 || level > b->Jmax) return bfail(b, MG_E_INVALID, "level must be in [2, %d] (use mg_curv_batch_level for 1)", b->Jmax);
    if (colour < 0 || colour > 3) return bfail(b, MG_E_INVALID, "colour must be in [0, 4)");
    const bool lazy = mgc::level_is_lazy(side_of(b, level));
    if (lazy && (st = batch_level_begin(b, b->user_stream, (const float*)u, (const float*)f, level)) != MG_OK) return st;
    if ((st = batch_sweep(b, b->user_stream, (float*)u, (const float*)f, level, colour)) != MG_OK) return st;
    if (lazy && (st = batch_level_end(b, b->user_stream, (float*)u, level)) != MG_OK) return st;
    return MG_OK;
}

mg_status mg_curv_batch_level(mg_curv_batch* b, void* u, const void* f, int32_t level)
{
    mg_status st = check_ptrs(b, u, f);
    if (st != MG_OK) return st;
    if (level < 1 || level > b->Jmax) return bfail(b, MG_E_INVALID, "level must be in [1, %d]", b->Jmax);
    return batch_level(b, b->user_stream, (float*)u, (const float*)f, level);
}

mg_status mg_curv_batch_energy(mg_curv_batch* b, const void* u, const void* f, double* energies)
{
    mg_status st = check_ptrs(b, u, f);
    if (st != MG_OK) return st;
    if (!energies) return bfail(b, MG_E_INVALID, "energies must be non-null");
    st = batch_energy_enqueue(b, b->user_stream, (const float*)u, (const float*)f);
    if (st != MG_OK) return st;
    hipError_t e = hipStreamSynchronize(b->user_stream);
    if (e != hipSuccess) return bhip(b, e, "stream synchronize");
    std::memcpy(energies, b->e_host, sizeof(double) * b->n);
    return MG_OK;
}

namespace {

// Shared driver: stop image i when its relative energy change is below rel_tol (rel_tol > 0) or,
// with targets, when its energy is at or below target[i] (checked before the first V-cycle too).
mg_status batch_solve_impl(mg_curv_batch* b, void* u, const void* f, double rel_tol, const double* target,
                           int32_t max_vcycles, int32_t* vcycles_done, double* final_energy, int32_t* status)
{
    mg_status st = check_ptrs(b, u, f);
    if (st != MG_OK) return st;
    if (max_vcycles < 0 || !std::isfinite(rel_tol)) return bfail(b, MG_E_INVALID, "bad rel_tol or max_vcycles");
    hipError_t e = hipStreamSynchronize(b->user_stream);
    if (e != hipSuccess) return bhip(b, e, "user stream synchronize");
    hipStream_t s = b->gstream;
    if ((st = set_all_active(b, s, 1)) != MG_OK) return st;
    if ((st = batch_energy_enqueue(b, s, (const float*)u, (const float*)f)) != MG_OK) return st;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return bhip(b, e, "stream synchronize");
    std::vector<double> prev(b->e_host, b->e_host + b->n), cur(b->n);
    std::vector<int> done(b->n, 0), conv(b->n, 0);
    int remaining = b->n;
    for (int i = 0; i < b->n; ++i) {
        if (!std::isfinite(prev[i])) return bfail(b, MG_E_NONFINITE, "energy of image %d is not finite", i);
        if (target && prev[i] <= target[i]) {
            conv[i] = 1;
            b->h_active[i] = 0;
            --remaining;
        }
    }
    if (remaining < b->n) {
        e = hipMemcpyAsync(b->d_active, b->h_active.data(), sizeof(int) * b->n, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return bhip(b, e, "active flags");
    }
    // capture one V-cycle + energies + host copy for these buffers
    drop_graph(b);
    if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal)) != hipSuccess) return bhip(b, e, "begin capture");
    st = batch_vcycle_enqueue(b, s, (float*)u, (const float*)f);
    if (st == MG_OK) st = batch_energy_enqueue(b, s, (const float*)u, (const float*)f);
    e = hipStreamEndCapture(s, &b->graph);
    if (st != MG_OK) { drop_graph(b); return st; }
    if (e != hipSuccess) return bhip(b, e, "end capture");
    if ((e = hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0)) != hipSuccess) return bhip(b, e, "graph instantiate");
    for (int l = 0; l < max_vcycles && remaining > 0; ++l) {
        if ((e = hipGraphLaunch(b->gexec, s)) != hipSuccess) return bhip(b, e, "graph launch");
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return bhip(b, e, "graph synchronize");
        bool changed = false;
        for (int i = 0; i < b->n; ++i) {
            if (!b->h_active[i]) continue;
            cur[i] = b->e_host[i];
            done[i] += 1;
            if (!std::isfinite(cur[i])) return bfail(b, MG_E_NONFINITE, "energy of image %d became non-finite", i);
            const bool stop = target ? cur[i] <= target[i]
                                     : (rel_tol > 0.0 && (cur[i] == prev[i] || std::fabs(cur[i] - prev[i]) < rel_tol * std::fabs(cur[i])));
            if (stop) {
                conv[i] = 1;
                b->h_active[i] = 0;
                --remaining;
                changed = true;
            }
            prev[i] = cur[i];
        }
        if (changed) {
            e = hipMemcpyAsync(b->d_active, b->h_active.data(), sizeof(int) * b->n, hipMemcpyHostToDevice, s);
            if (e != hipSuccess) return bhip(b, e, "active flags");
        }
    }
    if ((st = set_all_active(b, s, 1)) != MG_OK) return st;
    bool all_conv = true;
    const bool has_criterion = target != nullptr || rel_tol > 0.0;
    for (int i = 0; i < b->n; ++i) {
        if (vcycles_done) vcycles_done[i] = done[i];
        if (final_energy) final_energy[i] = prev[i];
        const int si = (has_criterion && !conv[i]) ? MG_NOT_CONVERGED : MG_OK;
        if (status) status[i] = si;
        all_conv = all_conv && si == MG_OK;
    }
    return all_conv ? MG_OK : MG_NOT_CONVERGED;
}

}  // namespace

mg_status mg_curv_batch_solve(mg_curv_batch* b, void* u, const void* f, double rel_tol, int32_t max_vcycles,
                              int32_t* vcycles_done, double* final_energy, int32_t* status)
{
    return batch_solve_impl(b, u, f, rel_tol, nullptr, max_vcycles, vcycles_done, final_energy, status);
}

mg_status mg_curv_batch_solve_target(mg_curv_batch* b, void* u, const void* f, const double* target_energy,
                                     int32_t max_vcycles, int32_t* vcycles_done, double* final_energy, int32_t* status)
{
    if (b && !target_energy) return bfail(b, MG_E_INVALID, "target_energy must be non-null");
    return batch_solve_impl(b, u, f, 0.0, target_energy, max_vcycles, vcycles_done, final_energy, status);
}

mg_status mg_curv_batch_tune(mg_curv_batch* b, void* u, const void* f, int32_t repeats)
{
    mg_status st = check_ptrs(b, u, f);
    if (st != MG_OK) return st;
    if (repeats < 1) repeats = 1;
    hipStream_t s = b->user_stream;
    hipError_t e;
    float* scratch = nullptr;
    if ((e = hipMalloc((void**)&scratch, sizeof(float) * b->total_elems)) != hipSuccess) return bhip(b, e, "tune scratch");
    hipEvent_t t0, t1;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    auto timeit = [&](auto&& fn) -> float {
        float best = 1e30f;
        for (int r = 0; r < repeats; ++r) {
            (void)hipMemcpyAsync(scratch, u, sizeof(float) * b->total_elems, hipMemcpyDeviceToDevice, s);
            (void)hipEventRecord(t0, s);
            fn();
            (void)hipEventRecord(t1, s);
            (void)hipEventSynchronize(t1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, t0, t1);
            best = std::min(best, ms);
        }
        return best;
    };
    const int grids[3] = {1024, 2048, 4096};
    // pixel level: persistent grid size
    {
        float best = 1e30f;
        int pick = b->grid[0];
        for (int g : grids) {
            b->grid[0] = g;
            const float ms = timeit([&] { (void)batch_level(b, s, scratch, (const float*)f, 1); });
            if (ms < best) { best = ms; pick = g; }
        }
        b->grid[0] = pick;
    }
    for (int level = 2; level <= b->Jmax; ++level) {
        const int li = level - 2;
        float best = 1e30f;
        mgc::BlockCfg pick = b->cfg[li];
        int gpick = b->grid[level - 1];
        for (const mgc::BlockCfg& c : candidates_of(b, level)) {
            for (int g : grids) {
                if (c.group > 64 && g != grids[0]) continue;  // one workgroup per item: grid is fixed
                b->cfg[li] = c;
                b->grid[level - 1] = g;
                const float ms = timeit([&] { (void)batch_level(b, s, scratch, (const float*)f, level); });
                if (ms < best) { best = ms; pick = c; gpick = g; }
            }
        }
        b->cfg[li] = pick;
        b->grid[level - 1] = gpick;
    }
    e = hipStreamSynchronize(s);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    (void)hipFree(scratch);
    drop_graph(b);
    if (e != hipSuccess) return bhip(b, e, "tune synchronize");
    return MG_OK;
}

int32_t mg_curv_batch_config(const mg_curv_batch* b, int32_t level, int32_t* group, int32_t* records, int32_t* grid)
{
    if (!b || level < 1 || level > b->Jmax) return -1;
    if (level == 1) {
        if (group) *group = 1;
        if (records) *records = 9;
    } else {
        if (group) *group = b->cfg[level - 2].group;
        if (records) *records = b->cfg[level - 2].rpl;
    }
    if (grid) *grid = b->grid[level - 1];
    return 0;
}

mg_status mg_curv_batch_set_config(mg_curv_batch* b, int32_t level, int32_t group, int32_t records, int32_t grid)
{
    if (!b || level < 1 || level > b->Jmax) return MG_E_INVALID;
    if (grid < 1 || grid > 65536) return bfail(b, MG_E_INVALID, "grid must be in [1, 65536]");
    if (level >= 2) {
        bool found = false;
        for (const mgc::BlockCfg& c : candidates_of(b, level))
            if (c.group == group && c.rpl == records) found = true;
        if (!found) return bfail(b, MG_E_INVALID, "no compiled lane-group shape (%d, %d) for level %d", group, records, level);
        b->cfg[level - 2] = mgc::BlockCfg{group, records};
    }
    b->grid[level - 1] = grid;
    drop_graph(b);
    return MG_OK;
}

int32_t mg_curv_batch_levels(const mg_curv_batch* b) { return b ? b->Jmax : 0; }

void mg_curv_batch_destroy(mg_curv_batch* b)
{
    if (!b) return;
    if (b->user_stream) (void)hipStreamSynchronize(b->user_stream);
    if (b->gstream) (void)hipStreamSynchronize(b->gstream);
    drop_graph(b);
    for (void* p : b->owned) (void)hipFree(p);
    if (b->e_host) (void)hipHostFree(b->e_host);
    if (b->gstream) (void)hipStreamDestroy(b->gstream);
    delete b;
}

const char* mg_curv_batch_last_error(const mg_curv_batch* b)
{
    if (b) return b->err.c_str();
    return g_batch_init_error.c_str();
}

}  // extern "C"
