// Colour-sweep and energy kernels for the multigrid curvature minimisation
// (Algorithm 3 of arXiv 2204.07921) on gfx950.
//
// Level j has block side b = 2^(j-1) (nested blocks) or, with the paper's
// schedule, 2^j - 1 (Section 2.2).  A colour sweep updates every block of
// one colour; blocks of one colour at b >= 2 never share a ring pixel, so they
// run in parallel and update u in place.  At b = 1 same-colour pixels of the
// four-colour map do share ring pixels, so the pixel level is two-phase: every
// c is computed from the input state and written to a second image
// (ping-pong), which makes the result independent of the schedule.
//
// The per-block work (sum of f - u, ring records, 1-D minimisation, apply)
// runs on a lane group: 1 lane per pixel at b = 1, 16..64 lanes of one
// wavefront for b <= 32, a whole workgroup (256 or 1024 lanes) for b >= 64.
#include "mgc_internal.h"
#include "mgc_sweep.h"

namespace mgc {

// ---------------------------------------------------------------------------
// Pixel level (b = 1), two-phase.  One thread per cell of the colour pattern
// (2x2 cells for four colours, 3x3 for nine); the thread solves the cell's
// pixel of the active colour and copies the cell's other pixels.
// ---------------------------------------------------------------------------
// One launch per colour.  The first `ring_blocks` workgroups take the outer
// ring of cells (first and last cell row and column) with a 16-lane group per
// cell (general form: the pixel may sit on the image border); they come first
// so their longer per-cell solves overlap the rest of the grid, which takes the
// interior cells one thread each (constant-slope form).
template <typename T, int KIND, int NC>
__global__ __launch_bounds__(256) void sweep_pixels_kernel(const T* __restrict__ uin, T* __restrict__ uout,
                                                           const T* __restrict__ f, int H, int W, int colour,
                                                           int cells_r, int cells_c, int ring_blocks, double alpha,
                                                           int M, int G)
{
    if ((int)blockIdx.x < ring_blocks) {
        const int k = (blockIdx.x * blockDim.x + threadIdx.x) >> 4;
        const int lane = threadIdx.x & 15;
        int cr, cc;
        if (!ring_cell(k, cells_r, cells_c, cr, cc)) return;   // whole groups exit together
        solve_ring_cell<T, KIND, NC>(uin, uout, f, H, W, colour, cr, cc, lane, alpha, M, G);
        return;
    }
    // interior workgroups: the dispatcher hands workgroups to the 8 XCDs round-robin (workgroup b
    // of the interior to XCD b % 8, ring_blocks being a multiple of 8); each XCD takes one
    // contiguous run of cell rows, so neighbouring cells share their halo rows in one XCD's L2
    // instead of every XCD fetching them
    const int ir = cells_r - 2, ic = cells_c - 2;
    const int nb_in = (int)gridDim.x - ring_blocks, b = (int)blockIdx.x - ring_blocks;
    const int x = b & 7, q = nb_in >> 3, r = nb_in & 7;
    const int run = x * q + min(x, r) + (b >> 3);
    const int cell = run * blockDim.x + threadIdx.x;
    if (ir <= 0 || ic <= 0 || cell >= ir * ic) return;
    const int cr = 1 + cell / ic, cc = 1 + cell % ic;
    solve_cell<T, KIND, NC, 1>(uin, uout, f, H, W, colour, cr, cc, alpha, M, G);
}

template <typename T, int KIND, int GROUP, int RPL, bool LAZY>
__global__ __launch_bounds__(GROUP > 64 ? GROUP : 256) void sweep_blocks_kernel(
    T* __restrict__ u, const T* __restrict__ f, int H, int W, int b, int pr, int pc, int nbr, int nbc,
    double alpha, int M, int G, CoarseArgs ca)
{
    if constexpr (GROUP <= 64) {
        const int gid = (blockIdx.x * blockDim.x + threadIdx.x) / GROUP;
        const int lane = threadIdx.x & (GROUP - 1);
        if (gid >= nbr * nbc) return;  // whole groups exit together
        const int bi = gid / nbc, bj = gid - bi * nbc;
        const int p = 2 * bi + pr, q = 2 * bj + pc;
        const int r0 = p * b, c0 = q * b;
        const int r1 = min(r0 + b, H), c1 = min(c0 + b, W);
        solve_block<T, KIND, GROUP, RPL, LAZY>(u, f, H, W, p, q, r0, r1, c0, c1, lane, alpha, M, G,
                                               WaveSum<GROUP>(), ca);
    } else {
        __shared__ double lds[2 * (GROUP / 64) * BlockSum<GROUP>::NMAX];
        const int gid = blockIdx.x;
        const int bi = gid / nbc, bj = gid - bi * nbc;
        const int p = 2 * bi + pr, q = 2 * bj + pc;
        const int r0 = p * b, c0 = q * b;
        const int r1 = min(r0 + b, H), c1 = min(c0 + b, W);
        BlockSum<GROUP> gs{lds, 0};
        CoarseArgs cb = ca;
        if (cb.rec) cb.rec += (size_t)gid * PolyRing<KIND>::NCOEF * cb.rec_stride;   // this block's region
        solve_block<T, KIND, GROUP, RPL, LAZY>(u, f, H, W, p, q, r0, r1, c0, c1, threadIdx.x, alpha, M, G, gs, cb);
    }
}

// b = 2 (nested schedule): QL lanes per block; blocks off the image border take the
// mirrored constant-slope form, the border blocks (numbered first) the general records.
template <typename T, int KIND, int QL>
__global__ __launch_bounds__(256) void sweep_b2_kernel(T* __restrict__ u, const T* __restrict__ f, int H, int W,
                                                       int pr, int pc, Split2 S, double alpha, int M, int G)
{
    const int k = (blockIdx.x * blockDim.x + threadIdx.x) / QL;
    if (k >= S.nbr * S.nbc) return;   // all lanes of a group exit together
    solve_b2_item<T, KIND, QL>(u, f, H, W, pr, pc, S, k, threadIdx.x & (QL - 1), alpha, M, G);
}

// Coarse levels: partial sums of f - u, one workgroup per (block, chunk of rows).
// partials[(p * nj + q) * nchunk + k] = sum over rows [r0 + k rows_per, ...) of
// block (p, q); the first chunk of each block also zeroes its pending correction.
// With cprev set, the previous coarse level's pending corrections (block side bp,
// njp blocks per row; lbp = log2(bp), or -1 when bp is not a power of two) are
// first added to u, rounded to the state type as the correction pass would store them.
template <typename T>
__global__ __launch_bounds__(256) void block_sums_kernel(T* __restrict__ u, const T* __restrict__ f, int H,
                                                         int W, int b, int nj, int nchunk, int rows_per,
                                                         double* __restrict__ partials, double* __restrict__ cpend,
                                                         const double* __restrict__ cprev, int bp, int lbp, int njp)
{
    __shared__ double lds[4];
    const int blk = blockIdx.x / nchunk, k = blockIdx.x - blk * nchunk;
    const int p = blk / nj, q = blk - p * nj;
    if (k == 0 && threadIdx.x == 0) cpend[blk] = 0.0;
    const int c0 = q * b, c1 = min(c0 + b, W), w = c1 - c0;
    const int ra = p * b + k * rows_per;
    const int rb = min(min(ra + rows_per, (p + 1) * b), H);
    double acc = 0.0;
    const int n = (rb > ra ? rb - ra : 0) * w;
    // element t = threadIdx.x + m blockDim.x of the chunk is pixel (ra + t / w, c0 + t % w);
    // its row and column advance by the step's quotient and remainder
    // U elements per round have their loads in flight together (one at a time, each waited on
    // its memory round trip); they are then applied and summed in the order of t.  Elements past
    // the chunk's end take the first element's address and are skipped.
    constexpr int U = 8;
    const int B = (int)blockDim.x;
    const int si = B / w, sj = B - si * w;
    int i = ra + (int)threadIdx.x / w, j = c0 + (int)threadIdx.x % w;
    for (int t0 = threadIdx.x; t0 < n; t0 += U * B) {
        int pi[U], pj[U];
#pragma unroll
        for (int m = 0; m < U; ++m) {
            const bool ok = m == 0 || t0 + m * B < n;   // element 0 is in the chunk (t0 < n)
            pi[m] = ok ? i : pi[0];
            pj[m] = ok ? j : pj[0];
            i += si;
            j += sj;
            if (j >= c1) { j -= w; ++i; }
        }
        double uv[U], fv[U], cv[U];
#pragma unroll
        for (int m = 0; m < U; ++m) {
            const size_t idx = (size_t)pi[m] * W + pj[m];
            uv[m] = (double)u[idx];
            fv[m] = (double)f[idx];
            cv[m] = cprev ? cprev[(size_t)side_div(pi[m], bp, lbp) * njp + side_div(pj[m], bp, lbp)] : 0.0;
        }
#pragma unroll
        for (int m = 0; m < U; ++m) {
            if (t0 + m * B >= n) break;
            double v = uv[m];
            if (cv[m] != 0.0) {
                const T r = (T)(v + cv[m]);
                u[(size_t)pi[m] * W + pj[m]] = r;
                v = (double)r;
            }
            acc += fv[m] - v;
        }
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

// End of a coarse level: u <- u + c of the pixel's block (rounded to the state type).
template <typename T>
__global__ __launch_bounds__(256) void apply_level_kernel(T* __restrict__ u, int H, int W, int b, int lb, int nj,
                                                          const double* __restrict__ cpend)
{
    const size_t n = (size_t)H * W;
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    if (t0 >= n) return;
    // U pixels per round have their loads in flight together (past n: pixel t0's address, skipped)
    constexpr int U = 4;
    PixelWalk pw(t0, stride, W);
    for (size_t t = t0; t < n; t += U * stride) {
        size_t px[U];
        double c[U];
        T uv[U];
        const int i0 = pw.i, j0 = pw.j;
#pragma unroll
        for (int m = 0; m < U; ++m) {
            const bool ok = m == 0 || t + m * stride < n;
            const int i = ok ? pw.i : i0, j = ok ? pw.j : j0;
            px[m] = ok ? t + m * stride : t;
            c[m] = cpend[(size_t)side_div(i, b, lb) * nj + side_div(j, b, lb)];
            uv[m] = u[px[m]];
            pw.next();
        }
#pragma unroll
        for (int m = 0; m < U; ++m) {
            if (t + m * stride >= n) break;
            if (c[m] != 0.0) u[px[m]] = (T)((double)uv[m] + c[m]);
        }
    }
}

// ---------------------------------------------------------------------------
// Energy F(u) = sum |kappa| + alpha/2 (u - f)^2 in FP64: fixed-size grid of
// partial sums, then one workgroup adds the partials in a fixed order.
// ---------------------------------------------------------------------------
template <typename T, int KIND>
__global__ __launch_bounds__(256) void energy_partial_kernel(const T* __restrict__ u, const T* __restrict__ f,
                                                             int H, int W, double alpha, double* __restrict__ partials)
{
    __shared__ double lds[4];
    const size_t n = (size_t)H * W;
    double acc = 0.0;
    const size_t p0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    if (p0 < n) {
        // U pixels per round have their loads in flight together and are summed in the order of
        // p; a pixel past n repeats pixel p's window and adds 0.0 (every term is >= 0, so the sum
        // is bitwise the one without it), which keeps the loads out of a branch
        constexpr int U = 2;
        PixelWalk pw(p0, stride, W);
        for (size_t p = p0; p < n; p += U * stride) {
            T v[U][3][3], fv[U];
            const int i0 = pw.i, j0 = pw.j;
#pragma unroll
            for (int m = 0; m < U; ++m) {
                const bool ok = m == 0 || p + m * stride < n;
                const int i = ok ? pw.i : i0, j = ok ? pw.j : j0;
                load_window(u, H, W, i, j, v[m]);
                fv[m] = f[(size_t)i * W + j];
                pw.next();
            }
#pragma unroll
            for (int m = 0; m < U; ++m) {
                const double d = (double)v[m][1][1] - (double)fv[m];
                const double e = abs_kappa_window<KIND>(v[m]) + 0.5 * alpha * d * d;
                acc += (m == 0 || p + m * stride < n) ? e : 0.0;
            }
        }
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

// Partial sums of (u - prev)^2 (partials[0 .. gridDim)) and u^2 (partials[gridDim ..)).
template <typename T>
__global__ __launch_bounds__(256) void diff_norms_kernel(const T* __restrict__ u, const T* __restrict__ prev,
                                                         size_t n, double* __restrict__ partials)
{
    __shared__ double lds[8];
    double a = 0.0, b = 0.0;
    // U elements per round have their loads in flight together and are summed in the order of p;
    // an element past n repeats element p and adds 0.0 (the terms are squares, so the sums are
    // bitwise the ones without it), which keeps the loads out of a branch
    constexpr int U = 4;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += U * stride) {
        T uv[U], pv[U];
#pragma unroll
        for (int m = 0; m < U; ++m) {
            const size_t q = (m == 0 || p + m * stride < n) ? p + m * stride : p;
            uv[m] = u[q];
            pv[m] = prev[q];
        }
#pragma unroll
        for (int m = 0; m < U; ++m) {
            const bool ok = m == 0 || p + m * stride < n;
            const double x = (double)uv[m], d = x - (double)pv[m];
            a += ok ? d * d : 0.0;
            b += ok ? x * x : 0.0;
        }
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
        partials[blockIdx.x] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
        partials[gridDim.x + blockIdx.x] = (lds[4] + lds[5]) + (lds[6] + lds[7]);
    }
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ partials, int n,
                                                           double* __restrict__ out)
{
    __shared__ double lds[4];
    double acc = 0.0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) acc += partials[k];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <typename T, int KIND, int NC>
static hipError_t launch_pixels_nc(const LaunchCtx& L, const void* uin, void* uout, const void* f, int colour)
{
    const int cells_r = (L.H + NC - 1) / NC, cells_c = (L.W + NC - 1) / NC;
    const int n_in = (cells_r > 2 && cells_c > 2) ? (cells_r - 2) * (cells_c - 2) : 0;
    const int rb = ((ring_cell_count(cells_r, cells_c) * 16 + 255) / 256 + 7) & ~7;   // a multiple of 8
    hipLaunchKernelGGL((sweep_pixels_kernel<T, KIND, NC>), dim3(rb + (n_in + 255) / 256), dim3(256), 0, L.stream,
                       (const T*)uin, (T*)uout, (const T*)f, L.H, L.W, colour, cells_r, cells_c, rb, L.alpha, L.M, L.G);
    return hipGetLastError();
}

template <typename T, int KIND>
static hipError_t launch_pixels_t(const LaunchCtx& L, const void* uin, void* uout, const void* f, int colour, int nc)
{
    return nc == 3 ? launch_pixels_nc<T, KIND, 3>(L, uin, uout, f, colour)
                   : launch_pixels_nc<T, KIND, 2>(L, uin, uout, f, colour);
}

hipError_t launch_sweep_pixels(const LaunchCtx& L, const void* uin, void* uout, const void* f, int colour, int ncolours)
{
    // nine colours use 3x3 cells, four colours 2x2 cells
    const int nc = (ncolours == 9) ? 3 : 2;
    if (L.f64) return L.kind ? launch_pixels_t<double, 1>(L, uin, uout, f, colour, nc)
                             : launch_pixels_t<double, 0>(L, uin, uout, f, colour, nc);
    return L.kind ? launch_pixels_t<float, 1>(L, uin, uout, f, colour, nc)
                  : launch_pixels_t<float, 0>(L, uin, uout, f, colour, nc);
}

template <typename T, int KIND, int GROUP, int RPL, bool LAZY>
static hipError_t launch_blocks_cfg(const LaunchCtx& L, void* u, const void* f, int b, int pr, int pc, int nbr,
                                    int nbc, const CoarseArgs& ca)
{
    const int groups = nbr * nbc;
    if (groups == 0) return hipSuccess;
    dim3 grid, block;
    if (GROUP <= 64) {
        block = dim3(256);  // several lane groups per workgroup
        grid = dim3((unsigned)(((size_t)groups * GROUP + 255) / 256));
    } else {
        block = dim3(GROUP);
        grid = dim3(groups);
    }
    hipLaunchKernelGGL((sweep_blocks_kernel<T, KIND, GROUP, RPL, LAZY>), grid, block, 0, L.stream, (T*)u,
                       (const T*)f, L.H, L.W, b, pr, pc, nbr, nbc, L.alpha, L.M, L.G, ca);
    return hipGetLastError();
}

template <typename T, int KIND>
static hipError_t launch_b2(const LaunchCtx& L, void* u, const void* f, int pr, int pc)
{
    constexpr int QL = 4;   // one quadrant per lane: four waves per SIMD at 1024 x 1024 (two lanes: two)
    const Split2 S = split2((L.H + 1) / 2, (L.W + 1) / 2, pr, pc);
    const size_t threads = (size_t)S.nbr * S.nbc * QL;
    if (threads == 0) return hipSuccess;
    hipLaunchKernelGGL((sweep_b2_kernel<T, KIND, QL>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, L.stream,
                       (T*)u, (const T*)f, L.H, L.W, pr, pc, S, L.alpha, L.M, L.G);
    return hipGetLastError();
}

template <typename T, int KIND>
static hipError_t launch_blocks_t(const LaunchCtx& L, void* u, const void* f, int b, int pr, int pc, int nbr,
                                  int nbc, const CoarseArgs& ca)
{
    if (b == 2) return launch_b2<T, KIND>(L, u, f, pr, pc);
    // ring size of an unclipped block is 8b (lanes x records per lane = 8b); per level the
    // fastest of the batched autotuner's candidate shapes, timed on a 1024x1024 image.  A
    // 2^j - 1 side takes the shape of 2^j.
    switch (shape_side(b)) {
    case 4: return launch_blocks_cfg<T, KIND, 8, 4, false>(L, u, f, b, pr, pc, nbr, nbc, ca);
    case 8: return launch_blocks_cfg<T, KIND, 32, 2, false>(L, u, f, b, pr, pc, nbr, nbc, ca);
    case 16: return launch_blocks_cfg<T, KIND, 64, 2, false>(L, u, f, b, pr, pc, nbr, nbc, ca);
    case 32: return launch_blocks_cfg<T, KIND, 256, 1, false>(L, u, f, b, pr, pc, nbr, nbc, ca);
    case 64: return launch_blocks_cfg<T, KIND, 256, 2, true>(L, u, f, b, pr, pc, nbr, nbc, ca);
    case 128: return launch_blocks_cfg<T, KIND, 256, 4, true>(L, u, f, b, pr, pc, nbr, nbc, ca);
    case 256: return launch_blocks_cfg<T, KIND, 512, 4, true>(L, u, f, b, pr, pc, nbr, nbc, ca);
    case 512: return launch_blocks_cfg<T, KIND, 512, 8, true>(L, u, f, b, pr, pc, nbr, nbc, ca);
    default: return launch_blocks_cfg<T, KIND, 1024, 0, true>(L, u, f, b, pr, pc, nbr, nbc, ca);   // shape side >= STREAMED_B
    }
}

bool level_is_lazy(int b) { return shape_side(b) >= 64; }

size_t record_scratch_doubles(int H, int W, int J, int schedule)
{
    size_t need = 0;
    for (int level = 2; level <= J; ++level) {
        const int b = block_side(level, schedule);
        if (shape_side(b) < STREAMED_B) continue;
        const size_t mj = (size_t)(H + b - 1) / b, nj = (size_t)(W + b - 1) / b;
        const size_t per_colour = ((mj + 1) / 2) * ((nj + 1) / 2);   // colour 0 has the most blocks
        const size_t n = per_colour * 7 * (size_t)(8 * b);
        if (n > need) need = n;
    }
    return need;
}

hipError_t launch_sweep_blocks(const LaunchCtx& L, void* u, const void* f, int b, int colour, CoarseScratch& cs)
{
    const int pr = colour >> 1, pc = colour & 1;
    const int mj = (L.H + b - 1) / b, nj = (L.W + b - 1) / b;
    const int nbr = (mj - pr + 1) / 2, nbc = (nj - pc + 1) / 2;
    CoarseArgs ca{cs.partials, cs.nchunk, cs.cpend, nj, nullptr, 8 * b};
    // streamed levels keep their expanded records in memory when the scratch holds a region per block
    if (shape_side(b) >= STREAMED_B && (size_t)nbr * nbc * 7 * (size_t)(8 * b) <= cs.rec_cap) ca.rec = cs.rec;
    // few blocks on a register-resident coarse level: each block on 2^d - 1 workgroups (same
    // results); not under stream capture, since a graph would replay the launch's tag
    if (cs.split_cus > 0 && level_is_lazy(b)) {
        const int nblk = nbr * nbc;
        const int d = split_depth(nblk, cs.split_cus, L.G, b);
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        const size_t rec_need = split_record_doubles(nblk, cs.split_cus, L.G, b);
        if (d > 0 && nblk <= cs.xblocks && split_slot_words(L.M, L.G, d) <= (size_t)cs.xstride &&
            (shape_side(b) < STREAMED_B || (cs.rec && rec_need <= cs.rec_cap)) &&
            hipStreamIsCapturing(L.stream, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone) {
            if (++cs.xepoch == 0) {   // tags wrapped: clear the words so no old tag can match
                const hipError_t e = hipMemsetAsync(cs.xslots, 0,
                                                     sizeof(unsigned long long) * (size_t)cs.xblocks * cs.xstride, L.stream);
                if (e != hipSuccess) return e;
                cs.xepoch = 1;
            }
            const SplitArgs sa{cs.xslots, (1 << d) - 1, d, cs.xstride, cs.xepoch, cs.split_polls};
            CoarseArgs cas = ca;
            if (shape_side(b) >= STREAMED_B) cas.rec = cs.rec;   // one region per workgroup
            return launch_sweep_split(L, u, f, b, pr, pc, nbr, nbc, cas, sa);
        }
    }
    if (L.f64) return L.kind ? launch_blocks_t<double, 1>(L, u, f, b, pr, pc, nbr, nbc, ca)
                             : launch_blocks_t<double, 0>(L, u, f, b, pr, pc, nbr, nbc, ca);
    return L.kind ? launch_blocks_t<float, 1>(L, u, f, b, pr, pc, nbr, nbc, ca)
                  : launch_blocks_t<float, 0>(L, u, f, b, pr, pc, nbr, nbc, ca);
}

void coarse_geometry(int H, int W, int b, int* nblocks, int* nchunk, int* rows_per)
{
    const int mj = (H + b - 1) / b, nj = (W + b - 1) / b;
    int rp = 2048 / b;               // about 2k pixels per chunk: hundreds of workgroups per pass
    if (rp < 1) rp = 1;
    if (rp > b) rp = b;
    *rows_per = rp;
    *nchunk = (b + rp - 1) / rp;
    *nblocks = mj * nj;
}

// log2(b) for a power of two, -1 otherwise
static int log2i(int b)
{
    int lb = 0;
    while ((1 << lb) < b) ++lb;
    return (1 << lb) == b ? lb : -1;
}

hipError_t launch_level_begin(const LaunchCtx& L, void* u, const void* f, int b, CoarseScratch& cs, int prev_b)
{
    int nblocks, nchunk, rows_per;
    coarse_geometry(L.H, L.W, b, &nblocks, &nchunk, &rows_per);
    cs.nchunk = nchunk;
    const int nj = (L.W + b - 1) / b;
    const double* cprev = nullptr;
    int lbp = 0, njp = 0;
    if (prev_b > 0) {   // the previous level's corrections move to the other buffer and are applied here
        double* t = cs.cpend;
        cs.cpend = cs.cpend_alt;
        cs.cpend_alt = t;
        cprev = cs.cpend_alt;
        lbp = log2i(prev_b);
        njp = (L.W + prev_b - 1) / prev_b;
    }
    dim3 grid((unsigned)nblocks * nchunk), block(256);
    if (L.f64)
        hipLaunchKernelGGL(block_sums_kernel<double>, grid, block, 0, L.stream, (double*)u, (const double*)f,
                           L.H, L.W, b, nj, nchunk, rows_per, cs.partials, cs.cpend, cprev, prev_b, lbp, njp);
    else
        hipLaunchKernelGGL(block_sums_kernel<float>, grid, block, 0, L.stream, (float*)u, (const float*)f,
                           L.H, L.W, b, nj, nchunk, rows_per, cs.partials, cs.cpend, cprev, prev_b, lbp, njp);
    return hipGetLastError();
}

hipError_t launch_level_end(const LaunchCtx& L, void* u, int b, const CoarseScratch& cs)
{
    const int nj = (L.W + b - 1) / b;
    const int lb = log2i(b);
    const size_t n = (size_t)L.H * L.W;
    size_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    if (L.f64)
        hipLaunchKernelGGL(apply_level_kernel<double>, dim3((unsigned)g), dim3(256), 0, L.stream, (double*)u, L.H, L.W,
                           b, lb, nj, (const double*)cs.cpend);
    else
        hipLaunchKernelGGL(apply_level_kernel<float>, dim3((unsigned)g), dim3(256), 0, L.stream, (float*)u, L.H, L.W,
                           b, lb, nj, (const double*)cs.cpend);
    return hipGetLastError();
}

hipError_t launch_diff_norms(const LaunchCtx& L, const void* u, const void* prev, double* partials, double* out)
{
    const int np = energy_partials_count(L.H, L.W);
    const size_t n = (size_t)L.H * L.W;
    if (L.f64)
        hipLaunchKernelGGL(diff_norms_kernel<double>, dim3(np), dim3(256), 0, L.stream, (const double*)u,
                           (const double*)prev, n, partials);
    else
        hipLaunchKernelGGL(diff_norms_kernel<float>, dim3(np), dim3(256), 0, L.stream, (const float*)u,
                           (const float*)prev, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, L.stream, partials, np, out);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, L.stream, partials + np, np, out + 1);
    return hipGetLastError();
}

int energy_partials_count(int H, int W)
{
    const size_t n = (size_t)H * W;
    size_t g = (n + 255) / 256;
    return (int)(g < 2048 ? g : 2048);
}

hipError_t launch_energy(const LaunchCtx& L, const void* u, const void* f, double* partials, double* out)
{
    const int np = energy_partials_count(L.H, L.W);
    dim3 grid(np), block(256);
    if (L.f64) {
        if (L.kind) hipLaunchKernelGGL((energy_partial_kernel<double, 1>), grid, block, 0, L.stream, (const double*)u, (const double*)f, L.H, L.W, L.alpha, partials);
        else hipLaunchKernelGGL((energy_partial_kernel<double, 0>), grid, block, 0, L.stream, (const double*)u, (const double*)f, L.H, L.W, L.alpha, partials);
    } else {
        if (L.kind) hipLaunchKernelGGL((energy_partial_kernel<float, 1>), grid, block, 0, L.stream, (const float*)u, (const float*)f, L.H, L.W, L.alpha, partials);
        else hipLaunchKernelGGL((energy_partial_kernel<float, 0>), grid, block, 0, L.stream, (const float*)u, (const float*)f, L.H, L.W, L.alpha, partials);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, L.stream, partials, np, out);
    return hipGetLastError();
}

}  // namespace mgc
