// Host runtime of libmgcurv.so: parameter validation, context and scratch
// ownership, the V-cycle and solve drivers of Algorithm 3, and the C ABI
// declared in include/mgcurv.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "../../include/mgcurv.h"
#include "mgc_internal.h"

struct mg_curv_ctx {
    mg_curv_params P;
    int J;
    int device;
    hipStream_t stream;
    void* pingpong;        // H x W state-dtype image for the two-phase pixel level
    double* partials;      // energy partial sums
    mgc::CoarseScratch coarse;  // block sums and pending corrections of the coarse levels
    double* energy_dev;    // one double
    double* energy_host;   // pinned host double
    void* prev;            // previous iterate for the relErr(u) rule (allocated on first use)
    double* norm_part;     // 2 x energy_partials_count partial sums of ||u - prev||^2 and ||u||^2
    double* norm_dev;      // the two sums
    double* norm_host;     // pinned host copy of the two sums
    std::string err;
};

namespace {

thread_local std::string g_init_error;

mg_status fail(mg_curv_ctx* ctx, mg_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf; else g_init_error = buf;
    return st;
}

mg_status hip_fail(mg_curv_ctx* ctx, hipError_t e, const char* what)
{
    return fail(ctx, MG_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int auto_levels(int H, int W)
{
    int m = H > W ? H : W, J = 0;
    while ((1 << J) < m) ++J;   // ceil(log2(max(H, W)))
    return J < 1 ? 1 : J;
}

size_t state_bytes(const mg_curv_ctx* c)
{
    return (size_t)c->P.height * c->P.width * (c->P.state_dtype == MG_F64 ? 8 : 4);
}

mgc::LaunchCtx launch_ctx(const mg_curv_ctx* c)
{
    mgc::LaunchCtx L;
    L.stream = c->stream;
    L.H = c->P.height;
    L.W = c->P.width;
    L.alpha = c->P.alpha;
    L.kind = c->P.curvature;
    L.f64 = c->P.state_dtype == MG_F64;
    L.M = c->P.samples;
    L.G = c->P.bisections;
    return L;
}

int colours_at(const mg_curv_ctx* c, int level) { return (level == 1 && c->P.fine_colours == 9) ? 9 : 4; }

int side_at(const mg_curv_ctx* c, int level) { return mgc::block_side(level, c->P.block_schedule); }

mg_status check_buffers(mg_curv_ctx* ctx, const void* u, const void* f)
{
    if (!ctx) return MG_E_INVALID;
    if (!u || !f) return fail(ctx, MG_E_INVALID, "u and f must be non-null device pointers");
    const size_t n = state_bytes(ctx);
    const char* a = (const char*)u;
    const char* b = (const char*)f;
    if (a < b + n && b < a + n) return fail(ctx, MG_E_INVALID, "u must not overlap f");
    return MG_OK;
}

// One colour sweep of one level, on u in place.
mg_status sweep(mg_curv_ctx* ctx, void* u, const void* f, int level, int colour)
{
    const mgc::LaunchCtx L = launch_ctx(ctx);
    hipError_t e;
    if (level == 1) {
        e = mgc::launch_sweep_pixels(L, u, ctx->pingpong, f, colour, colours_at(ctx, 1));
        if (e != hipSuccess) return hip_fail(ctx, e, "pixel sweep launch");
        e = hipMemcpyAsync(u, ctx->pingpong, state_bytes(ctx), hipMemcpyDeviceToDevice, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "pixel sweep copy");
        return MG_OK;
    }
    const int b = side_at(ctx, level);
    const bool lazy = mgc::level_is_lazy(b);
    if (lazy && (e = mgc::launch_level_begin(L, u, f, b, ctx->coarse)) != hipSuccess) return hip_fail(ctx, e, "level begin");
    e = mgc::launch_sweep_blocks(L, u, f, b, colour, ctx->coarse);
    if (e != hipSuccess) return hip_fail(ctx, e, "block sweep launch");
    if (lazy && (e = mgc::launch_level_end(L, u, b, ctx->coarse)) != hipSuccess) return hip_fail(ctx, e, "level end");
    return MG_OK;
}

// All colours of one level.  The pixel level ping-pongs between u and the
// scratch image (two-phase update); with an odd number of colours the result
// is copied back into u.  Coarse levels take their block sums first and apply
// the level's corrections after the last colour.
mg_status level_sweeps(mg_curv_ctx* ctx, void* u, const void* f, int level, int prev_b = 0, bool defer_end = false)
{
    const mgc::LaunchCtx L = launch_ctx(ctx);
    hipError_t e;
    if (level == 1) {
        const int nc = colours_at(ctx, 1);
        void* cur = u;
        void* nxt = ctx->pingpong;
        for (int colour = 0; colour < nc; ++colour) {
            e = mgc::launch_sweep_pixels(L, cur, nxt, f, colour, nc);
            if (e != hipSuccess) return hip_fail(ctx, e, "pixel sweep launch");
            void* t = cur; cur = nxt; nxt = t;
        }
        if (cur != u) {
            e = hipMemcpyAsync(u, cur, state_bytes(ctx), hipMemcpyDeviceToDevice, ctx->stream);
            if (e != hipSuccess) return hip_fail(ctx, e, "pixel level copy");
        }
        return MG_OK;
    }
    const int b = side_at(ctx, level);
    const bool lazy = mgc::level_is_lazy(b);
    if (lazy && (e = mgc::launch_level_begin(L, u, f, b, ctx->coarse, prev_b)) != hipSuccess)
        return hip_fail(ctx, e, "level begin");
    for (int colour = 0; colour < 4; ++colour) {
        e = mgc::launch_sweep_blocks(L, u, f, b, colour, ctx->coarse);
        if (e != hipSuccess) return hip_fail(ctx, e, "block sweep launch");
    }
    if (lazy && !defer_end && (e = mgc::launch_level_end(L, u, b, ctx->coarse)) != hipSuccess)
        return hip_fail(ctx, e, "level end");
    return MG_OK;
}

// All levels fine to coarse, all colours (one outer iteration of Algorithm 3).
mg_status vcycle(mg_curv_ctx* ctx, void* u, const void* f)
{
    // levels 1..J, and with the full cycle J-1..1 after them; a coarse level's
    // corrections are applied by the sums pass of the next level in this order when
    // that level is coarse too, otherwise by the level's own correction pass
    int order[2 * 32];
    int n = 0;
    for (int level = 1; level <= ctx->J; ++level) order[n++] = level;
    if (ctx->P.cycle == 1)
        for (int level = ctx->J - 1; level >= 1; --level) order[n++] = level;
    int pending = 0;
    for (int k = 0; k < n; ++k) {
        const int level = order[k], b = side_at(ctx, level);
        const bool defer = mgc::level_is_lazy(b) && k + 1 < n && mgc::level_is_lazy(side_at(ctx, order[k + 1]));
        mg_status st = level_sweeps(ctx, u, f, level, pending, defer);
        if (st != MG_OK) return st;
        pending = defer ? b : 0;
    }
    return MG_OK;
}

mg_status energy(mg_curv_ctx* ctx, const void* u, const void* f, double* out)
{
    const mgc::LaunchCtx L = launch_ctx(ctx);
    hipError_t e = mgc::launch_energy(L, u, f, ctx->partials, ctx->energy_dev);
    if (e != hipSuccess) return hip_fail(ctx, e, "energy launch");
    e = hipMemcpyAsync(ctx->energy_host, ctx->energy_dev, sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "energy copy");
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "stream synchronize");
    *out = *ctx->energy_host;
    return MG_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free energy (mg_curv_energy_noalloc).  Its partial sums live in a
// file-scope device array of fixed size instead of a context's allocation.
// In host code `scratch` names a host-side stand-in, not device memory: the
// array's device address on each GPU is looked up once (hipGetSymbolAddress,
// with that device current) and only that address is handed to kernels.
// Every call on one device shares the array; each launch overwrites the
// partials it reads, so nothing needs clearing, and calls that overlap in time
// on one device (two streams, two threads) race.
// ---------------------------------------------------------------------------
constexpr int NOALLOC_PARTIALS = 2048;   // = the most energy_partials_count returns
static __device__ __align__(256) double scratch[NOALLOC_PARTIALS];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of this device's copy of `scratch` (looked up on first use).
hipError_t noalloc_scratch(int device, double** out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = (double*)ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

extern "C" {

#ifndef MGC_SOURCE_HASH
#define MGC_SOURCE_HASH "unknown"
#endif
const char* mg_curv_build_id(void) { return MGC_SOURCE_HASH; }

void mg_curv_default_params(mg_curv_params* p, int32_t height, int32_t width)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->height = height;
    p->width = width;
    p->alpha = 20.0;
    p->curvature = MG_CURV_MEAN;
    p->levels = 0;
    p->state_dtype = MG_F32;
    p->fine_colours = 4;
    p->samples = 16;
    p->bisections = 32;
    p->cycle = 0;
    p->block_schedule = 0;
}

mg_status mg_curv_init(const mg_curv_params* params, void* hip_stream, mg_curv_ctx** out)
{
    if (!params || !out) return fail(nullptr, MG_E_INVALID, "params and out must be non-null");
    *out = nullptr;
    const mg_curv_params& p = *params;
    if (p.height < 2 || p.width < 2) return fail(nullptr, MG_E_SHAPE, "height and width must be >= 2 (got %d x %d)", p.height, p.width);
    if ((int64_t)p.height * p.width > ((int64_t)1 << 31) - 1)
        return fail(nullptr, MG_E_SHAPE, "image larger than 2^31 - 1 pixels");
    if (!(p.alpha > 0.0) || !std::isfinite(p.alpha)) return fail(nullptr, MG_E_INVALID, "alpha must be finite and > 0");
    if (p.curvature != MG_CURV_MEAN && p.curvature != MG_CURV_GAUSS) return fail(nullptr, MG_E_INVALID, "curvature must be 0 (mean) or 1 (Gaussian)");
    if (p.state_dtype != MG_F32 && p.state_dtype != MG_F64) return fail(nullptr, MG_E_DTYPE, "state_dtype must be MG_F32 or MG_F64");
    if (p.fine_colours != 4 && p.fine_colours != 9) return fail(nullptr, MG_E_INVALID, "fine_colours must be 4 or 9");
    if (p.samples < 2 || p.samples > 256 || (p.samples & 1)) return fail(nullptr, MG_E_INVALID, "samples must be even and in [2, 256]");
    if (p.bisections < 0 || p.bisections > 64) return fail(nullptr, MG_E_INVALID, "bisections must be in [0, 64]");
    if (p.cycle != 0 && p.cycle != 1) return fail(nullptr, MG_E_INVALID, "cycle must be 0 (half) or 1 (full)");
    const int Jmax = auto_levels(p.height, p.width) + 1;
    if (p.levels < 0 || p.levels > Jmax) return fail(nullptr, MG_E_INVALID, "levels must be in [0, %d]", Jmax);
    if (p.block_schedule != 0 && p.block_schedule != 1)
        return fail(nullptr, MG_E_INVALID, "block_schedule must be 0 (2^(j-1)) or 1 (2^j - 1)");
    {   // ring counts (8b) and record strides stay in int range
        const int J = p.levels > 0 ? p.levels : auto_levels(p.height, p.width);
        if (J > 27 || mgc::block_side(J, p.block_schedule) > (1 << 26))
            return fail(nullptr, MG_E_INVALID, "the block side at level %d exceeds 2^26 pixels; use fewer levels", J);
    }

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) return fail(nullptr, MG_E_DEVICE, "no HIP device available");
    mg_curv_ctx* c = new (std::nothrow) mg_curv_ctx();
    if (!c) return fail(nullptr, MG_E_NOMEM, "host allocation failed");
    c->P = p;
    c->J = p.levels > 0 ? p.levels : auto_levels(p.height, p.width);
    c->stream = (hipStream_t)hip_stream;
    c->pingpong = nullptr;
    c->partials = nullptr;
    c->energy_dev = nullptr;
    c->energy_host = nullptr;
    c->prev = nullptr;
    c->norm_part = nullptr;
    c->norm_dev = nullptr;
    c->norm_host = nullptr;
    c->coarse = mgc::CoarseScratch{nullptr, 0, nullptr, nullptr, nullptr, 0, nullptr, 0, 0, 0, 0, mgc::SPLIT_POLLS};
    (void)hipGetDevice(&c->device);
    const size_t nb = state_bytes(c);
    const int np = mgc::energy_partials_count(p.height, p.width);
    size_t n_part = 1, n_pend = 1;
    for (int level = 2; level <= c->J; ++level) {
        const int b = side_at(c, level);
        if (!mgc::level_is_lazy(b)) continue;
        int nblocks, nchunk, rows_per;
        mgc::coarse_geometry(p.height, p.width, b, &nblocks, &nchunk, &rows_per);
        if ((size_t)nblocks * nchunk > n_part) n_part = (size_t)nblocks * nchunk;
        if ((size_t)nblocks > n_pend) n_pend = (size_t)nblocks;
    }
    size_t n_rec = mgc::record_scratch_doubles(p.height, p.width, c->J, p.block_schedule);
    // split coarse solve: exchange words for every block of the largest split launch, all
    // regions with the stride of the widest tree; streamed sides also need one record region
    // per workgroup of their split launches
    int cus = 0;
    size_t xstride = 0, xblocks = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && cus > 0) {
        for (int level = 2; level <= c->J; ++level) {
            const int b = side_at(c, level);
            if (!mgc::level_is_lazy(b)) continue;
            const int mj = (p.height + b - 1) / b, nj = (p.width + b - 1) / b;
            for (int colour = 0; colour < 4; ++colour) {
                const int nblk = ((mj - (colour >> 1) + 1) / 2) * ((nj - (colour & 1) + 1) / 2);
                const int d = mgc::split_depth(nblk, cus, p.bisections, b);
                if (d == 0) continue;
                const size_t words = mgc::split_slot_words(p.samples, p.bisections, d);
                const size_t recs = mgc::split_record_doubles(nblk, cus, p.bisections, b);
                if (recs > n_rec) n_rec = recs;
                if (words > xstride) xstride = words;
                if ((size_t)nblk > xblocks) xblocks = (size_t)nblk;
            }
        }
    }
    c->coarse.rec_cap = n_rec;
    bool xok = true;
    if (xblocks > 0) {   // tag 0 is never used, so cleared words match no launch
        xok = hipMalloc((void**)&c->coarse.xslots, sizeof(unsigned long long) * xblocks * xstride) == hipSuccess &&
              hipMemsetAsync(c->coarse.xslots, 0, sizeof(unsigned long long) * xblocks * xstride, c->stream) == hipSuccess;
        c->coarse.xstride = (int)xstride;
        c->coarse.xblocks = (int)xblocks;
        c->coarse.split_cus = cus;
    }
    if (hipMalloc(&c->pingpong, nb) != hipSuccess || hipMalloc((void**)&c->partials, sizeof(double) * np) != hipSuccess ||
        hipMalloc((void**)&c->coarse.partials, sizeof(double) * n_part) != hipSuccess ||
        hipMalloc((void**)&c->coarse.cpend, sizeof(double) * n_pend) != hipSuccess ||
        hipMalloc((void**)&c->coarse.cpend_alt, sizeof(double) * n_pend) != hipSuccess ||
        (n_rec > 0 && hipMalloc((void**)&c->coarse.rec, sizeof(double) * n_rec) != hipSuccess) ||
        !xok || hipMalloc((void**)&c->energy_dev, sizeof(double)) != hipSuccess ||
        hipHostMalloc((void**)&c->energy_host, sizeof(double), hipHostMallocDefault) != hipSuccess) {
        mg_curv_destroy(c);
        (void)hipGetLastError();
        return fail(nullptr, MG_E_NOMEM, "device allocation of %zu bytes failed", nb);
    }
    *out = c;
    return MG_OK;
}

mg_status mg_curv_vcycle(mg_curv_ctx* ctx, void* u, const void* f, double* energy_after)
{
    mg_status st = check_buffers(ctx, u, f);
    if (st != MG_OK) return st;
    st = vcycle(ctx, u, f);
    if (st != MG_OK || !energy_after) return st;
    return energy(ctx, u, f, energy_after);
}

mg_status mg_curv_sweep(mg_curv_ctx* ctx, void* u, const void* f, int32_t level, int32_t colour)
{
    mg_status st = check_buffers(ctx, u, f);
    if (st != MG_OK) return st;
    if (level < 1 || level > ctx->J) return fail(ctx, MG_E_INVALID, "level must be in [1, %d]", ctx->J);
    if (colour < 0 || colour >= colours_at(ctx, level)) return fail(ctx, MG_E_INVALID, "colour out of range for level %d", level);
    return sweep(ctx, u, f, level, colour);
}

mg_status mg_curv_level(mg_curv_ctx* ctx, void* u, const void* f, int32_t level)
{
    mg_status st = check_buffers(ctx, u, f);
    if (st != MG_OK) return st;
    if (level < 1 || level > ctx->J) return fail(ctx, MG_E_INVALID, "level must be in [1, %d]", ctx->J);
    return level_sweeps(ctx, u, f, level);
}

mg_status mg_curv_energy(mg_curv_ctx* ctx, const void* u, const void* f, double* out)
{
    mg_status st = check_buffers(ctx, u, f);
    if (st != MG_OK) return st;
    if (!out) return fail(ctx, MG_E_INVALID, "energy output must be non-null");
    return energy(ctx, u, f, out);
}

mg_status mg_curv_solve(mg_curv_ctx* ctx, void* u, const void* f, double rel_tol, int32_t max_vcycles,
                        int32_t* vcycles_done, double* final_energy, double* energy_trace)
{
    mg_status st = check_buffers(ctx, u, f);
    if (st != MG_OK) return st;
    if (max_vcycles < 0) return fail(ctx, MG_E_INVALID, "max_vcycles must be >= 0");
    if (!std::isfinite(rel_tol)) return fail(ctx, MG_E_INVALID, "rel_tol must be finite");
    double e_prev;
    st = energy(ctx, u, f, &e_prev);
    if (st != MG_OK) return st;
    if (!std::isfinite(e_prev)) return fail(ctx, MG_E_NONFINITE, "energy of the initial state is not finite");
    if (energy_trace) energy_trace[0] = e_prev;
    int done = 0;
    bool converged = false;
    double e = e_prev;
    while (done < max_vcycles) {
        st = vcycle(ctx, u, f);
        if (st != MG_OK) return st;
        st = energy(ctx, u, f, &e);
        if (st != MG_OK) return st;
        ++done;
        if (energy_trace) energy_trace[done] = e;
        if (!std::isfinite(e)) return fail(ctx, MG_E_NONFINITE, "energy became non-finite after V-cycle %d", done);
        if (rel_tol > 0.0 && (e == e_prev || std::fabs(e - e_prev) < rel_tol * std::fabs(e))) { converged = true; break; }
        e_prev = e;
    }
    if (vcycles_done) *vcycles_done = done;
    if (final_energy) *final_energy = e;
    return (rel_tol > 0.0 && !converged) ? MG_NOT_CONVERGED : MG_OK;
}

mg_status mg_curv_solve_rule(mg_curv_ctx* ctx, void* u, const void* f, int32_t stop, double tol, int32_t max_vcycles,
                             int32_t* vcycles_done, double* final_energy)
{
    if (stop == MG_STOP_ENERGY) return mg_curv_solve(ctx, u, f, tol, max_vcycles, vcycles_done, final_energy, nullptr);
    mg_status st = check_buffers(ctx, u, f);
    if (st != MG_OK) return st;
    if (stop != MG_STOP_RELERR_U) return fail(ctx, MG_E_INVALID, "unknown stopping rule %d", stop);
    if (max_vcycles < 0) return fail(ctx, MG_E_INVALID, "max_vcycles must be >= 0");
    if (!std::isfinite(tol)) return fail(ctx, MG_E_INVALID, "tol must be finite");
    double e;
    st = energy(ctx, u, f, &e);
    if (st != MG_OK) return st;
    if (!std::isfinite(e)) return fail(ctx, MG_E_NONFINITE, "energy of the initial state is not finite");
    const int np = mgc::energy_partials_count(ctx->P.height, ctx->P.width);
    if (!ctx->prev) {
        if (hipMalloc(&ctx->prev, state_bytes(ctx)) != hipSuccess ||
            hipMalloc((void**)&ctx->norm_part, sizeof(double) * 2 * np) != hipSuccess ||
            hipMalloc((void**)&ctx->norm_dev, sizeof(double) * 2) != hipSuccess ||
            hipHostMalloc((void**)&ctx->norm_host, sizeof(double) * 2, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, MG_E_NOMEM, "allocation of the previous-iterate buffer failed");
        }
    }
    const mgc::LaunchCtx L = launch_ctx(ctx);
    int done = 0;
    bool converged = false;
    while (done < max_vcycles) {
        hipError_t he = hipMemcpyAsync(ctx->prev, u, state_bytes(ctx), hipMemcpyDeviceToDevice, ctx->stream);
        if (he != hipSuccess) return hip_fail(ctx, he, "previous-iterate copy");
        st = vcycle(ctx, u, f);
        if (st != MG_OK) return st;
        ++done;
        he = mgc::launch_diff_norms(L, u, ctx->prev, ctx->norm_part, ctx->norm_dev);
        if (he == hipSuccess)
            he = hipMemcpyAsync(ctx->norm_host, ctx->norm_dev, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
        if (he == hipSuccess) he = hipStreamSynchronize(ctx->stream);
        if (he != hipSuccess) return hip_fail(ctx, he, "relErr(u) norms");
        if (tol > 0.0 && std::sqrt(ctx->norm_host[0]) < tol * std::sqrt(ctx->norm_host[1])) { converged = true; break; }
    }
    st = energy(ctx, u, f, &e);
    if (st != MG_OK) return st;
    if (vcycles_done) *vcycles_done = done;
    if (final_energy) *final_energy = e;
    return (tol > 0.0 && !converged) ? MG_NOT_CONVERGED : MG_OK;
}

mg_status mg_curv_solve_target(mg_curv_ctx* ctx, void* u, const void* f, double target_energy, int32_t max_vcycles,
                               int32_t* vcycles_done, double* final_energy)
{
    mg_status st = check_buffers(ctx, u, f);
    if (st != MG_OK) return st;
    if (max_vcycles < 0 || std::isnan(target_energy)) return fail(ctx, MG_E_INVALID, "bad target_energy or max_vcycles");
    double e;
    st = energy(ctx, u, f, &e);
    if (st != MG_OK) return st;
    if (!std::isfinite(e)) return fail(ctx, MG_E_NONFINITE, "energy of the initial state is not finite");
    int done = 0;
    while (e > target_energy && done < max_vcycles) {
        if ((st = vcycle(ctx, u, f)) != MG_OK) return st;
        if ((st = energy(ctx, u, f, &e)) != MG_OK) return st;
        ++done;
        if (!std::isfinite(e)) return fail(ctx, MG_E_NONFINITE, "energy became non-finite after V-cycle %d", done);
    }
    if (vcycles_done) *vcycles_done = done;
    if (final_energy) *final_energy = e;
    return e <= target_energy ? MG_OK : MG_NOT_CONVERGED;
}

int32_t mg_curv_levels(const mg_curv_ctx* ctx) { return ctx ? ctx->J : 0; }

mg_status mg_curv_set_split(mg_curv_ctx* ctx, int32_t enable)
{
    if (!ctx) return MG_E_INVALID;
    if (enable != 0 && enable != 1) return fail(ctx, MG_E_INVALID, "enable must be 0 or 1");
    int cus = 0;
    if (enable && ctx->coarse.xblocks > 0 &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess)
        return fail(ctx, MG_E_DEVICE, "device attribute query failed");
    ctx->coarse.split_cus = (enable && ctx->coarse.xblocks > 0) ? cus : 0;
    return MG_OK;
}

int32_t mg_curv_split_active(const mg_curv_ctx* ctx) { return ctx && ctx->coarse.split_cus > 0 ? 1 : 0; }

mg_status mg_curv_set_split_polls(mg_curv_ctx* ctx, int32_t polls)
{
    if (!ctx) return MG_E_INVALID;
    if (polls < 0) return fail(ctx, MG_E_INVALID, "polls must be >= 0");
    ctx->coarse.split_polls = polls;
    return MG_OK;
}

void mg_curv_destroy(mg_curv_ctx* ctx)
{
    if (!ctx) return;
    if (ctx->stream || ctx->pingpong) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->pingpong) (void)hipFree(ctx->pingpong);
    if (ctx->partials) (void)hipFree(ctx->partials);
    if (ctx->coarse.partials) (void)hipFree(ctx->coarse.partials);
    if (ctx->coarse.cpend) (void)hipFree(ctx->coarse.cpend);
    if (ctx->coarse.cpend_alt) (void)hipFree(ctx->coarse.cpend_alt);
    if (ctx->coarse.rec) (void)hipFree(ctx->coarse.rec);
    if (ctx->coarse.xslots) (void)hipFree(ctx->coarse.xslots);
    if (ctx->energy_dev) (void)hipFree(ctx->energy_dev);
    if (ctx->energy_host) (void)hipHostFree(ctx->energy_host);
    if (ctx->prev) (void)hipFree(ctx->prev);
    if (ctx->norm_part) (void)hipFree(ctx->norm_part);
    if (ctx->norm_dev) (void)hipFree(ctx->norm_dev);
    if (ctx->norm_host) (void)hipHostFree(ctx->norm_host);
    delete ctx;
}

const char* mg_curv_last_error(const mg_curv_ctx* ctx)
{
    if (ctx) return ctx->err.c_str();
    return g_init_error.c_str();
}

}  // extern "C"

extern "C" mg_status mg_curv_energy_noalloc(const mg_curv_params* params, void* hip_stream, const void* u,
                                            const void* f, double* energy_dev)
{
    if (!params) return fail(nullptr, MG_E_INVALID, "params must be non-null");
    const mg_curv_params& p = *params;
    if (p.height < 2 || p.width < 2) return fail(nullptr, MG_E_SHAPE, "height and width must be >= 2 (got %d x %d)", p.height, p.width);
    if ((int64_t)p.height * p.width > ((int64_t)1 << 31) - 1)
        return fail(nullptr, MG_E_SHAPE, "image larger than 2^31 - 1 pixels");
    if (mgc::energy_partials_count(p.height, p.width) > NOALLOC_PARTIALS)
        return fail(nullptr, MG_E_SHAPE, "the energy needs more than %d partial sums", NOALLOC_PARTIALS);
    if (!(p.alpha > 0.0) || !std::isfinite(p.alpha)) return fail(nullptr, MG_E_INVALID, "alpha must be finite and > 0");
    if (p.curvature != MG_CURV_MEAN && p.curvature != MG_CURV_GAUSS) return fail(nullptr, MG_E_INVALID, "curvature must be 0 (mean) or 1 (Gaussian)");
    if (p.state_dtype != MG_F32 && p.state_dtype != MG_F64) return fail(nullptr, MG_E_DTYPE, "state_dtype must be MG_F32 or MG_F64");
    if (!u || !f || !energy_dev) return fail(nullptr, MG_E_INVALID, "u, f and energy must be non-null device pointers");
    const size_t n = (size_t)p.height * p.width * (p.state_dtype == MG_F64 ? 8 : 4);
    const char* a = (const char*)u;
    const char* b = (const char*)f;
    const char* o = (const char*)energy_dev;
    if (a < b + n && b < a + n) return fail(nullptr, MG_E_INVALID, "u must not overlap f");
    if ((o < a + n && a < o + sizeof(double)) || (o < b + n && b < o + sizeof(double)))
        return fail(nullptr, MG_E_INVALID, "the energy output must not overlap u or f");
    int device = -1;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return fail(nullptr, MG_E_DEVICE, "no HIP device available: %s", hipGetErrorString(e));
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return fail(nullptr, MG_E_DEVICE, "device index %d out of range", device);
    double* partials = nullptr;
    e = noalloc_scratch(device, &partials);
    if (e != hipSuccess) return fail(nullptr, MG_E_DEVICE, "scratch address lookup: %s", hipGetErrorString(e));
    mgc::LaunchCtx L;
    L.stream = (hipStream_t)hip_stream;
    L.H = p.height;
    L.W = p.width;
    L.alpha = p.alpha;
    L.kind = p.curvature;
    L.f64 = p.state_dtype == MG_F64;
    L.M = p.samples;
    L.G = p.bisections;
    e = mgc::launch_energy(L, u, f, partials, energy_dev);
    if (e != hipSuccess) return fail(nullptr, MG_E_DEVICE, "energy launch: %s", hipGetErrorString(e));
    return MG_OK;
}
