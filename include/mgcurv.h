/*
 * mgcurv.h -- C ABI of libmgcurv.so: multigrid minimisation of curvature
 * energies (arXiv 2204.07921) on AMD Instinct MI355X (gfx950).
 *
 * The library minimises, for an image f on an H x W pixel grid,
 *
 *     F(u) = sum_pixels |kappa(u)| + alpha/2 (u - f)^2              (eq. MCM / eq. GCM)
 *
 * where kappa is the mean curvature div(grad u / sqrt(1 + |grad u|^2)) or the
 * Gaussian curvature det(Hess u) / (1 + |grad u|^2)^2 of the image graph
 * (Table 1), discretised with 3x3 central differences and replicated ghost
 * pixels.  One V-cycle is the fine-to-coarse half cycle of Algorithm 3: for
 * level j = 1..J (block side b_j = 2^(j-1), blocks clipped at the right and
 * bottom edges), for each colour of the four-colour decomposition of
 * Section 2.3 (colour of block (p, q) = 2 (p mod 2) + (q mod 2)), every block
 * B of that colour receives u <- u + c_B chi_B with c_B the minimiser of the
 * local energy F(u + c chi_B) (Section 2.2, the arg min of Algorithm 3).
 * All c_B of one colour are computed from the state at the start of that
 * colour.  The one-dimensional minimisation samples the bracket
 * [f* - rho, f* + rho] (f* = mean of f - u over B, rho = sqrt(2 K(f*) / (alpha |B|)))
 * at `samples` + 1 points, refines the best one by `bisections` bisection
 * steps on the sign of the derivative, and keeps c = 0 unless the result
 * lowers the local energy by more than the rounding margin 1e-12 (1 + V(0))
 * of the computed change (V(0) = the block's local energy at c = 0).
 *
 * Conventions for every entry point:
 *   - u and f are DEVICE pointers to contiguous row-major H x W arrays of
 *     the context's state dtype (float or double).  The caller owns them.
 *     u is read and written, f is only read; u must not alias f.
 *   - Work is enqueued on the HIP stream given to mg_curv_init (NULL = the
 *     null stream).  Calls that return a host value (energy, solve) block
 *     until it is available; mg_curv_vcycle and mg_curv_sweep without a
 *     requested energy return after enqueueing.
 *   - Every entry point returns an mg_status and never throws.  A negative
 *     status means the request was rejected or failed; on validation
 *     failures u is not modified.  mg_curv_last_error describes the last
 *     failure.
 *   - A context is bound to one device and one stream; it is not thread-safe.
 */
#ifndef MGCURV_H
#define MGCURV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MG_OK = 0,
    MG_NOT_CONVERGED = 1,  /* warning: max_vcycles reached first; u holds the last iterate */
    MG_E_INVALID = -1,     /* bad argument (null pointer, alpha <= 0, aliasing, bad option) */
    MG_E_SHAPE = -2,       /* H or W < 2, or sizes beyond the supported range */
    MG_E_DTYPE = -3,       /* state dtype not MG_F32 / MG_F64 */
    MG_E_NOMEM = -4,       /* device allocation failed */
    MG_E_DEVICE = -5,      /* no usable GPU, or a HIP call failed */
    MG_E_NONFINITE = -6    /* the energy of the input state is NaN or infinite */
} mg_status;

typedef enum { MG_CURV_MEAN = 0, MG_CURV_GAUSS = 1 } mg_curv_kind;
typedef enum { MG_F32 = 0, MG_F64 = 1 } mg_dtype;

/* Stopping rules of the solves (Section 4). */
typedef enum {
    MG_STOP_ENERGY = 0,   /* |E_l - E_{l-1}| < tol |E_l| (Section 4) */
    MG_STOP_RELERR_U = 1  /* ||u_l - u_{l-1}||_2 < tol ||u_l||_2 (Section 4, relErr(u)) */
} mg_stop_rule;

typedef struct {
    int32_t height;        /* H >= 2 */
    int32_t width;         /* W >= 2 */
    double alpha;          /* data weight of eq. MCM / GCM, finite and > 0 */
    int32_t curvature;     /* mg_curv_kind */
    int32_t levels;        /* J >= 1, at most ceil(log2(max(H, W))) + 1, and the block side
                              at level J at most 2^26; 0 selects ceil(log2(max(H, W))) */
    int32_t state_dtype;   /* mg_dtype of u and f; the local minimisation always runs in FP64 */
    int32_t fine_colours;  /* colours at the pixel level (b = 1): 4 (Section 2.3) or 9
                              (3 x 3 pattern; pixels of one colour then share no ring pixel) */
    int32_t samples;       /* M, even, 2..256 (default 16) */
    int32_t bisections;    /* G, 0..64 (default 32) */
    int32_t cycle;         /* 0: levels 1..J, the half V-cycle of Algorithm 3 (default);
                              1: then J-1..1, the full V-cycle Section 2.2 compares it with.
                              Batches take 0 only. */
    int32_t block_schedule; /* block side at level j: 0: 2^(j-1), nested blocks (default);
                              1: 2^j - 1, the patch side of Section 2.2 (blocks of one
                              level then straddle those of the next).  Both are single
                              pixels at j = 1.  Equal across a batch. */
} mg_curv_params;

typedef struct mg_curv_ctx mg_curv_ctx;

/* Identifier of the sources the library was built from (a hash of its
 * source files and this header, fixed at build time); "unknown" for a build
 * that did not set it.  Lets a loader refuse a stale binary.  Never NULL. */
const char *mg_curv_build_id(void);

/* Fill *p with the defaults for an H x W image: alpha 20, mean curvature,
 * levels 0 (automatic), float state, 4 fine colours, M = 16, G = 32, half
 * V-cycle, power-of-two blocks. */
void mg_curv_default_params(mg_curv_params *p, int32_t height, int32_t width);

/* Validate *params, bind the current HIP device and `hip_stream`
 * (a hipStream_t, may be NULL), and allocate the context's scratch: one
 * H x W ping-pong image for the pixel level, the energy partial sums, the
 * coarse levels' block sums and two arrays of pending corrections, and, when
 * the levels reach blocks of side >= 1023, the expanded ring records of one
 * colour's blocks (7 doubles per ring pixel; 7.3 MB at 8192 x 8192), or, for
 * the split solve below, of each of its workgroups (at most 128 MB).
 * On success *out receives a context the caller releases with
 * mg_curv_destroy.  Errors: MG_E_INVALID / MG_E_SHAPE / MG_E_DTYPE for bad
 * parameters, MG_E_DEVICE without a GPU, MG_E_NOMEM. */
mg_status mg_curv_init(const mg_curv_params *params, void *hip_stream, mg_curv_ctx **out);

/* One fine-to-coarse V-cycle of Algorithm 3 on u (in place).  If
 * energy_after is non-null the call also evaluates F(u) afterwards and
 * waits for it. */
mg_status mg_curv_vcycle(mg_curv_ctx *ctx, void *u, const void *f, double *energy_after);

/* Run V-cycles on u (in place, starting from the u given; pass a copy of f
 * for the paper's usual start u0 = f) until the relative energy change
 * |E_l - E_{l-1}| / |E_l| drops below rel_tol (the stopping rule of the
 * paper's experiments, Section 4) or max_vcycles cycles have run.
 * rel_tol <= 0 runs exactly max_vcycles cycles.  Outputs (each nullable):
 * *vcycles_done, *final_energy, and energy_trace[0 .. done] (host array of
 * at least max_vcycles + 1 doubles, E_0 = F(u) on entry).
 * Returns MG_OK, MG_NOT_CONVERGED (rel_tol > 0 and the limit was hit) or an
 * error; MG_E_NONFINITE if F(u) on entry is not finite (u untouched). */
mg_status mg_curv_solve(mg_curv_ctx *ctx, void *u, const void *f, double rel_tol, int32_t max_vcycles,
                        int32_t *vcycles_done, double *final_energy, double *energy_trace);

/* As mg_curv_solve with the stopping rule chosen (mg_stop_rule): with
 * MG_STOP_ENERGY exactly mg_curv_solve; with MG_STOP_RELERR_U V-cycles run
 * until ||u_l - u_{l-1}||_2 < tol ||u_l||_2 (norms in FP64; tol <= 0 runs
 * exactly max_vcycles).  The iterate rule keeps a copy of the previous u,
 * which the context allocates on the first such call (MG_E_NOMEM if that
 * fails).  Returns MG_OK, MG_NOT_CONVERGED, MG_E_INVALID for an unknown rule,
 * or the errors of mg_curv_solve.  Outputs nullable; *final_energy is F(u)
 * at the end. */
mg_status mg_curv_solve_rule(mg_curv_ctx *ctx, void *u, const void *f, int32_t stop, double tol, int32_t max_vcycles,
                             int32_t *vcycles_done, double *final_energy);

/* Run V-cycles on u until F(u) <= target_energy (checked before the first
 * cycle as well) or max_vcycles cycles have run: the refinement step of a
 * warm-started solve that must reach a given energy.  Returns MG_OK when the
 * target was reached, MG_NOT_CONVERGED otherwise.  Outputs nullable. */
mg_status mg_curv_solve_target(mg_curv_ctx *ctx, void *u, const void *f, double target_energy, int32_t max_vcycles,
                               int32_t *vcycles_done, double *final_energy);

/* F(u) of eq. MCM / GCM, accumulated in FP64 in a fixed order (the result is
 * bitwise reproducible for a given size and launch). */
mg_status mg_curv_energy(mg_curv_ctx *ctx, const void *u, const void *f, double *energy);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the energy
 * of mg_curv_energy without a context.  params gives H, W, alpha, curvature
 * and state_dtype (the other fields are ignored); u and f are device arrays
 * as for every entry point, and energy is a DEVICE pointer to one double that
 * receives F(u) (same kernels and summation order as mg_curv_energy, so the
 * same value bit for bit).  Enqueued on hip_stream only; the call returns
 * without waiting.  The partial sums (at most 2048 doubles) live in a
 * static device array of the library, one per GPU, whose address is looked up
 * on the first call on each device; the call makes no device allocation.
 * Calls that overlap in time on one GPU (other streams or threads) share that
 * array and race.  Errors (before anything is enqueued): MG_E_INVALID /
 * MG_E_SHAPE / MG_E_DTYPE for bad parameters, null or overlapping pointers;
 * MG_E_SHAPE for more than 2^31 - 1 pixels; MG_E_DEVICE if no device is
 * current or a HIP call fails.  mg_curv_last_error(NULL) describes the
 * failure. */
mg_status mg_curv_energy_noalloc(const mg_curv_params *params, void *hip_stream, const void *u, const void *f,
                                 double *energy);

/* One colour sweep of one level (1-based level, colour in [0, 4) or
 * [0, 9) at level 1 with nine fine colours), in place on u.  This is the
 * unit a V-cycle repeats; it is exported so a caller can inspect single
 * steps.  Enqueued only. */
mg_status mg_curv_sweep(mg_curv_ctx *ctx, void *u, const void *f, int32_t level, int32_t colour);

/* All colours of one level (1-based), in place on u: the level-j part of one
 * V-cycle of Algorithm 3 (4 colour sweeps, or 9 at level 1 with nine fine
 * colours).  Enqueued only. */
mg_status mg_curv_level(mg_curv_ctx *ctx, void *u, const void *f, int32_t level);

/* Number of levels J the context uses (after resolving levels = 0). */
int32_t mg_curv_levels(const mg_curv_ctx *ctx);

/* Split solve of the coarse levels (the arg min of Algorithm 3, Section 2.2,
 * computed by several workgroups per block).  Where a colour of a coarse
 * level of block side >= 256 holds so few blocks that 2^d - 1 workgroups
 * per block fit on the device's CUs (d >= 4; for sides >= 1023, whose rings
 * are streamed from memory, 2 <= d <= 6 within a 128 MB budget of
 * per-workgroup record copies), each block's samples are spread over its
 * workgroups and its bisection takes d steps per exchange between them.  The corrections are bitwise those of the one-workgroup
 * solve; only the time differs (a workgroup that waits too long for a value
 * computes it itself, so results never depend on timing).  It is on by
 * default when the context's levels have such colours (mg_curv_init then
 * allocates the exchange words: 2 M + ceil(G / d)(2^d - 1) 64-bit words per
 * block of the largest such launch, 32 KB or less at the default M and G).
 * Launches under HIP stream capture use the one-workgroup solve.  enable: 1
 * on (no effect if the context has no such level), 0 off.  Returns MG_OK,
 * or MG_E_INVALID for a null context or another value. */
mg_status mg_curv_set_split(mg_curv_ctx *ctx, int32_t enable);

/* 1 if the context's coarse levels use the split solve, else 0 (also for NULL). */
int32_t mg_curv_split_active(const mg_curv_ctx *ctx);

/* Bound on the polls of each exchange wait of the split solve (default 16384,
 * some milliseconds).  A workgroup that has not seen a value within the bound
 * evaluates it itself, with the same records and sums, so the corrections do
 * not depend on this setting; 0 makes every workgroup evaluate every value
 * (each block then costs what it costs on one workgroup).  Meant for tests of
 * that fallback and for shared devices where workgroups of one launch may not
 * run at the same time.  Returns MG_OK, or MG_E_INVALID for a null context or
 * polls < 0. */
mg_status mg_curv_set_split_polls(mg_curv_ctx *ctx, int32_t polls);

/* Release the context (NULL is allowed).  Waits for its stream first. */
void mg_curv_destroy(mg_curv_ctx *ctx);

/* Text of the last error on this context, or of the calling thread's last
 * failed mg_curv_init when ctx is NULL.  Never NULL. */
const char *mg_curv_last_error(const mg_curv_ctx *ctx);


/* ------------------------------------------------------------------------
 * Batched images.  n images of independent sizes, alphas and curvature kinds
 * share one packed float32 buffer for u and one for f: image i occupies
 * elements [mg_curv_batch_offset(b, i), mg_curv_batch_offset(b, i + 1)) in
 * row-major H_i x W_i order.  Each image follows exactly the single-image
 * algorithm above with its own level count J_i; one V-cycle runs levels
 * 1 .. max J_i, and each (level, colour) is one persistent kernel over the
 * work items of all images (images with J_i < level have none).
 * Requirements: state_dtype MG_F32, fine_colours 4 and cycle 0 for every
 * image; samples, bisections and block_schedule equal across the batch.  The batch owns a packed
 * ping-pong buffer and small per-level tables; it is bound to one device and
 * stream and is not thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct mg_curv_batch mg_curv_batch;

/* Validate params[0 .. n-1] and allocate the batch.  Errors as mg_curv_init. */
mg_status mg_curv_batch_init(const mg_curv_params *params, int32_t n, void *hip_stream, mg_curv_batch **out);

/* Element offset of image i in the packed buffers; i = n gives the total
 * element count.  -1 for a bad argument. */
int64_t mg_curv_batch_offset(const mg_curv_batch *b, int32_t i);

/* Largest level count J_i of the batch. */
int32_t mg_curv_batch_levels(const mg_curv_batch *b);

/* One V-cycle for every image (enqueued on the batch's stream).  If
 * energies is non-null (host array of n doubles) it receives each image's
 * F(u) afterwards and the call waits. */
mg_status mg_curv_batch_vcycle(mg_curv_batch *b, void *u, const void *f, double *energies);

/* All colours of one level (1-based) for every image; enqueued only. */
mg_status mg_curv_batch_level(mg_curv_batch *b, void *u, const void *f, int32_t level);

/* One colour of one block level (level >= 2) for every image; enqueued only. */
mg_status mg_curv_batch_sweep(mg_curv_batch *b, void *u, const void *f, int32_t level, int32_t colour);

/* Per-image F(u) (host array of n doubles, FP64, fixed summation order). */
mg_status mg_curv_batch_energy(mg_curv_batch *b, const void *u, const void *f, double *energies);

/* Solve every image until its own relative energy change is below rel_tol
 * (or max_vcycles).  Converged images stop being updated while the others
 * continue.  One V-cycle plus the energies is captured once as a HIP graph
 * on the batch's internal stream and replayed.  Outputs are host arrays of n
 * entries (each nullable).  Returns MG_OK when every image converged,
 * MG_NOT_CONVERGED otherwise (status[i] tells which), or an error. */
mg_status mg_curv_batch_solve(mg_curv_batch *b, void *u, const void *f, double rel_tol, int32_t max_vcycles,
                              int32_t *vcycles_done, double *final_energy, int32_t *status);

/* As mg_curv_batch_solve, but image i stops when F(u_i) <= target_energy[i]
 * (host array of n doubles, checked before the first V-cycle too). */
mg_status mg_curv_batch_solve_target(mg_curv_batch *b, void *u, const void *f, const double *target_energy,
                                     int32_t max_vcycles, int32_t *vcycles_done, double *final_energy, int32_t *status);

/* Autotune: for each level, time the compiled lane-group shapes and
 * persistent grid sizes on these buffers (u is not modified; a scratch copy
 * is used) and keep the fastest.  `repeats` timings per candidate.
 * Different shapes change only the order of floating-point sums. */
mg_status mg_curv_batch_tune(mg_curv_batch *b, void *u, const void *f, int32_t repeats);

/* Inspect / force the lane-group shape (group lanes, ring records per lane)
 * and persistent grid of one level.  set_config rejects shapes that are not
 * compiled for that level.  At level 2 (b = 2), records = -1 with group = 4
 * (or 2) is the mirrored form: blocks off the image border read their ring as
 * four mirrored quadrants with constant slopes (one or two quadrants of four
 * records per lane), border blocks use the general (4, 4) (or (2, 8))
 * records; (4, -1) is that level's default. */
int32_t mg_curv_batch_config(const mg_curv_batch *b, int32_t level, int32_t *group, int32_t *records, int32_t *grid);
mg_status mg_curv_batch_set_config(mg_curv_batch *b, int32_t level, int32_t group, int32_t records, int32_t grid);

void mg_curv_batch_destroy(mg_curv_batch *b);
const char *mg_curv_batch_last_error(const mg_curv_batch *b);

/* ------------------------------------------------------------------------
 * Learned warm start.  A six-layer CNN g (3x3 convolutions with zero "same"
 * padding, channels 1 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, ReLU after the first
 * five) predicts an initial state u0 = f + g(f) for the multigrid solve; it is
 * trained by mean squared error against multigrid solutions with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8).  Weights are FP32 masters with bfloat16
 * copies; activations are stored in bfloat16; all sums accumulate in FP32.
 * Parameter vector (float32, mg_cnn_num_params() = 37601 entries), layer by
 * layer: W_l as (ky, kx, c_in, c_out) row-major, then b_l (c_out).
 * Images are float32 device arrays of n x height x width (row-major); the
 * context holds activation buffers for `max_pixels` = n * height * width.
 * ------------------------------------------------------------------------ */
typedef struct mg_cnn mg_cnn;

int32_t mg_cnn_num_params(void);

/* Allocate a network context for batches of up to max_pixels pixels
 * (about 450 bytes of device memory per pixel).  Parameters start unset:
 * call mg_cnn_set_params before use. */
mg_status mg_cnn_init(int64_t max_pixels, void *hip_stream, mg_cnn **out);

/* Copy parameters from a host array (and reset the Adam moments and step);
 * read them back into a host array.  Both wait for completion. */
mg_status mg_cnn_set_params(mg_cnn *c, const float *host_params);
mg_status mg_cnn_get_params(mg_cnn *c, float *host_params);

/* Training checkpoint: the FP32 parameters, both Adam moments (host arrays of
 * mg_cnn_num_params floats each) and the Adam step count.  A context restored
 * with mg_cnn_set_state continues training bit for bit as the one the state
 * was read from would have.  Both wait for completion. */
mg_status mg_cnn_get_state(mg_cnn *c, float *host_params, float *host_m, float *host_v, int32_t *step);
mg_status mg_cnn_set_state(mg_cnn *c, const float *host_params, const float *host_m, const float *host_v,
                           int32_t step);

/* u = f + g(f) for n images (device pointers, u may not alias f).  Enqueued only. */
mg_status mg_cnn_forward(mg_cnn *c, const float *f, float *u, int32_t n, int32_t height, int32_t width);

/* One Adam step on the mean squared error of f + g(f) against target; *loss
 * (nullable) receives the loss before the step (waits when non-null). */
mg_status mg_cnn_train_step(mg_cnn *c, const float *f, const float *target, int32_t n, int32_t height, int32_t width,
                            float lr, double *loss);

/* Loss and parameter gradient (host array of mg_cnn_num_params floats,
 * nullable) without updating the parameters.  Waits. */
mg_status mg_cnn_gradients(mg_cnn *c, const float *f, const float *target, int32_t n, int32_t height, int32_t width,
                           double *loss, float *host_grads);

/* One forward and backward pass as mg_cnn_gradients (no update), exporting the
 * backward pass's intermediate gradients for inspection: host_dz (host,
 * 5 x n x height x width x 32 bfloat16, NHWC, layer-major) receives
 * dL/dz_l for l = 0..4, z_l being the pre-activation of layer l (so a_{l+1} =
 * relu(z_l)), with the ReLU mask applied and rounded to bfloat16 as stored;
 * host_dz5 (host, n x height x width floats) receives dL/dz_5 = 2 (u - target) /
 * (n height width); host_grads (nullable) the parameter gradient.  The
 * activations of the same forward pass are then available from
 * mg_cnn_activation.  Waits. */
mg_status mg_cnn_gradient_trace(mg_cnn *c, const float *f, const float *target, int32_t n, int32_t height,
                                int32_t width, void *host_dz, float *host_dz5, float *host_grads);

/* Copy the first `count` bfloat16 values of activation a_layer (layer 1..5,
 * NHWC with 32 channels) of the last forward pass to a host buffer. */
mg_status mg_cnn_activation(mg_cnn *c, int32_t layer, void *host_out, int64_t count);

void mg_cnn_destroy(mg_cnn *c);
const char *mg_cnn_last_error(const mg_cnn *c);

/* ------------------------------------------------------------------------
 * The paper's own local step (Section 2.1-2.2, Algorithm 2, Propositions 1-2).
 * Patches of side b_j = 2^j - 1 on level j = 1..J (Section 2.2: m_j =
 * ceil(H / b_j) rows and n_j = ceil(W / b_j) columns of patches anchored at the
 * top-left pixel, clipped at the right and bottom edges; positions outside the
 * image take the value of the nearest image pixel), the four-colour order of
 * Section 2.3, and per patch `steps` forward-backward splitting updates:
 *     c_0 = 0, eta_0 = 1, eta_{t+1} = 1 / sqrt(1 + t),
 *     c_{t+1/2} = c_t + (tangent-plane estimate on u + c_t chi_patch),
 *     c_{t+1} = (c_t + c_{t+1/2} + eta_t alpha s f*) / (2 + eta_t alpha s),
 * s = pixels of the patch in the image, f* = their mean of f - u.  The estimate
 * uses the 8 planes of every ring r = 1 .. 2^(j-1) around the patch centre
 * (chords W-E, N-S, NW-SE, NE-SW through the centre, each with either ring
 * pixel perpendicular to it; 2^(j+2) planes on level j): the mean of the
 * signed distances from the centre point to the planes for mean curvature
 * (eq. (c-sol1)), or, for Gaussian curvature, the distance to the plane whose
 * normal curvature d / ds^2 (ds^2 = squared 3-D half chord) is, of the smallest
 * and the largest, the one of smaller magnitude (Proposition 2).  A patch's
 * update reads pixels at most one pixel outside it, so patches of one colour
 * do not interact.  These updates do not minimise F (eq. MCM / GCM) exactly;
 * F is still what mg_fbs_energy reports and the energy stopping rule uses.
 * Buffer conventions, stream semantics and errors are those of mg_curv_*.
 * ------------------------------------------------------------------------ */

typedef struct {
    int32_t height;       /* H >= 2 */
    int32_t width;        /* W >= 2 */
    double alpha;         /* data weight, finite and >= 0 */
    int32_t curvature;    /* mg_curv_kind */
    int32_t levels;       /* J in [1, 16]; the paper's experiments use 3 */
    int32_t state_dtype;  /* mg_dtype of u and f; the updates are computed in FP64 */
    int32_t steps;        /* FBS updates per patch, [1, 64]; 1 is the paper's t = 0 */
    int32_t cycle;        /* 0: levels 1..J (half V-cycle), 1: then J-1..1 (full V-cycle) */
    int32_t reserved;     /* must be 0 */
} mg_fbs_params;

typedef struct mg_fbs_ctx mg_fbs_ctx;

/* Defaults for an H x W image: alpha 20, mean curvature, J = 3, float state,
 * one FBS step, half V-cycle. */
void mg_fbs_default_params(mg_fbs_params *p, int32_t height, int32_t width);

/* Validate, bind the current device and stream, and allocate two H x W state
 * images (level-1 output and the previous iterate for relErr(u)) plus small
 * per-patch tables.  Errors as mg_curv_init. */
mg_status mg_fbs_init(const mg_fbs_params *params, void *hip_stream, mg_fbs_ctx **out);

/* One V-cycle on u (in place); F(u) afterwards into *energy_after if non-null
 * (then the call waits). */
mg_status mg_fbs_vcycle(mg_fbs_ctx *ctx, void *u, const void *f, double *energy_after);

/* All four colours of one level (1-based), in place.  Enqueued only. */
mg_status mg_fbs_level(mg_fbs_ctx *ctx, void *u, const void *f, int32_t level);

/* One colour of one level, in place.  Enqueued only. */
mg_status mg_fbs_sweep(mg_fbs_ctx *ctx, void *u, const void *f, int32_t level, int32_t colour);

/* F(u) of eq. MCM / GCM in FP64 (same kernel and order as mg_curv_energy). */
mg_status mg_fbs_energy(mg_fbs_ctx *ctx, const void *u, const void *f, double *energy);

/* V-cycles until the stopping rule `stop` (mg_stop_rule) holds with tolerance
 * tol, or max_vcycles cycles; tol <= 0 runs exactly max_vcycles.  Outputs as
 * mg_curv_solve (energy_trace holds F before and after every V-cycle).
 * Returns MG_OK, MG_NOT_CONVERGED or an error. */
mg_status mg_fbs_solve(mg_fbs_ctx *ctx, void *u, const void *f, double tol, int32_t max_vcycles, int32_t stop,
                       int32_t *vcycles_done, double *final_energy, double *energy_trace);

/* Release (NULL allowed; waits for the stream first). */
void mg_fbs_destroy(mg_fbs_ctx *ctx);

/* Last error of ctx, or of this thread's last failed mg_fbs_init (ctx NULL). */
const char *mg_fbs_last_error(const mg_fbs_ctx *ctx);

/* ------------------------------------------------------------------------
 * Reconstruction (Section 5): recover u from b = A u + noise by minimising
 *     1/2 ||A u - b||^2 + alpha sum |H(u)|          (H: mean curvature, as above).
 * A is a 5 x 5 Gaussian blur of width blur_sigma, normalised, positions outside
 * the image contributing nothing (the paper's Radon and Fourier operators need
 * data this library does not have; the blur is the operator this path is built
 * and measured with).  Patches of side 2^j - 1 and the four colours as for
 * mg_fbs_*.  For each colour the corrections c of all its patches solve the
 * coupled system of Section 5,
 *     (G + 2 alpha I) c = r,   G_il = <A phi_i, A phi_l>,
 *     r_i = <b - A u, A phi_i> + 2 alpha d_i,
 * d_i the tangent-plane estimate of Proposition 1 for patch i (mean of the
 * signed distances from the patch centre to its 2^(j+2) planes); the system is
 * solved by cg_iters conjugate-gradient iterations in FP64 from c = 0.
 * u and b: device arrays of the state dtype, caller-owned, u must not alias b.
 * ------------------------------------------------------------------------ */

typedef struct {
    int32_t height;       /* H >= 2 */
    int32_t width;        /* W >= 2 */
    double alpha;         /* weight of the curvature term, finite and >= 0 */
    double blur_sigma;    /* width of the Gaussian of A, > 0 */
    int32_t levels;       /* J in [1, 16] */
    int32_t state_dtype;  /* mg_dtype of u and b */
    int32_t cg_iters;     /* CG iterations per colour, [1, 1000] */
    int32_t reserved;     /* must be 0 */
} mg_recon_params;

typedef struct mg_recon_ctx mg_recon_ctx;

/* Defaults: alpha 0.01, blur_sigma 1, J = 3, float state, 20 CG iterations. */
void mg_recon_default_params(mg_recon_params *p, int32_t height, int32_t width);

/* Validate, bind the current device and stream, allocate three H x W FP64
 * images, one state-dtype image and per-patch CG vectors.  Errors as mg_curv_init. */
mg_status mg_recon_init(const mg_recon_params *params, void *hip_stream, mg_recon_ctx **out);

/* One colour of one level, in place (enqueued only). */
mg_status mg_recon_sweep(mg_recon_ctx *ctx, void *u, const void *b, int32_t level, int32_t colour);

/* One V-cycle (levels 1..J, four colours each), replayed from a graph captured
 * once per (u, b); the energy afterwards into *energy_after if non-null (waits). */
mg_status mg_recon_vcycle(mg_recon_ctx *ctx, void *u, const void *b, double *energy_after);

/* 1/2 ||A u - b||^2 + alpha sum |H(u)| in FP64. */
mg_status mg_recon_energy(mg_recon_ctx *ctx, const void *u, const void *b, double *energy);

/* V-cycles until ||u_l - u_{l-1}||_2 < tol ||u_l||_2 (Section 4's relErr(u)) or
 * max_vcycles; outputs nullable.  MG_OK, MG_NOT_CONVERGED or an error. */
mg_status mg_recon_solve(mg_recon_ctx *ctx, void *u, const void *b, double tol, int32_t max_vcycles,
                         int32_t *vcycles_done, double *final_energy);

void mg_recon_destroy(mg_recon_ctx *ctx);
const char *mg_recon_last_error(const mg_recon_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MGCURV_H */
