/*
 * fbs_oracle.c -- plain FP64 CPU oracle of the paper's own local step for the
 * multigrid curvature minimisation of arXiv 2204.07921: one or more
 * forward-backward splitting (FBS) updates per block (Algorithm 2) whose
 * forward step is the tangent-plane estimate of Proposition 1 (mean
 * curvature, eq. (c-sol1)) or Proposition 2 (Gaussian curvature), and whose
 * backward step is the closed form eq. (c-sol2) / its block form in
 * Section 2.2.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP implementation.
 *
 * What it computes, with the passage each part follows (readings named R..):
 *
 *  - blocks (Section 2.2): on level j = 1..J the image is cut into patches of
 *    side b_j = 2^j - 1 anchored at the top-left pixel, m_j = ceil(m / b_j)
 *    rows and n_j = ceil(n / b_j) columns of them, clipped at the right and
 *    bottom edges.  The image is prolonged by replicating its edge pixels, so
 *    every patch is complete and has a centre pixel at offset (b_j - 1) / 2
 *    (reading R16: positions outside the image take the value of the nearest
 *    image pixel);
 *  - colours (Section 2.3): colour of patch (p, q) is 2 (p mod 2) + (q mod 2),
 *    colours visited in the order 0, 1, 2, 3.  A patch's update reads pixels at
 *    most one pixel outside the patch, so patches of one colour do not
 *    interact and the order inside a colour is irrelevant;
 *  - tangent planes (Figs. 2-3 are missing; reading R17): on ring r = 1..2^(j-1)
 *    around the patch centre O the eight pixels at offsets r (di, dj),
 *    di, dj in {-1, 0, 1}, give four lines through O (W-E, N-S, NW-SE, NE-SW),
 *    and each line with either of the two ring pixels perpendicular to it
 *    spans a triangle plane: 8 planes per ring, iota = 8 * 2^(j-1) = 2^(j+2)
 *    planes on level j, as Section 2.2 counts them;
 *  - distance (eq. (distance to tri)): the signed distance from the centre
 *    point (O, u_O) of the surface to a plane through three surface points,
 *    positive when the plane lies above the centre point;
 *  - mean curvature (Proposition 1, eq. (c-sol1)): the forward estimate is the
 *    mean of the iota distances;
 *  - Gaussian curvature (Section 3, Proposition 2): normal curvature of plane l
 *    is kappa_l = d_l / ds_l^2, with ds_l^2 the squared length of the half
 *    chord of the plane's line in 3-D (reading R18); kappa_min / kappa_max are
 *    the first minimum / first maximum in plane order, the one of smaller
 *    magnitude (kappa_min on a tie) selects the plane T*, and the forward
 *    estimate is the distance d* to T*;
 *  - FBS (Algorithm 2): c_0 = 0, eta_0 = 1, eta_{t+1} = 1 / sqrt(1 + t); the
 *    forward estimate at step t is taken on the state with the patch shifted
 *    by c_t, c_{t+1/2} = c_t + estimate (reading R19), and the backward step is
 *    c_{t+1} = (c_t + c_{t+1/2} + eta_t alpha s f*) / (2 + eta_t alpha s) with
 *    s = number of image pixels in the patch and f* = mean of f - u over them;
 *    `steps` updates are made (the paper uses one, t = 0, in Section 2.1's
 *    remark, and 15 in its later study);
 *  - V-cycle (Section 2.2): levels 1..J fine to coarse (the half V-cycle the
 *    paper prefers) or, with cycle = 1, back again J-1..1;
 *  - stopping (Section 4): relative energy change, or relErr(u) =
 *    ||u_l - u_{l-1}||_2 / ||u_l||_2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FBS_MC 0
#define FBS_GC 1

typedef struct {
    int32_t height, width;
    double alpha;
    int32_t kind;       /* 0 mean curvature, 1 Gaussian curvature */
    int32_t levels;     /* J; patch side on level j (1-based) is 2^j - 1 */
    int32_t steps;      /* FBS updates per patch (>= 1) */
    int32_t cycle;      /* 0 fine-to-coarse, 1 fine-to-coarse-to-fine */
    int32_t round_f32;  /* 1: round the state to float after each update */
    int32_t threads;    /* OpenMP threads for the per-colour patch loop */
} fbs_params;

/* defined in mgc_oracle.c (same library): F(u) of eq. (MCM) / eq. (GCM) */
double orc_energy(int kind, const double *u, const double *f, int H, int W, double alpha);

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

int fbs_block_side(int level) { return (1 << level) - 1; }
int fbs_rings(int level) { return 1 << (level - 1); }
int fbs_grid_rows(const fbs_params *P, int level)
{
    int b = fbs_block_side(level);
    return (P->height + b - 1) / b;
}
int fbs_grid_cols(const fbs_params *P, int level)
{
    int b = fbs_block_side(level);
    return (P->width + b - 1) / b;
}
int fbs_colour(int p, int q) { return 2 * (p % 2) + (q % 2); }

typedef struct {
    int r0, r1, c0, c1;   /* image pixels of the patch: rows [r0, r1), columns [c0, c1) */
    int oi, oj;           /* centre position in the prolonged domain */
} patch;

static patch make_patch(const fbs_params *P, int level, int p, int q)
{
    patch B;
    int b = fbs_block_side(level);
    B.r0 = p * b;
    B.r1 = B.r0 + b < P->height ? B.r0 + b : P->height;
    B.c0 = q * b;
    B.c1 = B.c0 + b < P->width ? B.c0 + b : P->width;
    B.oi = B.r0 + (b - 1) / 2;
    B.oj = B.c0 + (b - 1) / 2;
    return B;
}

/* value of the state u + c chi_B at a position of the prolonged domain */
static double value_at(const fbs_params *P, const double *u, const patch *B, double c, int i, int j)
{
    int ci = clampi(i, 0, P->height - 1), cj = clampi(j, 0, P->width - 1);
    double v = u[(size_t)ci * P->width + cj];
    if (ci >= B->r0 && ci < B->r1 && cj >= B->c0 && cj < B->c1) v += c;
    return v;
}

/* the plane enumeration of one ring: line ends a, b and third vertex t as unit offsets */
static const int LINE_A[4][2] = {{0, -1}, {-1, 0}, {-1, -1}, {-1, 1}};
static const int THIRD[4][2][2] = {
    {{-1, 0}, {1, 0}},    /* W-E with N, S */
    {{0, -1}, {0, 1}},    /* N-S with W, E */
    {{-1, 1}, {1, -1}},   /* NW-SE with NE, SW */
    {{-1, -1}, {1, 1}},   /* NE-SW with NW, SE */
};

/*
 * Plane k (0..7) of ring r around the patch centre on the state u + c chi_B:
 * d = signed distance from the centre point to the plane through the three
 * surface points (positive when the plane is above it), ds2 = squared 3-D
 * length of half the plane's line (the chord through the centre).
 * Geometry from the definitions: normal n = (b - a) x (t - a) oriented
 * upwards, d = (a - o) . n / |n|.
 */
void fbs_plane(const fbs_params *P, const double *u, int level, int p, int q, double c, int r, int k,
               double *d, double *ds2)
{
    patch B = make_patch(P, level, p, q);
    int line = k / 2, side = k % 2;
    double a[3], b[3], t[3], o[3];
    a[0] = r * LINE_A[line][0];
    a[1] = r * LINE_A[line][1];
    b[0] = -a[0];
    b[1] = -a[1];
    t[0] = r * THIRD[line][side][0];
    t[1] = r * THIRD[line][side][1];
    o[0] = 0.0;
    o[1] = 0.0;
    a[2] = value_at(P, u, &B, c, B.oi + (int)a[0], B.oj + (int)a[1]);
    b[2] = value_at(P, u, &B, c, B.oi + (int)b[0], B.oj + (int)b[1]);
    t[2] = value_at(P, u, &B, c, B.oi + (int)t[0], B.oj + (int)t[1]);
    o[2] = value_at(P, u, &B, c, B.oi, B.oj);
    double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double e2[3] = {t[0] - a[0], t[1] - a[1], t[2] - a[2]};
    double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    if (n[2] < 0.0) {
        n[0] = -n[0];
        n[1] = -n[1];
        n[2] = -n[2];
    }
    double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    *d = ((a[0] - o[0]) * n[0] + (a[1] - o[1]) * n[1] + (a[2] - o[2]) * n[2]) / len;
    *ds2 = 0.25 * (e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
}

/* number of planes on a level: 8 per ring */
int fbs_planes(int level) { return 8 * fbs_rings(level); }

/* forward estimate on the state u + c chi_B: Proposition 1 (mean) or 2 (Gaussian) */
double fbs_estimate(const fbs_params *P, const double *u, int level, int p, int q, double c)
{
    int R = fbs_rings(level);
    if (P->kind == FBS_MC) {
        double acc = 0.0;
        for (int r = 1; r <= R; ++r)
            for (int k = 0; k < 8; ++k) {
                double d, ds2;
                fbs_plane(P, u, level, p, q, c, r, k, &d, &ds2);
                acc += d;
            }
        return acc / (double)(8 * R);
    }
    double kmin = 0.0, kmax = 0.0, dmin = 0.0, dmax = 0.0;
    int first = 1;
    for (int r = 1; r <= R; ++r)
        for (int k = 0; k < 8; ++k) {
            double d, ds2;
            fbs_plane(P, u, level, p, q, c, r, k, &d, &ds2);
            double kap = d / ds2;
            if (first || kap < kmin) { kmin = kap; dmin = d; }
            if (first || kap > kmax) { kmax = kap; dmax = d; }
            first = 0;
        }
    return fabs(kmin) <= fabs(kmax) ? dmin : dmax;
}

/*
 * Correction of patch (p, q) on level j from the state u (Algorithm 2).
 * trace (optional, 3 * steps doubles): per step c_t, c_{t+1/2}, eta_t.
 * info (optional, 2 doubles): s and f*.
 */
double fbs_block_step(const fbs_params *P, const double *u, const double *f, int level, int p, int q,
                      double *trace, double *info)
{
    patch B = make_patch(P, level, p, q);
    const int W = P->width;
    double acc = 0.0;
    for (int i = B.r0; i < B.r1; ++i)
        for (int j = B.c0; j < B.c1; ++j) acc += f[(size_t)i * W + j] - u[(size_t)i * W + j];
    const double s = (double)((B.r1 - B.r0) * (B.c1 - B.c0));
    const double fs = acc / s;
    if (info) {
        info[0] = s;
        info[1] = fs;
    }
    double c = 0.0, eta = 1.0;
    for (int t = 0; t < P->steps; ++t) {
        double half = c + fbs_estimate(P, u, level, p, q, c);
        double w = eta * P->alpha * s;
        double next = (c + half + w * fs) / (2.0 + w);
        if (trace) {
            trace[3 * t] = c;
            trace[3 * t + 1] = half;
            trace[3 * t + 2] = eta;
        }
        c = next;
        eta = 1.0 / sqrt(1.0 + (double)t);
    }
    return c;
}

/*
 * One colour sweep of level j: every patch of the colour computes its c from
 * the state at the start of the sweep, then all are applied.  cbuf
 * (optional, m_j * n_j doubles) receives c per patch (0 for other colours).
 * Returns the number of patches of the colour.
 */
int fbs_sweep(const fbs_params *P, double *u, const double *f, int level, int colour, double *cbuf)
{
    const int mj = fbs_grid_rows(P, level), nj = fbs_grid_cols(P, level);
    double *c = (double *)calloc((size_t)mj * nj, sizeof(double));
    int count = 0;
#pragma omp parallel for schedule(dynamic, 16) num_threads(P->threads > 0 ? P->threads : 1) reduction(+ : count)
    for (int blk = 0; blk < mj * nj; ++blk) {
        int p = blk / nj, q = blk % nj;
        if (fbs_colour(p, q) != colour) continue;
        c[blk] = fbs_block_step(P, u, f, level, p, q, NULL, NULL);
        ++count;
    }
    for (int blk = 0; blk < mj * nj; ++blk) {
        int p = blk / nj, q = blk % nj;
        if (fbs_colour(p, q) != colour || c[blk] == 0.0) continue;
        patch B = make_patch(P, level, p, q);
        for (int i = B.r0; i < B.r1; ++i)
            for (int j = B.c0; j < B.c1; ++j) {
                double v = u[(size_t)i * P->width + j] + c[blk];
                u[(size_t)i * P->width + j] = P->round_f32 ? (double)(float)v : v;
            }
    }
    if (cbuf) memcpy(cbuf, c, sizeof(double) * (size_t)mj * nj);
    free(c);
    return count;
}

void fbs_level(const fbs_params *P, double *u, const double *f, int level)
{
    for (int colour = 0; colour < 4; ++colour) fbs_sweep(P, u, f, level, colour, NULL);
}

void fbs_vcycle(const fbs_params *P, double *u, const double *f)
{
    for (int j = 1; j <= P->levels; ++j) fbs_level(P, u, f, j);
    if (P->cycle == 1)
        for (int j = P->levels - 1; j >= 1; --j) fbs_level(P, u, f, j);
}

/*
 * V-cycles until the stopping rule holds or max_vcycles are done.
 * stop = 0: |E_l - E_{l-1}| < tol |E_l| (energy of eq. (MCM) / (GCM));
 * stop = 1: ||u_l - u_{l-1}||_2 < tol ||u_l||_2.
 * trace (optional, max_vcycles + 1 doubles): energy before and after every
 * V-cycle.  Returns the number of V-cycles done.
 */
int fbs_solve(const fbs_params *P, double *u, const double *f, double tol, int max_vcycles, int stop, double *trace)
{
    const int H = P->height, W = P->width;
    const size_t n = (size_t)H * W;
    double *prev = (double *)malloc(sizeof(double) * n);
    double e = orc_energy(P->kind, u, f, H, W, P->alpha);
    if (trace) trace[0] = e;
    int done = 0;
    while (done < max_vcycles) {
        memcpy(prev, u, sizeof(double) * n);
        fbs_vcycle(P, u, f);
        ++done;
        double e_new = orc_energy(P->kind, u, f, H, W, P->alpha);
        if (trace) trace[done] = e_new;
        int stop_now;
        if (stop == 0) {
            stop_now = fabs(e_new - e) < tol * fabs(e_new);
        } else {
            double num = 0.0, den = 0.0;
            for (size_t k = 0; k < n; ++k) {
                num += (u[k] - prev[k]) * (u[k] - prev[k]);
                den += u[k] * u[k];
            }
            stop_now = sqrt(num) < tol * sqrt(den);
        }
        e = e_new;
        if (stop_now) break;
    }
    free(prev);
    return done;
}
