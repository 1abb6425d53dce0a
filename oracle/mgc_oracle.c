/*
 * mgc_oracle.c -- plain FP64 CPU oracle for the multigrid curvature-energy
 * minimisation of arXiv 2204.07921 (Pan, Duan, ... "Fast multi-grid methods for
 * minimizing curvature energies").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP implementation.
 *
 * What it computes, with the passage each part follows:
 *
 *  - curvature of the image graph (Table 1): mean curvature as the divergence
 *    of grad u / sqrt(1 + |grad u|^2) and Gaussian curvature as
 *    det(Hess u) / (1 + |grad u|^2)^2, discretised with 3x3 central differences
 *    (the paper gives no stencil; reading R1) and replicated ghost pixels
 *    outside the image (the paper only says the domain is prolonged by
 *    boundary conditions, Section 2.2; reading R3);
 *  - the discrete energy F(u) = sum |kappa(u)| + alpha/2 (u - f)^2 of
 *    eq. (MCM) and eq. (GCM);
 *  - the block hierarchy of Section 2.2, blocks clipped at the right and
 *    bottom edges, with block side b_j = 2^(j-1) (schedule 0, reading R4:
 *    nested blocks) or the paper's b_j = 2^j - 1 (schedule 1, Section 2.2's
 *    patch side, m_j = ceil(m / (2^j - 1)) blocks along a side of m pixels);
 *  - the four-colour decomposition of Section 2.3 (colour of block (p, q) is
 *    2 (p mod 2) + (q mod 2), colours visited in the order 0, 1, 2, 3);
 *  - Algorithm 3: fine-to-coarse half V-cycle (or, with cycle = 1, the full
 *    V-cycle that Section 2.2 compares it with: back again J-1..1); inside each colour every block
 *    B receives u <- u + c_B chi_B where c_B minimises the local energy
 *    F(u + c chi_B) (the arg min of the algorithm's inner step).  All c_B of
 *    one colour are computed from the state at the start of the colour and
 *    then applied together (reading R7).
 *
 * The one-dimensional minimisation is not specified by the paper for the
 * discrete energy (it uses a forward-backward splitting step instead); the
 * local solver here follows reading R8:
 *     s = |B|, f* = sum_B (f - u) / s,
 *     K(c) = sum over ring pixels of |kappa_p(u + c chi_B)|,
 *     V(c) = K(c) + alpha s / 2 (c - f*)^2   (= F(u + c chi_B) + const),
 *     rho = sqrt(2 K(f*) / (alpha s))        (every global minimiser of V
 *                                             lies in [f* - rho, f* + rho]),
 *     sample c_i = f* + rho (2 i - M) / M, i = 0..M; i* = first arg min V(c_i),
 *     bisection on the sign of V'(c) in [c_{i*-1}, c_{i*+1}] for G steps,
 *     choose the bisection point unless the best sample is lower by more than
 *     eta = 1e-12 (1 + V(0)), and accept the chosen point only when it lowers
 *     the local energy by more than eta (Delta < -eta): c = 0 is always a
 *     candidate of the arg min and wins every tie that rounding cannot resolve
 *     (eta bounds the rounding of the computed Delta, a difference of two ring
 *     sums), so an applied block update lowers F.
 *
 * The ring of a block B is the set of pixels p in the image whose clamped 3x3
 * tap set holds at least one tap in B and one tap outside B; every other
 * pixel's curvature does not depend on c.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MC 0
#define ORC_GC 1

typedef struct {
    int32_t height, width;
    double alpha;
    int32_t kind;          /* 0 mean curvature, 1 Gaussian curvature */
    int32_t levels;        /* J; block side at level j (1-based): see orc_block_side */
    int32_t fine_colours;  /* 4 (paper) or 9 (exactly non-interacting at b = 1) */
    int32_t samples;       /* M, even */
    int32_t bisections;    /* G */
    int32_t round_f32;     /* 1: round the state to float after each update */
    int32_t threads;       /* OpenMP threads for the per-colour block loop */
    int32_t cycle;         /* 0: levels 1..J (the half V-cycle of Algorithm 3); 1: then J-1..1 */
    int32_t schedule;      /* block side at level j: 0 -> 2^(j-1), 1 -> 2^j - 1 (Section 2.2) */
} orc_params;

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ------------------------------------------------------------------------ */
/* Table 1 curvatures from a 3x3 tap window t[row][col], row 0 = north       */
/* (i - 1), col 0 = west (j - 1); grid spacing h.                            */
/* ------------------------------------------------------------------------ */
static double curvature_taps(int kind, const double t[3][3], double h)
{
    double ux = (t[1][2] - t[1][0]) / (2.0 * h);
    double uy = (t[2][1] - t[0][1]) / (2.0 * h);
    double uxx = (t[1][2] - 2.0 * t[1][1] + t[1][0]) / (h * h);
    double uyy = (t[2][1] - 2.0 * t[1][1] + t[0][1]) / (h * h);
    double uxy = (t[2][2] - t[0][2] - t[2][0] + t[0][0]) / (4.0 * h * h);
    double q = 1.0 + ux * ux + uy * uy;
    if (kind == ORC_MC) {
        /* div( grad u / sqrt(1 + |grad u|^2) ) expanded */
        double num = (1.0 + uy * uy) * uxx - 2.0 * ux * uy * uxy + (1.0 + ux * ux) * uyy;
        return num / pow(q, 1.5);
    }
    return (uxx * uyy - uxy * uxy) / (q * q);
}

/* d kappa / d c when each tap value moves by m[r][k] * c (m = 1 for taps in
 * the block, 0 otherwise); same grid spacing h. */
static double curvature_taps_dc(int kind, const double t[3][3], const double m[3][3], double h)
{
    double ux = (t[1][2] - t[1][0]) / (2.0 * h);
    double uy = (t[2][1] - t[0][1]) / (2.0 * h);
    double uxx = (t[1][2] - 2.0 * t[1][1] + t[1][0]) / (h * h);
    double uyy = (t[2][1] - 2.0 * t[1][1] + t[0][1]) / (h * h);
    double uxy = (t[2][2] - t[0][2] - t[2][0] + t[0][0]) / (4.0 * h * h);
    double dux = (m[1][2] - m[1][0]) / (2.0 * h);
    double duy = (m[2][1] - m[0][1]) / (2.0 * h);
    double duxx = (m[1][2] - 2.0 * m[1][1] + m[1][0]) / (h * h);
    double duyy = (m[2][1] - 2.0 * m[1][1] + m[0][1]) / (h * h);
    double duxy = (m[2][2] - m[0][2] - m[2][0] + m[0][0]) / (4.0 * h * h);
    double q = 1.0 + ux * ux + uy * uy;
    double dq = 2.0 * ux * dux + 2.0 * uy * duy;
    if (kind == ORC_MC) {
        double num = (1.0 + uy * uy) * uxx - 2.0 * ux * uy * uxy + (1.0 + ux * ux) * uyy;
        double dnum = 2.0 * uy * duy * uxx + (1.0 + uy * uy) * duxx
                    - 2.0 * (dux * uy * uxy + ux * duy * uxy + ux * uy * duxy)
                    + 2.0 * ux * dux * uyy + (1.0 + ux * ux) * duyy;
        /* kappa = num q^{-3/2} */
        return dnum / pow(q, 1.5) - 1.5 * num * dq / pow(q, 2.5);
    }
    {
        double det = uxx * uyy - uxy * uxy;
        double ddet = duxx * uyy + uxx * duyy - 2.0 * uxy * duxy;
        /* kappa = det q^{-2} */
        return ddet / (q * q) - 2.0 * det * dq / (q * q * q);
    }
}

/* Gather the clamped 3x3 taps of pixel (i, j) of u (H x W, row-major). */
static void gather(const double *u, int H, int W, int i, int j, double t[3][3])
{
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx)
            t[dy + 1][dx + 1] = u[(size_t)clampi(i + dy, 0, H - 1) * W + clampi(j + dx, 0, W - 1)];
}

double orc_curvature_at(int kind, const double *u, int H, int W, int i, int j, double h)
{
    double t[3][3];
    gather(u, H, W, i, j, t);
    return curvature_taps(kind, t, h);
}

void orc_curvature_map(int kind, const double *u, int H, int W, double h, double *out)
{
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j)
            out[(size_t)i * W + j] = orc_curvature_at(kind, u, H, W, i, j, h);
}

/* eq. (MCM) / eq. (GCM): F(u) = sum_pixels |kappa(u)| + alpha/2 (u - f)^2,
 * summed in row-major order. */
double orc_energy(int kind, const double *u, const double *f, int H, int W, double alpha)
{
    double e = 0.0;
    for (int i = 0; i < H; ++i)
        for (int j = 0; j < W; ++j) {
            double d = u[(size_t)i * W + j] - f[(size_t)i * W + j];
            e += fabs(orc_curvature_at(kind, u, H, W, i, j, 1.0)) + 0.5 * alpha * d * d;
        }
    return e;
}

/* ------------------------------------------------------------------------ */
/* Local (one block) quantities.  Block B = rows [r0, r1) x cols [c0, c1).   */
/* ------------------------------------------------------------------------ */
static int in_block(int i, int j, int r0, int r1, int c0, int c1)
{
    return i >= r0 && i < r1 && j >= c0 && j < c1;
}

/* Taps of pixel (i, j) in u + c chi_B, and the mask of taps that lie in B.
 * Returns the number of the 9 tap positions that lie in B. */
static int shifted_taps(const double *u, int H, int W, int i, int j,
                        int r0, int r1, int c0, int c1, double c,
                        double t[3][3], double m[3][3])
{
    int n = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            int ci = clampi(i + dy, 0, H - 1), cj = clampi(j + dx, 0, W - 1);
            int inb = in_block(ci, cj, r0, r1, c0, c1);
            t[dy + 1][dx + 1] = u[(size_t)ci * W + cj] + (inb ? c : 0.0);
            m[dy + 1][dx + 1] = inb ? 1.0 : 0.0;
            n += inb;
        }
    return n;
}

/* K(c) = sum over the ring R(B) of |kappa_p(u + c chi_B)|. */
double orc_ring_K(int kind, const double *u, int H, int W, int r0, int r1, int c0, int c1, double c)
{
    double acc = 0.0;
    for (int i = r0 - 1; i <= r1; ++i) {
        if (i < 0 || i >= H) continue;
        for (int j = c0 - 1; j <= c1; ++j) {
            if (j < 0 || j >= W) continue;
            double t[3][3], m[3][3];
            int n = shifted_taps(u, H, W, i, j, r0, r1, c0, c1, c, t, m);
            if (n == 0 || n == 9) continue;
            acc += fabs(curvature_taps(kind, t, 1.0));
        }
    }
    return acc;
}

/* K at n points (brute-force pins evaluate many c for one block). */
void orc_ring_K_many(int kind, const double *u, int H, int W, int r0, int r1, int c0, int c1,
                     const double *cs, int n, double *out)
{
    for (int k = 0; k < n; ++k)
        out[k] = orc_ring_K(kind, u, H, W, r0, r1, c0, c1, cs[k]);
}

/* K'(c): sum over the ring of sign(kappa_p) d kappa_p / d c, sign(0) = 0. */
double orc_ring_dK(int kind, const double *u, int H, int W, int r0, int r1, int c0, int c1, double c)
{
    double acc = 0.0;
    for (int i = r0 - 1; i <= r1; ++i) {
        if (i < 0 || i >= H) continue;
        for (int j = c0 - 1; j <= c1; ++j) {
            if (j < 0 || j >= W) continue;
            double t[3][3], m[3][3];
            int n = shifted_taps(u, H, W, i, j, r0, r1, c0, c1, c, t, m);
            if (n == 0 || n == 9) continue;
            double k = curvature_taps(kind, t, 1.0);
            double s = (k > 0.0) - (k < 0.0);
            acc += s * curvature_taps_dc(kind, t, m, 1.0);
        }
    }
    return acc;
}

/* Number of ring pixels (diagnostics / tests). */
int orc_ring_size(const double *u, int H, int W, int r0, int r1, int c0, int c1)
{
    int cnt = 0;
    for (int i = r0 - 1; i <= r1; ++i) {
        if (i < 0 || i >= H) continue;
        for (int j = c0 - 1; j <= c1; ++j) {
            if (j < 0 || j >= W) continue;
            double t[3][3], m[3][3];
            int n = shifted_taps(u, H, W, i, j, r0, r1, c0, c1, 0.0, t, m);
            if (n != 0 && n != 9) ++cnt;
        }
    }
    return cnt;
}

/* s = |B| and r = sum_B (f - u) in row-major order. */
static void block_data(const double *u, const double *f, int W, int r0, int r1, int c0, int c1,
                       double *s, double *r)
{
    double acc = 0.0;
    for (int i = r0; i < r1; ++i)
        for (int j = c0; j < c1; ++j)
            acc += f[(size_t)i * W + j] - u[(size_t)i * W + j];
    *s = (double)(r1 - r0) * (double)(c1 - c0);
    *r = acc;
}

/* Local energy change Delta(c) = F(u + c chi_B) - F(u), evaluated on the ring:
 * (K(c) - K(0)) + alpha s / 2 (c^2 - 2 c f*). */
double orc_local_delta(const orc_params *P, const double *u, const double *f,
                       int r0, int r1, int c0, int c1, double c)
{
    double s, r;
    block_data(u, f, P->width, r0, r1, c0, c1, &s, &r);
    double fs = r / s;
    double K0 = orc_ring_K(P->kind, u, P->height, P->width, r0, r1, c0, c1, 0.0);
    double Kc = orc_ring_K(P->kind, u, P->height, P->width, r0, r1, c0, c1, c);
    return (Kc - K0) + 0.5 * P->alpha * s * c * (c - 2.0 * fs);
}

/* Output record of one local solve (tests read it through ctypes). */
typedef struct {
    double s, fs, K0, Kf, rho;
    double c_sample;   /* best sample c_{i*} */
    double c_bisect;   /* bisection point */
    double c_tilde;    /* chosen candidate */
    double delta;      /* Delta(c_tilde) */
    double c;          /* returned correction (c_tilde or 0) */
    int32_t istar;
    int32_t accepted;
} orc_solve_info;

/* The local solver of reading R8 for block B; returns c_B. */
double orc_local_solve(const orc_params *P, const double *u, const double *f,
                       int r0, int r1, int c0, int c1, orc_solve_info *info)
{
    const int H = P->height, W = P->width, kind = P->kind, M = P->samples, G = P->bisections;
    const double alpha = P->alpha;
    double s, r;
    block_data(u, f, W, r0, r1, c0, c1, &s, &r);
    const double fs = r / s;
    const double as = alpha * s;
    const double K0 = orc_ring_K(kind, u, H, W, r0, r1, c0, c1, 0.0);
    const double Kf = orc_ring_K(kind, u, H, W, r0, r1, c0, c1, fs);
    const double rho = sqrt(2.0 * Kf / as);
    const double V0 = K0 + 0.5 * as * fs * fs;
    const double eta = 1e-12 * (1.0 + V0);

    double c_tilde, c_best = fs, c_bis = fs;
    int istar = M / 2;
    if (rho == 0.0) {
        /* K(f*) = 0 and V >= 0 = V(f*): f* is a global minimiser. */
        c_tilde = fs;
    } else {
        /* Sample the bracket [f* - rho, f* + rho]. */
        double vbest = 0.0;
        for (int i = 0; i <= M; ++i) {
            double ci = fs + rho * ((double)(2 * i - M) / (double)M);
            double vi = orc_ring_K(kind, u, H, W, r0, r1, c0, c1, ci) + 0.5 * as * (ci - fs) * (ci - fs);
            if (i == 0 || vi < vbest) { vbest = vi; istar = i; }
        }
        c_best = fs + rho * ((double)(2 * istar - M) / (double)M);
        int ilo = istar > 0 ? istar - 1 : 0;
        int ihi = istar < M ? istar + 1 : M;
        double lo = fs + rho * ((double)(2 * ilo - M) / (double)M);
        double hi = fs + rho * ((double)(2 * ihi - M) / (double)M);
        /* Bisection on the sign of V'(c) = K'(c) + alpha s (c - f*). */
        for (int g = 0; g < G; ++g) {
            double mid = 0.5 * (lo + hi);
            double d = orc_ring_dK(kind, u, H, W, r0, r1, c0, c1, mid) + as * (mid - fs);
            if (d > 0.0) hi = mid; else lo = mid;
        }
        c_bis = 0.5 * (lo + hi);
        double vbis = orc_ring_K(kind, u, H, W, r0, r1, c0, c1, c_bis) + 0.5 * as * (c_bis - fs) * (c_bis - fs);
        c_tilde = (vbest < vbis - eta) ? c_best : c_bis;
    }
    double Kt = orc_ring_K(kind, u, H, W, r0, r1, c0, c1, c_tilde);
    double delta = (Kt - K0) + 0.5 * as * c_tilde * (c_tilde - 2.0 * fs);
    int accepted = delta < -eta;
    double c = accepted ? c_tilde : 0.0;
    if (info) {
        info->s = s; info->fs = fs; info->K0 = K0; info->Kf = Kf; info->rho = rho;
        info->c_sample = c_best; info->c_bisect = c_bis; info->c_tilde = c_tilde;
        info->delta = delta; info->c = c; info->istar = istar; info->accepted = accepted;
    }
    return c;
}

/* ------------------------------------------------------------------------ */
/* Level geometry and colour sweeps (Section 2.2-2.3, Algorithm 3).          */
/* ------------------------------------------------------------------------ */
/* Block side at level j (1-based): 2^(j-1) (schedule 0) or 2^j - 1 (schedule 1,
 * the patch side of Section 2.2).  Both give single pixels at j = 1. */
int orc_block_side(const orc_params *P, int level)
{
    return P->schedule == 1 ? (1 << level) - 1 : 1 << (level - 1);
}

int orc_num_colours(const orc_params *P, int level)
{
    return (level == 1 && P->fine_colours == 9) ? 9 : 4;
}

static int colour_of(int ncol, int p, int q)
{
    return ncol == 9 ? 3 * (p % 3) + (q % 3) : 2 * (p % 2) + (q % 2);
}

/* One colour sweep: compute c_B for every block of colour `colour` at `level`
 * from the current u, then add all of them.  If cbuf is non-null it receives
 * c_B at index p * n_j + q (other entries untouched).  Returns the number of
 * blocks of that colour. */
int orc_sweep(const orc_params *P, double *u, const double *f, int level, int colour, double *cbuf)
{
    const int H = P->height, W = P->width, b = orc_block_side(P, level);
    const int mj = (H + b - 1) / b, nj = (W + b - 1) / b;
    const int ncol = orc_num_colours(P, level);
    int nblk = 0;
    for (int p = 0; p < mj; ++p)
        for (int q = 0; q < nj; ++q)
            if (colour_of(ncol, p, q) == colour) ++nblk;
    if (nblk == 0) return 0;
    int *bp = (int *)malloc(sizeof(int) * 2 * (size_t)nblk);
    double *cs = (double *)malloc(sizeof(double) * (size_t)nblk);
    int k = 0;
    for (int p = 0; p < mj; ++p)
        for (int q = 0; q < nj; ++q)
            if (colour_of(ncol, p, q) == colour) { bp[2 * k] = p; bp[2 * k + 1] = q; ++k; }
    const int nt = P->threads > 0 ? P->threads : 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int t = 0; t < nblk; ++t) {
        int p = bp[2 * t], q = bp[2 * t + 1];
        int r0 = p * b, r1 = (p + 1) * b < H ? (p + 1) * b : H;
        int c0 = q * b, c1 = (q + 1) * b < W ? (q + 1) * b : W;
        cs[t] = orc_local_solve(P, u, f, r0, r1, c0, c1, NULL);
    }
    for (int t = 0; t < nblk; ++t) {
        int p = bp[2 * t], q = bp[2 * t + 1];
        int r0 = p * b, r1 = (p + 1) * b < H ? (p + 1) * b : H;
        int c0 = q * b, c1 = (q + 1) * b < W ? (q + 1) * b : W;
        for (int i = r0; i < r1; ++i)
            for (int j = c0; j < c1; ++j) {
                double v = u[(size_t)i * W + j] + cs[t];
                u[(size_t)i * W + j] = P->round_f32 ? (double)(float)v : v;
            }
        if (cbuf) cbuf[(size_t)p * nj + q] = cs[t];
    }
    free(bp);
    free(cs);
    return nblk;
}

static void orc_level(const orc_params *P, double *u, const double *f, int level)
{
    int ncol = orc_num_colours(P, level);
    for (int colour = 0; colour < ncol; ++colour)
        orc_sweep(P, u, f, level, colour, NULL);
}

/* One outer iteration of Algorithm 3: levels 1..J (fine to coarse), all colours;
 * with cycle = 1 the levels J-1..1 follow (the full V-cycle of Section 2.2). */
void orc_vcycle(const orc_params *P, double *u, const double *f)
{
    for (int level = 1; level <= P->levels; ++level) orc_level(P, u, f, level);
    if (P->cycle == 1)
        for (int level = P->levels - 1; level >= 1; --level) orc_level(P, u, f, level);
}

/* Repeat V-cycles from the given u until |E_l - E_{l-1}| / |E_l| < rel_tol
 * (the paper's relative energy-change stop, Section 4; an unchanged energy also
 * stops) or max_vcycles; rel_tol <= 0 runs
 * exactly max_vcycles.  energy_trace (nullable) receives E_0 .. E_done.
 * Returns the number of V-cycles run. */
int orc_solve(const orc_params *P, double *u, const double *f, double rel_tol, int max_vcycles,
              double *energy_trace)
{
    double e_prev = orc_energy(P->kind, u, f, P->height, P->width, P->alpha);
    if (energy_trace) energy_trace[0] = e_prev;
    int l = 0;
    while (l < max_vcycles) {
        orc_vcycle(P, u, f);
        ++l;
        double e = orc_energy(P->kind, u, f, P->height, P->width, P->alpha);
        if (energy_trace) energy_trace[l] = e;
        if (rel_tol > 0.0 && (e == e_prev || fabs(e - e_prev) < rel_tol * fabs(e))) break;
        e_prev = e;
    }
    return l;
}

/* As orc_solve with the stopping rule chosen: stop = 0 the relative energy change
 * above; stop = 1 the relative change of the iterate, ||u_l - u_{l-1}||_2 <
 * tol ||u_l||_2 (the rule of the paper's Tables 2-3, Section 4). */
int orc_solve_rule(const orc_params *P, double *u, const double *f, double tol, int max_vcycles, int stop,
                   double *energy_trace)
{
    if (stop == 0) return orc_solve(P, u, f, tol, max_vcycles, energy_trace);
    const size_t n = (size_t)P->height * P->width;
    double *prev = (double *)malloc(sizeof(double) * n);
    if (energy_trace) energy_trace[0] = orc_energy(P->kind, u, f, P->height, P->width, P->alpha);
    int l = 0;
    while (l < max_vcycles) {
        memcpy(prev, u, sizeof(double) * n);
        orc_vcycle(P, u, f);
        ++l;
        if (energy_trace) energy_trace[l] = orc_energy(P->kind, u, f, P->height, P->width, P->alpha);
        double num = 0.0, den = 0.0;
        for (size_t k = 0; k < n; ++k) {
            num += (u[k] - prev[k]) * (u[k] - prev[k]);
            den += u[k] * u[k];
        }
        if (tol > 0.0 && sqrt(num) < tol * sqrt(den)) break;
    }
    free(prev);
    return l;
}
