/* Sanitizer run of the C oracle (address and undefined-behaviour checks, CPU only): solves,
 * every local solve of every block of every level, sweeps with their correction grids, and the
 * FBS path, on ragged images down to 2 x 2, both curvatures, both block schedules, both cycle
 * shapes, four and nine fine colours, the float-state option, one and four threads.  The
 * parameter records repeat the oracle's layouts (the oracle has no header). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int32_t height, width;
    double alpha;
    int32_t kind, levels, fine_colours, samples, bisections, round_f32, threads, cycle, schedule;
} orc_params;

typedef struct {
    double s, fs, K0, Kf, rho, c_sample, c_bisect, c_tilde, delta, c;
    int32_t istar, accepted;
} orc_solve_info;

typedef struct {
    int32_t height, width;
    double alpha;
    int32_t kind, levels, steps, cycle, round_f32, threads;
} fbs_params;

double orc_energy(int kind, const double *u, const double *f, int H, int W, double alpha);
double orc_local_solve(const orc_params *P, const double *u, const double *f, int r0, int r1, int c0, int c1,
                       orc_solve_info *info);
int orc_block_side(const orc_params *P, int level);
int orc_num_colours(const orc_params *P, int level);
int orc_sweep(const orc_params *P, double *u, const double *f, int level, int colour, double *cbuf);
int orc_solve_rule(const orc_params *P, double *u, const double *f, double tol, int max_vcycles, int stop,
                   double *trace);
int fbs_grid_rows(const fbs_params *P, int level);
int fbs_grid_cols(const fbs_params *P, int level);
int fbs_solve(const fbs_params *P, double *u, const double *f, double tol, int max_vcycles, int stop, double *trace);

static double rnd(unsigned *s) { *s = *s * 1664525u + 1013904223u; return (double)(*s >> 8) / 16777216.0; }

static int levels_for(int H, int W)
{
    int m = H > W ? H : W, J = 0;
    while ((1 << J) < m) ++J;
    return J < 1 ? 1 : J;
}

int main(void)
{
    const int shapes[][2] = {{2, 2}, {2, 3}, {3, 2}, {5, 7}, {17, 13}, {24, 20}, {33, 40}};
    unsigned seed = 12345u;
    int runs = 0;
    for (size_t k = 0; k < sizeof shapes / sizeof shapes[0]; ++k) {
        const int H = shapes[k][0], W = shapes[k][1];
        double *f = malloc(sizeof(double) * H * W), *u = malloc(sizeof(double) * H * W);
        double trace[8];
        for (int t = 0; t < H * W; ++t) f[t] = (t % 7 < 3 ? 0.2 : 0.7) + 0.1 * (rnd(&seed) - 0.5);
        for (int kind = 0; kind < 2; ++kind)
            for (int sched = 0; sched < 2; ++sched)
                for (int cycle = 0; cycle < 2; ++cycle)
                    for (int col = 4; col <= 9; col += 5)
                        for (int rf = 0; rf < 2; ++rf) {
                            orc_params P = {H, W, 20.0, kind, levels_for(H, W), col, 16, 32, rf,
                                            (k & 1) ? 4 : 1, cycle, sched};
                            for (int t = 0; t < H * W; ++t) u[t] = f[t];
                            orc_solve_rule(&P, u, f, 0.0, 2, (k + kind) & 1, trace);
                            for (int level = 1; level <= P.levels; ++level) {
                                const int b = orc_block_side(&P, level);
                                const int mj = (H + b - 1) / b, nj = (W + b - 1) / b;
                                double *cb = malloc(sizeof(double) * mj * nj);
                                for (int p = 0; p < mj; ++p)
                                    for (int q = 0; q < nj; ++q) {
                                        orc_solve_info info;
                                        const int r1 = (p + 1) * b < H ? (p + 1) * b : H;
                                        const int c1 = (q + 1) * b < W ? (q + 1) * b : W;
                                        orc_local_solve(&P, u, f, p * b, r1, q * b, c1, &info);
                                        if (!isfinite(info.c)) { printf("non-finite c\n"); return 1; }
                                    }
                                for (int c = 0; c < orc_num_colours(&P, level); ++c) orc_sweep(&P, u, f, level, c, cb);
                                free(cb);
                            }
                            if (!isfinite(orc_energy(kind, u, f, H, W, 20.0))) { printf("non-finite F\n"); return 1; }
                            ++runs;
                        }
        for (int kind = 0; kind < 2; ++kind)
            for (int cycle = 0; cycle < 2; ++cycle)
                for (int levels = 1; levels <= 3; ++levels) {
                    fbs_params Q = {H, W, 0.05, kind, levels, 1 + cycle, cycle, 0, (k & 1) ? 4 : 1};
                    for (int t = 0; t < H * W; ++t) u[t] = 255.0 * f[t];
                    for (int t = 0; t < H * W; ++t) f[t] *= 255.0;
                    fbs_solve(&Q, u, f, 0.0, 2, 1, trace);
                    for (int t = 0; t < H * W; ++t) f[t] /= 255.0;
                    ++runs;
                }
        free(f);
        free(u);
    }
    printf("sanitized runs %d\n", runs);
    return 0;
}
