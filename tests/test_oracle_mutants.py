"""Mutation check of the oracle pins: each plausible mistake planted in a copy of the
oracle source (a dropped term, a wrong sign or index, a swapped branch) must make
at least one pin in test_oracle_pins.py fail.  Runs on the CPU only."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mgc_oracle.c")
SRC_FBS = os.path.join(ROOT, "oracle", "fbs_oracle.c")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")
PINS_FBS = os.path.join(ROOT, "tests", "test_fbs_oracle_pins.py")

# (name, original text, mutated text); every original must occur in the source.
MUTANTS = [
    ("mc_wrong_pairing", "double num = (1.0 + uy * uy) * uxx - 2.0 * ux * uy * uxy + (1.0 + ux * ux) * uyy;\n        return num",
     "double num = (1.0 + ux * ux) * uxx - 2.0 * ux * uy * uxy + (1.0 + uy * uy) * uyy;\n        return num"),
    ("mc_drop_cross_term", "double num = (1.0 + uy * uy) * uxx - 2.0 * ux * uy * uxy + (1.0 + ux * ux) * uyy;\n        return num",
     "double num = (1.0 + uy * uy) * uxx + (1.0 + ux * ux) * uyy;\n        return num"),
    ("uxy_sign", "double uxy = (t[2][2] - t[0][2] - t[2][0] + t[0][0]) / (4.0 * h * h);\n    double q = 1.0 + ux * ux + uy * uy;\n    if (kind == ORC_MC) {\n        /* div",
     "double uxy = (t[2][2] + t[0][2] - t[2][0] - t[0][0]) / (4.0 * h * h);\n    double q = 1.0 + ux * ux + uy * uy;\n    if (kind == ORC_MC) {\n        /* div"),
    ("mc_power", "return num / pow(q, 1.5);", "return num / pow(q, 1.0);"),
    ("gc_power", "return (uxx * uyy - uxy * uxy) / (q * q);", "return (uxx * uyy - uxy * uxy) / q;"),
    ("gc_det_sign", "return (uxx * uyy - uxy * uxy) / (q * q);", "return (uxx * uyy + uxy * uxy) / (q * q);"),
    ("ring_misses_outer", "double acc = 0.0;\n    for (int i = r0 - 1; i <= r1; ++i) {\n        if (i < 0 || i >= H) continue;\n        for (int j = c0 - 1; j <= c1; ++j) {\n            if (j < 0 || j >= W) continue;\n            double t[3][3], m[3][3];\n            int n = shifted_taps(u, H, W, i, j, r0, r1, c0, c1, c, t, m);\n            if (n == 0 || n == 9) continue;\n            acc += fabs",
     "double acc = 0.0;\n    for (int i = r0; i < r1; ++i) {\n        if (i < 0 || i >= H) continue;\n        for (int j = c0; j < c1; ++j) {\n            if (j < 0 || j >= W) continue;\n            double t[3][3], m[3][3];\n            int n = shifted_taps(u, H, W, i, j, r0, r1, c0, c1, c, t, m);\n            if (n == 0 || n == 9) continue;\n            acc += fabs"),
    ("border_wrap_not_clamp", "t[dy + 1][dx + 1] = u[(size_t)ci * W + cj] + (inb ? c : 0.0);",
     "t[dy + 1][dx + 1] = u[(size_t)ci * W + cj] + ((inb || (ci == i && cj == j)) ? c : 0.0);"),
    ("energy_data_factor", "e += fabs(orc_curvature_at(kind, u, H, W, i, j, 1.0)) + 0.5 * alpha * d * d;",
     "e += fabs(orc_curvature_at(kind, u, H, W, i, j, 1.0)) + alpha * d * d;"),
    ("delta_data_sign", "return (Kc - K0) + 0.5 * P->alpha * s * c * (c - 2.0 * fs);",
     "return (Kc - K0) + 0.5 * P->alpha * s * c * (c + 2.0 * fs);"),
    ("bisection_direction", "if (d > 0.0) hi = mid; else lo = mid;", "if (d > 0.0) lo = mid; else hi = mid;"),
    ("derivative_no_sign", "double s = (k > 0.0) - (k < 0.0);", "double s = 1.0;"),
    ("bracket_too_narrow", "const double rho = sqrt(2.0 * Kf / as);", "const double rho = sqrt(0.05 * Kf / as);"),
    ("mean_not_sum", "const double fs = r / s;", "const double fs = r;"),
    ("no_accept_test", "int accepted = delta < -eta;", "int accepted = 1;"),
    ("accept_within_eta", "int accepted = delta < -eta;", "int accepted = delta < eta;"),
    ("accept_unresolved_tie", "int accepted = delta < -eta;", "int accepted = delta < 0.0;"),
    ("sweep_in_place", "        cs[t] = orc_local_solve(P, u, f, r0, r1, c0, c1, NULL);\n    }",
     "        cs[t] = orc_local_solve(P, u, f, r0, r1, c0, c1, NULL);\n"
     "        for (int i = r0; i < r1; ++i)\n"
     "            for (int j = c0; j < c1; ++j) u[(size_t)i * W + j] += cs[t];\n"
     "        cs[t] = 0.0;\n    }"),
    ("stop_absolute_change", "fabs(e - e_prev) < rel_tol * fabs(e)", "fabs(e - e_prev) < rel_tol"),
    ("stop_against_first_energy", "        if (rel_tol > 0.0 && (e == e_prev || fabs(e - e_prev) < rel_tol * fabs(e))) break;\n        e_prev = e;",
     "        if (rel_tol > 0.0 && (e == e_prev || fabs(e - e_prev) < rel_tol * fabs(e))) break;"),
    ("colour_map", "return ncol == 9 ? 3 * (p % 3) + (q % 3) : 2 * (p % 2) + (q % 2);",
     "return ncol == 9 ? 3 * (p % 3) + (q % 3) : 2 * (q % 2) + (p % 2);"),
    ("schedule_side_pow2", "return P->schedule == 1 ? (1 << level) - 1 : 1 << (level - 1);",
     "return P->schedule == 1 ? (1 << level) : 1 << (level - 1);"),
    ("schedule_level_shift", "return P->schedule == 1 ? (1 << level) - 1 : 1 << (level - 1);",
     "return P->schedule == 1 ? (1 << (level + 1)) - 1 : 1 << (level - 1);"),
]


# Mistakes planted in the FBS oracle (the paper's own local step), caught by its pins.
MUTANTS_FBS = [
    ("fbs_diag_third_vertex", "{{-1, 1}, {1, -1}},   /* NW-SE with NE, SW */", "{{-1, 0}, {1, 0}},   /* NW-SE with NE, SW */"),
    ("fbs_normal_not_oriented", "if (n[2] < 0.0) {", "if (n[2] < -1e300) {"),
    ("fbs_distance_not_normalised", "/ len;\n    *ds2", "/ n[2];\n    *ds2"),
    ("fbs_ds2_factor", "*ds2 = 0.25 * (", "*ds2 = 0.5 * ("),
    ("fbs_ds2_flat", "*ds2 = 0.25 * (e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);",
     "*ds2 = 0.25 * (e1[0] * e1[0] + e1[1] * e1[1]);"),
    ("fbs_gc_larger_magnitude", "return fabs(kmin) <= fabs(kmax) ? dmin : dmax;", "return fabs(kmin) >= fabs(kmax) ? dmin : dmax;"),
    ("fbs_mc_mean_over_one_ring", "return acc / (double)(8 * R);", "return acc / 8.0;"),
    ("fbs_rings_short", "for (int r = 1; r <= R; ++r)\n            for (int k = 0; k < 8; ++k) {\n                double d, ds2;\n                fbs_plane(P, u, level, p, q, c, r, k, &d, &ds2);\n                acc",
     "for (int r = 1; r < R || r == 1; ++r)\n            for (int k = 0; k < 8; ++k) {\n                double d, ds2;\n                fbs_plane(P, u, level, p, q, c, r, k, &d, &ds2);\n                acc"),
    ("fbs_eta_schedule", "eta = 1.0 / sqrt(1.0 + (double)t);", "eta = 1.0 / sqrt(2.0 + (double)t);"),
    ("fbs_one_proximal_term", "double next = (c + half + w * fs) / (2.0 + w);", "double next = (half + w * fs) / (1.0 + w);"),
    ("fbs_half_not_shifted", "double half = c + fbs_estimate(", "double half = fbs_estimate("),
    ("fbs_estimate_unshifted_state", "double half = c + fbs_estimate(P, u, level, p, q, c);", "double half = c + fbs_estimate(P, u, level, p, q, 0.0);"),
    ("fbs_sum_not_mean", "const double fs = acc / s;", "const double fs = acc;"),
    ("fbs_centre_offset", "B.oi = B.r0 + (b - 1) / 2;", "B.oi = B.r0 + (b + 1) / 2;"),
    ("fbs_colour_map", "int fbs_colour(int p, int q) { return 2 * (p % 2) + (q % 2); }",
     "int fbs_colour(int p, int q) { return 2 * (q % 2) + (p % 2); }"),
    ("fbs_wrap_not_clamp", "int ci = clampi(i, 0, P->height - 1), cj", "int ci = (i + P->height) % P->height, cj"),
    ("fbs_block_side", "int fbs_block_side(int level) { return (1 << level) - 1; }",
     "int fbs_block_side(int level) { return 1 << (level - 1); }"),
]


def _build_mutant(tmp, name, old, new, src_path=SRC):
    src = open(src_path).read()
    assert old in src, name
    path_c = os.path.join(tmp, name + ".c")
    with open(path_c, "w") as fh:
        fh.write(src.replace(old, new, 1))
    others = [p for p in (SRC, SRC_FBS) if p != src_path]
    path_so = os.path.join(tmp, name + ".so")
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           path_c, *others, "-o", path_so, "-lm"])
    return path_so


def _run_pins(so, pins=PINS):
    env = dict(os.environ, MGC_ORACLE_LIB=so)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", pins],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    return r.returncode


def test_every_planted_mistake_is_caught():
    with tempfile.TemporaryDirectory() as tmp:
        jobs = [(m[0], _build_mutant(tmp, *m), PINS) for m in MUTANTS]
        jobs += [(m[0], _build_mutant(tmp, *m, src_path=SRC_FBS), PINS_FBS) for m in MUTANTS_FBS]
        with ThreadPoolExecutor(max_workers=6) as ex:
            codes = list(ex.map(lambda x: _run_pins(x[1], x[2]), jobs))
    survivors = [name for (name, _, _), code in zip(jobs, codes) if code == 0]
    assert not survivors, f"pins did not catch: {survivors}"
