"""ctypes front end of the FP64 C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mgc_oracle.c")
_SRC_FBS = os.path.join(_HERE, "fbs_oracle.c")
SOURCES = (_SRC, _SRC_FBS)


def lib_path() -> str:
    # MGC_ORACLE_LIB lets the mutation test load a deliberately broken build.
    return os.environ.get("MGC_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")


def build(force: bool = True, out: str | None = None, native: bool = False) -> str:
    """Compile the oracle library with gcc (FP64, OpenMP; no fast-math, no FMA contraction, so the
    results do not depend on the flags): -O2 for the portable build the tests load, or
    -O3 -march=native for a copy timed on the machine that builds it (out = its path)."""
    out = out or lib_path()
    if force or _stale(out):
        tmp = out + ".tmp"
        opt = ["-O3", "-march=native"] if native else ["-O2"]
        subprocess.check_call(["gcc", *opt, "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-fno-fast-math", "-ffp-contract=off", *SOURCES, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


def _stale(out: str) -> bool:
    return not os.path.exists(out) or any(os.path.getmtime(out) < os.path.getmtime(s) for s in SOURCES)


class OracleParams(C.Structure):
    _fields_ = [("height", C.c_int32), ("width", C.c_int32), ("alpha", C.c_double),
                ("kind", C.c_int32), ("levels", C.c_int32), ("fine_colours", C.c_int32),
                ("samples", C.c_int32), ("bisections", C.c_int32), ("round_f32", C.c_int32),
                ("threads", C.c_int32), ("cycle", C.c_int32), ("schedule", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("s", C.c_double), ("fs", C.c_double), ("K0", C.c_double), ("Kf", C.c_double),
                ("rho", C.c_double), ("c_sample", C.c_double), ("c_bisect", C.c_double),
                ("c_tilde", C.c_double), ("delta", C.c_double), ("c", C.c_double),
                ("istar", C.c_int32), ("accepted", C.c_int32)]


def default_levels(h: int, w: int) -> int:
    """J = ceil(log2(max(H, W))): the coarsest level still has two blocks along the longer side."""
    return max(1, int(math.ceil(math.log2(max(h, w)))))


_DP = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.environ.get("MGC_ORACLE_LIB") and _stale(lib_path()):
            build(force=True)
        L = C.CDLL(lib_path())
        P = C.POINTER(OracleParams)
        L.orc_curvature_at.restype = C.c_double
        L.orc_curvature_at.argtypes = [C.c_int, _DP, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double]
        L.orc_curvature_map.restype = None
        L.orc_curvature_map.argtypes = [C.c_int, _DP, C.c_int, C.c_int, C.c_double, _DP]
        L.orc_energy.restype = C.c_double
        L.orc_energy.argtypes = [C.c_int, _DP, _DP, C.c_int, C.c_int, C.c_double]
        for name in ("orc_ring_K", "orc_ring_dK"):
            fn = getattr(L, name)
            fn.restype = C.c_double
            fn.argtypes = [C.c_int, _DP, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double]
        L.orc_ring_K_many.restype = None
        L.orc_ring_K_many.argtypes = [C.c_int, _DP, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                      _DP, C.c_int, _DP]
        L.orc_ring_size.restype = C.c_int
        L.orc_ring_size.argtypes = [_DP, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        L.orc_local_delta.restype = C.c_double
        L.orc_local_delta.argtypes = [P, _DP, _DP, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double]
        L.orc_local_solve.restype = C.c_double
        L.orc_local_solve.argtypes = [P, _DP, _DP, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(SolveInfo)]
        L.orc_sweep.restype = C.c_int
        L.orc_sweep.argtypes = [P, _DP, _DP, C.c_int, C.c_int, C.c_void_p]
        L.orc_vcycle.restype = None
        L.orc_vcycle.argtypes = [P, _DP, _DP]
        L.orc_solve.restype = C.c_int
        L.orc_solve.argtypes = [P, _DP, _DP, C.c_double, C.c_int, C.c_void_p]
        L.orc_solve_rule.restype = C.c_int
        L.orc_solve_rule.argtypes = [P, _DP, _DP, C.c_double, C.c_int, C.c_int, C.c_void_p]
        L.orc_num_colours.restype = C.c_int
        L.orc_num_colours.argtypes = [P, C.c_int]
        L.orc_block_side.restype = C.c_int
        L.orc_block_side.argtypes = [P, C.c_int]
        FP = C.POINTER(FbsParams)
        L.fbs_plane.restype = None
        L.fbs_plane.argtypes = [FP, _DP, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.fbs_estimate.restype = C.c_double
        L.fbs_estimate.argtypes = [FP, _DP, C.c_int, C.c_int, C.c_int, C.c_double]
        L.fbs_block_step.restype = C.c_double
        L.fbs_block_step.argtypes = [FP, _DP, _DP, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
        L.fbs_sweep.restype = C.c_int
        L.fbs_sweep.argtypes = [FP, _DP, _DP, C.c_int, C.c_int, C.c_void_p]
        L.fbs_level.restype = None
        L.fbs_level.argtypes = [FP, _DP, _DP, C.c_int]
        L.fbs_vcycle.restype = None
        L.fbs_vcycle.argtypes = [FP, _DP, _DP]
        L.fbs_solve.restype = C.c_int
        L.fbs_solve.argtypes = [FP, _DP, _DP, C.c_double, C.c_int, C.c_int, C.c_void_p]
        for name in ("fbs_block_side", "fbs_rings", "fbs_planes"):
            getattr(L, name).restype = C.c_int
            getattr(L, name).argtypes = [C.c_int]
        for name in ("fbs_grid_rows", "fbs_grid_cols"):
            getattr(L, name).restype = C.c_int
            getattr(L, name).argtypes = [FP, C.c_int]
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def curvature_map(kind: int, u, h: float = 1.0) -> np.ndarray:
    u = _f64(u)
    out = np.empty_like(u)
    _load().orc_curvature_map(kind, u, u.shape[0], u.shape[1], h, out)
    return out


def energy(kind: int, u, f, alpha: float) -> float:
    u = _f64(u)
    f = _f64(f)
    return _load().orc_energy(kind, u, f, u.shape[0], u.shape[1], alpha)


class Oracle:
    """FP64 reference solver for one image (Algorithm 3 with the local solver of reading R8)."""

    def __init__(self, height: int, width: int, alpha: float, kind: int = 0, levels: int = 0,
                 fine_colours: int = 4, samples: int = 16, bisections: int = 32,
                 round_f32: bool = False, threads: int = 1, cycle: int = 0, schedule: int = 0):
        if levels <= 0:
            levels = default_levels(height, width)
        self.p = OracleParams(height, width, float(alpha), kind, levels, fine_colours,
                              samples, bisections, int(bool(round_f32)), threads, int(cycle), int(schedule))
        self.L = _load()

    # geometry -------------------------------------------------------------
    @property
    def levels(self) -> int:
        return self.p.levels

    def block_side(self, level: int) -> int:
        return self.L.orc_block_side(C.byref(self.p), level)

    def grid(self, level: int) -> tuple[int, int]:
        b = self.block_side(level)
        return (-(-self.p.height // b), -(-self.p.width // b))

    def block_bounds(self, level: int, p: int, q: int) -> tuple[int, int, int, int]:
        b = self.block_side(level)
        return (p * b, min((p + 1) * b, self.p.height), q * b, min((q + 1) * b, self.p.width))

    def num_colours(self, level: int) -> int:
        return self.L.orc_num_colours(C.byref(self.p), level)

    def colour_of(self, level: int, p: int, q: int) -> int:
        if self.num_colours(level) == 9:
            return 3 * (p % 3) + (q % 3)
        return 2 * (p % 2) + (q % 2)

    # local quantities -----------------------------------------------------
    def ring_K(self, u, bounds, c: float) -> float:
        u = _f64(u)
        return self.L.orc_ring_K(self.p.kind, u, self.p.height, self.p.width, *bounds, c)

    def ring_K_many(self, u, bounds, cs) -> np.ndarray:
        u = _f64(u)
        cs = _f64(cs)
        out = np.empty_like(cs)
        self.L.orc_ring_K_many(self.p.kind, u, self.p.height, self.p.width, *bounds, cs, cs.size, out)
        return out

    def ring_dK(self, u, bounds, c: float) -> float:
        u = _f64(u)
        return self.L.orc_ring_dK(self.p.kind, u, self.p.height, self.p.width, *bounds, c)

    def ring_size(self, u, bounds) -> int:
        u = _f64(u)
        return self.L.orc_ring_size(u, self.p.height, self.p.width, *bounds)

    def local_delta(self, u, f, bounds, c: float) -> float:
        return self.L.orc_local_delta(C.byref(self.p), _f64(u), _f64(f), *bounds, c)

    def local_solve(self, u, f, bounds) -> SolveInfo:
        info = SolveInfo()
        self.L.orc_local_solve(C.byref(self.p), _f64(u), _f64(f), *bounds, C.byref(info))
        return info

    # sweeps / cycles ------------------------------------------------------
    def sweep(self, u: np.ndarray, f, level: int, colour: int, want_c: bool = False):
        """In-place colour sweep on a float64 C-contiguous u; returns the c grid if asked."""
        assert u.dtype == np.float64 and u.flags.c_contiguous
        cb = None
        if want_c:
            cb = np.full(self.grid(level), np.nan)
        self.L.orc_sweep(C.byref(self.p), u, _f64(f), level, colour,
                         cb.ctypes.data if cb is not None else None)
        return cb

    def vcycle(self, u: np.ndarray, f) -> None:
        assert u.dtype == np.float64 and u.flags.c_contiguous
        self.L.orc_vcycle(C.byref(self.p), u, _f64(f))

    def solve(self, u: np.ndarray, f, rel_tol: float = 1e-6, max_vcycles: int = 1000):
        """In-place solve; returns (vcycles_done, energy trace E_0..E_done)."""
        assert u.dtype == np.float64 and u.flags.c_contiguous
        trace = np.zeros(max_vcycles + 1)
        n = self.L.orc_solve(C.byref(self.p), u, _f64(f), rel_tol, max_vcycles, trace.ctypes.data)
        return n, trace[: n + 1].copy()

    def solve_rule(self, u: np.ndarray, f, tol: float, max_vcycles: int = 1000, stop: int = 0):
        """In-place solve with stop 0 (relative energy change) or 1 (relative change of u);
        returns (vcycles_done, energy trace E_0..E_done)."""
        assert u.dtype == np.float64 and u.flags.c_contiguous
        trace = np.zeros(max_vcycles + 1)
        n = self.L.orc_solve_rule(C.byref(self.p), u, _f64(f), tol, max_vcycles, stop, trace.ctypes.data)
        return n, trace[: n + 1].copy()

    def energy(self, u, f) -> float:
        return energy(self.p.kind, u, f, self.p.alpha)


class FbsParams(C.Structure):
    _fields_ = [("height", C.c_int32), ("width", C.c_int32), ("alpha", C.c_double),
                ("kind", C.c_int32), ("levels", C.c_int32), ("steps", C.c_int32), ("cycle", C.c_int32),
                ("round_f32", C.c_int32), ("threads", C.c_int32)]


class FbsOracle:
    """FP64 reference of the paper's FBS local step (Algorithm 2, Propositions 1-2) on
    patches of side 2^j - 1 (Section 2.2)."""

    def __init__(self, height: int, width: int, alpha: float, kind: int = 0, levels: int = 3,
                 steps: int = 1, cycle: int = 0, round_f32: bool = False, threads: int = 1):
        self.p = FbsParams(height, width, float(alpha), kind, levels, steps, cycle,
                           int(bool(round_f32)), threads)
        self.L = _load()

    @property
    def levels(self) -> int:
        return self.p.levels

    def block_side(self, level: int) -> int:
        return self.L.fbs_block_side(level)

    def rings(self, level: int) -> int:
        return self.L.fbs_rings(level)

    def grid(self, level: int) -> tuple[int, int]:
        return (self.L.fbs_grid_rows(C.byref(self.p), level), self.L.fbs_grid_cols(C.byref(self.p), level))

    def block_bounds(self, level: int, p: int, q: int) -> tuple[int, int, int, int]:
        b = self.block_side(level)
        return (p * b, min((p + 1) * b, self.p.height), q * b, min((q + 1) * b, self.p.width))

    @staticmethod
    def colour_of(p: int, q: int) -> int:
        return 2 * (p % 2) + (q % 2)

    def plane(self, u, level: int, p: int, q: int, r: int, k: int, c: float = 0.0) -> tuple[float, float]:
        d, ds2 = C.c_double(), C.c_double()
        self.L.fbs_plane(C.byref(self.p), _f64(u), level, p, q, c, r, k, C.byref(d), C.byref(ds2))
        return d.value, ds2.value

    def estimate(self, u, level: int, p: int, q: int, c: float = 0.0) -> float:
        return self.L.fbs_estimate(C.byref(self.p), _f64(u), level, p, q, c)

    def block_step(self, u, f, level: int, p: int, q: int):
        """(c, trace[steps, 3] of (c_t, c_{t+1/2}, eta_t), s, f*)."""
        tr = np.zeros((self.p.steps, 3))
        info = np.zeros(2)
        c = self.L.fbs_block_step(C.byref(self.p), _f64(u), _f64(f), level, p, q, tr.ctypes.data, info.ctypes.data)
        return c, tr, info[0], info[1]

    def sweep(self, u: np.ndarray, f, level: int, colour: int, want_c: bool = False):
        assert u.dtype == np.float64 and u.flags.c_contiguous
        cb = np.zeros(self.grid(level)) if want_c else None
        self.L.fbs_sweep(C.byref(self.p), u, _f64(f), level, colour, cb.ctypes.data if cb is not None else None)
        return cb

    def level(self, u: np.ndarray, f, level: int) -> None:
        assert u.dtype == np.float64 and u.flags.c_contiguous
        self.L.fbs_level(C.byref(self.p), u, _f64(f), level)

    def vcycle(self, u: np.ndarray, f) -> None:
        assert u.dtype == np.float64 and u.flags.c_contiguous
        self.L.fbs_vcycle(C.byref(self.p), u, _f64(f))

    def solve(self, u: np.ndarray, f, tol: float = 1e-6, max_vcycles: int = 1000, stop: int = 0):
        """In-place solve; stop 0 = relative energy change, 1 = relErr(u).  Returns (done, energies)."""
        assert u.dtype == np.float64 and u.flags.c_contiguous
        trace = np.zeros(max_vcycles + 1)
        n = self.L.fbs_solve(C.byref(self.p), u, _f64(f), tol, max_vcycles, stop, trace.ctypes.data)
        return n, trace[: n + 1].copy()

    def energy(self, u, f) -> float:
        return energy(self.p.kind, u, f, self.p.alpha)
