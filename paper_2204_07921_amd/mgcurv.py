"""ctypes binding of libmgcurv.so (include/mgcurv.h).  Argument marshalling only.

Every function takes torch CUDA (HIP) tensors and passes their device pointers
and the current HIP stream to the library; no step of the method runs here.
If the library cannot be loaded the import fails loudly: there is no CPU or
PyTorch fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgcurv.so")

MG_OK, MG_NOT_CONVERGED = 0, 1
MG_CURV_MEAN, MG_CURV_GAUSS = 0, 1
MG_F32, MG_F64 = 0, 1
STATUS_NAMES = {0: "MG_OK", 1: "MG_NOT_CONVERGED", -1: "MG_E_INVALID", -2: "MG_E_SHAPE",
                -3: "MG_E_DTYPE", -4: "MG_E_NOMEM", -5: "MG_E_DEVICE", -6: "MG_E_NONFINITE"}


class MgCurvParams(C.Structure):
    _fields_ = [("height", C.c_int32), ("width", C.c_int32), ("alpha", C.c_double),
                ("curvature", C.c_int32), ("levels", C.c_int32), ("state_dtype", C.c_int32),
                ("fine_colours", C.c_int32), ("samples", C.c_int32), ("bisections", C.c_int32),
                ("cycle", C.c_int32), ("block_schedule", C.c_int32)]


class MgFbsParams(C.Structure):
    _fields_ = [("height", C.c_int32), ("width", C.c_int32), ("alpha", C.c_double),
                ("curvature", C.c_int32), ("levels", C.c_int32), ("state_dtype", C.c_int32),
                ("steps", C.c_int32), ("cycle", C.c_int32), ("reserved", C.c_int32)]


MG_STOP_ENERGY, MG_STOP_RELERR_U = 0, 1


class MgReconParams(C.Structure):
    _fields_ = [("height", C.c_int32), ("width", C.c_int32), ("alpha", C.c_double), ("blur_sigma", C.c_double),
                ("levels", C.c_int32), ("state_dtype", C.c_int32), ("cg_iters", C.c_int32), ("reserved", C.c_int32)]


class MgCurvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    L = C.CDLL(LIB_PATH)
    L.mg_curv_build_id.restype = C.c_char_p
    L.mg_curv_build_id.argtypes = []
    from . import build as _b
    want, got = _b.source_hash(), L.mg_curv_build_id().decode()
    if got != want:
        raise ImportError(f"{LIB_PATH} was built from other sources (build id {got}, sources {want}); "
                          "rebuild it with: python -m paper_2204_07921_amd.build")
    P = C.POINTER(MgCurvParams)
    vp, cvp = C.c_void_p, C.c_void_p
    L.mg_curv_default_params.restype = None
    L.mg_curv_default_params.argtypes = [P, C.c_int32, C.c_int32]
    L.mg_curv_init.restype = C.c_int
    L.mg_curv_init.argtypes = [P, vp, C.POINTER(vp)]
    L.mg_curv_energy_noalloc.restype = C.c_int
    L.mg_curv_energy_noalloc.argtypes = [P, vp, cvp, cvp, vp]
    L.mg_curv_vcycle.restype = C.c_int
    L.mg_curv_vcycle.argtypes = [vp, vp, cvp, C.POINTER(C.c_double)]
    L.mg_curv_solve.restype = C.c_int
    L.mg_curv_solve.argtypes = [vp, vp, cvp, C.c_double, C.c_int32, C.POINTER(C.c_int32),
                                C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.mg_curv_solve_target.restype = C.c_int
    L.mg_curv_solve_target.argtypes = [vp, vp, cvp, C.c_double, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    L.mg_curv_solve_rule.restype = C.c_int
    L.mg_curv_solve_rule.argtypes = [vp, vp, cvp, C.c_int32, C.c_double, C.c_int32, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double)]
    L.mg_curv_batch_solve_target.restype = C.c_int
    L.mg_curv_batch_solve_target.argtypes = [vp, vp, cvp, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32),
                                             C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    L.mg_curv_energy.restype = C.c_int
    L.mg_curv_energy.argtypes = [vp, cvp, cvp, C.POINTER(C.c_double)]
    L.mg_curv_sweep.restype = C.c_int
    L.mg_curv_sweep.argtypes = [vp, vp, cvp, C.c_int32, C.c_int32]
    L.mg_curv_level.restype = C.c_int
    L.mg_curv_level.argtypes = [vp, vp, cvp, C.c_int32]
    L.mg_curv_batch_init.restype = C.c_int
    L.mg_curv_batch_init.argtypes = [P, C.c_int32, vp, C.POINTER(vp)]
    L.mg_curv_batch_offset.restype = C.c_int64
    L.mg_curv_batch_offset.argtypes = [vp, C.c_int32]
    L.mg_curv_batch_levels.restype = C.c_int32
    L.mg_curv_batch_levels.argtypes = [vp]
    L.mg_curv_batch_vcycle.restype = C.c_int
    L.mg_curv_batch_vcycle.argtypes = [vp, vp, cvp, C.POINTER(C.c_double)]
    L.mg_curv_batch_level.restype = C.c_int
    L.mg_curv_batch_level.argtypes = [vp, vp, cvp, C.c_int32]
    L.mg_curv_batch_sweep.restype = C.c_int
    L.mg_curv_batch_sweep.argtypes = [vp, vp, cvp, C.c_int32, C.c_int32]
    L.mg_curv_batch_energy.restype = C.c_int
    L.mg_curv_batch_energy.argtypes = [vp, cvp, cvp, C.POINTER(C.c_double)]
    L.mg_curv_batch_solve.restype = C.c_int
    L.mg_curv_batch_solve.argtypes = [vp, vp, cvp, C.c_double, C.c_int32, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    L.mg_curv_batch_tune.restype = C.c_int
    L.mg_curv_batch_tune.argtypes = [vp, vp, cvp, C.c_int32]
    L.mg_curv_batch_config.restype = C.c_int32
    L.mg_curv_batch_config.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32)]
    L.mg_curv_batch_set_config.restype = C.c_int
    L.mg_curv_batch_set_config.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
    L.mg_curv_batch_destroy.restype = None
    L.mg_curv_batch_destroy.argtypes = [vp]
    L.mg_curv_batch_last_error.restype = C.c_char_p
    L.mg_curv_batch_last_error.argtypes = [vp]
    L.mg_curv_levels.restype = C.c_int32
    L.mg_curv_levels.argtypes = [vp]
    L.mg_curv_set_split.restype = C.c_int
    L.mg_curv_set_split.argtypes = [vp, C.c_int32]
    L.mg_curv_split_active.restype = C.c_int32
    L.mg_curv_split_active.argtypes = [vp]
    L.mg_curv_set_split_polls.restype = C.c_int
    L.mg_curv_set_split_polls.argtypes = [vp, C.c_int32]
    L.mg_cnn_num_params.restype = C.c_int32
    L.mg_cnn_num_params.argtypes = []
    L.mg_cnn_init.restype = C.c_int
    L.mg_cnn_init.argtypes = [C.c_int64, vp, C.POINTER(vp)]
    L.mg_cnn_set_params.restype = C.c_int
    L.mg_cnn_set_params.argtypes = [vp, vp]
    L.mg_cnn_get_params.restype = C.c_int
    L.mg_cnn_get_params.argtypes = [vp, vp]
    L.mg_cnn_forward.restype = C.c_int
    L.mg_cnn_forward.argtypes = [vp, cvp, vp, C.c_int32, C.c_int32, C.c_int32]
    L.mg_cnn_train_step.restype = C.c_int
    L.mg_cnn_train_step.argtypes = [vp, cvp, cvp, C.c_int32, C.c_int32, C.c_int32, C.c_float, C.POINTER(C.c_double)]
    L.mg_cnn_gradients.restype = C.c_int
    L.mg_cnn_gradients.argtypes = [vp, cvp, cvp, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double), vp]
    L.mg_cnn_get_state.restype = C.c_int
    L.mg_cnn_get_state.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_int32)]
    L.mg_cnn_set_state.restype = C.c_int
    L.mg_cnn_set_state.argtypes = [vp, vp, vp, vp, C.c_int32]
    L.mg_cnn_gradient_trace.restype = C.c_int
    L.mg_cnn_gradient_trace.argtypes = [vp, cvp, cvp, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp]
    L.mg_cnn_activation.restype = C.c_int
    L.mg_cnn_activation.argtypes = [vp, C.c_int32, vp, C.c_int64]
    L.mg_cnn_destroy.restype = None
    L.mg_cnn_destroy.argtypes = [vp]
    L.mg_cnn_last_error.restype = C.c_char_p
    L.mg_cnn_last_error.argtypes = [vp]
    L.mg_curv_destroy.restype = None
    L.mg_curv_destroy.argtypes = [vp]
    L.mg_curv_last_error.restype = C.c_char_p
    L.mg_curv_last_error.argtypes = [vp]
    FP = C.POINTER(MgFbsParams)
    L.mg_fbs_default_params.restype = None
    L.mg_fbs_default_params.argtypes = [FP, C.c_int32, C.c_int32]
    L.mg_fbs_init.restype = C.c_int
    L.mg_fbs_init.argtypes = [FP, vp, C.POINTER(vp)]
    L.mg_fbs_vcycle.restype = C.c_int
    L.mg_fbs_vcycle.argtypes = [vp, vp, cvp, C.POINTER(C.c_double)]
    L.mg_fbs_level.restype = C.c_int
    L.mg_fbs_level.argtypes = [vp, vp, cvp, C.c_int32]
    L.mg_fbs_sweep.restype = C.c_int
    L.mg_fbs_sweep.argtypes = [vp, vp, cvp, C.c_int32, C.c_int32]
    L.mg_fbs_energy.restype = C.c_int
    L.mg_fbs_energy.argtypes = [vp, cvp, cvp, C.POINTER(C.c_double)]
    L.mg_fbs_solve.restype = C.c_int
    L.mg_fbs_solve.argtypes = [vp, vp, cvp, C.c_double, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                               C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.mg_fbs_destroy.restype = None
    L.mg_fbs_destroy.argtypes = [vp]
    L.mg_fbs_last_error.restype = C.c_char_p
    L.mg_fbs_last_error.argtypes = [vp]
    RP = C.POINTER(MgReconParams)
    L.mg_recon_default_params.restype = None
    L.mg_recon_default_params.argtypes = [RP, C.c_int32, C.c_int32]
    L.mg_recon_init.restype = C.c_int
    L.mg_recon_init.argtypes = [RP, vp, C.POINTER(vp)]
    L.mg_recon_sweep.restype = C.c_int
    L.mg_recon_sweep.argtypes = [vp, vp, cvp, C.c_int32, C.c_int32]
    L.mg_recon_vcycle.restype = C.c_int
    L.mg_recon_vcycle.argtypes = [vp, vp, cvp, C.POINTER(C.c_double)]
    L.mg_recon_energy.restype = C.c_int
    L.mg_recon_energy.argtypes = [vp, cvp, cvp, C.POINTER(C.c_double)]
    L.mg_recon_solve.restype = C.c_int
    L.mg_recon_solve.argtypes = [vp, vp, cvp, C.c_double, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    L.mg_recon_destroy.restype = None
    L.mg_recon_destroy.argtypes = [vp]
    L.mg_recon_last_error.restype = C.c_char_p
    L.mg_recon_last_error.argtypes = [vp]
    return L


lib = _load()


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check(status: int, ctx=None) -> int:
    if status < 0:
        raise MgCurvError(status, lib.mg_curv_last_error(ctx).decode())
    return status


def default_params(height: int, width: int, **kw) -> MgCurvParams:
    p = MgCurvParams()
    lib.mg_curv_default_params(C.byref(p), height, width)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return MG_F32
    if t.dtype == torch.float64:
        return MG_F64
    raise TypeError(f"state tensors must be float32 or float64, got {t.dtype}")


def _tensor_ptr(t: torch.Tensor, p: MgCurvParams, name: str) -> int:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != (p.height, p.width):
        raise ValueError(f"{name} must have shape {(p.height, p.width)}, got {tuple(t.shape)}")
    if _dtype_code(t) != p.state_dtype:
        raise TypeError(f"{name} dtype does not match the context's state dtype")
    return t.data_ptr()


# --- functions with the ABI's names --------------------------------------------------

def mg_curv_init(params: MgCurvParams, stream=None) -> C.c_void_p:
    ctx = C.c_void_p()
    _check(lib.mg_curv_init(C.byref(params), C.c_void_p(_stream_handle(stream)), C.byref(ctx)))
    return ctx


def mg_curv_vcycle(ctx, params, u, f, want_energy: bool = False):
    e = C.c_double()
    _check(lib.mg_curv_vcycle(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(f, params, "f"),
                              C.byref(e) if want_energy else None), ctx)
    return e.value if want_energy else None


def mg_curv_solve(ctx, params, u, f, rel_tol: float = 1e-6, max_vcycles: int = 1000, trace: bool = False):
    done = C.c_int32()
    fin = C.c_double()
    buf = (C.c_double * (max_vcycles + 1))() if trace else None
    st = _check(lib.mg_curv_solve(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(f, params, "f"), rel_tol,
                                  max_vcycles, C.byref(done), C.byref(fin), buf), ctx)
    out = {"status": st, "vcycles": done.value, "energy": fin.value}
    if trace:
        out["trace"] = [buf[k] for k in range(done.value + 1)]
    return out


def mg_curv_solve_target(ctx, params, u, f, target_energy: float, max_vcycles: int = 1000):
    done = C.c_int32()
    fin = C.c_double()
    st = _check(lib.mg_curv_solve_target(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(f, params, "f"),
                                         float(target_energy), max_vcycles, C.byref(done), C.byref(fin)), ctx)
    return {"status": st, "vcycles": done.value, "energy": fin.value}


def mg_curv_solve_rule(ctx, params, u, f, stop: int, tol: float, max_vcycles: int = 1000):
    done = C.c_int32()
    fin = C.c_double()
    st = _check(lib.mg_curv_solve_rule(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(f, params, "f"), int(stop),
                                       float(tol), max_vcycles, C.byref(done), C.byref(fin)), ctx)
    return {"status": st, "vcycles": done.value, "energy": fin.value}


def mg_curv_energy(ctx, params, u, f) -> float:
    e = C.c_double()
    _check(lib.mg_curv_energy(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(f, params, "f"), C.byref(e)), ctx)
    return e.value


def mg_curv_energy_noalloc(params, u, f, out, stream=None) -> None:
    """F(u) into the one-element float64 device tensor `out`, enqueued only (no context, no allocation)."""
    if not (out.is_cuda and out.dtype == torch.float64 and out.numel() >= 1 and out.is_contiguous()):
        raise ValueError("out must be a contiguous float64 device tensor with at least one element")
    _check(lib.mg_curv_energy_noalloc(C.byref(params), C.c_void_p(_stream_handle(stream)),
                                      _tensor_ptr(u, params, "u"), _tensor_ptr(f, params, "f"),
                                      C.c_void_p(out.data_ptr())))


def mg_curv_sweep(ctx, params, u, f, level: int, colour: int) -> None:
    _check(lib.mg_curv_sweep(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(f, params, "f"), level, colour), ctx)


def mg_curv_level(ctx, params, u, f, level: int) -> None:
    _check(lib.mg_curv_level(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(f, params, "f"), level), ctx)


def mg_curv_destroy(ctx) -> None:
    lib.mg_curv_destroy(ctx)


def mg_curv_set_split(ctx, enable: bool) -> None:
    _check(lib.mg_curv_set_split(ctx, 1 if enable else 0), ctx)


def mg_curv_split_active(ctx) -> bool:
    return bool(lib.mg_curv_split_active(ctx))


def mg_curv_set_split_polls(ctx, polls: int) -> None:
    _check(lib.mg_curv_set_split_polls(ctx, int(polls)), ctx)


# --- convenience object ----------------------------------------------------------

class Solver:
    """One context: fixed image size, alpha, curvature kind, dtype and stream."""

    def __init__(self, height: int, width: int, alpha: float = 20.0, kind: int = MG_CURV_MEAN,
                 levels: int = 0, dtype=torch.float32, fine_colours: int = 4, samples: int = 16,
                 bisections: int = 32, stream=None, cycle: int = 0, block_schedule: int = 0):
        self.params = default_params(height, width, alpha=float(alpha), curvature=int(kind), levels=int(levels),
                                     state_dtype=MG_F64 if dtype == torch.float64 else MG_F32,
                                     fine_colours=int(fine_colours), samples=int(samples),
                                     bisections=int(bisections), cycle=int(cycle),
                                     block_schedule=int(block_schedule))
        self.dtype = dtype
        self.ctx = mg_curv_init(self.params, stream)
        self.levels = lib.mg_curv_levels(self.ctx)

    def close(self):
        if self.ctx:
            mg_curv_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def vcycle(self, u, f, want_energy=False):
        return mg_curv_vcycle(self.ctx, self.params, u, f, want_energy)

    def solve(self, u, f, rel_tol=1e-6, max_vcycles=1000, trace=False):
        return mg_curv_solve(self.ctx, self.params, u, f, rel_tol, max_vcycles, trace)

    def energy(self, u, f):
        return mg_curv_energy(self.ctx, self.params, u, f)

    def solve_target(self, u, f, target_energy, max_vcycles=1000):
        return mg_curv_solve_target(self.ctx, self.params, u, f, target_energy, max_vcycles)

    def solve_rule(self, u, f, tol, max_vcycles=1000, stop=MG_STOP_RELERR_U):
        return mg_curv_solve_rule(self.ctx, self.params, u, f, stop, tol, max_vcycles)

    def sweep(self, u, f, level, colour):
        return mg_curv_sweep(self.ctx, self.params, u, f, level, colour)

    def level(self, u, f, level):
        return mg_curv_level(self.ctx, self.params, u, f, level)

    def set_split(self, enable: bool) -> None:
        mg_curv_set_split(self.ctx, enable)

    @property
    def split_active(self) -> bool:
        return mg_curv_split_active(self.ctx)

    def set_split_polls(self, polls: int) -> None:
        mg_curv_set_split_polls(self.ctx, polls)


# --- the paper's own local step (FBS with tangent-plane estimates) ------------------

def _fcheck(status: int, ctx=None) -> int:
    if status < 0:
        raise MgCurvError(status, lib.mg_fbs_last_error(ctx).decode())
    return status


def fbs_default_params(height: int, width: int, **kw) -> MgFbsParams:
    p = MgFbsParams()
    lib.mg_fbs_default_params(C.byref(p), height, width)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def mg_fbs_init(params: MgFbsParams, stream=None) -> C.c_void_p:
    ctx = C.c_void_p()
    _fcheck(lib.mg_fbs_init(C.byref(params), C.c_void_p(_stream_handle(stream)), C.byref(ctx)))
    return ctx


def mg_fbs_vcycle(ctx, params, u, f, want_energy: bool = False):
    e = C.c_double()
    _fcheck(lib.mg_fbs_vcycle(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(f, params, "f"),
                              C.byref(e) if want_energy else None), ctx)
    return e.value if want_energy else None


def mg_fbs_level(ctx, params, u, f, level: int) -> None:
    _fcheck(lib.mg_fbs_level(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(f, params, "f"), level), ctx)


def mg_fbs_sweep(ctx, params, u, f, level: int, colour: int) -> None:
    _fcheck(lib.mg_fbs_sweep(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(f, params, "f"), level, colour), ctx)


def mg_fbs_energy(ctx, params, u, f) -> float:
    e = C.c_double()
    _fcheck(lib.mg_fbs_energy(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(f, params, "f"), C.byref(e)), ctx)
    return e.value


def mg_fbs_solve(ctx, params, u, f, tol: float = 1e-4, max_vcycles: int = 1000, stop: int = MG_STOP_RELERR_U,
                 trace: bool = False):
    done = C.c_int32()
    fin = C.c_double()
    buf = (C.c_double * (max_vcycles + 1))() if trace else None
    st = _fcheck(lib.mg_fbs_solve(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(f, params, "f"), tol, max_vcycles,
                                  stop, C.byref(done), C.byref(fin), buf), ctx)
    out = {"status": st, "vcycles": done.value, "energy": fin.value}
    if trace:
        out["trace"] = [buf[k] for k in range(done.value + 1)]
    return out


def mg_fbs_destroy(ctx) -> None:
    lib.mg_fbs_destroy(ctx)


class FbsSolver:
    """The paper's own local step on patches of side 2^j - 1: one context per image size."""

    def __init__(self, height: int, width: int, alpha: float = 20.0, kind: int = MG_CURV_MEAN, levels: int = 3,
                 dtype=torch.float32, steps: int = 1, cycle: int = 0, stream=None):
        self.params = fbs_default_params(height, width, alpha=float(alpha), curvature=int(kind), levels=int(levels),
                                         state_dtype=MG_F64 if dtype == torch.float64 else MG_F32,
                                         steps=int(steps), cycle=int(cycle))
        self.dtype = dtype
        self.levels = int(levels)
        self.ctx = mg_fbs_init(self.params, stream)

    def close(self):
        if self.ctx:
            mg_fbs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def vcycle(self, u, f, want_energy=False):
        return mg_fbs_vcycle(self.ctx, self.params, u, f, want_energy)

    def level(self, u, f, level):
        return mg_fbs_level(self.ctx, self.params, u, f, level)

    def sweep(self, u, f, level, colour):
        return mg_fbs_sweep(self.ctx, self.params, u, f, level, colour)

    def energy(self, u, f):
        return mg_fbs_energy(self.ctx, self.params, u, f)

    def solve(self, u, f, tol=1e-4, max_vcycles=1000, stop=MG_STOP_RELERR_U, trace=False):
        return mg_fbs_solve(self.ctx, self.params, u, f, tol, max_vcycles, stop, trace)


# --- reconstruction b = A u + noise (Section 5) ---------------------------------------

def _rcheck(status: int, ctx=None) -> int:
    if status < 0:
        raise MgCurvError(status, lib.mg_recon_last_error(ctx).decode())
    return status


def recon_default_params(height: int, width: int, **kw) -> MgReconParams:
    p = MgReconParams()
    lib.mg_recon_default_params(C.byref(p), height, width)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def mg_recon_init(params: MgReconParams, stream=None) -> C.c_void_p:
    ctx = C.c_void_p()
    _rcheck(lib.mg_recon_init(C.byref(params), C.c_void_p(_stream_handle(stream)), C.byref(ctx)))
    return ctx


def mg_recon_sweep(ctx, params, u, b, level: int, colour: int) -> None:
    _rcheck(lib.mg_recon_sweep(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(b, params, "b"), level, colour), ctx)


def mg_recon_vcycle(ctx, params, u, b, want_energy: bool = False):
    e = C.c_double()
    _rcheck(lib.mg_recon_vcycle(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(b, params, "b"),
                                C.byref(e) if want_energy else None), ctx)
    return e.value if want_energy else None


def mg_recon_energy(ctx, params, u, b) -> float:
    e = C.c_double()
    _rcheck(lib.mg_recon_energy(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(b, params, "b"), C.byref(e)), ctx)
    return e.value


def mg_recon_solve(ctx, params, u, b, tol: float = 1e-4, max_vcycles: int = 200):
    done = C.c_int32()
    fin = C.c_double()
    st = _rcheck(lib.mg_recon_solve(ctx, _tensor_ptr(u, params, "u"), _tensor_ptr(b, params, "b"), tol, max_vcycles,
                                    C.byref(done), C.byref(fin)), ctx)
    return {"status": st, "vcycles": done.value, "energy": fin.value}


def mg_recon_destroy(ctx) -> None:
    lib.mg_recon_destroy(ctx)


class ReconSolver:
    """Reconstruction from b = A u + noise with a 5 x 5 Gaussian blur as A (one context per size)."""

    def __init__(self, height: int, width: int, alpha: float = 0.01, blur_sigma: float = 1.0, levels: int = 3,
                 dtype=torch.float32, cg_iters: int = 20, stream=None):
        self.params = recon_default_params(height, width, alpha=float(alpha), blur_sigma=float(blur_sigma),
                                           levels=int(levels), state_dtype=MG_F64 if dtype == torch.float64 else MG_F32,
                                           cg_iters=int(cg_iters))
        self.dtype = dtype
        self.ctx = mg_recon_init(self.params, stream)

    def close(self):
        if self.ctx:
            mg_recon_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, u, b, level, colour):
        return mg_recon_sweep(self.ctx, self.params, u, b, level, colour)

    def vcycle(self, u, b, want_energy=False):
        return mg_recon_vcycle(self.ctx, self.params, u, b, want_energy)

    def energy(self, u, b):
        return mg_recon_energy(self.ctx, self.params, u, b)

    def solve(self, u, b, tol=1e-4, max_vcycles=200):
        return mg_recon_solve(self.ctx, self.params, u, b, tol, max_vcycles)


# --- batched images ----------------------------------------------------------------

def _bcheck(status: int, b=None) -> int:
    if status < 0:
        raise MgCurvError(status, lib.mg_curv_batch_last_error(b).decode())
    return status


class BatchSolver:
    """Many images of independent sizes, alphas and curvature kinds in packed float32 buffers.

    ``specs`` is a list of dicts with keys height, width, alpha, kind (0 mean, 1 Gaussian) and
    optionally levels.  ``block_schedule`` (0: sides 2^(j-1), 1: 2^j - 1) applies to every image.
    Use :meth:`pack` / :meth:`unpack` to move between the packed device buffer and per-image 2-D
    views."""

    def __init__(self, specs, samples: int = 16, bisections: int = 32, stream=None, block_schedule: int = 0):
        n = len(specs)
        arr = (MgCurvParams * n)()
        for i, sp in enumerate(specs):
            p = default_params(int(sp["height"]), int(sp["width"]), alpha=float(sp["alpha"]),
                               curvature=int(sp.get("kind", 0)), levels=int(sp.get("levels", 0)),
                               state_dtype=MG_F32, fine_colours=4, samples=samples, bisections=bisections,
                               block_schedule=int(block_schedule))
            arr[i] = p
        self.n = n
        self.specs = [dict(sp) for sp in specs]
        self.b = C.c_void_p()
        _bcheck(lib.mg_curv_batch_init(arr, n, C.c_void_p(_stream_handle(stream)), C.byref(self.b)))
        self.offsets = [lib.mg_curv_batch_offset(self.b, i) for i in range(n + 1)]
        self.total = self.offsets[-1]
        self.levels = lib.mg_curv_batch_levels(self.b)

    def close(self):
        if self.b:
            lib.mg_curv_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, images) -> torch.Tensor:
        out = torch.empty(self.total, dtype=torch.float32, device="cuda")
        for i, im in enumerate(images):
            t = torch.as_tensor(im, dtype=torch.float32)
            out[self.offsets[i]:self.offsets[i + 1]].copy_(t.reshape(-1))
        return out

    def unpack(self, packed: torch.Tensor):
        return [packed[self.offsets[i]:self.offsets[i + 1]].view(self.specs[i]["height"], self.specs[i]["width"])
                for i in range(self.n)]

    def _ptr(self, t: torch.Tensor, name: str) -> int:
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != self.total:
            raise ValueError(f"{name} must be a contiguous float32 device tensor of {self.total} elements")
        return t.data_ptr()

    def vcycle(self, u, f, want_energy: bool = False):
        e = (C.c_double * self.n)() if want_energy else None
        _bcheck(lib.mg_curv_batch_vcycle(self.b, self._ptr(u, "u"), self._ptr(f, "f"), e), self.b)
        return list(e) if want_energy else None

    def level(self, u, f, level: int):
        _bcheck(lib.mg_curv_batch_level(self.b, self._ptr(u, "u"), self._ptr(f, "f"), level), self.b)

    def sweep(self, u, f, level: int, colour: int):
        _bcheck(lib.mg_curv_batch_sweep(self.b, self._ptr(u, "u"), self._ptr(f, "f"), level, colour), self.b)

    def energy(self, u, f):
        e = (C.c_double * self.n)()
        _bcheck(lib.mg_curv_batch_energy(self.b, self._ptr(u, "u"), self._ptr(f, "f"), e), self.b)
        return list(e)

    def solve(self, u, f, rel_tol: float = 1e-6, max_vcycles: int = 1000):
        done = (C.c_int32 * self.n)()
        fin = (C.c_double * self.n)()
        st = (C.c_int32 * self.n)()
        s = _bcheck(lib.mg_curv_batch_solve(self.b, self._ptr(u, "u"), self._ptr(f, "f"), rel_tol, max_vcycles,
                                            done, fin, st), self.b)
        return {"status": s, "vcycles": list(done), "energy": list(fin), "image_status": list(st)}

    def solve_target(self, u, f, target_energy, max_vcycles: int = 1000):
        done = (C.c_int32 * self.n)()
        fin = (C.c_double * self.n)()
        st = (C.c_int32 * self.n)()
        tg = (C.c_double * self.n)(*[float(x) for x in target_energy])
        s = _bcheck(lib.mg_curv_batch_solve_target(self.b, self._ptr(u, "u"), self._ptr(f, "f"), tg, max_vcycles,
                                                   done, fin, st), self.b)
        return {"status": s, "vcycles": list(done), "energy": list(fin), "image_status": list(st)}

    def tune(self, u, f, repeats: int = 2):
        _bcheck(lib.mg_curv_batch_tune(self.b, self._ptr(u, "u"), self._ptr(f, "f"), repeats), self.b)

    def config(self, level: int):
        g, r, gr = C.c_int32(), C.c_int32(), C.c_int32()
        lib.mg_curv_batch_config(self.b, level, C.byref(g), C.byref(r), C.byref(gr))
        return {"group": g.value, "records": r.value, "grid": gr.value}

    def set_config(self, level: int, group: int, records: int, grid: int):
        _bcheck(lib.mg_curv_batch_set_config(self.b, level, group, records, grid), self.b)


# --- warm-start CNN ---------------------------------------------------------------

def _ccheck(status: int, c=None) -> int:
    if status < 0:
        raise MgCurvError(status, lib.mg_cnn_last_error(c).decode())
    return status


class WarmStartCNN:
    """The six-layer warm-start network (bfloat16 MFMA kernels in libmgcurv.so).

    Images are float32 device tensors of shape (n, height, width)."""

    def __init__(self, max_pixels: int, params=None, stream=None):
        self.c = C.c_void_p()
        _ccheck(lib.mg_cnn_init(int(max_pixels), C.c_void_p(_stream_handle(stream)), C.byref(self.c)))
        self.n_params = lib.mg_cnn_num_params()
        self.max_pixels = int(max_pixels)
        if params is not None:
            self.set_params(params)

    def close(self):
        if self.c:
            lib.mg_cnn_destroy(self.c)
            self.c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if p.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {p.size}")
        _ccheck(lib.mg_cnn_set_params(self.c, p.ctypes.data), self.c)

    def get_params(self):
        import numpy as np
        p = np.empty(self.n_params, dtype=np.float32)
        _ccheck(lib.mg_cnn_get_params(self.c, p.ctypes.data), self.c)
        return p

    def get_state(self) -> dict:
        """Training checkpoint: parameters, Adam moments m and v (float32 numpy) and the step count."""
        import numpy as np
        w, m, v = (np.empty(self.n_params, dtype=np.float32) for _ in range(3))
        step = C.c_int32()
        _ccheck(lib.mg_cnn_get_state(self.c, w.ctypes.data, m.ctypes.data, v.ctypes.data, C.byref(step)), self.c)
        return {"params": w, "m": m, "v": v, "step": int(step.value)}

    def set_state(self, state: dict) -> None:
        import numpy as np
        arrs = [np.ascontiguousarray(np.asarray(state[k], dtype=np.float32)) for k in ("params", "m", "v")]
        if any(a.size != self.n_params for a in arrs):
            raise ValueError(f"expected {self.n_params} values per array")
        _ccheck(lib.mg_cnn_set_state(self.c, arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data,
                                     int(state["step"])), self.c)

    @staticmethod
    def _img(t: torch.Tensor, name: str):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous() or t.dim() != 3:
            raise ValueError(f"{name} must be a contiguous float32 device tensor (n, height, width)")
        return t.data_ptr()

    def forward(self, f: torch.Tensor, out: torch.Tensor = None) -> torch.Tensor:
        n, h, w = f.shape
        u = torch.empty_like(f) if out is None else out
        _ccheck(lib.mg_cnn_forward(self.c, self._img(f, "f"), self._img(u, "u"), n, h, w), self.c)
        return u

    def train_step(self, f: torch.Tensor, target: torch.Tensor, lr: float, want_loss: bool = True):
        n, h, w = f.shape
        loss = C.c_double()
        _ccheck(lib.mg_cnn_train_step(self.c, self._img(f, "f"), self._img(target, "target"), n, h, w, float(lr),
                                      C.byref(loss) if want_loss else None), self.c)
        return loss.value if want_loss else None

    def gradients(self, f: torch.Tensor, target: torch.Tensor):
        import numpy as np
        n, h, w = f.shape
        loss = C.c_double()
        g = np.empty(self.n_params, dtype=np.float32)
        _ccheck(lib.mg_cnn_gradients(self.c, self._img(f, "f"), self._img(target, "target"), n, h, w,
                                     C.byref(loss), g.ctypes.data), self.c)
        return loss.value, g

    def gradient_trace(self, f: torch.Tensor, target: torch.Tensor):
        """Intermediate gradients of one backward pass: ([dL/dz_l for l = 0..4] as float32 numpy
        (n, h, w, 32) from their bfloat16 storage, dL/dz_5 as (n, h, w), parameter gradient)."""
        import numpy as np
        n, h, w = f.shape
        raw = np.empty(5 * n * h * w * 32, dtype=np.uint16)
        dz5 = np.empty(n * h * w, dtype=np.float32)
        g = np.empty(self.n_params, dtype=np.float32)
        _ccheck(lib.mg_cnn_gradient_trace(self.c, self._img(f, "f"), self._img(target, "target"), n, h, w,
                                          raw.ctypes.data, dz5.ctypes.data, g.ctypes.data), self.c)
        dz = (raw.astype(np.uint32) << 16).view(np.float32).reshape(5, n, h, w, 32)
        return [dz[l] for l in range(5)], dz5.reshape(n, h, w), g

    def activation(self, layer: int, shape):
        """Activation a_layer (1..5) of the last forward pass as float32 numpy (n, h, w, 32)."""
        import numpy as np
        n, h, w = shape
        count = n * h * w * 32
        raw = np.empty(count, dtype=np.uint16)
        _ccheck(lib.mg_cnn_activation(self.c, layer, raw.ctypes.data, count), self.c)
        return (raw.astype(np.uint32) << 16).view(np.float32).reshape(n, h, w, 32)
