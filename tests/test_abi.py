"""C-ABI contract of libmgcurv.so on a machine without a GPU: the library loads,
exports every entry point include/mgcurv.h declares, validates parameters before
touching a device and reports MG_E_DEVICE when no GPU is present.  No compute
call is made here."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgcurv.h")
LIB = os.path.join(ROOT, "paper_2204_07921_amd", "libmgcurv.so")


class Params(C.Structure):
    _fields_ = [("height", C.c_int32), ("width", C.c_int32), ("alpha", C.c_double),
                ("curvature", C.c_int32), ("levels", C.c_int32), ("state_dtype", C.c_int32),
                ("fine_colours", C.c_int32), ("samples", C.c_int32), ("bisections", C.c_int32),
                ("cycle", C.c_int32), ("block_schedule", C.c_int32)]


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2204_07921_amd import build
        build.build()
    L = C.CDLL(LIB)
    L.mg_curv_init.restype = C.c_int
    L.mg_curv_init.argtypes = [C.POINTER(Params), C.c_void_p, C.POINTER(C.c_void_p)]
    L.mg_curv_last_error.restype = C.c_char_p
    L.mg_curv_last_error.argtypes = [C.c_void_p]
    L.mg_curv_default_params.argtypes = [C.POINTER(Params), C.c_int32, C.c_int32]
    for name in ("mg_curv_vcycle", "mg_curv_energy", "mg_curv_sweep", "mg_curv_solve", "mg_curv_level",
                 "mg_curv_batch_init", "mg_curv_batch_vcycle", "mg_curv_batch_solve"):
        getattr(L, name).restype = C.c_int
    return L


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared_symbols()
    for required in ("mg_curv_init", "mg_curv_vcycle", "mg_curv_solve", "mg_curv_energy",
                     "mg_curv_destroy", "mg_curv_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_params_struct_layout(lib):
    assert C.sizeof(Params) == 48
    p = Params()
    lib.mg_curv_default_params(C.byref(p), 64, 48)
    assert (p.height, p.width, p.alpha, p.curvature, p.levels, p.state_dtype) == (64, 48, 20.0, 0, 0, 0)
    assert (p.fine_colours, p.samples, p.bisections, p.cycle, p.block_schedule) == (4, 16, 32, 0, 0)


@pytest.mark.parametrize("field,value,status", [
    ("height", 1, -2), ("width", 0, -2), ("alpha", 0.0, -1), ("alpha", float("nan"), -1), ("cycle", 2, -1),
    ("alpha", float("inf"), -1), ("curvature", 2, -1), ("state_dtype", 7, -3), ("fine_colours", 5, -1),
    ("samples", 3, -1), ("samples", 0, -1), ("bisections", -1, -1), ("bisections", 65, -1), ("levels", 99, -1),
    ("block_schedule", 2, -1), ("block_schedule", -1, -1),
])
def test_invalid_params_rejected_before_device(lib, field, value, status):
    p = Params()
    lib.mg_curv_default_params(C.byref(p), 64, 64)
    setattr(p, field, value)
    ctx = C.c_void_p(1234)
    st = lib.mg_curv_init(C.byref(p), None, C.byref(ctx))
    assert st == status
    assert not ctx.value
    assert lib.mg_curv_last_error(None)


def test_null_arguments(lib):
    ctx = C.c_void_p()
    assert lib.mg_curv_init(None, None, C.byref(ctx)) == -1
    assert lib.mg_curv_vcycle(None, None, None, None) == -1
    assert lib.mg_curv_energy(None, None, None, None) == -1
    assert lib.mg_curv_sweep(None, None, None, 1, 0) == -1
    assert lib.mg_curv_level(None, None, None, 1) == -1
    lib.mg_curv_solve_rule.restype = C.c_int
    lib.mg_curv_solve_rule.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_int32,
                                       C.c_void_p, C.c_void_p]
    for stop in (0, 1, 7):
        assert lib.mg_curv_solve_rule(None, None, None, stop, 1e-4, 10, None, None) == -1
    lib.mg_curv_destroy(None)


def test_split_controls_reject_a_null_context(lib):
    """The split coarse solve's switch, status query and wait bound check their context first."""
    lib.mg_curv_set_split.restype = C.c_int
    lib.mg_curv_set_split.argtypes = [C.c_void_p, C.c_int32]
    lib.mg_curv_set_split_polls.restype = C.c_int
    lib.mg_curv_set_split_polls.argtypes = [C.c_void_p, C.c_int32]
    lib.mg_curv_split_active.restype = C.c_int32
    lib.mg_curv_split_active.argtypes = [C.c_void_p]
    assert lib.mg_curv_set_split(None, 1) == -1
    assert lib.mg_curv_set_split(None, 0) == -1
    assert lib.mg_curv_set_split_polls(None, 16) == -1
    assert lib.mg_curv_split_active(None) == 0


def test_no_device_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    p = Params()
    lib.mg_curv_default_params(C.byref(p), 64, 64)
    ctx = C.c_void_p()
    assert lib.mg_curv_init(C.byref(p), None, C.byref(ctx)) == -5
    assert b"device" in lib.mg_curv_last_error(None).lower()


def _batch_params(lib, shapes, **over):
    arr = (Params * len(shapes))()
    for i, (h, w) in enumerate(shapes):
        lib.mg_curv_default_params(C.byref(arr[i]), h, w)
        for k, v in over.items():
            setattr(arr[i], k, v)
    return arr


@pytest.mark.parametrize("over,status", [
    ({"state_dtype": 1}, -3), ({"fine_colours": 9}, -1), ({"height": 1}, -2), ({"alpha": -1.0}, -1),
    ({"curvature": 5}, -1), ({"block_schedule": 2}, -1),
])
def test_batch_invalid_params(lib, over, status):
    lib.mg_curv_batch_init.restype = C.c_int
    lib.mg_curv_batch_init.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.mg_curv_batch_last_error.restype = C.c_char_p
    arr = _batch_params(lib, [(32, 40), (64, 64)], **over)
    b = C.c_void_p()
    assert lib.mg_curv_batch_init(arr, 2, None, C.byref(b)) == status
    assert not b.value
    assert lib.mg_curv_batch_last_error(None)


def test_batch_mismatched_search_constants_and_empty(lib):
    lib.mg_curv_batch_init.restype = C.c_int
    lib.mg_curv_batch_init.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
    arr = _batch_params(lib, [(32, 40), (64, 64)])
    arr[1].samples = 8
    b = C.c_void_p()
    assert lib.mg_curv_batch_init(arr, 2, None, C.byref(b)) == -1
    lib.mg_curv_batch_last_error.restype = C.c_char_p
    mixed = _batch_params(lib, [(32, 40), (64, 64)])
    mixed[1].block_schedule = 1
    assert lib.mg_curv_batch_init(mixed, 2, None, C.byref(b)) == -1
    assert b"block_schedule" in lib.mg_curv_batch_last_error(None)
    assert lib.mg_curv_batch_init(arr, 0, None, C.byref(b)) == -1
    assert lib.mg_curv_batch_init(None, 2, None, C.byref(b)) == -1


@pytest.mark.parametrize("levels,schedule,status", [
    (0, 0, -1), (31, 1, -1), (28, 0, -1), (27, 1, -1), (27, 0, -5), (26, 1, -5)])
def test_block_side_limit(lib, levels, schedule, status):
    """Ring counts (8b) must stay in int range: a level whose block side exceeds 2^26 is rejected
    before any device work, for single images and batches.  A 2^29 + 1 by 2 image would default
    to J = 30 (side 2^29); J = 27 is the largest with nested blocks (2^26) and J = 26 with
    2^j - 1 blocks.  Allowed cases reach the device check (-5 without a GPU)."""
    import torch
    if status == -5 and torch.cuda.is_available():
        pytest.skip("a GPU is present; the allowed cases would allocate a 2^30-pixel image")
    p = Params()
    lib.mg_curv_default_params(C.byref(p), (1 << 29) + 1, 2)
    p.levels, p.block_schedule = levels, schedule
    ctx = C.c_void_p(1234)
    assert lib.mg_curv_init(C.byref(p), None, C.byref(ctx)) == status
    if status == -1:
        assert b"2^26" in lib.mg_curv_last_error(None)
        lib.mg_curv_batch_init.restype = C.c_int
        lib.mg_curv_batch_init.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
        arr = (Params * 1)(p)
        b = C.c_void_p()
        assert lib.mg_curv_batch_init(arr, 1, None, C.byref(b)) == -1


def test_batch_no_device(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib.mg_curv_batch_init.restype = C.c_int
    lib.mg_curv_batch_init.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]
    arr = _batch_params(lib, [(32, 40), (64, 64)])
    b = C.c_void_p()
    assert lib.mg_curv_batch_init(arr, 2, None, C.byref(b)) == -5


class FbsParams(C.Structure):
    _fields_ = [("height", C.c_int32), ("width", C.c_int32), ("alpha", C.c_double),
                ("curvature", C.c_int32), ("levels", C.c_int32), ("state_dtype", C.c_int32),
                ("steps", C.c_int32), ("cycle", C.c_int32), ("reserved", C.c_int32)]


def _fbs(lib):
    lib.mg_fbs_init.restype = C.c_int
    lib.mg_fbs_init.argtypes = [C.POINTER(FbsParams), C.c_void_p, C.POINTER(C.c_void_p)]
    lib.mg_fbs_default_params.argtypes = [C.POINTER(FbsParams), C.c_int32, C.c_int32]
    lib.mg_fbs_last_error.restype = C.c_char_p
    lib.mg_fbs_last_error.argtypes = [C.c_void_p]
    for name in ("mg_fbs_vcycle", "mg_fbs_energy", "mg_fbs_sweep", "mg_fbs_level", "mg_fbs_solve"):
        getattr(lib, name).restype = C.c_int
    return lib


def test_fbs_params_struct_layout(lib):
    _fbs(lib)
    assert C.sizeof(FbsParams) == 40
    p = FbsParams()
    lib.mg_fbs_default_params(C.byref(p), 64, 48)
    assert (p.height, p.width, p.alpha, p.curvature, p.levels, p.state_dtype) == (64, 48, 20.0, 0, 3, 0)
    assert (p.steps, p.cycle, p.reserved) == (1, 0, 0)


@pytest.mark.parametrize("field,value,status", [
    ("height", 1, -2), ("width", 0, -2), ("alpha", -1.0, -1), ("alpha", float("nan"), -1),
    ("curvature", 2, -1), ("state_dtype", 7, -3), ("levels", 0, -1), ("levels", 17, -1),
    ("steps", 0, -1), ("steps", 65, -1), ("cycle", 2, -1), ("reserved", 1, -1),
])
def test_fbs_invalid_params_rejected_before_device(lib, field, value, status):
    _fbs(lib)
    p = FbsParams()
    lib.mg_fbs_default_params(C.byref(p), 64, 64)
    setattr(p, field, value)
    ctx = C.c_void_p(1234)
    assert lib.mg_fbs_init(C.byref(p), None, C.byref(ctx)) == status
    assert not ctx.value
    assert lib.mg_fbs_last_error(None)


def test_fbs_null_arguments_and_no_device(lib):
    import torch
    _fbs(lib)
    ctx = C.c_void_p()
    assert lib.mg_fbs_init(None, None, C.byref(ctx)) == -1
    assert lib.mg_fbs_vcycle(None, None, None, None) == -1
    assert lib.mg_fbs_energy(None, None, None, None) == -1
    assert lib.mg_fbs_sweep(None, None, None, 1, 0) == -1
    assert lib.mg_fbs_level(None, None, None, 1) == -1
    lib.mg_fbs_destroy(None)
    if torch.cuda.is_available():
        return
    p = FbsParams()
    lib.mg_fbs_default_params(C.byref(p), 64, 64)
    assert lib.mg_fbs_init(C.byref(p), None, C.byref(ctx)) == -5
    assert b"device" in lib.mg_fbs_last_error(None).lower()


class ReconParams(C.Structure):
    _fields_ = [("height", C.c_int32), ("width", C.c_int32), ("alpha", C.c_double), ("blur_sigma", C.c_double),
                ("levels", C.c_int32), ("state_dtype", C.c_int32), ("cg_iters", C.c_int32), ("reserved", C.c_int32)]


def _recon(lib):
    lib.mg_recon_init.restype = C.c_int
    lib.mg_recon_init.argtypes = [C.POINTER(ReconParams), C.c_void_p, C.POINTER(C.c_void_p)]
    lib.mg_recon_default_params.argtypes = [C.POINTER(ReconParams), C.c_int32, C.c_int32]
    lib.mg_recon_last_error.restype = C.c_char_p
    lib.mg_recon_last_error.argtypes = [C.c_void_p]
    for name in ("mg_recon_vcycle", "mg_recon_energy", "mg_recon_sweep", "mg_recon_solve"):
        getattr(lib, name).restype = C.c_int
    return lib


def test_recon_params_layout_and_validation(lib):
    import torch
    _recon(lib)
    assert C.sizeof(ReconParams) == 40
    p = ReconParams()
    lib.mg_recon_default_params(C.byref(p), 32, 24)
    assert (p.height, p.width, p.alpha, p.blur_sigma, p.levels, p.state_dtype, p.cg_iters, p.reserved) == \
        (32, 24, 0.01, 1.0, 3, 0, 20, 0)
    for field, value, status in [("height", 1, -2), ("alpha", -1.0, -1), ("blur_sigma", 0.0, -1),
                                 ("state_dtype", 3, -3), ("levels", 0, -1), ("cg_iters", 0, -1), ("reserved", 2, -1)]:
        q = ReconParams()
        lib.mg_recon_default_params(C.byref(q), 32, 24)
        setattr(q, field, value)
        ctx = C.c_void_p(99)
        assert lib.mg_recon_init(C.byref(q), None, C.byref(ctx)) == status, field
        assert not ctx.value
    ctx = C.c_void_p()
    assert lib.mg_recon_init(None, None, C.byref(ctx)) == -1
    assert lib.mg_recon_vcycle(None, None, None, None) == -1
    assert lib.mg_recon_energy(None, None, None, None) == -1
    assert lib.mg_recon_sweep(None, None, None, 1, 0) == -1
    lib.mg_recon_destroy(None)
    if not torch.cuda.is_available():
        assert lib.mg_recon_init(C.byref(p), None, C.byref(ctx)) == -5


@pytest.mark.parametrize("field,value,status", [
    ("height", 1, -2), ("alpha", 0.0, -1), ("curvature", 3, -1), ("state_dtype", 4, -3),
])
def test_energy_noalloc_validates_before_device(lib, field, value, status):
    lib.mg_curv_energy_noalloc.restype = C.c_int
    lib.mg_curv_energy_noalloc.argtypes = [C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    p = Params()
    lib.mg_curv_default_params(C.byref(p), 64, 64)
    setattr(p, field, value)
    assert lib.mg_curv_energy_noalloc(C.byref(p), None, C.c_void_p(4096), C.c_void_p(1 << 20),
                                      C.c_void_p(1 << 24)) == status
    assert lib.mg_curv_last_error(None)
    assert lib.mg_curv_energy_noalloc(None, None, None, None, None) == -1
    lib.mg_curv_default_params(C.byref(p), 64, 64)
    # u overlapping f, and a null output, are rejected before any device call
    assert lib.mg_curv_energy_noalloc(C.byref(p), None, C.c_void_p(4096), C.c_void_p(4096 + 64),
                                      C.c_void_p(1 << 24)) == -1
    assert lib.mg_curv_energy_noalloc(C.byref(p), None, C.c_void_p(4096), C.c_void_p(1 << 20), None) == -1


def test_library_carries_its_source_hash(lib):
    from paper_2204_07921_amd import build
    lib.mg_curv_build_id.restype = C.c_char_p
    assert lib.mg_curv_build_id().decode() == build.source_hash()


def test_binding_refuses_a_stale_library(monkeypatch):
    from paper_2204_07921_amd import build, mgcurv
    monkeypatch.setattr(build, "source_hash", lambda: "0" * 16)
    with pytest.raises(ImportError, match="built from other sources"):
        mgcurv._load()
