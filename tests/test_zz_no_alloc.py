"""mg_curv_energy_noalloc (the energy without a context, its partial sums in the library's static
device array) against mg_curv_energy on the same inputs: the same kernels and summation order, so
the same value bit for bit, and the oracle's energy to 2 N eps.  Two calls in a row, the second on
a smaller image, for both state dtypes and both curvature kinds."""
import numpy as np
import pytest
import torch

from synth import noisy_image

pytestmark = pytest.mark.gpu


def _inputs(h, w, seed, dtype):
    f, _ = noisy_image(h, w, seed, 0.1, dtype=np.float32 if dtype == torch.float32 else np.float64)
    f = f.astype(np.float64)
    u = f + 0.05 * np.random.default_rng(seed + 3).standard_normal(f.shape)
    if dtype == torch.float32:
        u = u.astype(np.float32).astype(np.float64)
    return u, f


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("kind", [0, 1])
def test_energy_noalloc_matches_context_energy(orc, dtype, kind):
    from paper_2204_07921_amd import mgcurv as mg
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    for call, (h, w) in enumerate([(1024, 768), (37, 53)]):
        print(f"\n[case] energy_noalloc call {call} {h}x{w} kind={kind} {dtype}", flush=True)
        u, f = _inputs(h, w, 11 + call, dtype)
        ud = torch.tensor(u, dtype=dtype, device="cuda")
        fd = torch.tensor(f, dtype=dtype, device="cuda")
        params = mg.default_params(h, w, alpha=20.0, curvature=kind,
                                   state_dtype=mg.MG_F64 if dtype == torch.float64 else mg.MG_F32)
        out.fill_(float("nan"))
        mg.mg_curv_energy_noalloc(params, ud, fd, out)
        torch.cuda.synchronize()
        e_noalloc = float(out.item())
        s = mg.Solver(h, w, alpha=20.0, kind=kind, dtype=dtype)
        e_ctx = s.energy(ud, fd)
        s.close()
        e_orc = orc.oracle.energy(kind, u, f, 20.0)
        assert e_noalloc == e_ctx, (call, e_noalloc, e_ctx)
        assert abs(e_noalloc - e_orc) <= 2.2e-16 * h * w * abs(e_orc), (call, e_noalloc, e_orc)


def test_energy_noalloc_rejects_bad_arguments():
    from paper_2204_07921_amd import mgcurv as mg
    u, f = _inputs(32, 32, 1, torch.float32)
    ud = torch.tensor(u, dtype=torch.float32, device="cuda")
    fd = torch.tensor(f, dtype=torch.float32, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    params = mg.default_params(32, 32)
    with pytest.raises(mg.MgCurvError) as ei:
        mg.mg_curv_energy_noalloc(params, fd, fd, out)
    assert ei.value.status == -1
    bad = mg.default_params(32, 32, alpha=-1.0)
    with pytest.raises(mg.MgCurvError) as ei:
        mg.mg_curv_energy_noalloc(bad, ud, fd, out)
    assert ei.value.status == -1
