"""The split coarse-level solve (several workgroups per block, cooperative launch) against the
one-workgroup solve: bitwise equal states after every V-cycle.

Both compute the arg min of Algorithm 3 (Section 2.2) with the same group sums over the same ring
records, in the same order of decisions, so the corrections must agree bit for bit.  The oracle
comparisons of the other GPU tests run with the split solve on (it is the default), so this file
only ties the two GPU forms together, over shapes whose colours give the split launches different
tree depths (one, two and four blocks per colour; ragged edges; rings held in registers and rings
streamed from per-workgroup record copies at sides 1023-2048), both block schedules, both
curvatures and both state types."""
import numpy as np
import pytest
import torch

from synth import noisy_image

pytestmark = pytest.mark.gpu


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("shape", [(1024, 1024), (1000, 700), (777, 1030), (2048, 2048), (2100, 1500)])
def test_split_equals_one_workgroup(shape, kind, dtype, schedule):
    from paper_2204_07921_amd import mgcurv as mg
    h, w = shape
    f, _ = noisy_image(h, w, 5, 0.1, dtype=np.float32 if dtype == torch.float32 else np.float64)
    a = mg.Solver(h, w, alpha=20.0, kind=kind, dtype=dtype, block_schedule=schedule)
    b = mg.Solver(h, w, alpha=20.0, kind=kind, dtype=dtype, block_schedule=schedule)
    b.set_split(False)
    assert a.split_active, "the split solve should be on for this size on a 256-CU device"
    assert not b.split_active
    fd = torch.tensor(f, dtype=dtype, device="cuda")
    ua = fd.clone()
    ub = fd.clone()
    for cyc in range(3):
        _case(f"split vs one workgroup {shape} kind {kind} {dtype} schedule {schedule} V-cycle {cyc}")
        a.vcycle(ua, fd)
        b.vcycle(ub, fd)
        torch.cuda.synchronize()
        assert torch.isfinite(ua).all()
        diff = (ua != ub).sum().item()
        assert diff == 0, f"{diff} pixels differ after V-cycle {cyc}"
    a.close()
    b.close()


def test_split_switch_round_trip():
    from paper_2204_07921_amd import mgcurv as mg
    s = mg.Solver(1024, 1024)
    assert s.split_active
    s.set_split(False)
    assert not s.split_active
    s.set_split(True)
    assert s.split_active
    assert mg.lib.mg_curv_set_split(s.ctx, 2) == -1   # MG_E_INVALID
    assert s.split_active
    small = mg.Solver(64, 64)   # no coarse colour with 7 or more workgroups per block fits: nothing to split
    assert not small.split_active
    s.close()
    small.close()


@pytest.mark.parametrize("samples,bisections", [(10, 7), (2, 5), (256, 64), (6, 4)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_split_equals_one_workgroup_other_search_constants(samples, bisections, dtype):
    """M not a power of two (the sample offsets are quotients), M below the workgroups per block,
    G below the tree depth of 6 and 8 (partial rounds; the split needs G >= 4), and the largest M
    and G the parameters allow (512 sample words)."""
    from paper_2204_07921_amd import mgcurv as mg
    h, w = 1024, 1024
    f, _ = noisy_image(h, w, 9, 0.1, dtype=np.float32 if dtype == torch.float32 else np.float64)
    kw = dict(alpha=20.0, kind=0, dtype=dtype, samples=samples, bisections=bisections)
    a = mg.Solver(h, w, **kw)
    b = mg.Solver(h, w, **kw)
    b.set_split(False)
    assert a.split_active
    fd = torch.tensor(f, dtype=dtype, device="cuda")
    ua = fd.clone()
    ub = fd.clone()
    for cyc in range(2):
        _case(f"split vs one workgroup M {samples} G {bisections} {dtype} V-cycle {cyc}")
        a.vcycle(ua, fd)
        b.vcycle(ub, fd)
        torch.cuda.synchronize()
        assert torch.isfinite(ua).all()
        assert torch.equal(ua, ub)
    a.close()
    b.close()


@pytest.mark.parametrize("polls", [0, 1, 4])
@pytest.mark.parametrize("shape", [(1024, 1024), (2048, 2048)])
def test_split_local_fallback_is_bitwise_equal(shape, polls):
    """Exchange waits cut short from the host: with 0 polls every workgroup evaluates every sample
    and tree node itself; with 1 or 4 polls some values arrive in time and the rest are evaluated
    locally, a mix that depends on timing.  The corrections must not depend on it (register and
    streamed rings)."""
    from paper_2204_07921_amd import mgcurv as mg
    h, w = shape
    f, _ = noisy_image(h, w, 13, 0.1, dtype=np.float32)
    a = mg.Solver(h, w, alpha=20.0, kind=0)
    b = mg.Solver(h, w, alpha=20.0, kind=0)
    a.set_split_polls(polls)
    b.set_split(False)
    assert a.split_active
    fd = torch.tensor(f, device="cuda")
    ua = fd.clone()
    ub = fd.clone()
    for cyc in range(2):
        _case(f"split with {polls} polls per wait {shape} V-cycle {cyc}")
        a.vcycle(ua, fd)
        b.vcycle(ub, fd)
        torch.cuda.synchronize()
        assert torch.equal(ua, ub)
    assert mg.lib.mg_curv_set_split_polls(a.ctx, -1) == -1   # MG_E_INVALID
    a.close()
    b.close()


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("shape", [(260, 4100), (4100, 260)])
def test_split_equals_one_workgroup_clipped_blocks(shape, kind):
    """Long thin images: colours of 3-9 blocks at sides 256-1024 and single blocks clipped to a
    few pixels across (260 x 4096 and 260 x 4 at side 4096), register and streamed rings."""
    from paper_2204_07921_amd import mgcurv as mg
    h, w = shape
    f, _ = noisy_image(h, w, 17, 0.1, dtype=np.float32)
    a = mg.Solver(h, w, alpha=20.0, kind=kind)
    b = mg.Solver(h, w, alpha=20.0, kind=kind)
    b.set_split(False)
    assert a.split_active
    fd = torch.tensor(f, device="cuda")
    ua = fd.clone()
    ub = fd.clone()
    for cyc in range(2):
        _case(f"split vs one workgroup {shape} kind {kind} V-cycle {cyc}")
        a.vcycle(ua, fd)
        b.vcycle(ub, fd)
        torch.cuda.synchronize()
        assert torch.isfinite(ua).all()
        assert torch.equal(ua, ub)
    a.close()
    b.close()
