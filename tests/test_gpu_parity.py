"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances, derived from the arithmetic:
  * FP64 state: the two sides differ only in summation order and in rounding
    of algebraically equal expressions (about 1e-16 relative per term); the
    local searches take the same branches unless a derivative is within
    rounding of zero, so u agrees to <= 1e-10 after 20 V-cycles (the target
    stated for the FP64 mode) and a single sweep to <= 1e-12.
  * FP32 state: both sides run the local solve in FP64 on the same float
    inputs and round the result to float, so they agree to an ulp or two
    (<= 1e-6 at unit scale) with the oracle's float-state option; against the
    pure FP64 oracle the target is <= 1e-4.
  * Energy: two summation orders of N non-negative terms differ by at most
    about 2 N eps relative.
"""
import json
import os

import numpy as np
import pytest
import torch

from synth import noisy_image
from tests.parity_helpers import _blocks_of, _check_sweep_against_oracle, assert_untouched, full_grid_check

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def mg():
    from paper_2204_07921_amd import mgcurv
    return mgcurv


def dev(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _f_and_u(h, w, seed, sigma, dtype, perturb=0.0):
    f, _ = noisy_image(h, w, seed, sigma, dtype=np.float32 if dtype == torch.float32 else np.float64)
    f = f.astype(np.float64)
    u = f.copy()
    if perturb:
        rng = np.random.default_rng(seed + 77)
        u = u + perturb * rng.standard_normal(u.shape)
        if dtype == torch.float32:
            u = u.astype(np.float32).astype(np.float64)
    return f, u


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("shape", [(2, 2), (37, 53), (64, 64), (1024, 1024)])
def test_energy_parity(mg, orc, dtype, kind, shape):
    h, w = shape
    _case(f"energy {shape} kind={kind} {dtype}")
    f, u = _f_and_u(h, w, 3, 0.1, dtype, perturb=0.05)
    s = mg.Solver(h, w, alpha=20.0, kind=kind, dtype=dtype)
    e_gpu = s.energy(dev(u, dtype), dev(f, dtype))
    e_orc = orc.oracle.energy(kind, u, f, 20.0)
    assert abs(e_gpu - e_orc) <= 2.2e-16 * max(h * w, 8) * abs(e_orc), (e_gpu, e_orc)


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("colours", [4, 9])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_single_sweep_parity_every_level(mg, orc, kind, colours, dtype):
    """Every level and colour of a ragged image (clipped blocks at every level)."""
    h, w = 45, 37
    f, u0 = _f_and_u(h, w, 5, 0.1, dtype, perturb=0.05)
    s = mg.Solver(h, w, alpha=20.0, kind=kind, dtype=dtype, fine_colours=colours)
    o = orc.Oracle(h, w, 20.0, kind, fine_colours=colours, round_f32=(dtype == torch.float32), threads=THREADS)
    assert s.levels == o.levels
    fd = dev(f, dtype)
    for level in range(1, o.levels + 1):
        for colour in range(o.num_colours(level)):
            _case(f"sweep kind={kind} colours={colours} {dtype} level={level} colour={colour}")
            ug = dev(u0, dtype)
            s.sweep(ug, fd, level, colour)
            worst, n_equal = _check_sweep_against_oracle(o, f, u0, host(ug), level, colour,
                                                         fp64=dtype == torch.float64)
            assert n_equal <= 1, (level, colour, n_equal)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind", [0, 1])
def test_single_sweep_parity_coarse_levels(mg, orc, kind, dtype):
    """A ragged 300x260 image: the coarse levels (block side 64..256, corrections applied lazily at the
    end of a level) against the oracle, sweep by sweep, plus one whole level through mg_curv_level."""
    h, w = 300, 260
    f, u0 = _f_and_u(h, w, 8, 0.1, dtype, perturb=0.05)
    s = mg.Solver(h, w, alpha=20.0, kind=kind, dtype=dtype)
    o = orc.Oracle(h, w, 20.0, kind, round_f32=(dtype == torch.float32), threads=THREADS)
    fd = dev(f, dtype)
    for level in range(2, o.levels + 1):
        ug = dev(u0, dtype)
        before = u0.copy()
        for colour in range(4):
            _case(f"coarse sweep {h}x{w} kind={kind} {dtype} level={level} colour={colour}")
            s.sweep(ug, fd, level, colour)
            after = host(ug)
            worst, n_equal = _check_sweep_against_oracle(o, f, before, after, level, colour,
                                                         fp64=dtype == torch.float64)
            assert n_equal <= 1, (level, colour, n_equal)
            before = after
        # the same four colours through one mg_curv_level call (pending corrections)
        ul = dev(u0, dtype)
        s.level(ul, fd, level)
        assert torch.equal(ul, ug), level


def _trajectory(mg, orc, h, w, kind, colours, dtype, cycles, seed, sigma, levels=0):
    """Run the GPU sweep by sweep for `cycles` V-cycles, checking every sweep against the oracle
    from the GPU's own state; then compare with the free-running oracle."""
    fp64 = dtype == torch.float64
    f, _ = _f_and_u(h, w, seed, sigma, dtype)
    s = mg.Solver(h, w, alpha=20.0, kind=kind, levels=levels, dtype=dtype, fine_colours=colours)
    o = orc.Oracle(h, w, 20.0, kind, levels=s.levels, fine_colours=colours, round_f32=not fp64, threads=THREADS)
    fd = dev(f, dtype)
    ug = dev(f, dtype)
    uv = dev(f, dtype)   # same run through mg_curv_vcycle
    worst, n_equal, n_blocks = 0.0, 0, 0
    for cyc in range(cycles):
        for level in range(1, s.levels + 1):
            for colour in range(o.num_colours(level)):
                before = host(ug)
                s.sweep(ug, fd, level, colour)
                after = host(ug)
                wv, ne = _check_sweep_against_oracle(o, f, before, after, level, colour, fp64)
                worst = max(worst, wv)
                n_equal += ne
                n_blocks += len(_blocks_of(o, level, colour))
        s.vcycle(uv, fd)
        assert torch.equal(uv, ug), "mg_curv_vcycle and the sweep sequence must agree bitwise"
    uo = f.copy()
    n, trace = o.solve(uo, f, rel_tol=0.0, max_vcycles=cycles)
    e_gpu = s.energy(ug, fd)
    du = float(np.max(np.abs(host(ug) - uo)))
    print(f"sweep parity: max|dc| = {worst:.3e}, equal-minimum blocks {n_equal}/{n_blocks}; "
          f"free-running max|u_gpu - u_oracle| = {du:.3e}, energy {e_gpu:.10f} vs {trace[-1]:.10f}")
    assert n_equal <= max(2, n_blocks // 1000)
    return e_gpu, trace[-1], du


# Free-running energies.  The 20-cycle energy of this nonconvex, chaotic iteration moves when the
# state changes at the rounding level: tests/golden/free_run_spread.json holds, per case, the
# relative spread of the oracle's own 20-cycle energy over 200 runs from u_0 = f (1 + 1e-15 z)
# (written by tests/golden/free_run_spread.py, which calls only the oracle).  The GPU computes its
# sums in another order, so its energy is one more draw from that spread; it is held to 1.5 times
# the largest of the 200 (for seed 1 of the mean-curvature case that is 1.2e-5, for the others
# 1.5e-7 .. 1.3e-6).
_SPREAD = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                      "free_run_spread.json")))["cases"]


def free_run_tol(name):
    return 1.5 * _SPREAD[name]["rel_spread"]["max"]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_config_64_mean_fp64_20_vcycles(mg, orc, seed):
    """64x64, sigma 0.05, mean curvature, alpha 20, 6 levels, 4 colours, 20 V-cycles, FP64 state:
    every colour sweep of the GPU trajectory matches the oracle from the same state; the free-running
    energies agree to the amplification level the oracle itself shows under a 1e-15 perturbation."""
    _case(f"64x64 MC fp64 seed={seed}")
    e_gpu, e_orc, du = _trajectory(mg, orc, 64, 64, 0, 4, torch.float64, 20, seed, 0.05, levels=6)
    print(f"free-running energy gap {abs(e_gpu - e_orc) / e_orc:.3e}, tolerance {free_run_tol(f'mean_4_seed{seed}'):.3e}")
    assert abs(e_gpu - e_orc) <= free_run_tol(f"mean_4_seed{seed}") * e_orc


@pytest.mark.parametrize("kind,colours", [(1, 4), (0, 9), (1, 9)])
def test_config_64_variants_fp64(mg, orc, kind, colours):
    _case(f"64x64 kind={kind} colours={colours} fp64")
    e_gpu, e_orc, du = _trajectory(mg, orc, 64, 64, kind, colours, torch.float64, 20, 0, 0.05, levels=6)
    name = f"{'gauss' if kind else 'mean'}_{colours}_seed0"
    print(f"free-running energy gap {abs(e_gpu - e_orc) / e_orc:.3e}, tolerance {free_run_tol(name):.3e}")
    assert abs(e_gpu - e_orc) <= free_run_tol(name) * e_orc


@pytest.mark.parametrize("kind", [0, 1])
def test_fp32_state_parity(mg, orc, kind):
    """FP32 state, FP64 local math: every sweep matches the float-state oracle from the same state, and
    the free-running run matches it too; against the pure FP64 oracle the energy gap and max |du| are
    reported (FP32 rounding of the state changes later kink decisions, as any 1e-15 perturbation does)."""
    h, w = 96, 80
    _case(f"fp32 state {h}x{w} kind={kind}")
    e_gpu, e_orc, du = _trajectory(mg, orc, h, w, kind, 4, torch.float32, 15, 4, 0.1)
    assert du <= 1e-6
    f, _ = _f_and_u(h, w, 4, 0.1, torch.float32)
    o64 = orc.Oracle(h, w, 20.0, kind, threads=THREADS)
    u64 = f.copy()
    n, t64 = o64.solve(u64, f, rel_tol=0.0, max_vcycles=15)
    gap = abs(e_gpu - t64[-1]) / t64[-1]
    print(f"FP32-state GPU vs FP64 oracle: energy gap {gap:.3e}")
    assert gap <= 1e-4


def test_solve_stop_rule_matches_oracle(mg, orc):
    """Relative energy-change stop: same number of V-cycles and final energy as the oracle."""
    h, w = 80, 72
    _case("solve stop rule fp32")
    f, _ = _f_and_u(h, w, 9, 0.08, torch.float32)
    s = mg.Solver(h, w, alpha=20.0, kind=0, dtype=torch.float32)
    ug = dev(f, torch.float32)
    res = s.solve(ug, dev(f, torch.float32), rel_tol=1e-6, max_vcycles=300)
    o = orc.Oracle(h, w, 20.0, 0, round_f32=True, threads=THREADS)
    uo = f.copy()
    n, trace = o.solve(uo, f, rel_tol=1e-6, max_vcycles=300)
    print(f"gpu vcycles={res['vcycles']} oracle={n}")
    assert res["status"] == 0
    assert res["vcycles"] == n
    assert abs(res["energy"] - trace[-1]) <= 1e-9 * trace[-1]
    assert np.max(np.abs(host(ug) - uo)) <= 1e-6


@pytest.mark.parametrize("kind", [0, 1])
def test_full_cycle_matches_level_composition_and_oracle(mg, orc, kind):
    """Full V-cycle (levels 1..J then J-1..1, Section 2.2): the V-cycle call, in which coarse
    levels hand their corrections to the next level's sums pass in both directions, equals the
    same levels run one self-contained call at a time, bit for bit; and it matches the float-state
    oracle's full cycle from the same start."""
    h, w = 200, 170   # J = 8: levels 7 and 8 (b = 64, 128) are the lazily applied ones
    _case(f"full cycle {h}x{w} kind={kind}")
    f, _ = _f_and_u(h, w, 12, 0.1, torch.float32)
    s = mg.Solver(h, w, alpha=20.0, kind=kind, dtype=torch.float32, cycle=1)
    J = s.levels
    fd = dev(f, torch.float32)
    ua, ub = dev(f, torch.float32), dev(f, torch.float32)
    o = orc.Oracle(h, w, 20.0, kind, round_f32=True, threads=THREADS, cycle=1)
    uo = f.copy()
    for rep in range(2):
        s.vcycle(ua, fd)
        for level in list(range(1, J + 1)) + list(range(J - 1, 0, -1)):
            s.level(ub, fd, level)
        assert torch.equal(ua, ub), rep
        o.vcycle(uo, f)
        du = np.max(np.abs(host(ua) - uo))
        print(f"full cycle {rep + 1}: max |du| vs oracle {du:.3e}")
        assert du <= 1e-6
    half = mg.Solver(h, w, alpha=20.0, kind=kind, dtype=torch.float32)
    uh = dev(f, torch.float32)
    half.vcycle(uh, fd)
    assert not torch.equal(uh, ua)


@pytest.mark.parametrize("cycle", [0, 1])
def test_relerr_stop_rule_matches_oracle(mg, orc, cycle):
    """relErr(u) stop (Section 4): same number of V-cycles, final energy and state as the oracle."""
    h, w = 80, 72
    _case(f"relErr stop cycle={cycle}")
    # float state against the oracle's float-state option, as for the energy rule: both sides
    # round the same FP64 corrections to float, so states and norms agree
    f, _ = _f_and_u(h, w, 9, 0.08, torch.float32)
    s = mg.Solver(h, w, alpha=20.0, kind=0, dtype=torch.float32, cycle=cycle)
    ug = dev(f, torch.float32)
    res = s.solve_rule(ug, dev(f, torch.float32), 1e-3, max_vcycles=200, stop=mg.MG_STOP_RELERR_U)
    o = orc.Oracle(h, w, 20.0, 0, round_f32=True, threads=THREADS, cycle=cycle)
    uo = f.copy()
    n, trace = o.solve_rule(uo, f, 1e-3, max_vcycles=200, stop=1)
    print(f"gpu vcycles={res['vcycles']} oracle={n}")
    assert res["status"] == 0
    assert res["vcycles"] == n
    assert abs(res["energy"] - trace[-1]) <= 1e-9 * trace[-1]
    assert np.max(np.abs(host(ug) - uo)) <= 1e-6
    # the energy rule through the same entry point is mg_curv_solve
    ue = dev(f, torch.float32)
    r2 = s.solve_rule(ue, dev(f, torch.float32), 1e-6, max_vcycles=300, stop=mg.MG_STOP_ENERGY)
    r3 = s.solve(dev(f, torch.float32), dev(f, torch.float32), rel_tol=1e-6, max_vcycles=300)
    assert r2["vcycles"] == r3["vcycles"] and r2["energy"] == r3["energy"]


def test_not_converged_status(mg):
    f, _ = _f_and_u(32, 32, 1, 0.1, torch.float32)
    s = mg.Solver(32, 32, dtype=torch.float32)
    res = s.solve(dev(f, torch.float32), dev(f, torch.float32).clone(), rel_tol=1e-14, max_vcycles=2)
    assert res["status"] == mg.MG_NOT_CONVERGED and res["vcycles"] == 2


def _sampled_check(mg, orc, h, w, kind, dtype, levels_to_check, n_samples, warm_cycles, seed=0, sigma=0.1):
    f, _ = _f_and_u(h, w, seed, sigma, dtype)
    s = mg.Solver(h, w, alpha=20.0, kind=kind, dtype=dtype)
    o = orc.Oracle(h, w, 20.0, kind, round_f32=(dtype == torch.float32))
    fd = dev(f, dtype)
    ug = dev(f, dtype)
    for _ in range(warm_cycles):
        s.vcycle(ug, fd)
    rng = np.random.default_rng(seed)
    worst = 0.0
    for level in levels_to_check:
        colour = int(rng.integers(0, 4))
        _case(f"sampled {h}x{w} kind={kind} {dtype} level={level} colour={colour}")
        before = host(ug)
        s.sweep(ug, fd, level, colour)
        after = host(ug)
        assert_untouched(o, before, after, level, colour)
        m, n = o.grid(level)
        cand = [(p, q) for p in range(m) for q in range(n) if o.colour_of(level, p, q) == colour]
        pick = rng.choice(len(cand), size=min(n_samples, len(cand)), replace=False)
        for k in pick:
            p, q = cand[int(k)]
            r0, r1, c0, c1 = o.block_bounds(level, p, q)
            info = o.local_solve(before, f, (r0, r1, c0, c1))
            expect = before[r0:r1, c0:c1] + info.c
            if dtype == torch.float32:
                expect = expect.astype(np.float32).astype(np.float64)
            err = np.max(np.abs(after[r0:r1, c0:c1] - expect))
            worst = max(worst, err)
            tol = 1e-12 if dtype == torch.float64 else 2.5e-7
            assert err <= tol, (level, p, q, err, info.c)
    return worst


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("sigma", [0.05, 0.1])
@pytest.mark.parametrize("kind", [0, 1])
def test_full_grid_parity_1024(mg, orc, kind, sigma, dtype):
    """1024x1024, J = 10, the benchmark's launch configuration: after 3 V-cycles from u = f, every
    colour sweep of one more V-cycle (all ten levels) is compared pixel by pixel with the oracle's
    sweep from the GPU's own state (float state against the oracle's float-state option, bitwise
    except where the arg-min is ill-conditioned; FP64 state to 1e-10)."""
    h = w = 1024
    fp64 = dtype == torch.float64
    f, _ = _f_and_u(h, w, 0, sigma, dtype)
    s = mg.Solver(h, w, alpha=20.0, kind=kind, dtype=dtype)
    o = orc.Oracle(h, w, 20.0, kind, round_f32=not fp64, threads=THREADS)
    assert s.levels == o.levels == 10
    fd = dev(f, dtype)
    ug = dev(f, dtype)
    for _ in range(3):
        s.vcycle(ug, fd)
    total_blocks = total_equal = 0
    worst = 0.0
    for level in range(1, s.levels + 1):
        for colour in range(4):
            _case(f"full grid 1024 kind={kind} sigma={sigma} {dtype} level={level} colour={colour}")
            before = host(ug)
            s.sweep(ug, fd, level, colour)
            after = host(ug)
            n_blocks, n_equal, w_ = full_grid_check(o, f, before, after, level, colour, fp64)
            # ill-conditioned arg-mins are rare: at most 1 in 1000 blocks of a sweep (and 2 at coarse levels)
            assert n_equal <= max(2, n_blocks // 1000), (level, colour, n_equal, n_blocks)
            total_blocks += n_blocks
            total_equal += n_equal
            worst = max(worst, w_)
    print(f"full-grid parity: {total_blocks} blocks, {total_equal} on the equal-minimum criterion, "
          f"max |u_gpu - u_oracle| elsewhere {worst:.3e}")
    assert worst <= (1e-10 if fp64 else 0.0)


@pytest.mark.parametrize("sigma", [0.05, 0.1])
@pytest.mark.parametrize("kind", [0, 1])
def test_converged_state_1024_is_stationary_under_oracle(mg, orc, kind, sigma):
    """The end state of a 1024x1024 solve (float state, stop at a relative energy change below 1e-6):
    the method is nonconvex and its iteration chaotic at kinks of |kappa|, so the end state is
    judged by whether it is a stopping point of the oracle's own iteration.  From the GPU's final u,
    one oracle V-cycle (float-state option) lowers F by less than 1e-6 relative, and by the same
    amount as the GPU's own next V-cycle from that state.

    Mean curvature at sigma 0.05 does not reach the 1e-6 rule: its energy keeps falling by about
    1.4e-6 of itself per V-cycle for thousands of V-cycles (0.23 % between V-cycles 400 and 2000).
    There the end state after 400 V-cycles is checked the same way: the oracle's next V-cycle
    lowers F by the same amount as the GPU's (both still about 1.4e-6)."""
    h = w = 1024
    creeps = (kind, sigma) == (0, 0.05)
    _case(f"converged 1024 kind={kind} sigma={sigma}")
    f, _ = _f_and_u(h, w, 0, sigma, torch.float32)
    s = mg.Solver(h, w, alpha=20.0, kind=kind, dtype=torch.float32)
    fd = dev(f, torch.float32)
    ug = dev(f, torch.float32)
    res = s.solve(ug, fd, rel_tol=1e-6, max_vcycles=400 if creeps else 2000, trace=True)
    tr = res["trace"]
    last = abs(tr[-1] - tr[-2]) / tr[-1]
    u_end = host(ug)
    e_end = res["energy"]
    # the GPU's own next V-cycle from the end state
    un = ug.clone()
    e_next = s.vcycle(un, fd, want_energy=True)
    g = (e_end - e_next) / e_end
    # the oracle's V-cycle from the same state
    o = orc.Oracle(h, w, 20.0, kind, round_f32=True, threads=THREADS)
    e0 = o.energy(u_end, f)
    x = u_end.copy()
    o.vcycle(x, f)
    e1 = o.energy(x, f)
    r = (e0 - e1) / e0
    du_next = float(np.max(np.abs(host(un) - x)))
    print(f"status {res['status']} after {res['vcycles']} V-cycles, last change {last:.3e}; "
          f"next V-cycle: GPU {g:.3e}, oracle {r:.3e}; max |u_gpu - u_oracle| after it {du_next:.3e}; "
          f"energy GPU {e_end:.10f} oracle {e0:.10f}")
    assert abs(e0 - e_end) <= 2.2e-16 * h * w * e_end
    if creeps:
        assert res["status"] == 1 and 0.0 < r < 2e-6
    else:
        assert res["status"] == 0
        assert -1e-12 <= r < 1e-6
    assert abs(r - g) <= 1e-8


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("size,levels", [(4096, [1, 2, 7, 11, 12]), (8192, [1, 3, 10, 12, 13])])
def test_sampled_parity_large_fp32(mg, orc, kind, size, levels):
    """The large-scale configurations (4096^2 with J = 12 and 8192^2 with J = 13, sigma 0.1,
    float32 state) in the benchmark's launch configuration: sampled blocks of one colour per level
    against the oracle's local solve on the same state.  Levels with b >= 1024 run the
    streamed-record path."""
    worst = _sampled_check(mg, orc, size, size, kind, torch.float32, levels, 6, 1)
    print(f"worst sampled error {worst:.3e}")


def test_sampled_parity_streamed_coarse_blocks(mg, orc):
    """Blocks of side >= 1024 stream their ring from memory at every evaluation."""
    worst = _sampled_check(mg, orc, 1536, 1200, 0, torch.float32, [11, 9], 4, 1)
    print(f"worst sampled error {worst:.3e}")


@pytest.mark.parametrize("shape", [(2, 2), (2, 3), (3, 2), (5, 7), (33, 65), (65, 33)])
def test_small_and_ragged_shapes_fp64(mg, orc, shape):
    h, w = shape
    _case(f"ragged {shape}")
    _trajectory(mg, orc, h, w, 0, 4, torch.float64, 4, 6, 0.1)


def test_deterministic_bitwise(mg):
    _case("determinism 256x256")
    f, _ = _f_and_u(256, 256, 2, 0.1, torch.float32)
    s = mg.Solver(256, 256, dtype=torch.float32)
    fd = dev(f, torch.float32)
    outs = []
    for _ in range(2):
        ug = dev(f, torch.float32)
        for _ in range(3):
            s.vcycle(ug, fd)
        outs.append(host(ug))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_constant_image_is_fixed_point(mg, dtype):
    f = np.full((40, 56), 0.375)
    s = mg.Solver(40, 56, dtype=dtype)
    ug = dev(f, dtype)
    s.solve(ug, dev(f, dtype), rel_tol=0.0, max_vcycles=3)
    assert np.array_equal(host(ug), f)


def test_error_paths(mg):
    f, _ = _f_and_u(32, 32, 1, 0.1, torch.float32)
    s = mg.Solver(32, 32, dtype=torch.float32)
    fd = dev(f, torch.float32)
    with pytest.raises(mg.MgCurvError) as ei:
        s.vcycle(fd, fd)
    assert ei.value.status == -1
    bad = f.copy()
    bad[3, 4] = np.nan
    ub = dev(f, torch.float32)
    before = host(ub)
    with pytest.raises(mg.MgCurvError) as ei:
        s.solve(ub, dev(bad, torch.float32), rel_tol=1e-6, max_vcycles=3)
    assert ei.value.status == -6
    assert np.array_equal(host(ub), before)
    with pytest.raises(ValueError):
        s.vcycle(dev(f[:16], torch.float32), fd)
    with pytest.raises(TypeError):
        s.vcycle(dev(f, torch.float64), fd)
    with pytest.raises(mg.MgCurvError) as ei:
        s.solve_rule(dev(f, torch.float32), fd, 1e-4, max_vcycles=3, stop=7)
    assert ei.value.status == -1
    r = s.solve_rule(dev(f, torch.float32), fd, 0.0, max_vcycles=3, stop=mg.MG_STOP_RELERR_U)
    assert r["status"] == 0 and r["vcycles"] == 3
    with pytest.raises(mg.MgCurvError) as ei:
        mg.Solver(32, 32, dtype=torch.float32, cycle=2)
    assert ei.value.status == -1
