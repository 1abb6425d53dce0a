"""GPU tests of the learned warm start with the committed trained weights.

The gain test runs the plain batched solve from u0 = f (relative energy change 1e-6) and the
warm-started one (u0 = f + g(f), then V-cycles until the plain final energy (1 + 1e-6) is
reached) on images the network never saw, and checks that the warm start reaches the plain
energy in fewer V-cycles and less wall time, CNN included.  The fallback test forces an
unreachable target and checks that the refinement reports it."""
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws():
    from paper_2204_07921_amd import warmstart
    if not os.path.exists(warmstart.DEFAULT_WEIGHTS):
        pytest.skip("trained weights are not in the tree")
    return warmstart


def test_weights_load_and_match_layout(ws):
    from paper_2204_07921_amd import mgcurv
    params, meta = ws.load()
    assert params.size == 37601 and np.all(np.isfinite(params))
    net = mgcurv.WarmStartCNN(64 * 64, params)
    assert np.array_equal(net.get_params(), params)


def test_warm_start_gain(ws):
    from paper_2204_07921_amd import mgcurv
    params, _ = ws.load()
    print("\n[case] warm-start gain, 6 images of 512x512", flush=True)
    f = ws.make_inputs(6, 512, seed0=200000)
    net = mgcurv.WarmStartCNN(4 * 512 * 512, params)
    ws.forward_chunked(net, f)   # warm-up
    r = ws.evaluate(net, f, max_vcycles=600)
    print(r)
    assert r["warm"]["reached_plain_energy"] >= 5
    assert r["warm"]["vcycles_mean"] < r["plain"]["vcycles_mean"]
    assert r["warm"]["seconds"] < r["plain"]["seconds"]
    assert r["final_energy_gap_rel_max"] <= 1e-6


def test_unreachable_target_reports_not_converged(ws):
    from paper_2204_07921_amd import mgcurv
    params, _ = ws.load()
    f = ws.make_inputs(2, 128, seed0=300000)
    net = mgcurv.WarmStartCNN(2 * 128 * 128, params)
    u0 = ws.forward_chunked(net, f)
    _, res = ws.solve_batch(f, u0=u0, targets=[0.0, 0.0], max_vcycles=3, tune=False)
    assert res["status"] == 1 and res["image_status"] == [1, 1] and res["vcycles"] == [3, 3]
    s = mgcurv.Solver(128, 128, dtype=torch.float32)
    r1 = s.solve_target(u0[0].contiguous(), f[0].contiguous(), 0.0, max_vcycles=2)
    assert r1["status"] == 1 and r1["vcycles"] == 2
    r2 = s.solve_target(u0[0].contiguous(), f[0].contiguous(), 1e30, max_vcycles=5)
    assert r2["status"] == 0 and r2["vcycles"] == 0


def test_warm_start_refines_to_the_nine_colour_plain_energy(ws):
    """With the nine-colour pixel level the plain solve settles far below the four-colour one, and the
    network's prediction starts above that energy, so the warm start must refine.  On three unseen
    1024x1024 images: the prediction's energy is above F_plain; nine-colour V-cycles from it reach
    F_plain (1 + 1e-6) after at least one V-cycle and without fallback, in fewer V-cycles and less
    wall time (CNN included) than the plain nine-colour solve from u = f."""
    from paper_2204_07921_amd import mgcurv
    params, _ = ws.load()
    print("\n[case] nine-colour warm start, 3 images of 1024x1024", flush=True)
    f = ws.make_inputs(3, 1024, seed0=100000)
    net = mgcurv.WarmStartCNN(1024 * 1024, params)
    r = ws.evaluate_single(net, f, fine_colours=9)
    print({k: v for k, v in r.items() if k != "per_image"})
    for row in r["per_image"]:
        assert row["plain_status"] == 0
        assert row["cnn_energy"] > row["plain_energy"]
        assert 1 <= row["warm_vcycles"] < row["plain_vcycles"] and not row["fallback"]
        assert row["warm_energy"] <= row["plain_energy"] * (1 + 1e-6)
    assert r["warm"]["seconds"] < r["plain"]["seconds"]


def test_warm_start_refines_outside_the_training_noise(ws):
    """Noise sigma 0.2, outside the training range U[0.03, 0.12]: the batched protocol needs at least
    one refinement V-cycle per image and still reaches the plain energy sooner."""
    from paper_2204_07921_amd import mgcurv
    from synth import noisy_image
    params, _ = ws.load()
    print("\n[case] warm start at sigma 0.2, 4 images of 512x512", flush=True)
    f = torch.tensor(np.stack([noisy_image(512, 512, 400000 + k, 0.2, dtype=np.float32)[0] for k in range(4)]),
                     device="cuda")
    net = mgcurv.WarmStartCNN(4 * 512 * 512, params)
    ws.forward_chunked(net, f)   # warm-up
    r = ws.evaluate(net, f, max_vcycles=600)
    print(r)
    assert r["plain"]["converged"] == 4
    assert r["warm"]["reached_plain_energy"] == 4 and r["warm"]["fallbacks"] == 0
    assert r["warm"]["vcycles_max"] >= 1
    assert r["warm"]["vcycles_mean"] < r["plain"]["vcycles_mean"]
    assert r["final_energy_gap_rel_max"] <= 1e-6
