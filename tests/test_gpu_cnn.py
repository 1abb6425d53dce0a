"""GPU tests of the warm-start CNN against the FP64 NumPy reference (oracle/cnn_ref.py).

Tolerances follow from bfloat16 storage: both sides round weights, activations and activation
gradients to bfloat16 at the same points (round to nearest even); the GPU accumulates in FP32,
the reference in FP64, so a stored value can land one bfloat16 step (2^-8 relative) away when
the two accumulations straddle a rounding boundary.  Layers are compared from the GPU's own
inputs (teacher forcing) so such steps do not compound.  The backward pass is compared element by
element in the same way (each layer from the GPU's own gradient of the layer above), and the
end-to-end parameter gradient by relative norm and direction per layer."""
import numpy as np
import pytest
import torch

from oracle import cnn_ref
from synth import init_params, noisy_image

pytestmark = pytest.mark.gpu

LAYER_SLICES = []
_k = 0
for _ci, _co in zip(cnn_ref.CHANNELS[:-1], cnn_ref.CHANNELS[1:]):
    LAYER_SLICES.append(slice(_k, _k + 9 * _ci * _co + _co))
    _k += 9 * _ci * _co + _co


@pytest.fixture(scope="module")
def mg():
    from paper_2204_07921_amd import mgcurv
    return mgcurv


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _batch(shapes, seed=0):
    fs = [noisy_image(h, w, seed + k, 0.08, dtype=np.float32)[0] for k, (h, w) in enumerate(shapes)]
    return fs


def _params(seed, scale=2.0):
    p = init_params(seed)
    p *= scale          # larger weights: ReLUs switch inside the test images
    p[LAYER_SLICES[-1]] *= 5.0
    for sl in LAYER_SLICES:  # non-zero biases exercise the bias paths
        stop = sl.stop
        co = 32 if sl is not LAYER_SLICES[-1] else 1
        p[stop - co:stop] = 0.05 * np.cos(np.arange(co))
    return p.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("shape", [(2, 20, 40), (1, 9, 45), (3, 33, 17)])
def test_forward_per_layer_matches_reference(mg, shape):
    n, h, w = shape
    _case(f"forward {shape}")
    f = np.stack(_batch([(h, w)] * n))
    p = _params(1)
    net = mg.WarmStartCNN(n * h * w, p)
    fd = torch.tensor(f, device="cuda")
    u = net.forward(fd).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    layers = cnn_ref.unpack(p)
    a = f[..., None].astype(np.float64)
    for l in range(5):
        W, b = layers[l]
        ref = cnn_ref.round_bf16(np.maximum(cnn_ref.conv(a, cnn_ref.round_bf16(W), b), 0.0))
        got = net.activation(l + 1, (n, h, w)).astype(np.float64)
        step = 2.0 ** -7 * np.maximum(np.abs(ref), 1e-30)   # one bfloat16 step at the value
        bad = np.abs(got - ref) > step + 1e-4 * np.max(np.abs(ref))
        assert np.count_nonzero(bad) == 0, (l, np.max(np.abs(got - ref)))
        a = got                                             # teacher forcing
    W5, b5 = layers[5]
    ref_u = f + cnn_ref.conv(a, cnn_ref.round_bf16(W5), b5)[..., 0]
    assert np.max(np.abs(u - ref_u)) <= 1e-5 * (1 + np.max(np.abs(ref_u - f)))


def test_gradients_match_reference(mg):
    n, h, w = 2, 24, 40
    _case("gradients")
    f = np.stack(_batch([(h, w)] * n, seed=10))
    target = (f + 0.05 * np.sin(np.arange(w))[None, None, :]).astype(np.float32)
    p = _params(2)
    net = mg.WarmStartCNN(n * h * w, p)
    loss_g, g = net.gradients(torch.tensor(f, device="cuda"), torch.tensor(target, device="cuda"))
    loss_r, gr = cnn_ref.loss_and_grad(p, f.astype(np.float64), target.astype(np.float64), bf16=True)
    assert abs(loss_g - loss_r) <= 1e-3 * loss_r, (loss_g, loss_r)
    for l, sl in enumerate(LAYER_SLICES):
        a, b = g[sl].astype(np.float64), gr[sl]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
        print(f"layer {l}: relative gradient error {rel:.2e}, cosine {cos:.6f}")
        assert rel <= 2e-2 and cos >= 0.9995, (l, rel, cos)


@pytest.mark.parametrize("shape", [(2, 24, 40), (1, 19, 70), (3, 9, 33)])
def test_backward_per_layer_matches_reference(mg, shape):
    """Element-wise, teacher-forced backward pass.  From the GPU's own activations and its own
    gradient of each layer's output, the FP64 reference computes that layer's input gradient (3x3
    transposed convolution with the bfloat16 weights, ReLU mask, bfloat16 rounding) and its weight
    and bias gradients; every element is compared.  Input gradients may differ by one bfloat16 step
    (FP32 vs FP64 accumulation straddling a rounding boundary); weight gradients by the FP32
    accumulation error, at most 1e-4 of the sum of the absolute products of each element."""
    n, h, w = shape
    _case(f"backward per layer {shape}")
    f = np.stack(_batch([(h, w)] * n, seed=40))
    target = (f + 0.05 * np.cos(0.3 * np.arange(w))[None, None, :] - 0.02).astype(np.float32)
    p = _params(4)
    net = mg.WarmStartCNN(n * h * w, p)
    fd, td = torch.tensor(f, device="cuda"), torch.tensor(target, device="cuda")
    u = net.forward(fd).cpu().numpy()
    dz, dz5, g = net.gradient_trace(fd, td)
    acts = [f[..., None].astype(np.float64)] + [net.activation(l, (n, h, w)).astype(np.float64) for l in range(1, 6)]
    layers = cnn_ref.unpack(p)
    # output gradient of the loss: 2 (u - target) / N from the GPU's own prediction, in float32
    r32 = (u - target).astype(np.float32).astype(np.float64)
    ref5 = 2.0 * r32 / (n * h * w)
    assert np.max(np.abs(dz5 - ref5)) <= 2.0 ** -23 * np.max(np.abs(ref5)), np.max(np.abs(dz5 - ref5))
    # input gradients, layer by layer from the GPU's gradient of the layer above
    g_up = dz5.astype(np.float64)[..., None]
    for l in range(5, 0, -1):
        W, _ = layers[l]
        ref = cnn_ref.round_bf16(cnn_ref.conv_transpose_taps(g_up, cnn_ref.round_bf16(W)) * (acts[l] > 0))
        got = dz[l - 1].astype(np.float64)
        step = 2.0 ** -7 * np.abs(ref) + 1e-4 * np.max(np.abs(ref))
        bad = np.abs(got - ref) > step
        print(f"dz_{l - 1}: max |got - ref| {np.max(np.abs(got - ref)):.3e}, "
              f"elements off by a bfloat16 step {np.count_nonzero(got != ref)} of {ref.size}")
        assert np.count_nonzero(bad) == 0, (l, np.max(np.abs(got - ref)))
        # a wrong tap or channel would move most elements; rounding-boundary splits stay rare
        assert np.count_nonzero(got != ref) <= max(4, ref.size // 50), l
        g_up = got
    # weight and bias gradients of every layer from the GPU's inputs and output gradients
    for l, sl in enumerate(LAYER_SLICES):
        a = acts[l]
        d = dz5.astype(np.float64)[..., None] if l == 5 else dz[l].astype(np.float64)
        refW = cnn_ref.weight_grad(a, d)
        absW = cnn_ref.weight_grad(np.abs(a), np.abs(d))
        refb = d.sum(axis=(0, 1, 2))
        absb = np.abs(d).sum(axis=(0, 1, 2))
        gl = g[sl].astype(np.float64)
        gotW, gotb = gl[:refW.size].reshape(refW.shape), gl[refW.size:]
        errW = np.abs(gotW - refW) / (absW + 1e-30)
        errb = np.abs(gotb - refb) / (absb + 1e-30)
        print(f"layer {l}: weight gradient max error {errW.max():.2e}, bias {errb.max():.2e} of the absolute sums")
        assert np.all(np.abs(gotW - refW) <= 1e-4 * absW + 1e-12), (l, errW.max())
        assert np.all(np.abs(gotb - refb) <= 1e-4 * absb + 1e-12), (l, errb.max())


def test_adam_step_matches_reference(mg):
    n, h, w = 1, 16, 32
    _case("adam")
    f = np.stack(_batch([(h, w)], seed=20))
    target = (f * 0.9).astype(np.float32)
    p = _params(3)
    net = mg.WarmStartCNN(n * h * w, p)
    fd, td = torch.tensor(f, device="cuda"), torch.tensor(target, device="cuda")
    w64, m, v = p.copy(), np.zeros_like(p), np.zeros_like(p)
    for t in (1, 2):
        _, g = net.gradients(fd, td)
        net.train_step(fd, td, lr=1e-3, want_loss=False)
        w64, m, v = cnn_ref.adam_step(w64, g.astype(np.float64), m, v, t, lr=1e-3)
        got = net.get_params().astype(np.float64)
        assert np.max(np.abs(got - w64)) <= 1e-6, t
        w64 = got  # continue from the GPU's float32 state


def test_training_reduces_loss_and_is_deterministic(mg):
    _case("training")
    n, h, w = 8, 32, 32
    rng = np.random.default_rng(0)
    f = np.stack(_batch([(h, w)] * n, seed=30))
    # a smooth target: the 3x3 box mean of f (a learnable denoiser)
    fp = np.pad(f, ((0, 0), (1, 1), (1, 1)), mode="edge")
    target = sum(fp[:, dy:dy + h, dx:dx + w] for dy in range(3) for dx in range(3)) / 9.0
    target = target.astype(np.float32)
    fd, td = torch.tensor(f, device="cuda"), torch.tensor(target, device="cuda")
    runs = []
    for _ in range(2):
        net = mg.WarmStartCNN(n * h * w, init_params(7))
        losses = [net.train_step(fd, td, lr=2e-3) for _ in range(150)]
        runs.append(net.get_params())
        print(f"loss {losses[0]:.3e} -> {losses[-1]:.3e}")
        assert losses[-1] < 0.3 * losses[0]
    assert np.array_equal(runs[0], runs[1])


def test_input_validation(mg):
    net = mg.WarmStartCNN(1000, init_params(0))
    f = torch.zeros(2, 30, 30, device="cuda")
    with pytest.raises(mg.MgCurvError):
        net.forward(f)          # 1800 pixels > capacity 1000
    with pytest.raises(ValueError):
        net.set_params(np.zeros(10))


def test_checkpoint_resume_is_bitwise(mg, tmp_path):
    """Train 6 Adam steps, checkpoint (parameters, moments, step) to a file, train 6 more; a fresh
    context restored from the file and trained the same 6 steps ends bit for bit equal."""
    from paper_2204_07921_amd import warmstart
    _case("checkpoint resume")
    n, h, w = 4, 24, 32
    f = np.stack(_batch([(h, w)] * n, seed=50))
    target = (0.9 * f + 0.05).astype(np.float32)
    fd, td = torch.tensor(f, device="cuda"), torch.tensor(target, device="cuda")
    a = mg.WarmStartCNN(n * h * w, init_params(11))
    for _ in range(6):
        a.train_step(fd, td, lr=1e-3, want_loss=False)
    path = str(tmp_path / "ckpt.npz")
    warmstart.save_checkpoint(path, a.get_state())
    for _ in range(6):
        a.train_step(fd, td, lr=1e-3, want_loss=False)
    b = mg.WarmStartCNN(n * h * w, init_params(99))
    st = warmstart.load_checkpoint(path)
    assert st["step"] == 6 and np.any(st["m"] != 0) and np.any(st["v"] != 0)
    b.set_state(st)
    for _ in range(6):
        b.train_step(fd, td, lr=1e-3, want_loss=False)
    assert np.array_equal(a.get_params(), b.get_params())
    sa, sb = a.get_state(), b.get_state()
    assert sa["step"] == sb["step"] == 12
    assert np.array_equal(sa["m"], sb["m"]) and np.array_equal(sa["v"], sb["v"])
    # restoring parameters alone (moments reset) does not reproduce the run
    c = mg.WarmStartCNN(n * h * w, st["params"])
    for _ in range(6):
        c.train_step(fd, td, lr=1e-3, want_loss=False)
    assert not np.array_equal(a.get_params(), c.get_params())
