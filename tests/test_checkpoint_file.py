"""The warm-start training checkpoint file (CPU): parameters, both Adam moments and the step survive a
save/load round trip exactly, and the file holds plain arrays only (it loads without pickle)."""
import numpy as np


def test_checkpoint_round_trip(tmp_path):
    from paper_2204_07921_amd import warmstart
    rng = np.random.default_rng(0)
    st = {"params": rng.standard_normal(37601).astype(np.float32),
          "m": rng.standard_normal(37601).astype(np.float32),
          "v": rng.random(37601).astype(np.float32), "step": 123}
    path = str(tmp_path / "c.npz")
    warmstart.save_checkpoint(path, st, {"note": "test"})
    back = warmstart.load_checkpoint(path)
    for k in ("params", "m", "v"):
        assert back[k].dtype == np.float32 and np.array_equal(back[k], st[k])
    assert back["step"] == 123 and back["meta"] == {"note": "test"}
    with np.load(path, allow_pickle=False) as z:
        assert sorted(z.files) == ["m", "meta", "params", "step", "v"]
