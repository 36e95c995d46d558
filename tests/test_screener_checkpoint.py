"""Screener checkpoints (host only): the safetensors round trip keeps the FP32
weights, the Adam state and the metadata exactly, and the BF16 copy is the
round-to-nearest-even image of the weights."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytest.importorskip("safetensors")

from paper_2607_04310_amd import inputs, screener


def _bf16_rne(x):
    u = x.astype(np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def test_checkpoint_round_trip(tmp_path):
    rng = np.random.default_rng(4)
    theta = torch.tensor(inputs.mlp_init_params(3))
    m = torch.tensor(rng.normal(size=inputs.MLP_PARAMS).astype(np.float32))
    v = torch.tensor(rng.random(inputs.MLP_PARAMS).astype(np.float32))
    path = tmp_path / "screener.safetensors"
    screener.save_checkpoint(path, theta, m, v, step=123, seed=3, hist=[1.5, 0.25])
    st = screener.load_checkpoint(path)
    assert torch.equal(st["theta"], theta)
    assert torch.equal(st["adam_m"], m) and torch.equal(st["adam_v"], v)
    assert st["step"] == 123 and st["seed"] == 3 and st["hist"] == [1.5, 0.25]
    bf = st["theta_bf16"].view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(bf, _bf16_rne(theta.numpy()))


def test_checkpoint_without_optimizer_state(tmp_path):
    theta = torch.tensor(inputs.mlp_init_params(0))
    path = tmp_path / "w.safetensors"
    screener.save_checkpoint(path, theta)
    st = screener.load_checkpoint(path)
    assert st["adam_m"] is None and st["adam_v"] is None and st["step"] == 0


def test_checkpoint_rejects_other_files(tmp_path):
    from safetensors.torch import save_file
    path = tmp_path / "other.safetensors"
    save_file({"theta": torch.zeros(7)}, str(path))
    with pytest.raises(ValueError):
        screener.load_checkpoint(path)
