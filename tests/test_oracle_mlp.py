"""Pins of the FP64 MLP reference: backward against central finite differences
of the forward pass, and the bfloat16 rounding against PyTorch's conversion."""
import numpy as np
import pytest

from oracle import mlp


def test_parameter_count():
    assert mlp.N_PARAMS == 8577


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    flat = mlp.init(3) * 0.8
    f = rng.uniform(-1.2, 1.2, (37, 2))
    t = rng.normal(-3.0, 2.0, 37)
    loss, g = mlp.mse_grad(flat, f, t)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False), [0, 1, 127, 128, 8576]])
    for i in idx:
        h = 1e-6 * max(1.0, abs(flat[i]))
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        lp, _ = mlp.mse_grad(fp, f, t)
        lm, _ = mlp.mse_grad(fm, f, t)
        num = (lp - lm) / (2 * h)
        assert g[i] == pytest.approx(num, rel=1e-5, abs=1e-9), i


def test_features_map_ranges():
    f = mlp.features([1e-4, 1e2], [2.0 ** -24, 1 - 2.0 ** -24])
    assert np.allclose(f[:, 0], [-1.0, 1.0])
    # logit of the extreme 23-bit midpoints is -+ 24 ln 2 (to 1e-7), scaled by 1/16
    assert np.allclose(f[:, 1], [-24 * np.log(2) / 16, 24 * np.log(2) / 16], atol=1e-6)


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    a = np.concatenate([rng.normal(0, 10, 10000), [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3e38]])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(a), ref)
