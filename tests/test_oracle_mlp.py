"""Pins of the FP64 surrogate-MLP reference (CPU)."""
import numpy as np

from oracle import mlp


def test_parameter_count():
    assert mlp.N_PARAMS == 134918


def test_bf16_rounding_is_nearest_even():
    one = 1.0
    ulp = 2.0 ** -7                       # bfloat16 spacing at 1
    vals = np.array([one, one + ulp / 2, one + 3 * ulp / 2, one + ulp / 4, -(one + 3 * ulp / 4), 3.0e38])
    r = mlp.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                    # tie -> even (1.0)
    assert r[2] == one + 2 * ulp          # tie -> even (1 + 2 ulp)
    assert r[3] == 1.0
    assert r[4] == -(one + ulp)
    assert np.isfinite(r[5])


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    p = mlp.init_params(5) * 0.5
    x = rng.normal(size=(7, 6))
    t = rng.normal(size=(7, 6))
    loss, g = mlp.loss_and_grad(p, x, t)
    idx = rng.choice(mlp.N_PARAMS, size=60, replace=False)
    # include every block: W1, b1, W2, b2, W3, b3, W4, b4
    offs = np.cumsum([0] + [s for o, i in mlp.SIZES for s in (o * i, o)])
    idx = np.concatenate([idx, offs[:-1] + 1])
    eps = 1e-6
    for k in idx:
        pp = p.copy()
        pp[k] += eps
        pm = p.copy()
        pm[k] -= eps
        fd = (mlp.loss_and_grad(pp, x, t)[0] - mlp.loss_and_grad(pm, x, t)[0]) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_silu_derivative():
    z = np.linspace(-6, 6, 101)
    fd = (mlp.silu(z + 1e-6) - mlp.silu(z - 1e-6)) / 2e-6
    assert np.allclose(mlp.dsilu(z), fd, atol=1e-8)


def test_bf16_emulation_is_close_to_fp64():
    rng = np.random.default_rng(4)
    p = mlp.init_params(6)
    x = rng.normal(size=(32, 6))
    y64, _ = mlp.forward(p, x)
    y16, _ = mlp.forward(p, x, bf16=True)
    assert np.abs(y16 - y64).max() <= 0.05 * np.abs(y64).max()


def test_split_bf16_product_is_near_fp32():
    """Three-term split bf16 (Ah Bh + Ah Bl + Al Bh) recovers the product to
    ~2^-16 relative, where a single bf16 rounding leaves ~2^-9."""
    rng = np.random.default_rng(7)
    A = rng.normal(size=(64, 256))
    B = rng.normal(size=(256, 32))
    ref = A @ B
    norm = np.abs(A) @ np.abs(B)
    e3 = np.abs(mlp.split_product(A, B) - ref) / norm
    e1 = np.abs(mlp.bf16_round(A) @ mlp.bf16_round(B) - ref) / norm
    assert e3.max() < 2.0 ** -14
    assert e1.max() > 2.0 ** -11
    hi, lo = mlp.split_bf16(A)
    assert np.array_equal(mlp.bf16_round(hi), hi) and np.array_equal(mlp.bf16_round(lo), lo)
    assert np.abs(hi + lo - A).max() <= 2.0 ** -16 * np.abs(A).max()
