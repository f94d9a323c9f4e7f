"""GPU BF16-MFMA MLP kernels against the FP64 oracle MLP (which emulates
the same bfloat16 rounding points)."""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_05386_amd import rt
    return rt, torch, rt.Tracer(0)


def _params(torch, n, scale=1.0):
    p = np.stack([mlp.init_params(10 + i) for i in range(n)]) * scale
    rng = np.random.default_rng(1)
    for i in range(n):   # non-zero biases
        for k, (o, _) in zip(range(4), mlp.SIZES):
            mlp.split(p[i])[2 * k + 1][:] = rng.normal(0, 0.1, size=o)
    pt = torch.tensor(p, dtype=torch.float32, device="cuda")
    return p, pt, pt.to(torch.bfloat16)


# batches that are multiples of 8 take the vector-staged backward products,
# multiples of 128 the split-K weight gradient and the LDS-staged epilogue
# (264: a ragged last tile of 8 rows), the others the element-wise ones
@pytest.mark.parametrize("n,batch", [(3, 37), (2, 300), (1, 1), (2, 264), (1, 1024), (3, 512)])
def test_mlp_forward_backward_match_oracle(env, n, batch):
    rt, torch, tr = env
    say("mlp fwd/bwd n_nets=%d batch=%d" % (n, batch))
    p, pt, pb = _params(torch, n)
    rng = np.random.default_rng(2)
    x = rng.normal(size=(n, batch, 6)).astype(np.float32)
    dy = rng.normal(size=(n, batch, 6)).astype(np.float32)
    work = tr.mlp_work(n, batch)
    y = tr.mlp_fwd(pb, pt, torch.tensor(x, device="cuda"), work).cpu().numpy()
    g = tr.mlp_bwd(pb, pt, torch.tensor(dy, device="cuda"), work).cpu().numpy()
    p32 = p.astype(np.float32).astype(np.float64)
    worst_f = worst_b = 0.0
    for i in range(n):
        yr, _ = mlp.forward(p32[i], x[i].astype(np.float64), bf16=True)
        ef = np.abs(y[i] - yr).max() / max(1.0, np.abs(yr).max())
        worst_f = max(worst_f, ef)
        # the oracle rounds at the same bf16 points; what remains is FP32
        # accumulation order (measured worst 4.1e-6)
        assert ef <= 2e-5, (i, ef)
        gr = mlp.backward(p32[i], x[i].astype(np.float64), dy[i].astype(np.float64), bf16=True)
        for blk, (a, b) in enumerate(zip(mlp.split(g[i].astype(np.float64)), mlp.split(gr))):
            err = np.abs(a - b).max() / max(1e-3, np.abs(b).max())
            worst_b = max(worst_b, err)
            # backward operands are rounded to bf16 from FP32 values that
            # differ from the oracle's FP64 ones by accumulation order; an
            # element that lies that close to a rounding boundary goes to
            # the neighbouring bf16 value (2^-8 relative), so a sum of 256
            # terms can move by about one bf16 ulp of one term (measured
            # worst 9.8e-4 of the largest component)
            assert err <= 3e-3, (i, blk, err, np.abs(b).max())
    say("worst relative error: forward %.2e, backward %.2e" % (worst_f, worst_b))


@pytest.mark.parametrize("n,batch", [(2, 1024), (3, 264)])
def test_mlp_backward_is_deterministic(env, n, batch):
    """The weight gradients split K over the waves of a block and sum the
    partial tiles in a fixed order, the FP32 layers sum fixed row chunks in
    order: two backward passes give the same bits."""
    rt, torch, tr = env
    say("mlp backward determinism n_nets=%d batch=%d" % (n, batch))
    p, pt, pb = _params(torch, n)
    rng = np.random.default_rng(5)
    x = torch.tensor(rng.normal(size=(n, batch, 6)).astype(np.float32), device="cuda")
    dy = torch.tensor(rng.normal(size=(n, batch, 6)).astype(np.float32), device="cuda")
    out = []
    for _ in range(2):
        work = tr.mlp_work(n, batch)
        tr.mlp_fwd(pb, pt, x, work)
        out.append(tr.mlp_bwd(pb, pt, dy, work).cpu().numpy())
    assert np.array_equal(out[0], out[1])


def test_adamw_step(env):
    rt, torch, tr = env
    say("adamw")
    rng = np.random.default_rng(3)
    n = 1000
    p = rng.normal(size=n).astype(np.float32)
    m = rng.normal(size=n).astype(np.float32) * 0.1
    v = np.abs(rng.normal(size=n)).astype(np.float32) * 0.01
    g = rng.normal(size=n).astype(np.float32)
    P, M, V, G = (torch.tensor(a, device="cuda") for a in (p, m, v, g))
    PB = P.to(torch.bfloat16)
    lr, b1, b2, eps, wd, step = 1e-3, 0.9, 0.999, 1e-8, 0.01, 7
    tr.adamw(P, PB, M, V, G, lr, step, b1, b2, eps, wd)
    m2 = b1 * m + (1 - b1) * g
    v2 = b2 * v + (1 - b2) * g * g
    p2 = p - lr * ((m2 / (1 - b1 ** step)) / (np.sqrt(v2 / (1 - b2 ** step)) + eps) + wd * p)
    assert np.allclose(P.cpu().numpy(), p2, rtol=1e-5, atol=1e-6)
    assert np.allclose(PB.float().cpu().numpy(), p2, rtol=1e-2, atol=1e-3)


def test_training_reduces_loss(env):
    rt, torch, tr = env
    say("mlp training on a smooth 6->6 map")
    n, batch = 2, 512
    p, pt, pb = _params(torch, n, scale=0.5)
    rng = np.random.default_rng(4)
    x = torch.tensor(rng.uniform(-1, 1, size=(n, batch, 6)), dtype=torch.float32, device="cuda")
    t = torch.sin(2.0 * x) * 0.5 + x.roll(1, dims=2) * 0.3
    m = torch.zeros_like(pt)
    v = torch.zeros_like(pt)
    work = tr.mlp_work(n, batch)
    losses = []
    for step in range(1, 301):
        y = tr.mlp_fwd(pb, pt, x, work)
        diff = y - t
        losses.append(float((diff * diff).sum() / (n * batch)))
        g = tr.mlp_bwd(pb, pt, 2.0 * diff / batch, work)
        tr.adamw(pt, pb, m, v, g, 2e-3, step)
    say("loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.05 * losses[0]
