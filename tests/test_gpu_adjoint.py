"""GPU adjoint of the RK4 trace against central finite differences of the
FP64 oracle, plus the exact special cases of the gradient."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_05386_amd import rt
    return rt, torch


def gpu_grad(rt, torch, wl, theta, target_hit, target_id, mask, ckpt_every=100):
    """Full-frame GPU trace with tape, masked L2 loss, adjoint.  target_* and
    mask are full-frame numpy arrays [n_sets*H*W]."""
    tr = rt.Tracer(0)
    tr.set_metric(dict(wl["metric"], bumps=theta))
    tr.set_scene(wl["scene"])
    cam, rule = wl["camera"], wl["rule"]
    out, tape = tr.trace_fwd_ckpt(cam, rule, rule["max_steps"], ckpt_every)
    th = torch.from_numpy(np.ascontiguousarray(target_hit, np.float32)).cuda()
    ti = torch.from_numpy(np.ascontiguousarray(target_id, np.int32)).cuda()
    mk = torch.from_numpy(np.ascontiguousarray(mask, np.uint8)).cuda()
    loss, gh = tr.loss_l2(cam, out["hit"], out["id"], th, ti, mk)
    g = tr.trace_bwd(tape, gh, theta.shape[1])
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64), loss.cpu().numpy(), {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def fd_case(wl, set_index, pix):
    tm = dict(wl["metric"], bumps=wl["target_bumps"])
    tgt = oracle.Oracle(tm, wl["scene"], set_index).trace(wl["camera"], wl["rule"], pix)
    g, L, m = oracle.fd_gradient(wl["metric"], wl["scene"], wl["camera"], wl["rule"], pix, tgt["hit"], tgt["id"],
                                 set_index=set_index)
    return g, L, m, tgt


def check_close(g_gpu, g_fd):
    scale = np.abs(g_fd).max()
    tol = 1e-4 + 1e-3 * scale
    err = np.abs(g_gpu - g_fd).max()
    cos = float((g_gpu * g_fd).sum() / (np.linalg.norm(g_gpu) * np.linalg.norm(g_fd) + 1e-300))
    return err, tol, cos


def run_fd_parity(env, n_sets, size, sets, n_pix, seed):
    rt, torch = env
    wl = W.with_size(W.get("adjoint_64x512", n_sets=n_sets), size, size)
    HW = size * size
    theta = wl["metric"]["bumps"]
    target_hit = np.zeros((n_sets * HW, 3), np.float32)
    target_id = np.full(n_sets * HW, -7, np.int32)
    mask = np.zeros(n_sets * HW, np.uint8)
    fds = {}
    for s in sets:
        pix = W.pixel_sample(size, size, n_pix, seed=seed + s)
        g, L, m, tgt = fd_case(wl, s, pix)
        fds[s] = (g, L)
        target_hit[s * HW + pix] = tgt["hit"]
        target_id[s * HW + pix] = tgt["id"]
        mask[s * HW + pix[m]] = 1
        say("set", s, "FD loss", L, "stable masked pixels", int(m.sum()))
    g_gpu, loss, _ = gpu_grad(rt, torch, wl, theta, target_hit, target_id, mask)
    for s in sets:
        g_fd, L = fds[s]
        err, tol, cos = check_close(g_gpu[s], g_fd)
        say("set", s, "loss gpu %.6g fd %.6g" % (loss[s], L), "max err %.3g tol %.3g cos %.6f" % (err, tol, cos))
        assert abs(loss[s] - L) <= 1e-3 * max(1.0, L)
        assert err <= tol and cos >= 0.9999, (g_gpu[s], g_fd)
    return g_gpu


def test_adjoint_matches_fd_small(env):
    say("adjoint vs FP64 central FD (eps 1e-4), 2 sets x 8 bumps, 96x96 frame")
    run_fd_parity(env, n_sets=2, size=96, sets=[0, 1], n_pix=160, seed=40)


def test_adjoint_matches_fd_full_size(env):
    """64 sets x 512^2 in one launch (the benchmark configuration); the
    loss is restricted by the mask to seeded pixel samples of two sets,
    whose FD gradients the oracle computes pixel by pixel."""
    say("adjoint at full size (64 x 512^2), FD on sampled pixels of sets 0 and 37")
    g = run_fd_parity(env, n_sets=64, size=512, sets=[0, 37], n_pix=96, seed=70)
    others = [s for s in range(64) if s not in (0, 37)]
    assert np.all(g[others] == 0.0)


def _zero_target(wl, n_sets, HW):
    # target = the map itself shifted: any fixed target works for these checks
    return np.zeros((n_sets * HW, 3), np.float32)


def test_adjoint_exact_special_cases(env):
    rt, torch = env
    say("special cases: a = 0 everywhere; a_b = 0; a -> -a")
    n_sets, size = 3, 64
    wl = W.with_size(W.get("adjoint_64x512", n_sets=n_sets), size, size)
    HW = size * size
    theta = wl["metric"]["bumps"].copy()
    # a realistic target: the oracle-free GPU map of the target parameters
    tr = rt.Tracer(0)
    tr.set_metric(dict(wl["metric"], bumps=wl["target_bumps"]))
    tr.set_scene(wl["scene"])
    t_out = rt.to_numpy(tr.trace(wl["camera"], wl["rule"]))
    ones = np.ones(n_sets * HW, np.uint8)
    # (1) all amplitudes zero: flat metric, every gradient component vanishes
    th0 = theta.copy()
    th0[..., 0] = 0.0
    g0, _, _ = gpu_grad(rt, torch, wl, th0, t_out["hit"], t_out["id"], ones)
    assert np.all(g0 == 0.0)
    # (2) one bump with a = 0: its centre and sigma receive exactly zero
    th1 = theta.copy()
    th1[:, 3, 0] = 0.0
    g1, _, _ = gpu_grad(rt, torch, wl, th1, t_out["hit"], t_out["id"], ones)
    assert np.all(g1[:, 3, 1:] == 0.0)
    assert np.any(g1[:, 3, 0] != 0.0)
    # (3) a -> -a: same hits, d/da flips sign, d/dc and d/dsigma unchanged (bitwise)
    g2, l2, o2 = gpu_grad(rt, torch, wl, theta, t_out["hit"], t_out["id"], ones)
    thn = theta.copy()
    thn[..., 0] *= -1
    g3, l3, o3 = gpu_grad(rt, torch, wl, thn, t_out["hit"], t_out["id"], ones)
    assert np.array_equal(o2["hit"], o3["hit"]) and np.array_equal(l2, l3)
    assert np.array_equal(g2[..., 0], -g3[..., 0])
    assert np.array_equal(g2[..., 1:], g3[..., 1:])


@pytest.mark.parametrize("ck", [1, 37, 2000])
def test_adjoint_independent_of_checkpoint_interval(env, ck):
    rt, torch = env
    say("checkpoint interval %d vs 100: bitwise identical gradients" % ck)
    n_sets, size = 2, 48
    wl = W.with_size(W.get("adjoint_64x512", n_sets=n_sets), size, size)
    tr = rt.Tracer(0)
    tr.set_metric(dict(wl["metric"], bumps=wl["target_bumps"]))
    tr.set_scene(wl["scene"])
    t_out = rt.to_numpy(tr.trace(wl["camera"], wl["rule"]))
    ones = np.ones(n_sets * size * size, np.uint8)
    ga, _, _ = gpu_grad(rt, torch, wl, wl["metric"]["bumps"], t_out["hit"], t_out["id"], ones, ckpt_every=100)
    gb, _, _ = gpu_grad(rt, torch, wl, wl["metric"]["bumps"], t_out["hit"], t_out["id"], ones, ckpt_every=ck)
    assert np.array_equal(ga, gb)


def test_autograd_function(env):
    rt, torch = env
    say("torch.autograd.Function around the adjoint")
    n_sets, size = 2, 40
    wl = W.with_size(W.get("adjoint_64x512", n_sets=n_sets), size, size)
    tr = rt.Tracer(0)
    tr.set_metric(dict(wl["metric"], bumps=wl["target_bumps"]))
    tr.set_scene(wl["scene"])
    t_out = tr.trace(wl["camera"], wl["rule"])
    TraceFn = rt.make_trace_function()
    params = torch.tensor(wl["metric"]["bumps"], dtype=torch.float32, requires_grad=True)
    hit, ids = TraceFn.apply(params, tr, wl["metric"], wl["camera"], wl["rule"], 100)
    m = ((ids == t_out["id"]) & (ids >= 0)).float()[:, None]
    loss = (((hit - t_out["hit"]) ** 2) * m).sum()
    loss.backward()
    g_auto = params.grad.numpy().astype(np.float64)
    ones = np.ones(n_sets * size * size, np.uint8)
    g_api, l_api, _ = gpu_grad(rt, torch, wl, wl["metric"]["bumps"], t_out["hit"].cpu().numpy(),
                               t_out["id"].cpu().numpy(), ones)
    assert abs(float(loss.detach()) - float(l_api.sum())) <= 1e-4 * max(1.0, float(loss.detach()))
    assert np.allclose(g_auto, g_api, rtol=1e-5, atol=1e-5 * np.abs(g_api).max())


def test_new_scene_invalidates_tape(env):
    rt, torch = env
    say("rt_trace_bwd after rt_set_scene: RT_ESTATE, nothing launched")
    n_sets, size = 1, 16
    wl = W.with_size(W.get("adjoint_64x512", n_sets=n_sets), size, size)
    tr = rt.Tracer(0)
    tr.set_metric(wl["metric"])
    tr.set_scene(wl["scene"])
    cam, rule = wl["camera"], wl["rule"]
    out, tape = tr.trace_fwd_ckpt(cam, rule, rule["max_steps"], 100)
    gh = torch.zeros(n_sets * size * size, 3, dtype=torch.float32, device="cuda")
    tr.trace_bwd(tape, gh, wl["metric"]["bumps"].shape[1])
    torch.cuda.synchronize()
    tr.set_scene(wl["scene"])
    with pytest.raises(rt.RtError) as ei:
        tr.trace_bwd(tape, gh, wl["metric"]["bumps"].shape[1])
    assert ei.value.status == -5


def test_adjoint_directional_derivative(env):
    """Dot-product check of the adjoint: for seeded random directions u in
    parameter space, <grad L, u> from the GPU adjoint equals the FP64
    oracle's central difference of L along u, (L(theta + eps u) -
    L(theta - eps u)) / (2 eps), over pixels whose object is the same at
    theta and at both perturbed points.  Every parameter moves at once, so
    this also catches cross terms that coordinate differences see only one
    at a time."""
    rt, torch = env
    say("adjoint: <grad, u> against the FP64 directional difference, 3 random directions, 2 sets x 64x64")
    n_sets, size, eps = 2, 64, 1e-4
    wl = W.with_size(W.get("adjoint_64x512", n_sets=n_sets), size, size)
    HW = size * size
    theta = wl["metric"]["bumps"]
    pix = W.pixel_sample(size, size, 400, seed=90)
    rng = np.random.default_rng(91)
    for s in range(n_sets):
        tm = dict(wl["metric"], bumps=wl["target_bumps"])
        tgt = oracle.Oracle(tm, wl["scene"], s).trace(wl["camera"], wl["rule"], pix)
        base = theta[s].astype(np.float64)
        for trial in range(3):
            u = rng.normal(size=base.shape)
            u /= np.linalg.norm(u)
            r0 = oracle.Oracle(wl["metric"], wl["scene"], bumps64=base).trace(wl["camera"], wl["rule"], pix)
            rp = oracle.Oracle(wl["metric"], wl["scene"], bumps64=base + eps * u).trace(wl["camera"], wl["rule"], pix)
            rm = oracle.Oracle(wl["metric"], wl["scene"], bumps64=base - eps * u).trace(wl["camera"], wl["rule"], pix)
            m = (r0["id"] == tgt["id"]) & (r0["id"] >= 0) & (rp["id"] == r0["id"]) & (rm["id"] == r0["id"])
            fd = (oracle.l2_loss(rp["hit"], tgt["hit"], m) - oracle.l2_loss(rm["hit"], tgt["hit"], m)) / (2 * eps)
            target_hit = np.zeros((n_sets * HW, 3), np.float32)
            target_id = np.full(n_sets * HW, -7, np.int32)
            mask = np.zeros(n_sets * HW, np.uint8)
            target_hit[s * HW + pix] = tgt["hit"]
            target_id[s * HW + pix] = tgt["id"]
            mask[s * HW + pix[m]] = 1
            g, _, _ = gpu_grad(rt, torch, wl, theta, target_hit, target_id, mask)
            dot = float((g[s] * u).sum())
            scale = np.linalg.norm(g[s])
            say("set %d dir %d: <g,u> %.6g  FD %.6g  |g| %.4g  pixels %d" % (s, trial, dot, fd, scale, int(m.sum())))
            assert m.sum() > 100
            assert abs(dot - fd) <= 1e-4 + 1e-3 * scale, (dot, fd, scale)


def test_metric_speed_conserved_along_gpu_rays(env):
    """g(y, y) is a first integral of the geodesic flow: the GPU trace starts
    every ray at g-unit speed and RK4 at h = 0.01 keeps it to within its
    truncation and FP32 rounding.  The velocities come from the adjoint
    tape's checkpoints (x_hi, x_lo, y every 100 steps, blocked by 64 ray
    ids); g at x is the oracle's FP64 metric tensor."""
    rt, torch = env
    say("g(y,y) along GPU rays from the tape checkpoints, 2 sets x 64x64, RK4 h = 0.01")
    n_sets, size, ck = 2, 64, 100
    wl = W.with_size(W.get("adjoint_64x512", n_sets=n_sets), size, size)
    tr = rt.Tracer(0)
    tr.set_metric(wl["metric"])
    tr.set_scene(wl["scene"])
    cam, rule = wl["camera"], wl["rule"]
    out, tape = tr.trace_fwd_ckpt(cam, rule, rule["max_steps"], ck)
    torch.cuda.synchronize()
    steps = out["steps"].cpu().numpy()
    n_ck = (rule["max_steps"] + ck - 1) // ck
    T = (size // 8) * (size // 8) * 64
    ckpt = tape.cpu().numpy()[:n_sets * T * n_ck * 9].reshape(n_sets * T // 64, n_ck, 9, 64)
    rng = np.random.default_rng(92)
    worst = 0.0
    n_pts = 0
    for s in range(n_sets):
        orc = oracle.Oracle(wl["metric"], wl["scene"], s)
        for p in rng.choice(size * size, 150, replace=False):
            pi, pj = p % size, p // size
            rid = s * T + ((pj // 8) * (size // 8) + pi // 8) * 64 + (pj % 8) * 8 + (pi % 8)
            for c in range(n_ck):
                if c * ck >= steps[s * size * size + p]:
                    break
                v = ckpt[rid // 64, c, :, rid % 64].astype(np.float64)
                x = v[0:3] + v[3:6]
                y = v[6:9]
                worst = max(worst, abs(y @ orc.metric_tensor(x) @ y - 1.0))
                n_pts += 1
    say("worst |g(y,y) - 1| over %d checkpoints: %.3g" % (n_pts, worst))
    assert n_pts > 1000
    assert worst < 1e-5
