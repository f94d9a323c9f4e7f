"""GPU parity of the HIP trace path against the FP64 oracle, through the
C ABI.  Every test names its case on stdout before touching the GPU."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from tests import exact
from tests.parity import assert_parity, compare

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_05386_amd import rt as _rt
    return _rt


def gpu_trace(rt, wl, rule=None, max_steps=None, tracer=None):
    rule = rule or wl["rule"]
    tr = tracer or rt.Tracer(0)
    tr.set_metric(wl["metric"])
    tr.set_scene(wl["scene"])
    out = tr.trace(wl["camera"], rule, max_steps or rule["max_steps"])
    tr.sync()
    res = rt.to_numpy(out)
    res["_stats"] = tr.stats()
    return res


def oracle_trace(wl, pixels=None, rule=None, set_index=0):
    return oracle.Oracle(wl["metric"], wl["scene"], set_index).trace(wl["camera"], rule or wl["rule"], pixels)


def test_single_bump_full_frame(rt):
    say("single_bump_64 full frame 64x64 RK4 h=0.01")
    wl = W.get("single_bump_64")
    g = gpu_trace(rt, wl)
    ref = oracle_trace(wl)
    rep = compare(g, ref)
    say(rep)
    assert_parity(rep)
    assert rep["max_t_err"] < 1e-3
    st = g["_stats"]
    assert st["rays"] == 64 * 64
    assert st["ray_steps"] == int(g["steps"].sum())
    assert np.array_equal(g["steps"], ref["steps"]) or (g["steps"] != ref["steps"]).mean() < 0.002


def test_single_bump_matches_quadrature(rt):
    """GPU against the exact continuous single-bump geodesics (tighter than
    the parity tolerance: RK4 truncation + FP32 rounding)."""
    say("single_bump_64 vs quadrature")
    wl = W.get("single_bump_64")
    g = gpu_trace(rt, wl)
    pix = W.pixel_sample(64, 64, 300, seed=21)
    d = exact.camera_dirs(wl["camera"], pix)
    b = np.linalg.norm(np.cross(np.float64(wl["camera"]["eye"]), d), axis=1)
    pix = pix[(b > 0.02) & (b < 1.2) & (g["id"][pix] >= 0)][:25]
    d = exact.camera_dirs(wl["camera"], pix)
    bump = wl["metric"]["bumps"][0, 0].astype(np.float64)
    sph = np.float64(wl["scene"]["spheres"][0])
    pl = np.float64(wl["scene"]["planes"][0])
    objs = [lambda x: (x - sph[:3]) @ (x - sph[:3]) - sph[3] ** 2, lambda x: pl[:3] @ x - pl[3]]
    worst = 0.0
    for q, p in enumerate(pix):
        ray = exact.SingleBumpRay(bump[0], bump[1:4], bump[4], np.float64(wl["camera"]["eye"]), d[q]).tabulate(10.0)
        t, oid, x = ray.first_hit(objs, 10.0)
        assert g["id"][p] == oid
        worst = max(worst, np.abs(g["hit"][p] - x).max())
    say("worst hit error vs quadrature", worst)
    assert worst < 2e-4


def test_flat_space_is_straight(rt):
    say("flat space (EUCLID) bumps16 scene 96x54")
    wl = W.with_size(W.get("bumps16_1080p"), 96, 54)
    wl["metric"] = W.metric(W.EUCLID)
    rule = dict(wl["rule"], max_steps=2000)
    g = gpu_trace(rt, wl, rule=rule)
    pix = np.arange(96 * 54)
    d = exact.camera_dirs(wl["camera"], pix)
    t, ids = exact.line_hits(np.float64(wl["camera"]["eye"]), d, wl["scene"], 2000 * np.float64(np.float32(0.005)))
    same = g["id"] == ids
    assert same.mean() >= 0.999
    hit = same & (ids >= 0)
    exp_hit = np.float64(wl["camera"]["eye"]) + t[hit, None] * d[hit]
    say("max flat hit err", np.abs(g["hit"][hit] - exp_hit).max())
    assert np.abs(g["hit"][hit] - exp_hit).max() < 2e-5


def test_bumps16_small_full_frame(rt):
    say("bumps16 192x108 full frame RK4 h=0.005 4000 steps")
    wl = W.with_size(W.get("bumps16_1080p"), 192, 108)
    g = gpu_trace(rt, wl)
    ref = oracle_trace(wl)
    rep = compare(g, ref)
    say(rep)
    assert_parity(rep)


def test_bumps16_1080p_sampled(rt):
    """Full 1080p frame in the benchmark's launch configuration; a seeded
    sample of pixels recomputed one by one by the oracle."""
    say("bumps16_1080p full frame, 32400 sampled pixels vs oracle")
    wl = W.get("bumps16_1080p")
    g = gpu_trace(rt, wl)
    pix = W.pixel_sample(1920, 1080, 32400, seed=7)
    ref = oracle_trace(wl, pix)
    rep = compare(g, ref, pix)
    say(rep, g["_stats"])
    assert_parity(rep)
    assert g["_stats"]["rays"] == 1920 * 1080
    assert (g["id"] >= -1).all()


def test_rk45_small(rt):
    say("bumps16 RK45 tol 1e-6, 96x54")
    wl = W.with_size(W.get("bumps16_1080p_rk45"), 96, 54)
    g = gpu_trace(rt, wl)
    ref = oracle_trace(wl)
    rep = compare(g, ref)
    say(rep, g["_stats"])
    assert_parity(rep)


def test_rk45_1080p_sampled(rt):
    say("bumps16 RK45 1080p, 32400 sampled pixels")
    wl = W.get("bumps16_1080p_rk45")
    g = gpu_trace(rt, wl)
    pix = W.pixel_sample(1920, 1080, 32400, seed=8)
    rep = compare(g, oracle_trace(wl, pix), pix)
    say(rep, g["_stats"])
    assert_parity(rep)


def failing_rk45_case():
    """A frame in which the rays through a steep bump fail (id -2): RK45
    with h = h_min = h_max = 0.08, so the step never grows back and an
    attempt whose error norm exceeds 1 cannot be retried above h_min.  A
    ray fails where the error norm along its path exceeds 1, which varies
    smoothly with the pixel: FP32 and FP64 take the same decision except
    within rounding of the boundary of the failed region."""
    wl = W.with_size(W.get("single_bump_64"), 64, 64)
    wl["camera"] = W.camera(64, 64, vfov_deg=20.0)
    wl["metric"] = dict(wl["metric"], bumps=W.f32([[[1.5, 0.0, 0.0, 0.0, 0.3]]]))
    rule = W.rule(kind=W.RK45, h=0.08, max_steps=4000, t_max=10.0, rtol=1e-6, atol=1e-6)
    rule.update(h_min=rule["h"], h_max=rule["h"])
    wl["rule"] = rule
    return wl


def test_failed_rays_match_the_oracle(rt):
    say("id -2: RK45 pinned at h_min = h_max = 0.08 through a steep bump, 64x64")
    wl = failing_rk45_case()
    g = gpu_trace(rt, wl)
    ref = oracle_trace(wl)
    rep = compare(g, ref)
    n_fail = int((ref["id"] == -2).sum())
    say(rep, "oracle failed", n_fail, "gpu failed", int((g["id"] == -2).sum()),
        "id -2 disagreements", int(((g["id"] == -2) != (ref["id"] == -2)).sum()))
    assert n_fail > 150
    assert_parity(rep)
    # the failed rays stop where the oracle's stop (their last accepted state)
    f = (g["id"] == -2) & (ref["id"] == -2)
    assert f.sum() >= n_fail - 2
    assert np.linalg.norm(g["hit"][f] - ref["hit"][f], axis=1).max() < 1e-4
    assert np.array_equal(g["steps"][f], ref["steps"][f])


def test_twist_rays_near_its_centre(rt):
    """The twist is only C^1 at its centre: rays aimed at it, or passing
    within a few steps of it, against the oracle.  The central pixel of the
    odd-sized frame looks straight down the z axis through the centre."""
    say("twist: 33x33 frame, 1 degree field of view aimed at the centre, plane z = 3")
    wl = W.with_size(W.get("twist_4k"), 33, 33)
    wl["camera"] = W.camera(33, 33, vfov_deg=1.0)
    wl["scene"] = W.scene(planes=[[0.0, 0.0, 1.0, 3.0]])
    wl["rule"] = W.rule(W.RK4, h=0.005, max_steps=4000)
    g = gpu_trace(rt, wl)
    ref = oracle_trace(wl)
    rep = compare(g, ref)
    say(rep)
    assert (ref["id"] == 0).all() and (g["id"] == 0).all()
    assert_parity(rep)
    # the central ray stays on the axis
    c = 16 * 33 + 16
    assert abs(g["hit"][c, 0]) < 1e-6 and abs(g["hit"][c, 1]) < 1e-6


def test_refinement_brackets_the_root(rt):
    """The hit refinement brackets the step fraction s of the sign change to
    a width of 2^-bisect_iters and returns the bracket's midpoint: within
    h 2^-(n+1) of the root in s, so t within that and the hit point within
    that times the Euclidean speed (<= 1 for the graph metric, plus the
    step's own curvature), up to the
    FP32 rounding of the outputs.  Checked against a 40-iteration trace of
    the same frame; object ids do not depend on the refinement."""
    say("refinement precision: bumps16 160x90, bisect_iters 8 / 16 / 24 against 40")
    wl = W.with_size(W.get("bumps16_1080p"), 160, 90)
    h = wl["rule"]["h"]
    ref = gpu_trace(rt, wl, rule=dict(wl["rule"], bisect_iters=40))
    hit = ref["id"] >= 0
    assert hit.sum() > 2000
    for n in (8, 16, 24):
        g = gpu_trace(rt, wl, rule=dict(wl["rule"], bisect_iters=n))
        assert np.array_equal(g["id"], ref["id"])
        bound = h * 2.0 ** -(n + 1) * 1.001
        ulp_t = np.spacing(np.abs(ref["t"][hit])).astype(np.float64)
        dt = np.abs(g["t"][hit].astype(np.float64) - ref["t"][hit])
        assert np.all(dt <= bound + 2 * ulp_t), (n, dt.max())
        ulp_x = np.spacing(np.abs(ref["hit"][hit])).max(axis=1).astype(np.float64)
        dx = np.linalg.norm(g["hit"][hit].astype(np.float64) - ref["hit"][hit], axis=1)
        # the partial step's end moves at h (|y| + O(h |a|)) per unit of s
        assert np.all(dx <= 1.1 * bound + 4 * ulp_x), (n, dx.max())
        say("  bisect_iters=%d: max |dt| %.3g, max |dx| %.3g, bound %.3g" % (n, dt.max(), dx.max(), bound))


def test_euler_single_bump(rt):
    say("single_bump Euler h=0.01")
    wl = W.get("single_bump_64")
    rule = dict(wl["rule"], kind=W.EULER)
    g = gpu_trace(rt, wl, rule=rule)
    rep = compare(g, oracle_trace(wl, rule=rule))
    say(rep)
    assert_parity(rep)


def test_sign_invariance_bitwise(rt):
    say("f -> -f bitwise, bumps16 96x54")
    wl = W.with_size(W.get("bumps16_1080p"), 96, 54)
    g1 = gpu_trace(rt, wl)
    wl2 = dict(wl)
    wl2["metric"] = dict(wl["metric"], bumps=wl["metric"]["bumps"] * np.array([-1, 1, 1, 1, 1], np.float32))
    g2 = gpu_trace(rt, wl2)
    for k in ("hit", "t", "id", "dir", "steps"):
        assert np.array_equal(g1[k], g2[k]), k


def test_concurrent_contexts_bitwise(rt):
    """Frames in flight on two streams, each with its own context, equal a
    frame traced alone bit for bit (the throughput figure traces this way)."""
    import torch
    say("two contexts on two streams, bumps16 320x180, 3 frames each")
    wl = W.with_size(W.get("bumps16_1080p"), 320, 180)
    ref = gpu_trace(rt, wl)
    cam, rule = wl["camera"], wl["rule"]
    trs, outs, streams = [], [], []
    for _ in range(2):
        tr = rt.Tracer(0)
        tr.set_metric(wl["metric"])
        tr.set_scene(wl["scene"])
        trs.append(tr)
        outs.append(tr.alloc_outputs(cam))
        streams.append(torch.cuda.Stream())
    for i in range(6):
        trs[i % 2].trace_into(cam, rule, rule["max_steps"], outs[i % 2], stream=streams[i % 2])
    torch.cuda.synchronize()
    for o in outs:
        g = {k: v.cpu().numpy() for k, v in o.items() if hasattr(v, "cpu")}
        for k in ("hit", "t", "id", "dir", "steps"):
            assert np.array_equal(g[k].reshape(ref[k].shape), ref[k]), k


@pytest.mark.parametrize("grid,K,S", [("1", 16, 256), ("7", 4, 64), ("", 64, 16)])
def test_deterministic_across_launch_shapes(rt, grid, K, S):
    """Per-lane 6-sigma selection and ordered bump walks make every ray's
    arithmetic independent of the grid size, the culling period K and the
    pass length S: outputs must be bitwise identical."""
    say("determinism grid=%s K=%d S=%d" % (grid or "default", K, S))
    wl = W.with_size(W.get("bumps16_1080p"), 64, 40)
    ref = gpu_trace(rt, wl)
    old = os.environ.get("RT_GRID_BLOCKS")
    try:
        if grid:
            os.environ["RT_GRID_BLOCKS"] = grid
        g = gpu_trace(rt, wl, rule=dict(wl["rule"], cull_every=K, pass_steps=S))
    finally:
        if old is None:
            os.environ.pop("RT_GRID_BLOCKS", None)
        else:
            os.environ["RT_GRID_BLOCKS"] = old
    for k in ("hit", "t", "id", "dir", "steps"):
        assert np.array_equal(ref[k], g[k]), k


def test_ragged_and_tiny_frames(rt):
    for (w, h) in [(61, 37), (1, 1), (9, 3)]:
        say("ragged frame %dx%d" % (w, h))
        wl = W.with_size(W.get("single_bump_64"), w, h)
        g = gpu_trace(rt, wl)
        rep = compare(g, oracle_trace(wl))
        assert rep["frac_ok"] == 1.0 or (w * h > 1000 and rep["frac_ok"] >= 0.999), rep
        assert g["_stats"]["rays"] == w * h


def test_multi_set_equals_single_sets(rt):
    say("3 parameter sets in one launch vs one by one")
    wl = W.with_size(W.get("adjoint_64x512", n_sets=3), 40, 32)
    g = gpu_trace(rt, wl)
    n = 40 * 32
    for s in range(3):
        one = dict(wl)
        one["metric"] = dict(wl["metric"], bumps=wl["metric"]["bumps"][s:s + 1])
        gs = gpu_trace(rt, one)
        for k in ("hit", "t", "id", "dir", "steps"):
            assert np.array_equal(g[k][s * n:(s + 1) * n], gs[k]), (s, k)
    ref = oracle_trace(wl, set_index=2)
    assert_parity(compare({k: v[2 * n:] for k, v in g.items() if k != "_stats"}, ref))


def test_twist_small_full_frame(rt):
    say("twist pullback 128x72 full frame")
    wl = W.with_size(W.get("twist_4k"), 128, 72)
    g = gpu_trace(rt, wl)
    rep = compare(g, oracle_trace(wl))
    say(rep)
    assert_parity(rep)


def test_twist_4k_sampled(rt):
    say("twist_4k full frame, 32400 sampled pixels")
    wl = W.get("twist_4k")
    g = gpu_trace(rt, wl)
    pix = W.pixel_sample(3840, 2160, 32400, seed=3)
    rep = compare(g, oracle_trace(wl, pix), pix)
    say(rep, g["_stats"])
    assert_parity(rep)


def test_ztwist_small(rt):
    say("paper z-twist 64x48")
    wl = W.with_size(W.get("single_bump_64"), 64, 48)
    wl["metric"] = W.metric(W.PULLBACK_ZTWIST)
    wl["scene"] = W.scene(spheres=W.random_spheres(32, 1), planes=W.PLANE_Y_MINUS_1)
    rule = dict(wl["rule"], h=0.005, max_steps=2000, t_max=10.0)
    g = gpu_trace(rt, wl, rule=rule)
    rep = compare(g, oracle_trace(wl, rule=rule))
    say(rep)
    assert_parity(rep)


# --------------------------------------- composed local deformations (Sec. 6.2)
# deform16: constant fields; rdeform16: fields with a rotation part
@pytest.mark.parametrize("name", ["deform16_1080p", "rdeform16_1080p"])
def test_deform_small_full_frame(rt, name):
    say("%s (16 composed local deformations) 96x54 full frame" % name)
    wl = W.with_size(W.get(name), 96, 54)
    g = gpu_trace(rt, wl)
    rep = compare(g, oracle_trace(wl))
    say(rep)
    assert_parity(rep)


@pytest.mark.parametrize("name", ["deform16_1080p", "rdeform16_1080p"])
def test_deform_1080p_sampled(rt, name):
    say("%s full frame, 1000 sampled pixels" % name)
    wl = W.get(name)
    g = gpu_trace(rt, wl)
    pix = W.pixel_sample(1920, 1080, 1000, seed=4)
    rep = compare(g, oracle_trace(wl, pix), pix)
    say(rep, g["_stats"])
    assert_parity(rep)


def _strong_deform_wl(w=96, h=64, rotating=False):
    """Six strong, overlapping deformations around the origin (the oracle
    pins' sets, with constant or rotating fields): the order of the
    composition matters and the culling bounds are far from trivial."""
    from tests.test_oracle_pins import DEFORMS, RDEFORMS
    wl = W.with_size(W.get("single_bump_64"), w, h)
    wl["metric"] = W.metric(W.PULLBACK_DEFORM, deforms=RDEFORMS if rotating else DEFORMS)
    wl["scene"] = W.scene(spheres=W.random_spheres(24, 1, box=1.5, radius=(0.1, 0.3)),
                          planes=W.PLANE_Y_MINUS_1, tori=W.TORUS_Z)
    wl["rule"] = dict(wl["rule"], h=0.005, max_steps=2000, t_max=10.0)
    return wl


@pytest.mark.parametrize("rotating", [False, True])
def test_deform_strong_small(rt, rotating):
    say("strong overlapping deformations 96x64, rotating fields %s" % rotating)
    wl = _strong_deform_wl(rotating=rotating)
    g = gpu_trace(rt, wl)
    rep = compare(g, oracle_trace(wl))
    say(rep, g["_stats"])
    assert_parity(rep)


@pytest.mark.parametrize("K,S,rotating", [(4, 64, False), (64, 2000, False), (4, 64, True)])
def test_deform_deterministic_across_culling(rt, K, S, rotating):
    """The per-lane cut makes each deformation the identity outside its
    region, so any superset list gives the same arithmetic: a culling period
    or pass length change must leave the frame bitwise unchanged (a list
    that missed a deformation a lane needs would change it)."""
    say("deform determinism K=%d S=%d rotating fields %s" % (K, S, rotating))
    wl = _strong_deform_wl(64, 40, rotating=rotating)
    ref = gpu_trace(rt, wl)
    g = gpu_trace(rt, wl, rule=dict(wl["rule"], cull_every=K, pass_steps=S))
    for k in ("hit", "t", "id", "dir", "steps"):
        assert np.array_equal(ref[k], g[k]), k


# ------------------ more graph metrics: anisotropic bumps, Sec. 5.1 quadratic
@pytest.mark.parametrize("name", ["abumps16_1080p", "quadric_1080p"])
def test_graph2_small_full_frame(rt, name):
    say("%s 96x54 full frame" % name)
    wl = W.with_size(W.get(name), 96, 54)
    g = gpu_trace(rt, wl)
    rep = compare(g, oracle_trace(wl))
    say(rep)
    assert_parity(rep)


@pytest.mark.parametrize("name", ["abumps16_1080p", "quadric_1080p"])
def test_graph2_1080p_sampled(rt, name):
    say("%s full frame, 1000 sampled pixels" % name)
    wl = W.get(name)
    g = gpu_trace(rt, wl)
    pix = W.pixel_sample(1920, 1080, 1000, seed=6)
    rep = compare(g, oracle_trace(wl, pix), pix)
    say(rep, g["_stats"])
    assert_parity(rep)


def test_aniso_deterministic_across_culling(rt):
    """Per-lane ellipsoid cut: any superset bump list gives the same
    arithmetic, so the frame is bitwise independent of the culling period."""
    say("anisotropic bumps determinism K=4 S=64")
    wl = W.with_size(W.get("abumps16_1080p"), 64, 40)
    ref = gpu_trace(rt, wl)
    g = gpu_trace(rt, wl, rule=dict(wl["rule"], cull_every=4, pass_steps=64))
    for k in ("hit", "t", "id", "dir", "steps"):
        assert np.array_equal(ref[k], g[k]), k


@pytest.mark.parametrize("name,kind", [("deform16_1080p", W.RK45), ("abumps16_1080p", W.RK45),
                                       ("quadric_1080p", W.EULER), ("twist_4k", W.EULER)])
def test_other_integrators_on_new_metrics(rt, name, kind):
    """DP5(4) and the paper's Euler march on the newer metric kinds, small
    frames, against the oracle running the same discrete method."""
    say("%s with step kind %d, 64x36" % (name, kind))
    wl = W.with_size(W.get(name), 64, 36)
    if kind == W.RK45:
        rule = W.rule(W.RK45, h=0.005, max_steps=4000, t_max=20.0, rtol=1e-6, atol=1e-6, h_min=1e-6, h_max=0.02,
                      pass_steps=4000)
    else:
        rule = W.rule(W.EULER, h=0.005, max_steps=4000, t_max=20.0, pass_steps=4000)
    g = gpu_trace(rt, wl, rule=rule)
    rep = compare(g, oracle_trace(wl, rule=rule))
    say(rep)
    assert_parity(rep)
