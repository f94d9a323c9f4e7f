"""Batched multi-segment intersection (RT_FLAG_BATCH_SEGMENTS): a window of
segments is marched without scene tests and its polygon boxes are tested at
once; lanes whose box meets an object march the window again with per-step
tests.  The outputs must equal the plain trace's bit for bit, on every metric
kind, both fixed-step integrators, several culling periods and pass lengths,
and the full benchmarked frame; one frame is also checked against the oracle
directly.  Every test names its case on stdout before touching the GPU."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.parity import assert_parity, compare

pytestmark = pytest.mark.gpu

FIELDS = ("hit", "t", "id", "dir", "steps")


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_05386_amd import rt as _rt
    return _rt


def trace(rt, wl, rule):
    tr = rt.Tracer(0)
    tr.set_metric(wl["metric"])
    tr.set_scene(wl["scene"])
    out = tr.trace(wl["camera"], rule, rule["max_steps"])
    tr.sync()
    res = rt.to_numpy(out)
    res["_stats"] = tr.stats()
    return res


def plain_and_batched(rt, wl, rule):
    g0 = trace(rt, wl, rule)
    g1 = trace(rt, wl, dict(rule, flags=rule.get("flags", 0) | rt.FLAG_BATCH_SEGMENTS))
    for k in FIELDS:
        assert np.array_equal(g0[k], g1[k]), k
    s0, s1 = g0["_stats"], g1["_stats"]
    assert s1["ray_steps"] == s0["ray_steps"] and s1["refined"] == s0["refined"]
    assert s1["batch_windows"] > 0 and s0["batch_windows"] == 0
    return g0, g1


CASES = [
    ("bumps16_1080p", 192, 108, {}),
    ("bumps16_1080p", 96, 54, {"kind": W.EULER}),
    ("bumps16_1080p", 61, 37, {"cull_every": 4, "pass_steps": 64}),
    ("bumps16_1080p", 64, 40, {"cull_every": 64, "pass_steps": 16}),
    ("bumps16_1080p", 64, 40, {"cull_every": 1}),
    ("twist_4k", 128, 72, {}),
    ("deform16_1080p", 64, 40, {}),
    ("rdeform16_1080p", 48, 32, {}),
    ("abumps16_1080p", 64, 40, {}),
    ("quadric_1080p", 64, 40, {}),
    ("single_bump_64", 9, 3, {}),
]


@pytest.mark.parametrize("name,w,h,mod", CASES)
def test_batched_equals_plain(rt, name, w, h, mod):
    say("batched segments vs plain trace: %s %dx%d %s" % (name, w, h, mod))
    wl = W.with_size(W.get(name), w, h)
    _, g1 = plain_and_batched(rt, wl, dict(wl["rule"], **mod))
    st = g1["_stats"]
    say("windows", st["batch_windows"], "replayed", st["batch_replays"])


def test_batched_flat_space(rt):
    """Flat space (the test kind): straight rays, so every replay comes from a
    box that meets an object; hits equal the closed form via the plain
    trace's pins."""
    say("batched segments vs plain trace: flat space 64x48")
    wl = W.with_size(W.get("single_bump_64"), 64, 48)
    wl["metric"] = W.metric(W.EUCLID)
    plain_and_batched(rt, wl, wl["rule"])


def test_batched_small_vs_oracle(rt):
    say("batched segments 96x54 bumps16 vs oracle")
    wl = W.with_size(W.get("bumps16_1080p"), 96, 54)
    rule = dict(wl["rule"], flags=rt.FLAG_BATCH_SEGMENTS)
    g = trace(rt, wl, rule)
    ref = oracle.Oracle(wl["metric"], wl["scene"], 0).trace(wl["camera"], wl["rule"])
    rep = compare(g, ref)
    say(rep)
    assert_parity(rep)


def test_batched_1080p_equals_plain(rt):
    """The benchmarked frame and launch configuration."""
    say("batched segments vs plain trace: bumps16_1080p full frame")
    wl = W.get("bumps16_1080p")
    _, g1 = plain_and_batched(rt, wl, wl["rule"])
    st = g1["_stats"]
    say("windows", st["batch_windows"], "replayed", st["batch_replays"])
    assert 0 < st["batch_replays"] < st["batch_windows"]
