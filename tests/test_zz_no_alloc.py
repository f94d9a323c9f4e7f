"""The allocation-free trace (rt_trace_noalloc, static per-GPU workspace)
against rt_trace on the same inputs: the same kernels run, so every output
must be bitwise identical.  Two calls in a row, the second on a smaller
frame (the workspace keeps the first call's contents), a multi-pass trace
(survivor lists in the workspace) and the size limit."""
import numpy as np
import pytest

import workloads as W

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


def _both(rt, tr, wl, rule):
    import torch
    cam = wl["camera"]
    a = tr.trace_into(cam, rule, rule["max_steps"], tr.alloc_outputs(cam))
    torch.cuda.synchronize()
    sa = tr.stats()
    b = tr.trace_into(cam, rule, rule["max_steps"], tr.alloc_outputs(cam), noalloc=True)
    torch.cuda.synchronize()
    sb = tr.stats()
    return rt.to_numpy(a), rt.to_numpy(b), sa, sb


@pytest.mark.parametrize("name,size,pass_steps", [
    ("bumps16_1080p", (480, 360), None),     # first call: 172,800 ray ids, one pass
    ("bumps16_1080p", (96, 54), None),       # second call, smaller frame
    ("twist_4k", (160, 90), 256),            # multi-pass: survivor lists in the workspace
])
def test_noalloc_equals_trace(rt, name, size, pass_steps):
    say("rt_trace_noalloc vs rt_trace: %s %dx%d pass_steps=%s" % (name, size[0], size[1], pass_steps))
    wl = W.with_size(W.get(name), *size)
    rule = dict(wl["rule"], flags=rt.FLAG_COUNT_WORK)
    if pass_steps:
        rule["pass_steps"] = pass_steps
    tr = rt.Tracer(0)
    tr.set_metric(wl["metric"])
    tr.set_scene(wl["scene"])
    a, b, sa, sb = _both(rt, tr, wl, rule)
    for k in ("hit", "t", "id", "dir", "steps"):
        assert np.array_equal(a[k], b[k]), k
    for k in ("rays", "ray_steps", "refined", "bump_evals", "passes"):
        assert sa[k] == sb[k], (k, sa[k], sb[k])
    assert sa["rays"] == size[0] * size[1]
    assert (a["id"] >= 0).any()


def test_noalloc_rejects_oversize_frames(rt):
    say("rt_trace_noalloc: a 1080p frame exceeds the static workspace (host check, nothing launched)")
    wl = W.get("bumps16_1080p")
    tr = rt.Tracer(0)
    tr.set_metric(wl["metric"])
    tr.set_scene(wl["scene"])
    cam = wl["camera"]
    with pytest.raises(rt.RtError) as e:
        tr.trace_into(cam, wl["rule"], wl["rule"]["max_steps"], tr.alloc_outputs(cam), noalloc=True)
    assert e.value.status == rt.RT_EINVAL
    assert "RT_NOALLOC_SCRATCH_BYTES" in str(e.value)
