"""C-ABI checks that need no GPU: the library loads, exports every function
include/rt.h declares, and the host-side validation returns the documented
status codes (host-only context, device -1)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rt():
    from paper_2005_05386_amd import rt
    return rt


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rt.h")).read()
    return sorted(set(re.findall(r"^\s*(?:rt_status|void|int|size_t|const char \*)\s*\*?\s*(rt_\w+)\s*\(", src, re.M)))


def test_every_declared_symbol_is_exported():
    rt = _rt()
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(rt.lib(), n), n
    assert sorted(rt.EXPORTS) == names
    assert rt.abi_version() == 6


def test_host_only_context_validates():
    rt = _rt()
    tr = rt.Tracer(-1)
    wl = W.get("bumps16_1080p")
    tr.set_metric(wl["metric"])
    tr.set_scene(wl["scene"])
    cam, rule = wl["camera"], wl["rule"]
    # a valid trace on a host-only context stops after validation
    with pytest.raises(rt.RtError) as e:
        tr.trace_raw(cam, rule, rule["max_steps"], (16, 16, 16, 16, 0), 0)
    assert e.value.status == rt.RT_ESTATE
    bad = [
        (dict(cam, width=0), rule, 10, rt.RT_EINVAL),
        (dict(cam, vfov_deg=180.0), rule, 10, rt.RT_EINVAL),
        (dict(cam, up=[0, 0, 1.0]), rule, 10, rt.RT_EINVAL),
        (cam, dict(rule, h=0.0), 10, rt.RT_EINVAL),
        (cam, dict(rule, h=float("nan")), 10, rt.RT_EINVAL),
        (cam, dict(rule, kind=7), 10, rt.RT_EUNSUPPORTED),
        (cam, dict(rule, cull_every=0), 10, rt.RT_EINVAL),
        (cam, dict(rule, pass_steps=4), 10, rt.RT_EINVAL),
        (cam, dict(rule, bisect_iters=61), 10, rt.RT_EINVAL),
        (cam, dict(rule, kind=W.RK45, rtol=0.0), 10, rt.RT_EINVAL),
        (cam, rule, 0, rt.RT_EINVAL),
        (cam, rule, 2000000, rt.RT_EINVAL),
    ]
    for c_, r_, ms, want in bad:
        with pytest.raises(rt.RtError) as e:
            tr.trace_raw(c_, r_, ms, (16, 16, 16, 16, 0), 0)
        assert e.value.status == want, (c_, r_, ms, e.value)
        assert rt.lib().rt_last_error(tr._h)
    with pytest.raises(rt.RtError) as e:
        tr.trace_raw(cam, rule, 10, (0, 16, 16, 16, 0), 0)
    assert e.value.status == rt.RT_EINVAL


def test_noalloc_trace_validates():
    """rt_trace_noalloc shares rt_trace's validation; it also refuses the
    flags that need allocations, before looking at the device."""
    rt = _rt()
    tr = rt.Tracer(-1)
    wl = W.get("bumps16_1080p")
    tr.set_metric(wl["metric"])
    tr.set_scene(wl["scene"])
    cam, rule = wl["camera"], wl["rule"]
    for flags in (rt.FLAG_TIMING, rt.FLAG_SURROGATE, rt.FLAG_TIMING | rt.FLAG_COUNT_WORK):
        with pytest.raises(rt.RtError) as e:
            tr.trace_raw(cam, dict(rule, flags=flags), 10, (16, 16, 16, 16, 0), 0, noalloc=True)
        assert e.value.status == rt.RT_EUNSUPPORTED
    for c_, r_, ms, want in [(dict(cam, width=0), rule, 10, rt.RT_EINVAL), (cam, dict(rule, h=0.0), 10, rt.RT_EINVAL),
                             (cam, rule, 0, rt.RT_EINVAL), (cam, rule, 10, rt.RT_ESTATE)]:
        with pytest.raises(rt.RtError) as e:
            tr.trace_raw(c_, r_, ms, (16, 16, 16, 16, 0), 0, noalloc=True)
        assert e.value.status == want


def test_batched_segments_validate():
    """RT_FLAG_BATCH_SEGMENTS serves fixed-step plain traces: DP5(4), work
    counting and the surrogate are refused before the device is touched; a
    valid request gets as far as the host-only context check."""
    rt = _rt()
    tr = rt.Tracer(-1)
    wl = W.get("bumps16_1080p")
    tr.set_metric(wl["metric"])
    tr.set_scene(wl["scene"])
    cam, rule = wl["camera"], wl["rule"]
    B = rt.FLAG_BATCH_SEGMENTS
    rk45 = W.get("bumps16_1080p_rk45")["rule"]
    for r_ in (dict(rk45, flags=B), dict(rule, flags=B | rt.FLAG_COUNT_WORK), dict(rule, flags=B | rt.FLAG_SURROGATE)):
        with pytest.raises(rt.RtError) as e:
            tr.trace_raw(cam, r_, 10, (16, 16, 16, 16, 0), 0)
        assert e.value.status == rt.RT_EUNSUPPORTED
    for r_ in (dict(rule, flags=B), dict(rule, kind=rt.EULER, flags=B | rt.FLAG_TIMING)):
        with pytest.raises(rt.RtError) as e:
            tr.trace_raw(cam, r_, 10, (16, 16, 16, 16, 0), 0)
        assert e.value.status == rt.RT_ESTATE
    with pytest.raises(rt.RtError) as e:
        tr.trace_raw(cam, dict(rule, flags=16), 10, (16, 16, 16, 16, 0), 0)
    assert e.value.status == rt.RT_EINVAL


def test_metric_and_scene_validation():
    rt = _rt()
    tr = rt.Tracer(-1)
    b = W.random_bumps(4, 0)
    for mod, want in [(lambda x: x.__setitem__((0, 4), 0.0), rt.RT_EINVAL),
                      (lambda x: x.__setitem__((1, 4), -1.0), rt.RT_EINVAL),
                      (lambda x: x.__setitem__((2, 0), np.nan), rt.RT_EINVAL),
                      (lambda x: x.__setitem__((3, 1), np.inf), rt.RT_EINVAL)]:
        bb = b.copy()
        mod(bb)
        with pytest.raises(rt.RtError) as e:
            tr.set_metric(W.metric(W.GRAPH_GAUSS, bb))
        assert e.value.status == want
    with pytest.raises(rt.RtError) as e:
        tr.set_metric(W.metric(W.GRAPH_GAUSS, W.random_bumps(65, 0)))
    assert e.value.status == rt.RT_EINVAL
    with pytest.raises(rt.RtError) as e:
        tr.set_metric(dict(W.metric(W.GRAPH_GAUSS, b), kind=9))
    assert e.value.status == rt.RT_EUNSUPPORTED
    with pytest.raises(rt.RtError) as e:
        tr.set_metric(dict(W.metric(W.PULLBACK_TWIST), twist_amp=2.0))
    assert e.value.status == rt.RT_EINVAL
    with pytest.raises(rt.RtError) as e:
        tr.set_metric(dict(W.metric(W.GRAPH_GAUSS, b), cull_sigmas=2.0))
    assert e.value.status == rt.RT_EINVAL
    with pytest.raises(rt.RtError) as e:
        tr.set_scene(W.scene(spheres=W.random_spheres(257, 1)))
    assert e.value.status == rt.RT_EINVAL
    with pytest.raises(rt.RtError) as e:
        tr.set_scene(W.scene(planes=[[0.0, 2.0, 0.0, -1.0]]))
    assert e.value.status == rt.RT_EINVAL
    with pytest.raises(rt.RtError) as e:
        tr.set_scene(W.scene(tori=[[0, 0, 0, 0, 0, 1, 0.1, 0.2]]))
    assert e.value.status == rt.RT_EINVAL
    sp = W.random_spheres(3, 1)
    sp[1, 3] = -0.1
    with pytest.raises(rt.RtError) as e:
        tr.set_scene(W.scene(spheres=sp))
    assert e.value.status == rt.RT_EINVAL
    # composed local deformations: accepted as generated, rejected when a
    # deformation is not a diffeomorphism with margin, has a zero spread or
    # a non-finite value, or the count is out of range
    d = W.random_deforms(5, 0)
    tr.set_metric(W.metric(W.PULLBACK_DEFORM, deforms=d))
    for mod in [lambda x: x.__setitem__((0, 0), 50.0 * x[0, 0]),
                lambda x: x.__setitem__((1, 5), 0.0),
                lambda x: x.__setitem__((2, 8), np.nan)]:
        dd = d.copy()
        mod(dd)
        with pytest.raises(rt.RtError) as e:
            tr.set_metric(W.metric(W.PULLBACK_DEFORM, deforms=dd))
        assert e.value.status == rt.RT_EINVAL
    for n in (0, 65):
        with pytest.raises(rt.RtError) as e:
            tr.set_metric(W.metric(W.PULLBACK_DEFORM, deforms=W.random_deforms(n, 0).reshape(n, 10)))
        assert e.value.status == rt.RT_EINVAL
    # rotating fields: accepted as generated; rejected when the rotation
    # pushes the Lipschitz bound past the margin or is not finite
    rd = W.random_deforms(5, 0, rot=(0.3, 0.5))
    assert rd.shape == (5, 13)
    tr.set_metric(W.metric(W.PULLBACK_DEFORM, deforms=rd))
    for mod in [lambda x: x.__setitem__((3, 10), 20.0 * x[3, 10] + 20.0),
                lambda x: x.__setitem__((4, 12), np.inf)]:
        dd = rd.copy()
        mod(dd)
        with pytest.raises(rt.RtError) as e:
            tr.set_metric(W.metric(W.PULLBACK_DEFORM, deforms=dd))
        assert e.value.status == rt.RT_EINVAL
    # anisotropic bumps and the quadric
    ab = W.random_abumps(4, 0)
    tr.set_metric(W.metric(W.GRAPH_ANISO, abumps=ab))
    for mod in [lambda x: x.__setitem__((0, 4), 0.0), lambda x: x.__setitem__((1, 6), -0.2),
                lambda x: x.__setitem__((2, 1), np.inf)]:
        bb = ab.copy()
        mod(bb)
        with pytest.raises(rt.RtError) as e:
            tr.set_metric(W.metric(W.GRAPH_ANISO, abumps=bb))
        assert e.value.status == rt.RT_EINVAL
    tr.set_metric(W.metric(W.GRAPH_QUADRIC, quadric=(1.0, 1.0, -1.0)))
    with pytest.raises(rt.RtError) as e:
        tr.set_metric(W.metric(W.GRAPH_QUADRIC, quadric=(1.0, 200.0, -1.0)))
    assert e.value.status == rt.RT_EINVAL
    # trace before a scene is set
    tr2 = rt.Tracer(-1)
    tr2.set_metric(W.metric(W.GRAPH_GAUSS, b))
    wl = W.get("single_bump_64")
    with pytest.raises(rt.RtError) as e:
        tr2.trace_raw(wl["camera"], wl["rule"], 10, (16, 16, 16, 16, 0), 0)
    assert e.value.status == rt.RT_ESTATE


def test_create_errors():
    rt = _rt()
    h = C.c_void_p()
    assert rt.lib().rt_create(-2, C.byref(h)) == rt.RT_EINVAL
    assert rt.lib().rt_last_error(None)
    assert not h.value
    rt.lib().rt_destroy(None)


def test_surrogate_and_mlp_entry_points_validate():
    """Argument checks of the surrogate and MLP entry points, host-only
    context (no device work is ever launched)."""
    rt = _rt()
    tr = rt.Tracer(-1)
    L = rt.lib()
    wl = W.get("single_bump_64")
    tr.set_metric(wl["metric"])
    tr.set_scene(wl["scene"])
    cam, rule = wl["camera"], wl["rule"]
    # surrogate traces need networks, the graph metric, RK4, one set
    with pytest.raises(rt.RtError) as e:
        tr.trace_raw(cam, dict(rule, flags=rt.FLAG_SURROGATE), 10, (16, 16, 16, 16, 0), 0)
    assert e.value.status == rt.RT_ESTATE
    with pytest.raises(rt.RtError) as e:
        tr.trace_raw(cam, dict(rule, kind=W.RK45, flags=rt.FLAG_SURROGATE), 10, (16, 16, 16, 16, 0), 0)
    assert e.value.status == rt.RT_EUNSUPPORTED
    with pytest.raises(rt.RtError) as e:
        tr.trace_raw(cam, dict(rule, flags=16), 10, (16, 16, 16, 16, 0), 0)
    assert e.value.status == rt.RT_EINVAL
    P = C.c_void_p(16)
    one = np.ones(4, np.float32)
    nob = np.zeros(1, np.int32)
    # load: bad sizes first, then the host-only state
    assert L.rt_surrogate_load(tr._h, 65, P, P, one.ctypes.data, P, 2, P, 1, nob.ctypes.data, 1, 1e-3) == rt.RT_EINVAL
    assert L.rt_surrogate_load(tr._h, 1, P, P, one.ctypes.data, P, 1, P, 1, nob.ctypes.data, 1, 1e-3) == rt.RT_EINVAL
    assert L.rt_surrogate_load(tr._h, 1, P, P, one.ctypes.data, P, 2, P, 1, nob.ctypes.data, 1, 0.0) == rt.RT_EINVAL
    bad_nob = np.array([3], np.int32)
    assert L.rt_surrogate_load(tr._h, 1, P, P, one.ctypes.data, P, 2, P, 1, bad_nob.ctypes.data, 1,
                               1e-3) == rt.RT_EINVAL
    neg = -one
    assert L.rt_surrogate_load(tr._h, 1, P, P, neg.ctypes.data, P, 2, P, 1, nob.ctypes.data, 1, 1e-3) == rt.RT_EINVAL
    assert L.rt_surrogate_load(tr._h, 1, P, P, one.ctypes.data, P, 2, P, 1, nob.ctypes.data, 1, 1e-3) == rt.RT_ESTATE
    assert L.rt_surrogate_load(tr._h, 0, None, None, None, None, 2, None, 1, None, 0, 1.0) == rt.RT_OK
    # data generation and calibration
    k = np.array([1.0], np.float32)
    assert L.rt_surrogate_gen(tr._h, 1, k.ctypes.data, one.ctypes.data, 16, 0.0, 0, 1, P, P, P, None) == rt.RT_EINVAL
    assert L.rt_surrogate_gen(tr._h, 1, k.ctypes.data, one.ctypes.data, 16, 0.01, 3, 1, P, P, P, None) == rt.RT_EINVAL
    assert L.rt_surrogate_gen(tr._h, 1, k.ctypes.data, neg.ctypes.data, 16, 0.01, 0, 1, P, P, P,
                              None) == rt.RT_EINVAL
    assert L.rt_surrogate_gen(tr._h, 1, k.ctypes.data, one.ctypes.data, 16, 0.01, 0, 1, P, P, P, None) == rt.RT_ESTATE
    assert L.rt_surrogate_calibrate(tr._h, 1, 16, P, P, P, one.ctypes.data, 0, P, None) == rt.RT_EINVAL
    assert L.rt_surrogate_calibrate(tr._h, 1, 16, P, P, P, one.ctypes.data, 8, P, None) == rt.RT_ESTATE
    # MLP entry points
    rows = np.array([3, -1], np.int32)
    assert L.rt_mlp_fwd_grouped(tr._h, 2, rows.ctypes.data, P, P, P, P, None) == rt.RT_EINVAL
    assert L.rt_mlp_fwd_grouped(tr._h, 65, rows.ctypes.data, P, P, P, P, None) == rt.RT_EINVAL
    assert L.rt_mlp_work_bytes(0, 5) == 0 and L.rt_mlp_work_bytes(2, 5) > 0
    assert L.rt_mlp_fwd(tr._h, 2, 5, P, P, P, P, P, 0, None) == rt.RT_EINVAL       # workspace too small
    nb = L.rt_mlp_work_bytes(2, 5)
    assert L.rt_mlp_fwd(tr._h, 2, 5, P, P, P, P, P, nb, None) == rt.RT_ESTATE
    assert L.rt_mlp_bwd(tr._h, 2, 5, P, None, P, P, P, nb, None) == rt.RT_EINVAL
    assert L.rt_adamw_step(tr._h, P, P, P, P, P, 10, 1e-3, 0.9, 0.999, 1e-8, 0.0, 0, None) == rt.RT_EINVAL
    assert L.rt_adamw_step(tr._h, P, P, P, P, P, 10, 1e-3, 0.9, 0.999, 1e-8, 0.0, 1, None) == rt.RT_ESTATE
    assert L.rt_mse_grad(tr._h, P, P, P, 10, 0, P, None) == rt.RT_EINVAL


def test_surrogate_train_validates():
    rt = _rt()
    tr = rt.Tracer(-1)
    L = rt.lib()
    P = C.c_void_p(16)
    k = np.array([1.0, 0.5], np.float32)
    sc = np.array([0.1, 0.2], np.float32)
    nb = L.rt_surrogate_train_bytes(2, 64)
    assert nb > 0 and L.rt_surrogate_train_bytes(0, 64) == 0

    def call(**kw):
        a = dict(n=2, kappa=k.ctypes.data, scale=sc.ctypes.data, batch=64, steps=10, h=0.01, mode=0, lr=1e-3,
                 warm=5, work_bytes=nb, log=None, log_every=1)
        a.update(kw)
        return L.rt_surrogate_train(tr._h, a["n"], a["kappa"], a["scale"], a["batch"], a["steps"], a["h"],
                                    a["mode"], 1, a["lr"], 1e-5, a["warm"], 0.9, 0.999, 1e-8, 0.0, P, P, P, P, P,
                                    a["work_bytes"], a["log"], a["log_every"], None)
    assert call(n=0) == rt.RT_EINVAL
    assert call(steps=0) == rt.RT_EINVAL
    assert call(mode=1) == rt.RT_EINVAL          # the grid is for calibration, not training
    assert call(h=0.0) == rt.RT_EINVAL
    assert call(lr=0.0) == rt.RT_EINVAL
    assert call(work_bytes=nb - 1) == rt.RT_EINVAL
    assert call(log=P, log_every=0) == rt.RT_EINVAL
    bad = np.array([-0.1, 0.2], np.float32)
    assert call(scale=bad.ctypes.data) == rt.RT_EINVAL
    assert call() == rt.RT_ESTATE


def test_illuminate_validates():
    rt = _rt()
    tr = rt.Tracer(-1)
    wl = W.get("single_bump_64")
    light = dict(pos=(1.0, 2.0, -1.0))
    with pytest.raises(rt.RtError) as e:  # no metric yet
        tr.illuminate_raw(wl["camera"], 16, 16, light, 16, 16)
    assert e.value.status == rt.RT_ESTATE
    tr.set_metric(wl["metric"])
    tr.set_scene(wl["scene"])
    for bad, ptrs in [(dict(light, h=0.5), (16, 16, 16, 16)), (dict(light, h=0.0), (16, 16, 16, 16)),
                      (dict(light, tol=-1.0), (16, 16, 16, 16)), (dict(light, max_iters=0), (16, 16, 16, 16)),
                      (dict(light, pos=(np.nan, 0.0, 0.0)), (16, 16, 16, 16)), (light, (0, 16, 16, 16)),
                      (light, (16, 16, 0, 16))]:
        with pytest.raises(rt.RtError) as e:
            tr.illuminate_raw(wl["camera"], ptrs[0], ptrs[1], bad, ptrs[2], ptrs[3])
        assert e.value.status == rt.RT_EINVAL, bad
    # every argument valid: a host-only context stops after validation
    with pytest.raises(rt.RtError) as e:
        tr.illuminate_raw(wl["camera"], 16, 16, light, 16, 16)
    assert e.value.status == rt.RT_ESTATE
