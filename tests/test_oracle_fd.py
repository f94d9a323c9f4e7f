"""Pins of the oracle's finite-difference gradient (the reference the GPU
adjoint is checked against).

The loss is L(theta) = sum over masked pixels of |hit(theta) - target|^2,
with theta the bump parameters (a, cx, cy, cz, sigma) of Eq. 6.1.  These
facts fix the derivative without reference to the oracle itself:

  * g = I + grad f grad f^T (Eq. 5.2) is even in f, so rays, and hence L,
    are even in the amplitudes as a whole: with every a = 0, all central
    differences vanish exactly; a global a -> -a flips dL/da and leaves
    dL/dc, dL/dsigma unchanged, bit for bit;
  * a bump of amplitude 0 contributes nothing whatever its centre and
    spread: dL/dc_b = dL/dsigma_b = 0 exactly;
  * for one isotropic bump the exact continuous hits follow from 1-D
    quadratures (planar geodesics conserving (x - c) x y), so central
    differences of the exact loss give the gradient with its signs,
    magnitudes and parameter order; RK4 at h = 0.01 must agree to its
    truncation error.
"""
import numpy as np

import oracle
import workloads as W

from . import exact


def _small(n_w=10, n_h=8):
    wl = W.get("single_bump_64")
    return W.with_size(wl, n_w, n_h)


def _bumps3():
    return np.array([[0.45, -0.35, 0.1, 0.2, 0.35],
                     [-0.5, 0.3, -0.15, -0.1, 0.3],
                     [0.4, 0.05, 0.35, 0.6, 0.25]])


def _target(wl, bumps):
    """Target hit map of a perturbed parameter set (oracle trace)."""
    tb = np.asarray(bumps, np.float64).copy()
    tb[:, 0] *= 0.9
    tb[:, 1:4] += np.array([0.03, -0.02, 0.04])
    tb[:, 4] *= 1.05
    r = oracle.Oracle(wl["metric"], wl["scene"], bumps64=tb).trace(wl["camera"], wl["rule"])
    return r["hit"], r["id"]


def _fd(wl, bumps, target_hit, target_id):
    wl = dict(wl, metric=W.metric(W.GRAPH_GAUSS, np.asarray(bumps, np.float32)))
    W_, H_ = wl["camera"]["width"], wl["camera"]["height"]
    pix = np.arange(W_ * H_, dtype=np.int64)
    return oracle.fd_gradient(wl["metric"], wl["scene"], wl["camera"], wl["rule"], pix, target_hit, target_id)


def test_fd_gradient_vanishes_with_zero_amplitudes():
    wl = _small()
    b = _bumps3()
    target_hit, target_id = _target(wl, b)
    b0 = b.copy()
    b0[:, 0] = 0.0
    g, L, mask = _fd(wl, b0, target_hit, target_id)
    assert mask.sum() >= 20 and L > 0.0
    assert np.all(g == 0.0), g


def test_fd_gradient_of_a_zero_amplitude_bump_position_and_spread():
    wl = _small()
    b = _bumps3()
    target_hit, target_id = _target(wl, b)
    b1 = b.copy()
    b1[1, 0] = 0.0
    g, L, mask = _fd(wl, b1, target_hit, target_id)
    assert mask.sum() >= 20
    assert np.all(g[1, 1:] == 0.0), g[1]
    # the other bumps act, so their components do not vanish
    assert np.all(np.abs(g[[0, 2]]) > 0.0), g


def test_fd_gradient_under_global_amplitude_flip():
    wl = _small()
    b = _bumps3()
    target_hit, target_id = _target(wl, b)
    g, L, mask = _fd(wl, b, target_hit, target_id)
    bn = b.copy()
    bn[:, 0] = -bn[:, 0]
    gn, Ln, maskn = _fd(wl, bn, target_hit, target_id)
    assert np.array_equal(mask, maskn) and L == Ln
    assert np.array_equal(gn[:, 0], -g[:, 0]), (g[:, 0], gn[:, 0])
    assert np.array_equal(gn[:, 1:], g[:, 1:])
    assert np.abs(g).min() > 0.0


def test_fd_gradient_matches_quadrature_derivative():
    """One bump (a = 0.5, sigma = 0.3 at the origin), the 64x64 camera and
    scene: the oracle's central differences of RK4 hits (h = 0.01,
    eps = 1e-4) against central differences of the exact hits.  Measured
    agreement is ~1e-6 of the largest component; 1e-4 leaves room for the
    RK4 truncation error and the quadrature's tolerance while a wrong sign,
    a factor 2 or a swapped parameter fails by orders of magnitude."""
    wl = W.get("single_bump_64")
    cam, scene, rule = wl["camera"], wl["scene"], wl["rule"]
    theta = np.array([0.5, 0.0, 0.0, 0.0, 0.3])
    target = np.array([0.45, 0.03, -0.02, 0.04, 0.32])
    eye = np.float64(cam["eye"])
    pix = W.pixel_sample(64, 64, 4096, seed=5)
    d = exact.camera_dirs(cam, pix)
    b = np.linalg.norm(np.cross(eye, d), axis=1)
    sph = np.float64(scene["spheres"][0])
    pl = np.float64(scene["planes"][0])
    objs = [lambda x: (x - sph[:3]) @ (x - sph[:3]) - sph[3] ** 2, lambda x: pl[:3] @ x - pl[3]]
    # rays passing the bump closely (strongly bent) that hit the sphere
    # (impact parameter below ~0.45 reaches it) or the plane
    cand = pix[(b > 0.05) & (b < 0.9)]
    rng = np.random.default_rng(3)
    cand = np.sort(rng.choice(cand, 48, replace=False))
    dc = exact.camera_dirs(cam, cand)

    def exact_hits(p, sel):
        ids, xs = [], []
        for q in sel:
            ray = exact.SingleBumpRay(p[0], p[1:4], p[4], eye, dc[q]).tabulate(rule["t_max"])
            t, oid, x = ray.first_hit(objs, rule["t_max"])
            ids.append(oid)
            xs.append(x if x is not None else np.zeros(3))
        return np.array(ids), np.array(xs)

    tid, thit = exact_hits(target, range(len(cand)))
    id0, _ = exact_hits(theta, range(len(cand)))
    keep = np.nonzero((tid >= 0) & (id0 == tid))[0][:20]
    assert len(keep) == 20
    px, tid, thit = cand[keep], tid[keep], thit[keep]
    sel = keep

    g, L, mask = oracle.fd_gradient(W.metric(W.GRAPH_GAUSS, theta[None].astype(np.float32)), scene, cam, rule,
                                    px, thit, tid)
    assert mask.all()
    eps = 1e-4
    ge = np.zeros(5)
    for j in range(5):
        tp, tm = theta.copy(), theta.copy()
        tp[j] += eps
        tm[j] -= eps
        ip, hp = exact_hits(tp, sel)
        im, hm = exact_hits(tm, sel)
        assert np.array_equal(ip, tid) and np.array_equal(im, tid)
        ge[j] = (((hp - thit) ** 2).sum() - ((hm - thit) ** 2).sum()) / (2 * eps)
    scale = np.abs(ge).max()
    assert np.all(np.abs(ge) > 0.05 * scale), ge  # every component carries signal
    err = np.abs(g[0] - ge).max() / scale
    assert err < 1e-4, (g[0], ge, err)
