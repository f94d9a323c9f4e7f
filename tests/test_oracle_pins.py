"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test compares the oracle with something that is not the oracle: a
closed form, a generic formula computed a different way, an invariant or a
convergence order.  All CPU-only.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests import exact

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _flat(wl):
    m = W.metric(W.EUCLID)
    return oracle.Oracle(m, wl["scene"])


# ------------------------------------------------------------ flat space
@pytest.mark.parametrize("name", ["single_bump_64", "bumps16_1080p"])
def test_flat_space_hits_are_analytic(name):
    """f = 0: rays are straight lines; hits equal the closed-form
    intersections (sphere, plane) and the torus quartic roots."""
    wl = W.with_size(W.get(name), 48, 32)
    cam, rule = wl["camera"], dict(wl["rule"])
    orc = _flat(wl)
    pix = np.arange(48 * 32)
    res = orc.trace(cam, rule, pix)
    d = exact.camera_dirs(cam, pix)
    t, ids = exact.line_hits(np.float64(cam["eye"]), d, wl["scene"], rule["t_max"])
    same = res["id"] == ids
    assert same.mean() >= 0.995, same.mean()
    hit = (ids >= 0) & same
    assert hit.sum() > 100
    exp_hit = np.float64(cam["eye"]) + t[hit, None] * d[hit]
    assert np.max(np.abs(res["hit"][hit] - exp_hit)) < 1e-9
    assert np.max(np.abs(res["t"][hit] - t[hit])) < 1e-9
    assert np.max(np.abs(res["dir"] - d)) < 1e-12
    miss = (ids < 0) & same
    assert np.allclose(res["t"][miss], rule["max_steps"] * np.float64(np.float32(rule["h"])), atol=1e-9)


def test_graph_metric_with_zero_amplitude_is_flat():
    wl = W.with_size(W.get("bumps16_1080p"), 24, 16)
    b = wl["metric"]["bumps"].copy()
    b[..., 0] = 0.0
    m = W.metric(W.GRAPH_GAUSS, b)
    r1 = oracle.Oracle(m, wl["scene"]).trace(wl["camera"], wl["rule"])
    r2 = _flat(wl).trace(wl["camera"], wl["rule"])
    for k in ("hit", "t", "dir", "id"):
        assert np.array_equal(r1[k], r2[k])


def test_camera_directions():
    cam = W.camera(64, 48)
    orc = _flat(W.get("single_bump_64"))
    pix = np.array([0, 63, 64 * 47, 64 * 48 - 1, 64 * 24 + 32])
    d = exact.camera_dirs(cam, pix)
    for q, p in enumerate(pix):
        assert np.allclose(orc.camera_dir(cam, p % 64, p // 64), d[q], atol=1e-15)
    # top-left pixel looks up and left (+y, -x) of +z
    assert d[0][0] < 0 and d[0][1] > 0


# ------------------------------------------------- graph metric algebra
def _rand_points(n, seed, box=2.0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-box, box, size=(n, 3))
    y = rng.normal(size=(n, 3))
    return x, y


@pytest.mark.parametrize("name", ["single_bump_64", "bumps16_1080p"])
def test_graph_accel_matches_generic_christoffel(name):
    """Eq. 5.4 (Gamma = f_m f_ij / (1+|grad f|^2)) equals the generic
    Levi-Civita symbols of Eq. 3.4 computed from finite differences of
    g = I + grad f grad f^T."""
    wl = W.get(name)
    bumps = wl["metric"]["bumps"][0].astype(np.float64)
    orc = oracle.Oracle(wl["metric"], wl["scene"])
    # points near the bumps so that the curvature is not negligible
    x, y = _rand_points(40, 3, box=1.0)
    if name == "bumps16_1080p":
        x = bumps[np.arange(40) % len(bumps), 1:4] + 0.3 * np.random.default_rng(4).normal(size=(40, 3))
    worst = 0.0
    for q in range(len(x)):
        a, ok = orc.accel(x[q], y[q])
        ref = exact.generic_accel(lambda z: exact.graph_g(bumps, z), x[q], y[q])
        scale = max(1e-3, np.abs(ref).max())
        worst = max(worst, np.abs(a - ref).max() / scale)
    assert worst < 2e-7, worst


def _graph2(kind):
    """Metric, scalar function f and sample points for the anisotropic and
    quadric graph kinds."""
    if kind == W.GRAPH_ANISO:
        ab = W.random_abumps(16, seed=0)
        x = ab[np.arange(40) % 16, 1:4].astype(np.float64) + 0.3 * np.random.default_rng(6).normal(size=(40, 3))
        return W.metric(kind, abumps=ab), (lambda z: exact.gauss_aniso_f(ab, z)), x
    q = (1.0, 1.0, -1.0)
    return W.metric(kind, quadric=q), (lambda z: exact.quadric_f(q, z)), _rand_points(40, 8, box=1.5)[0]


@pytest.mark.parametrize("kind", [W.GRAPH_ANISO, W.GRAPH_QUADRIC])
def test_graph2_accel_matches_generic_christoffel(kind):
    """Eq. 5.4 for anisotropic Gaussian sums and the quadratic of Sec. 5.1
    equals the generic symbols of g = I + grad f grad f^T, with grad f by
    complex step from an independent f; det g = 1 + |grad f|^2."""
    m, f, x = _graph2(kind)
    orc = oracle.Oracle(m, W.scene())
    y = np.random.default_rng(9).normal(size=(len(x), 3))
    worst = 0.0
    for q in range(len(x)):
        a, ok = orc.accel(x[q], y[q])
        assert ok
        ref = exact.generic_accel(lambda z: exact.graph_g(None, z, f), x[q], y[q])
        worst = max(worst, np.abs(a - ref).max() / max(1e-3, np.abs(ref).max()))
        g = orc.metric_tensor(x[q])
        gr = exact.cs_grad(f, x[q])
        assert abs(np.linalg.det(g) - (1.0 + gr @ gr)) < 1e-10 * (1.0 + gr @ gr)
    assert worst < 2e-7, worst


def test_aniso_with_equal_spreads_is_isotropic():
    """Three equal spreads reduce Eq. 6.1 to the isotropic bump: the two
    oracle kinds agree to rounding."""
    b = W.random_bumps(8, seed=2).astype(np.float64)
    ab = np.concatenate([b[:, :4], np.repeat(b[:, 4:5], 3, axis=1)], axis=1)
    o1 = oracle.Oracle(W.metric(W.GRAPH_GAUSS, b), W.scene())
    o2 = oracle.Oracle(W.metric(W.GRAPH_ANISO, abumps=ab), W.scene())
    x, y = _rand_points(30, 10, box=1.5)
    for q in range(len(x)):
        a1, _ = o1.accel(x[q], y[q])
        a2, _ = o2.accel(x[q], y[q])
        assert np.allclose(a1, a2, rtol=1e-12, atol=1e-15)


def test_graph2_sign_invariance_is_bitwise():
    """f -> -f leaves g, hence every traced ray, unchanged bit for bit."""
    for kind in (W.GRAPH_ANISO, W.GRAPH_QUADRIC):
        wl = W.with_size(W.get("abumps16_1080p" if kind == W.GRAPH_ANISO else "quadric_1080p"), 24, 14)
        m2 = dict(wl["metric"])
        if kind == W.GRAPH_ANISO:
            m2["abumps"] = wl["metric"]["abumps"].copy()
            m2["abumps"][..., 0] *= -1
        else:
            m2["quadric"] = [-q for q in wl["metric"]["quadric"]]
        r1 = oracle.Oracle(wl["metric"], wl["scene"]).trace(wl["camera"], wl["rule"])
        r2 = oracle.Oracle(m2, wl["scene"]).trace(wl["camera"], wl["rule"])
        for k in ("hit", "t", "dir", "id", "steps"):
            assert np.array_equal(r1[k], r2[k]), (kind, k)


def test_graph_det_g_volume_element():
    """det g = 1 + |grad f|^2 (Sec. 5.1)."""
    wl = W.get("bumps16_1080p")
    bumps = wl["metric"]["bumps"][0].astype(np.float64)
    orc = oracle.Oracle(wl["metric"], wl["scene"])
    x, _ = _rand_points(50, 5, box=2.0)
    for q in range(len(x)):
        g = orc.metric_tensor(x[q])
        gr = exact.cs_grad(lambda z: exact.gauss_f(bumps, z), x[q])
        assert abs(np.linalg.det(g) - (1.0 + gr @ gr)) < 1e-12
        # corrected inverse: g^-1 = I - grad f grad f^T / (1 + |grad f|^2)
        ginv = np.eye(3) - np.outer(gr, gr) / (1.0 + gr @ gr)
        assert np.allclose(g @ ginv, np.eye(3), atol=1e-13)


def test_sign_invariance_is_bitwise():
    """g depends on grad f grad f^T only, so f -> -f traces identical rays."""
    wl = W.with_size(W.get("bumps16_1080p"), 32, 18)
    m2 = dict(wl["metric"])
    m2["bumps"] = wl["metric"]["bumps"].copy()
    m2["bumps"][..., 0] *= -1
    r1 = oracle.Oracle(wl["metric"], wl["scene"]).trace(wl["camera"], wl["rule"])
    r2 = oracle.Oracle(m2, wl["scene"]).trace(wl["camera"], wl["rule"])
    for k in ("hit", "t", "dir", "id", "steps"):
        assert np.array_equal(r1[k], r2[k]), k


# ------------------------------------------------------ pullback algebra
# Strong local deformations around the origin (six of them, overlapping, so
# that the order of the composition matters).
DEFORMS = W.random_deforms(6, seed=21, box=0.8, spread=(0.4, 0.9), kappa=(0.4, 0.8))
# The same with fields that also rotate about an axis through each centre.
RDEFORMS = W.random_deforms(6, seed=22, box=0.8, spread=(0.4, 0.9), kappa=(0.2, 0.4), rot=(0.3, 0.5))
ROTATING = "rotating deformations"


def _pullback(kind):
    if kind == W.PULLBACK_DEFORM:
        return W.metric(kind, deforms=DEFORMS), lambda z: exact.deform_phi(z, DEFORMS)
    if kind == ROTATING:
        return W.metric(W.PULLBACK_DEFORM, deforms=RDEFORMS), lambda z: exact.deform_phi(z, RDEFORMS)
    return W.metric(kind), (exact.twist_phi if kind == W.PULLBACK_TWIST else exact.ztwist_phi)


PULLBACKS = [W.PULLBACK_TWIST, W.PULLBACK_ZTWIST, W.PULLBACK_DEFORM, ROTATING]


@pytest.mark.parametrize("kind", PULLBACKS)
def test_pullback_accel_matches_generic_christoffel(kind):
    """Thm 5.1 / Eq. 5.8 equals the generic symbols of g = J^T J."""
    m, phi = _pullback(kind)
    orc = oracle.Oracle(m, W.scene())
    x, y = _rand_points(30, 7, box=1.5)
    worst = 0.0
    for q in range(len(x)):
        a, ok = orc.accel(x[q], y[q])
        assert ok
        ref = exact.generic_accel(lambda z: exact.pullback_g(phi, z), x[q], y[q])
        worst = max(worst, np.abs(a - ref).max() / max(1e-3, np.abs(ref).max()))
        g = orc.metric_tensor(x[q])
        assert np.allclose(g, exact.pullback_g(phi, x[q]), rtol=1e-13, atol=1e-13)
    assert worst < 2e-7, worst


def _straight_line_residual(kind, h, n, seed=11):
    m, phi = _pullback(kind)
    orc = oracle.Oracle(m, W.scene())
    rng = np.random.default_rng(seed)
    worst = 0.0
    for _ in range(4):
        p = rng.uniform(-1.2, 1.2, 3)
        v = rng.normal(size=3)
        g = orc.metric_tensor(p)
        v = v / np.sqrt(v @ g @ v)
        rule = W.rule(W.RK4, h=h, max_steps=n)
        rule["h"] = h
        traj = orc.trajectory(rule, np.concatenate([p, v]), n)
        J = exact.cs_jac(phi, p)
        tk = float(np.float32(h)) * np.arange(n + 1)
        line = phi(p)[None, :] + tk[:, None] * (J @ v)[None, :]
        img = np.array([phi(z[:3]) for z in traj])
        worst = max(worst, np.abs(img - line).max())
    return worst


@pytest.mark.parametrize("kind", PULLBACKS)
def test_pullback_geodesics_are_preimages_of_lines(kind):
    """phi(x(t)) = phi(p) + t J(p) v; RK4 error O(h^4)."""
    e1 = _straight_line_residual(kind, 0.02, 150)
    e2 = _straight_line_residual(kind, 0.01, 300)
    assert e1 < 1e-5, e1
    assert 10.0 < e1 / e2 < 24.0, (e1, e2)


def test_deform_composition_order_matters():
    """The pins above would fail for the reversed composition: the two
    orders give different maps for these deformations."""
    x = np.array([0.1, -0.2, 0.15])
    fwd = exact.deform_phi(x, DEFORMS)
    rev = exact.deform_phi(x, DEFORMS[::-1])
    assert np.abs(fwd - rev).max() > 1e-2
    orc = oracle.Oracle(W.metric(W.PULLBACK_DEFORM, deforms=DEFORMS), W.scene())
    J = exact.cs_jac(lambda z: exact.deform_phi(z, DEFORMS), x)
    assert np.allclose(orc.metric_tensor(x), J.T @ J, rtol=1e-12, atol=1e-12)


def test_deform_diffeomorphism_margin():
    """Each Phi_i of the generator satisfies |a| |v/s| exp(-1/2) = kappa < 1,
    the condition for 1 + grad f . v > 0 everywhere; check it by brute force
    on a grid around each centre."""
    for a, cx, cy, cz, sx, sy, sz, vx, vy, vz in DEFORMS.astype(np.float64):
        g = np.linspace(-3, 3, 41)
        X, Y, Z = np.meshgrid(g * sx, g * sy, g * sz, indexing="ij")
        f = a * np.exp(-0.5 * ((X / sx) ** 2 + (Y / sy) ** 2 + (Z / sz) ** 2))
        gv = -f * (X / sx ** 2 * vx + Y / sy ** 2 * vy + Z / sz ** 2 * vz)
        kap = abs(a) * np.sqrt((vx / sx) ** 2 + (vy / sy) ** 2 + (vz / sz) ** 2) * np.exp(-0.5)
        assert kap < 0.95
        assert (1.0 + gv).min() > 0.0
        assert np.isclose(np.abs(gv).max(), kap, rtol=0.05)


def test_rotating_deformation_lipschitz_margin():
    """Each Phi_i of the rotating generator has |D(f V)| <= kappa + share
    < 1 (spectral norm, brute force on a grid around each centre), so it is
    a diffeomorphism; and the rotation part is not negligible."""
    rot_part = 0.0
    for a, cx, cy, cz, sx, sy, sz, vx, vy, vz, wx, wy, wz in RDEFORMS.astype(np.float64):
        s = np.array([sx, sy, sz])
        v, w = np.array([vx, vy, vz]), np.array([wx, wy, wz])
        bound = abs(a) * (np.exp(-0.5) * np.linalg.norm(v) / s.min()
                          + np.linalg.norm(w) * (2.0 / np.e * s.max() / s.min() + 1.0))
        assert bound <= 0.95
        W_ = np.array([[0.0, -wz, wy], [wz, 0.0, -wx], [-wy, wx, 0.0]])
        worst = 0.0
        grid = np.linspace(-3, 3, 13)
        for i in grid:
            for j in grid:
                for k in grid:
                    d = np.array([i, j, k]) * s
                    f = a * np.exp(-0.5 * ((d / s) ** 2).sum())
                    gf = -f * d / s ** 2
                    DF = np.outer(v + np.cross(w, d), gf) + f * W_
                    worst = max(worst, np.linalg.norm(DF, 2))
                    rot_part = max(rot_part, abs(f) * np.linalg.norm(np.cross(w, d)))
        assert worst <= bound + 1e-12, (worst, bound)
        assert worst < 1.0
    assert rot_part > 0.02


def test_ztwist_closed_form_geodesic():
    """The z-twist of Sec. 5.2: x(t) = Phi^-1(Phi(p) + t J(p) v)."""
    orc = oracle.Oracle(W.metric(W.PULLBACK_ZTWIST), W.scene())
    p = np.array([0.3, -0.2, 0.1])
    v = np.array([0.2, 0.5, 0.7])
    g = orc.metric_tensor(p)
    v = v / np.sqrt(v @ g @ v)
    h, n = 0.005, 800
    rule = W.rule(W.RK4, h=h, max_steps=n)
    rule["h"] = h
    traj = orc.trajectory(rule, np.concatenate([p, v]), n)
    J = exact.cs_jac(exact.ztwist_phi, p)
    tk = float(np.float32(h)) * np.arange(n + 1)
    X = exact.ztwist_phi(p)[None, :] + tk[:, None] * (J @ v)[None, :]
    x_exact = exact.ztwist_inv(X)
    assert np.abs(traj[:, :3] - x_exact).max() < 1e-8


# ---------------------------------------------- conservation, convergence
def test_speed_is_conserved():
    """g(y, y) is constant along a geodesic; RK4 drift scales like h^4."""
    wl = W.get("bumps16_1080p")
    orc = oracle.Oracle(wl["metric"], wl["scene"])
    bumps = wl["metric"]["bumps"][0]
    p = np.array([-1.5, 0.2, -2.5])
    v = (bumps[0, 1:4] - p)
    v = v / np.sqrt(v @ orc.metric_tensor(p) @ v)
    drift = []
    for h in (0.02, 0.01):
        n = int(round(4.0 / h))
        rule = W.rule(W.RK4, h=h, max_steps=n)
        rule["h"] = h
        traj = orc.trajectory(rule, np.concatenate([p, v]), n)
        sp = [z[3:] @ orc.metric_tensor(z[:3]) @ z[3:] for z in traj]
        drift.append(np.abs(np.array(sp) - 1.0).max())
    assert drift[0] < 1e-5
    assert 8.0 < drift[0] / drift[1] < 40.0, drift


def _single_bump_exact(wl, pixels):
    cam = wl["camera"]
    bump = wl["metric"]["bumps"][0, 0].astype(np.float64)
    sc = wl["scene"]
    sph = np.float64(sc["spheres"][0])
    pl = np.float64(sc["planes"][0])
    objs = [lambda x: (x - sph[:3]) @ (x - sph[:3]) - sph[3] ** 2,
            lambda x: pl[:3] @ x - pl[3]]
    d = exact.camera_dirs(cam, pixels)
    out = []
    for q in range(len(pixels)):
        ray = exact.SingleBumpRay(bump[0], bump[1:4], bump[4], np.float64(cam["eye"]), d[q]).tabulate(
            wl["rule"]["t_max"])
        out.append(ray.first_hit(objs, wl["rule"]["t_max"]))
    return out


def test_single_bump_rays_match_quadrature():
    """One isotropic bump: exact hits from the 1-D quadratures of the planar,
    angular-momentum-conserving geodesic.  RK4 at h = 0.01 agrees to
    truncation error and converges at fourth order."""
    wl = W.get("single_bump_64")
    orc = oracle.Oracle(wl["metric"], wl["scene"])
    pix = W.pixel_sample(64, 64, 400, seed=5)
    # keep rays that pass the bump closely enough to be bent noticeably and
    # that hit something
    d = exact.camera_dirs(wl["camera"], pix)
    b = np.linalg.norm(np.cross(np.float64(wl["camera"]["eye"]), d), axis=1)
    hits = oracle.Oracle(wl["metric"], wl["scene"]).trace(wl["camera"], wl["rule"], pix)["id"] >= 0
    pix = pix[(b > 0.02) & (b < 1.2) & hits][:30]
    ex = _single_bump_exact(wl, pix)
    errs = {}
    for h in (0.01, 0.005):
        rule = dict(wl["rule"])
        rule["h"] = h
        rule["max_steps"] = int(round(10.0 / h))
        res = orc.trace(wl["camera"], rule, pix)
        e = []
        for q, (t, oid, x) in enumerate(ex):
            assert res["id"][q] == oid, (q, res["id"][q], oid)
            if oid >= 0:
                e.append(max(np.abs(res["hit"][q] - x).max(), abs(res["t"][q] - t)))
        errs[h] = np.array(e)
    assert len(errs[0.01]) >= 10
    assert errs[0.01].max() < 2e-5, errs[0.01].max()
    big = errs[0.01] > 1e-9
    ratio = np.median(errs[0.01][big] / errs[0.005][big])
    assert 10.0 < ratio < 24.0, ratio


def test_single_bump_angular_momentum_and_planarity():
    wl = W.get("single_bump_64")
    orc = oracle.Oracle(wl["metric"], wl["scene"])
    p = np.float64(wl["camera"]["eye"])
    d = np.array([0.05, 0.03, 1.0])
    d /= np.linalg.norm(d)
    rule = dict(wl["rule"])
    traj = orc.trajectory(rule, np.concatenate([p, d]), 800)
    L = np.cross(traj[:, :3], traj[:, 3:])
    # continuous flow: L exactly conserved; RK4 keeps it to O(h^4)
    assert np.abs(L - L[0]).max() < 1e-8
    # every stage moves within the plane spanned by x - c and y
    n = L[0] / np.linalg.norm(L[0])
    assert np.abs(traj[:, :3] @ n).max() < 1e-13


def test_rk45_converged_matches_quadrature():
    """Dormand-Prince 5(4) with tight tolerances reaches the exact hits."""
    wl = W.get("single_bump_64")
    orc = oracle.Oracle(wl["metric"], wl["scene"])
    pix = W.pixel_sample(64, 64, 40, seed=9)
    d = exact.camera_dirs(wl["camera"], pix)
    b = np.linalg.norm(np.cross(np.float64(wl["camera"]["eye"]), d), axis=1)
    pix = pix[(b > 0.02) & (b < 1.0)][:12]
    ex = _single_bump_exact(wl, pix)
    rule = W.rule(W.RK45, h=0.01, max_steps=20000, t_max=10.0, rtol=1e-11, atol=1e-11,
                  h_min=1e-9, h_max=0.02)
    rule.update(rtol=1e-11, atol=1e-11, h_min=1e-9)
    res = orc.trace(wl["camera"], rule, pix)
    for q, (t, oid, x) in enumerate(ex):
        assert res["id"][q] == oid
        if oid >= 0:
            assert np.abs(res["hit"][q] - x).max() < 1e-8
            assert abs(res["t"][q] - t) < 1e-8


def test_dp5_orders():
    """The 5th-order solution has local error O(h^6), the embedded error
    estimate is O(h^5): checks every tableau coefficient at once."""
    wl = W.get("single_bump_64")
    orc = oracle.Oracle(wl["metric"], wl["scene"])
    z0 = np.array([-0.2, 0.1, -0.5, 0.2, 0.1, 1.0])
    z0[3:] /= np.sqrt(z0[3:] @ orc.metric_tensor(z0[:3]) @ z0[3:])
    loc, est = [], []
    for H in (0.08, 0.04, 0.02):
        out, err, _ = orc.step(W.RK45, z0, H)
        ref = z0.copy()
        for _ in range(400):
            ref, _, _ = orc.step(W.RK4, ref, H / 400)
        loc.append(np.abs(out - ref).max())
        est.append(np.abs(err).max())
    r_loc = loc[1] / loc[2]
    r_est = est[1] / est[2]
    assert 40 < r_loc < 100, loc
    assert 20 < r_est < 48, est


def test_euler_is_first_order():
    """The paper's Eq. 4.1 integrator: global error halves with h."""
    wl = W.get("single_bump_64")
    orc = oracle.Oracle(wl["metric"], wl["scene"])
    z0 = np.array([-0.2, 0.1, -1.0, 0.1, 0.05, 1.0])
    z0[3:] /= np.linalg.norm(z0[3:])
    ref_rule = W.rule(W.RK4, h=0.001, max_steps=2000)
    ref_rule["h"] = 0.001
    ref = orc.trajectory(ref_rule, z0, 2000)[-1]
    errs = []
    for h in (0.004, 0.002):
        r = W.rule(W.EULER, h=h, max_steps=int(round(2.0 / h)))
        r["h"] = h
        errs.append(np.abs(orc.trajectory(r, z0, int(round(2.0 / h)))[-1] - ref).max())
    assert 1.7 < errs[0] / errs[1] < 2.3, errs


# --------------------------------------------------- direct illumination
def test_shoot_and_visibility_flat_space():
    """g = I: the shot geodesic is the segment q + t v, and it is clear
    exactly when the segment meets no object (closed form)."""
    wl = W.get("bumps16_1080p")
    orc = oracle.Oracle(W.metric(W.EUCLID), wl["scene"])
    rng = np.random.default_rng(12)
    n_clear = 0
    for _ in range(200):
        q = rng.uniform(-2.5, 2.5, 3)
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        T = rng.uniform(0.5, 4.0)
        z, ok = orc.shoot(q, v, T, 0.01)
        assert ok
        assert np.allclose(z[:3], q + T * v, atol=1e-12) and np.allclose(z[3:], v, atol=1e-14)
        t, oid = exact.line_hits(q, v[None, :], wl["scene"], T)
        inside = any(np.linalg.norm(q - s[:3]) < s[3] for s in wl["scene"]["spheres"])
        if inside:
            continue
        clear = orc.geodesic_clear(q, v, T, 0.01, 0.0)
        n_clear += clear
        assert clear == (oid[0] < 0), (q, v, T, t, oid)
    assert 20 < n_clear < 190


def test_shoot_matches_the_trajectory():
    """Shooting over a whole number of steps is the trajectory itself."""
    wl = W.get("bumps16_1080p")
    orc = oracle.Oracle(wl["metric"], wl["scene"])
    z0 = np.array([0.3, -0.2, -1.5, 0.1, 0.05, 0.9])
    z0[3:] /= np.sqrt(z0[3:] @ orc.metric_tensor(z0[:3]) @ z0[3:])
    traj = orc.trajectory(W.rule(W.RK4, h=0.01, max_steps=300), z0, 300)
    z, ok = orc.shoot(z0[:3], z0[3:], float(np.float32(0.01)) * 300, float(np.float32(0.01)))
    assert ok and np.allclose(z, traj[-1], atol=1e-12)


def test_twist_rays_through_the_origin():
    """The twist phi(x) = x + 0.4 tanh|x| R_z(1.2 e^{-|x|^2}) x is C^1 but
    not C^2 at the origin (tanh|x| ~ |x|): D^2 phi[y, y] there depends on
    the side from which the ray arrives, so the flow's right-hand side jumps
    across the origin.  The oracle stays finite on rays aimed at the origin
    and their images stay on the straight line phi(p) + t J(p) v to within a
    step's jump, O(h |a| t) rather than RK4's O(h^4); from a distance of a
    few h on, fourth order returns."""
    m = W.metric(W.PULLBACK_TWIST)
    orc = oracle.Oracle(m, W.scene())
    phi = exact.twist_phi

    def resid(b, h, T=3.0):
        n = int(round(T / h))
        p = np.array([b, 0.3 * b, -1.5])
        d = np.array([0.0, 0.0, 1.0])
        v = d / np.sqrt(d @ orc.metric_tensor(p) @ d)
        rule = W.rule(W.RK4, h=h, max_steps=n)
        rule["h"] = h
        traj = orc.trajectory(rule, np.concatenate([p, v]), n)
        assert np.isfinite(traj).all()
        tk = float(np.float32(h)) * np.arange(n + 1)
        line = phi(p)[None, :] + tk[:, None] * (exact.cs_jac(phi, p) @ v)[None, :]
        img = np.array([phi(z[:3]) for z in traj])
        return np.abs(img - line).max(), traj

    e, traj = resid(0.0, 0.005)
    # on the axis the ray stays on it exactly (the acceleration has no x, y part)
    assert np.all(traj[:, 0] == 0.0) and np.all(traj[:, 1] == 0.0)
    for b in (0.0, 1e-4, 1e-3):
        for h in (0.01, 0.005):
            assert resid(b, h)[0] < 4e-3
    # away from the origin by two steps: fourth order again
    e1, e2 = resid(0.01, 0.01)[0], resid(0.01, 0.005)[0]
    assert e2 < 1e-7 and e1 / e2 > 16.0, (e1, e2)


def test_failed_rays_stop_at_their_last_accepted_state():
    """id -2 (the error-controlled step of the RK45 march would have to fall
    below h_min).  With h = h_min = h_max = 0.08 the step can never grow
    back, and a ray fails at the first attempt whose error norm exceeds 1:
    on the rays through the bump's steep core.  A failed ray reports the
    state after its accepted steps: bitwise the output of the same run
    stopped there by max_steps (a miss, id -1).  Rays that keep away from
    the bump never see a large error and are bitwise the rays of a run with
    tolerances so loose that no attempt is rejected."""
    n = 32
    wl = W.with_size(W.get("single_bump_64"), n, n)
    wl["camera"] = W.camera(n, n, vfov_deg=20.0)
    m = dict(wl["metric"], bumps=W.f32([[[1.5, 0.0, 0.0, 0.0, 0.3]]]))
    strict = W.rule(kind=W.RK45, h=0.08, max_steps=4000, t_max=10.0, rtol=1e-6, atol=1e-6)
    strict.update(h_min=strict["h"], h_max=strict["h"])
    loose = dict(strict, rtol=1e9, atol=1e9)
    orc = oracle.Oracle(m, wl["scene"])
    a = orc.trace(wl["camera"], strict)
    b = orc.trace(wl["camera"], loose)
    fail = a["id"] == -2
    assert 10 < fail.sum() < 0.5 * fail.size
    assert (b["id"] != -2).all() and (b["rejected"] == 0).all()
    for p in np.flatnonzero(fail):
        c = orc.trace(wl["camera"], dict(strict, max_steps=int(a["steps"][p])), np.array([p]))
        assert c["id"][0] == -1 and c["steps"][0] == a["steps"][p]
        assert np.array_equal(c["hit"][0], a["hit"][p]) and c["t"][0] == a["t"][p]
    ii, jj = np.unravel_index(np.arange(n * n), (n, n))
    r = np.hypot(ii - (n - 1) / 2, jj - (n - 1) / 2)
    assert r[fail].max() < 6 and fail.reshape(n, n)[n // 2 - 1:n // 2 + 1, n // 2 - 1:n // 2 + 1].all()
    same = np.all(a["hit"] == b["hit"], axis=1) & (a["id"] == b["id"])
    assert same[r > 10].all() and same.mean() > 0.7
