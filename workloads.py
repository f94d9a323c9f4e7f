"""Seeded synthetic inputs for the Riemannian ray tracer.

This module only draws numbers and packs them into plain arrays and dicts:
cameras, Gaussian bump sets, scenes and step rules.  It contains none of the
method's arithmetic (no camera rays, no metric, no integrator, no
intersection), so both the FP64 oracle and the HIP path can consume it
without sharing any computation.

Every floating-point parameter is rounded to float32 here, once.  The GPU
path consumes these float32 values directly; the oracle converts the very
same float32 values to float64 (exactly), so both sides start from
bit-identical inputs.

Array formats (all float32, C-contiguous):
  bumps    [n_sets, n_bumps, 5]  (a, cx, cy, cz, sigma)   isotropic Eq. 6.1
  spheres  [n, 4]                (cx, cy, cz, r)
  planes   [n, 4]                (nx, ny, nz, d)  surface n.x = d, |n| = 1
  tori     [n, 8]                (cx, cy, cz, ax, ay, az, R, r), |a| = 1
Object ids run over spheres, then planes, then tori.

Workloads (sizes are the ones the throughput and parity runs use):
  single_bump_64      64x64, one bump a=0.5 sigma=0.3 at the origin, unit
                      sphere at (0,0,2) + plane y=-1, RK4 h=0.01, 1000 steps
  bumps16_1080p       1920x1080, 16 random bumps (seed 0), 64 random
                      spheres (seed 1) + plane y=-1 + torus, RK4 h=0.005,
                      4000 steps (t_max 20), one pass; RK45 variant tol 1e-6
  twist_4k            3840x2160, twist pullback
                      phi(x) = x + 0.4 tanh|x| R_z(1.2 exp(-|x|^2)) x,
                      256 random spheres (seed 1), RK4 h=0.005, 4000 steps
  adjoint_64x512      64 parameter sets x 8 bumps, 512x512, RK4 h=0.01,
                      2000 steps, scene of single_bump_64
  surrogate_64_4k     3840x2160, 64 random bumps, scene of bumps16_1080p
  surrogate_isolated_4k
                      3840x2160, 64 bumps with the distributions of
                      surrogate_64_4k but centres in [-8,8]^3 drawn by
                      rejection so that no bump's 6-sigma cut sphere reaches
                      another's 3-sigma support sphere (seed 3), 64 spheres
                      (seed 4) kept outside every support, plane y=-1, torus
"""
from __future__ import annotations

import copy
import numpy as np

# Metric kinds (same integer codes as the C-ABI and the oracle use).
EUCLID = 0
GRAPH_GAUSS = 1
PULLBACK_TWIST = 2
PULLBACK_ZTWIST = 3
PULLBACK_DEFORM = 4
GRAPH_ANISO = 5
GRAPH_QUADRIC = 6

# Step rules.
RK4 = 0
RK45 = 1
EULER = 2


def f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def camera(width, height, eye=(0.0, 0.0, -4.0), forward=(0.0, 0.0, 1.0),
           up=(0.0, 1.0, 0.0), vfov_deg=60.0):
    return dict(eye=f32(eye), forward=f32(forward), up=f32(up),
                vfov_deg=float(np.float32(vfov_deg)),
                width=int(width), height=int(height))


def random_bumps(n, seed, box=2.0, amp=0.6, sigma=(0.15, 0.5)):
    """Centres U[-box,box]^3, then amplitudes U(-amp,amp), then sigmas
    U(sigma) -- drawn in that order from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-box, box, size=(n, 3))
    a = rng.uniform(-amp, amp, size=n)
    s = rng.uniform(sigma[0], sigma[1], size=n)
    return f32(np.concatenate([a[:, None], c, s[:, None]], axis=1))


def isolated_bumps(n, seed, box=8.0, amp=0.6, sigma=(0.15, 0.5), gap=0.1):
    """Amplitudes U(-amp,amp), then sigmas U(sigma), then centres
    U[-box,box]^3 redrawn until |c_i - c_j| >= max(3 s_i + 6 s_j,
    3 s_j + 6 s_i) + gap for every earlier bump j."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-amp, amp, size=n)
    s = rng.uniform(sigma[0], sigma[1], size=n)
    c = np.zeros((n, 3))
    for i in range(n):
        for _ in range(100000):
            p = rng.uniform(-box, box, size=3)
            d = np.linalg.norm(c[:i] - p, axis=1)
            need = np.maximum(3 * s[i] + 6 * s[:i], 3 * s[:i] + 6 * s[i]) + gap
            if np.all(d >= need):
                break
        else:
            raise RuntimeError("isolated_bumps: could not place bump %d" % i)
        c[i] = p
    return f32(np.concatenate([a[:, None], c, s[:, None]], axis=1))


def spheres_outside(n, seed, bumps, box=2.0, radius=(0.1, 0.4), gap=0.05):
    """Radii U(radius), then centres U[-box,box]^3 redrawn until the sphere
    stays outside every bump's 3-sigma support sphere."""
    rng = np.random.default_rng(seed)
    b = np.asarray(bumps, np.float64).reshape(-1, 5)
    r = rng.uniform(radius[0], radius[1], size=n)
    c = np.zeros((n, 3))
    for i in range(n):
        for _ in range(100000):
            p = rng.uniform(-box, box, size=3)
            if np.all(np.linalg.norm(b[:, 1:4] - p, axis=1) >= 3 * b[:, 4] + r[i] + gap):
                break
        else:
            raise RuntimeError("spheres_outside: could not place sphere %d" % i)
        c[i] = p
    return f32(np.concatenate([c, r[:, None]], axis=1))


def random_spheres(n, seed, box=2.0, radius=(0.1, 0.4)):
    """Centres U[-box,box]^3, then radii U(radius), from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-box, box, size=(n, 3))
    r = rng.uniform(radius[0], radius[1], size=n)
    return f32(np.concatenate([c, r[:, None]], axis=1))


def empty4():
    return np.zeros((0, 4), np.float32)


def empty8():
    return np.zeros((0, 8), np.float32)


def rule(kind=RK4, h=0.01, max_steps=1000, t_max=None, rtol=1e-6, atol=1e-6,
         h_min=1e-6, h_max=0.02, cull_every=16, pass_steps=256,
         bisect_iters=24):
    if t_max is None:
        t_max = float(np.float32(h) * max_steps) if kind != RK45 else 20.0
    return dict(kind=int(kind), h=float(np.float32(h)), max_steps=int(max_steps),
                t_max=float(np.float32(t_max)), rtol=float(np.float32(rtol)),
                atol=float(np.float32(atol)), h_min=float(np.float32(h_min)),
                h_max=float(np.float32(h_max)), cull_every=int(cull_every),
                pass_steps=int(pass_steps), bisect_iters=int(bisect_iters))


def metric(kind, bumps=None, twist_amp=0.4, twist_theta0=1.2, cull_sigmas=6.0, deforms=None, abumps=None,
           quadric=None):
    if bumps is None:
        bumps = np.zeros((1, 0, 5), np.float32)
    bumps = f32(bumps)
    if bumps.ndim == 2:
        bumps = bumps[None]
    m = dict(kind=int(kind), bumps=bumps,
             twist_amp=float(np.float32(twist_amp)),
             twist_theta0=float(np.float32(twist_theta0)),
             cull_sigmas=float(np.float32(cull_sigmas)))
    if deforms is not None:
        d = f32(deforms)
        m["deforms"] = d[None] if d.ndim == 2 else d
    if abumps is not None:
        d = f32(abumps)
        m["abumps"] = d[None] if d.ndim == 2 else d
    if quadric is not None:
        m["quadric"] = [float(np.float32(q)) for q in quadric]
    return m


def random_abumps(n, seed, box=2.0, amp=0.6, spread=(0.15, 0.5)):
    """Anisotropic bumps (Eq. 6.1 with three spreads): rows (a, cx, cy, cz,
    sx, sy, sz).  Draw order: centres U[-box, box]^3 (n, 3), amplitudes
    U(-amp, amp) (n), spreads U(spread) (n, 3)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-box, box, size=(n, 3))
    a = rng.uniform(-amp, amp, size=n)
    s = rng.uniform(spread[0], spread[1], size=(n, 3))
    return f32(np.concatenate([a[:, None], c, s], axis=1))


def random_deforms(n, seed, box=3.0, amp=(0.4, 1.0), spread=(0.15, 0.35), kappa=(0.1, 0.4), rot=None):
    """Local deformations Phi_i(p) = p + f_i(p) V_i(p) with anisotropic
    Gaussians f_i: rows (a, cx, cy, cz, sx, sy, sz, vx, vy, vz) for a
    constant field V_i = v_i.  Draw order: centres U[-box, box]^3 (n, 3);
    spreads U(spread)^3 (n, 3); |a| U(amp) (n); sign of a (n); direction on
    the unit sphere (n, 3, normalised normals); kappa U(kappa) (n).  |v| is
    set so that |a| |v/s| exp(-1/2) = kappa: each Phi_i is a diffeomorphism
    with margin 1 - kappa.

    rot = (lo, hi) adds the rotation part of V_i(p) = v_i + w_i x (p - c_i):
    rows gain (wx, wy, wz), drawn after the above as an axis on the unit
    sphere (n, 3) and a share U(rot) (n).  Then |v| is set so that
    |a| exp(-1/2) |v| / s_min = kappa and |w| so that
    |a| |w| (2/e s_max / s_min + 1) = share: the Lipschitz bound of
    f_i V_i is kappa + share."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-box, box, size=(n, 3))
    s = rng.uniform(spread[0], spread[1], size=(n, 3))
    a = rng.uniform(amp[0], amp[1], size=n) * np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    k = rng.uniform(kappa[0], kappa[1], size=n)
    if rot is None:
        vn = k / (np.abs(a) * np.linalg.norm(u / s, axis=1) * np.exp(-0.5))
        v = u * vn[:, None]
        return f32(np.concatenate([a[:, None], c, s, v], axis=1))
    ax = rng.normal(size=(n, 3))
    ax /= np.linalg.norm(ax, axis=1, keepdims=True)
    share = rng.uniform(rot[0], rot[1], size=n)
    smin, smax = s.min(axis=1), s.max(axis=1)
    v = u * (k * smin / (np.abs(a) * np.exp(-0.5)))[:, None]
    w = ax * (share / (np.abs(a) * (2.0 / np.e * smax / smin + 1.0)))[:, None]
    return f32(np.concatenate([a[:, None], c, s, v, w], axis=1))


def scene(spheres=None, planes=None, tori=None):
    return dict(spheres=f32(spheres) if spheres is not None else empty4(),
                planes=f32(planes) if planes is not None else empty4(),
                tori=f32(tori) if tori is not None else empty8())


PLANE_Y_MINUS_1 = [[0.0, 1.0, 0.0, -1.0]]
TORUS_Z = [[0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 1.2, 0.15]]


def single_bump_64(width=64, height=64):
    bump = [[0.5, 0.0, 0.0, 0.0, 0.3]]
    return dict(name="single_bump_64",
                camera=camera(width, height),
                metric=metric(GRAPH_GAUSS, [bump]),
                scene=scene(spheres=[[0.0, 0.0, 2.0, 1.0]], planes=PLANE_Y_MINUS_1),
                rule=rule(RK4, h=0.01, max_steps=1000))


def bumps16_1080p(width=1920, height=1080, kind=RK4):
    # one pass (no compaction): measured fastest for this frame
    if kind == RK45:
        r = rule(RK45, h=0.005, max_steps=4000, t_max=20.0, rtol=1e-6, atol=1e-6,
                 h_min=1e-6, h_max=0.02, pass_steps=4000)
    else:
        r = rule(kind, h=0.005, max_steps=4000, t_max=20.0, pass_steps=4000)
    return dict(name="bumps16_1080p" + {RK4: "", RK45: "_rk45", EULER: "_euler"}[kind],
                camera=camera(width, height),
                metric=metric(GRAPH_GAUSS, random_bumps(16, seed=0)),
                scene=scene(spheres=random_spheres(64, seed=1),
                            planes=PLANE_Y_MINUS_1, tori=TORUS_Z),
                rule=r)


def twist_4k(width=3840, height=2160):
    return dict(name="twist_4k",
                camera=camera(width, height),
                metric=metric(PULLBACK_TWIST, twist_amp=0.4, twist_theta0=1.2),
                scene=scene(spheres=random_spheres(256, seed=1)),
                rule=rule(RK4, h=0.005, max_steps=4000, t_max=20.0))


def deform16_1080p(width=1920, height=1080):
    """The composition Phi_1 o ... o Phi_16 of local deformations (Sec. 6.2)
    in the bumps16 scene, RK4 as the headline workload."""
    base = bumps16_1080p(width, height)
    return dict(name="deform16_1080p", camera=base["camera"],
                metric=metric(PULLBACK_DEFORM, deforms=random_deforms(16, seed=5)),
                scene=base["scene"],
                rule=rule(RK4, h=0.005, max_steps=4000, t_max=20.0, pass_steps=4000))


def rdeform16_1080p(width=1920, height=1080):
    """Sixteen local deformations whose fields also rotate about an axis
    through their centres (V_i(p) = v_i + w_i x (p - c_i)), in the bumps16
    scene, RK4 as the headline workload."""
    base = bumps16_1080p(width, height)
    return dict(name="rdeform16_1080p", camera=base["camera"],
                metric=metric(PULLBACK_DEFORM, deforms=random_deforms(16, seed=6, kappa=(0.1, 0.3), rot=(0.2, 0.5))),
                scene=base["scene"],
                rule=rule(RK4, h=0.005, max_steps=4000, t_max=20.0, pass_steps=4000))


def abumps16_1080p(width=1920, height=1080):
    """The headline frame with anisotropic bumps (three spreads each)."""
    base = bumps16_1080p(width, height)
    return dict(name="abumps16_1080p", camera=base["camera"],
                metric=metric(GRAPH_ANISO, abumps=random_abumps(16, seed=0)),
                scene=base["scene"], rule=base["rule"])


def quadric_1080p(width=1920, height=1080):
    """The graph of the paper's quadratic f = x^2 + y^2 - z^2 (Sec. 5.1),
    camera inside the scene box looking +x (the paper's left view)."""
    base = bumps16_1080p(width, height)
    return dict(name="quadric_1080p", camera=camera(width, height, eye=(-1.0, 0.1, 0.2), forward=(1.0, 0.0, 0.0)),
                metric=metric(GRAPH_QUADRIC, quadric=(1.0, 1.0, -1.0)),
                scene=base["scene"], rule=base["rule"])


def adjoint_sets(n_sets=64, n_bumps=8):
    """Per set b: bumps from the bumps16 distributions with seed 2+b; the
    target set perturbs them with seed 1000+b: a + N(0,0.05), c + N(0,0.1),
    sigma * exp(N(0,0.1))."""
    theta = np.stack([random_bumps(n_bumps, seed=2 + b) for b in range(n_sets)])
    target = np.empty_like(theta)
    for b in range(n_sets):
        rng = np.random.default_rng(1000 + b)
        da = rng.normal(0.0, 0.05, size=n_bumps)
        dc = rng.normal(0.0, 0.1, size=(n_bumps, 3))
        ds = rng.normal(0.0, 0.1, size=n_bumps)
        t = theta[b].astype(np.float64)
        t[:, 0] += da
        t[:, 1:4] += dc
        t[:, 4] *= np.exp(ds)
        target[b] = t.astype(np.float32)
    return f32(theta), f32(target)


def adjoint_64x512(n_sets=64, width=512, height=512, n_bumps=8):
    theta, target = adjoint_sets(n_sets, n_bumps)
    base = single_bump_64(width, height)
    return dict(name="adjoint_64x512", camera=base["camera"],
                metric=metric(GRAPH_GAUSS, theta), target_bumps=target,
                scene=base["scene"],
                rule=rule(RK4, h=0.01, max_steps=2000), ckpt_every=100)


def surrogate_64_4k(width=3840, height=2160):
    base = bumps16_1080p(width, height)
    return dict(name="surrogate_64_4k", camera=base["camera"],
                metric=metric(GRAPH_GAUSS, random_bumps(64, seed=0)),
                scene=base["scene"],
                rule=rule(RK4, h=0.005, max_steps=4000, t_max=20.0, pass_steps=4000))


def surrogate_isolated_4k(width=3840, height=2160):
    bumps = isolated_bumps(64, seed=3)
    return dict(name="surrogate_isolated_4k", camera=camera(width, height),
                metric=metric(GRAPH_GAUSS, bumps),
                scene=scene(spheres=spheres_outside(64, seed=4, bumps=bumps),
                            planes=PLANE_Y_MINUS_1, tori=TORUS_Z),
                rule=rule(RK4, h=0.005, max_steps=4000, t_max=20.0, pass_steps=4000))


WORKLOADS = {
    "single_bump_64": single_bump_64,
    "bumps16_1080p": bumps16_1080p,
    "bumps16_1080p_rk45": lambda **kw: bumps16_1080p(kind=RK45, **kw),
    "bumps16_1080p_euler": lambda **kw: bumps16_1080p(kind=EULER, **kw),
    "euler_vs_rk4_1080p": lambda **kw: bumps16_1080p(kind=EULER, **kw),
    # batched multi-segment intersection against the per-step test, on the
    # 1080p frame (and on the 4K twist scene of 256 spheres)
    "batch_segments_1080p": lambda **kw: bumps16_1080p(**kw),
    "twist_4k": twist_4k,
    "deform16_1080p": deform16_1080p,
    "rdeform16_1080p": rdeform16_1080p,
    "illum_1080p": lambda **kw: dict(bumps16_1080p(**kw), name="illum_1080p",
                                     light=dict(pos=(2.5, 3.5, -3.0), h=0.01, tol=1e-4, max_iters=16,
                                                max_steps=4000)),
    "abumps16_1080p": abumps16_1080p,
    "quadric_1080p": quadric_1080p,
    "adjoint_64x512": adjoint_64x512,
    "surrogate_64_4k": surrogate_64_4k,
    "surrogate_isolated_4k": surrogate_isolated_4k,
}


def get(name, **kw):
    return WORKLOADS[name](**kw)


def with_size(wl, width, height):
    """Same workload on a smaller or larger image."""
    w = copy.deepcopy(wl)
    w["camera"]["width"] = int(width)
    w["camera"]["height"] = int(height)
    return w


def pixel_sample(width, height, n, seed):
    """Seeded sample of n distinct pixel indices (row-major j*W+i)."""
    rng = np.random.default_rng(seed)
    n = min(n, width * height)
    return np.sort(rng.choice(width * height, size=n, replace=False)).astype(np.int64)
