"""FP64 CPU oracle of the Riemannian ray tracer -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does, and
the oracle imports nothing from it: the two share only the seeded inputs of
``workloads.py``.

The C source ``rt_oracle.c`` holds the arithmetic (double precision, scalar,
no culling).  This module builds it with gcc and marshals arguments.

Pinning status (what fixes each function to something other than itself):
  camera + chord test + bisection   flat-space analytic hits (sphere, plane,
                                    torus quartic)          -- pinned
  graph acceleration (Eq. 5.4)      generic Christoffel symbols (Eq. 3.4)
  (isotropic and anisotropic        from finite differences of g; det g
  bumps, the Sec. 5.1 quadratic)    = 1 + |grad f|^2; f -> -f invariance;
                                    single-bump quadrature   -- pinned
  pullback acceleration (Eq. 5.8)   generic Christoffel symbols; geodesics are
                                    preimages of straight lines
                                    (closed form for the z-twist) -- pinned;
                                    for the composed local deformations
                                    (Sec. 6.2) also the map and its Jacobian
                                    against an independent evaluation and
                                    finite differences        -- pinned
  RK4 / DP5 / Euler                 step-convergence orders, g(y,y)
                                    conservation, DP5 order conditions,
                                    quadrature hits           -- pinned
  multi-bump trajectories           no closed form: invariants and agreement
                                    of independent integrators only
  FD gradient (fd_gradient)         exact zeros for a = 0 and for the centre
                                    and spread of a zero-amplitude bump,
                                    bitwise parity under a -> -a, and the
                                    single-bump quadrature derivative
                                    (tests/test_oracle_fd.py) -- pinned
  twist at its centre               the hyper-dual square root divides by
                                    |x|: an evaluation exactly at x = 0
                                    gives NaN (the ray would fail, id -2);
                                    rays aimed at the centre stay finite and
                                    on their line preimage to a step's jump
  failed rays (id -2)               a failed ray reports the state of the
                                    same run stopped by max_steps; rays away
                                    from the failure region equal a run that
                                    never rejects               -- pinned
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rt_oracle.c")
_LIB = os.path.join(_HERE, "_rt_oracle.so")

EUCLID, GRAPH_GAUSS, PULLBACK_TWIST, PULLBACK_ZTWIST, PULLBACK_DEFORM, GRAPH_ANISO, GRAPH_QUADRIC = 0, 1, 2, 3, 4, 5, 6
RK4, RK45, EULER = 0, 1, 2


def build(force=True):
    """Compile the oracle with gcc (plain C, OpenMP over pixels)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC",
                           "-shared", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class _Metric(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_bumps", C.c_int), ("bumps", C.POINTER(C.c_double)),
                ("twist_amp", C.c_double), ("twist_theta0", C.c_double),
                ("n_deforms", C.c_int), ("deforms", C.POINTER(C.c_double)),
                ("n_abumps", C.c_int), ("abumps", C.POINTER(C.c_double)), ("quadric", C.c_double * 3)]


class _Scene(C.Structure):
    _fields_ = [("n_spheres", C.c_int), ("spheres", C.POINTER(C.c_double)),
                ("n_planes", C.c_int), ("planes", C.POINTER(C.c_double)),
                ("n_tori", C.c_int), ("tori", C.POINTER(C.c_double))]


class _Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("fwd", C.c_double * 3), ("up", C.c_double * 3),
                ("vfov_deg", C.c_double), ("width", C.c_int), ("height", C.c_int)]


class _Rule(C.Structure):
    _fields_ = [("kind", C.c_int), ("h", C.c_double), ("rtol", C.c_double),
                ("atol", C.c_double), ("h_min", C.c_double), ("h_max", C.c_double),
                ("t_max", C.c_double), ("max_steps", C.c_int), ("bisect_iters", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.orc_camera_dir.argtypes = [C.POINTER(_Camera), C.c_int, C.c_int, dp]
        L.orc_accel.argtypes = [C.POINTER(_Metric), dp, dp, dp]
        L.orc_accel.restype = C.c_int
        L.orc_metric_tensor.argtypes = [C.POINTER(_Metric), dp, dp]
        L.orc_step.argtypes = [C.POINTER(_Metric), C.c_int, dp, C.c_double, dp, dp]
        L.orc_step.restype = C.c_int
        L.orc_trace_pixels.argtypes = [C.POINTER(_Metric), C.POINTER(_Scene), C.POINTER(_Camera),
                                       C.POINTER(_Rule), C.c_int64, C.POINTER(C.c_int64), dp,
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32), C.c_int]
        L.orc_shoot.argtypes = [C.POINTER(_Metric), dp, C.c_double, C.c_double, dp]
        L.orc_shoot.restype = C.c_int
        L.orc_geodesic_clear.argtypes = [C.POINTER(_Metric), C.POINTER(_Scene), dp, C.c_double, C.c_double,
                                         C.c_double]
        L.orc_geodesic_clear.restype = C.c_int
        L.orc_trajectory.argtypes = [C.POINTER(_Metric), C.POINTER(_Rule), dp, C.c_int, dp]
        L.orc_trajectory.restype = C.c_int
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Oracle:
    """Holds FP64 copies of one metric (one parameter set) and one scene."""

    def __init__(self, metric, scene, set_index=0, bumps64=None):
        """bumps64: optional float64 [n_bumps, 5] parameters used as given
        (finite-difference perturbations must not be rounded to float32)."""
        if bumps64 is not None:
            b = np.asarray(bumps64, np.float64)
        else:
            b = np.asarray(metric["bumps"], np.float32)
            if b.ndim == 3:
                b = b[set_index]
            b = b.astype(np.float64)
        self._bumps = np.ascontiguousarray(b.reshape(-1, 5))
        # deformation rows: a, c, spreads, v and the rotation w of the field
        # V(p) = v + w x (p - c) (w = 0 when a row has 10 values)
        dfm = metric.get("deforms")
        if dfm is None:
            dfm = np.zeros((0, 13))
        dfm = np.asarray(dfm, np.float32)
        if dfm.ndim == 3:
            dfm = dfm[set_index]
        if dfm.shape[-1] == 10:
            dfm = np.concatenate([dfm, np.zeros(dfm.shape[:-1] + (3,), np.float32)], axis=-1)
        self._deforms = np.ascontiguousarray(dfm.astype(np.float64).reshape(-1, 13))
        ab = metric.get("abumps")
        ab = np.zeros((0, 7)) if ab is None else np.asarray(ab, np.float32)
        if ab.ndim == 3:
            ab = ab[set_index]
        self._abumps = np.ascontiguousarray(ab.astype(np.float64).reshape(-1, 7))
        q = [float(np.float32(x)) for x in metric.get("quadric", (0.0, 0.0, 0.0))]
        self.m = _Metric(int(metric["kind"]), int(self._bumps.shape[0]), _dptr(self._bumps),
                         float(metric.get("twist_amp", 0.4)), float(metric.get("twist_theta0", 1.2)),
                         int(self._deforms.shape[0]), _dptr(self._deforms),
                         int(self._abumps.shape[0]), _dptr(self._abumps), (C.c_double * 3)(*q))
        self._sp = np.ascontiguousarray(np.asarray(scene["spheres"], np.float32).astype(np.float64).reshape(-1, 4))
        self._pl = np.ascontiguousarray(np.asarray(scene["planes"], np.float32).astype(np.float64).reshape(-1, 4))
        self._to = np.ascontiguousarray(np.asarray(scene["tori"], np.float32).astype(np.float64).reshape(-1, 8))
        self.s = _Scene(self._sp.shape[0], _dptr(self._sp), self._pl.shape[0], _dptr(self._pl),
                        self._to.shape[0], _dptr(self._to))

    # ---- pointwise quantities
    def accel(self, x, y):
        x = np.ascontiguousarray(x, np.float64)
        y = np.ascontiguousarray(y, np.float64)
        a = np.zeros(3)
        ok = lib().orc_accel(C.byref(self.m), _dptr(x), _dptr(y), _dptr(a))
        return a, bool(ok)

    def metric_tensor(self, x):
        x = np.ascontiguousarray(x, np.float64)
        g = np.zeros(9)
        lib().orc_metric_tensor(C.byref(self.m), _dptr(x), _dptr(g))
        return g.reshape(3, 3)

    def step(self, kind, z, h):
        z = np.ascontiguousarray(z, np.float64)
        o = np.zeros(6)
        e = np.zeros(6)
        ok = lib().orc_step(C.byref(self.m), int(kind), _dptr(z), float(h), _dptr(o), _dptr(e))
        return o, e, bool(ok)

    def trajectory(self, rule, z0, n_steps):
        z0 = np.ascontiguousarray(z0, np.float64)
        out = np.zeros((n_steps + 1, 6))
        r = _rule(rule)
        lib().orc_trajectory(C.byref(self.m), C.byref(r), _dptr(z0), int(n_steps), _dptr(out))
        return out

    # ---- direct illumination
    def shoot(self, q, v, T, h):
        """End state (x, y) of the geodesic from (q, v) over arc length T
        (RK4, step h, last step shortened)."""
        z0 = np.ascontiguousarray(np.concatenate([q, v]), np.float64)
        out = np.zeros(6)
        ok = lib().orc_shoot(C.byref(self.m), _dptr(z0), float(T), float(h), _dptr(out))
        return out, bool(ok)

    def geodesic_clear(self, q, v, T, h, skip=1e-3):
        """True when that geodesic crosses no object between skip and T."""
        z0 = np.ascontiguousarray(np.concatenate([q, v]), np.float64)
        return bool(lib().orc_geodesic_clear(C.byref(self.m), C.byref(self.s), _dptr(z0), float(T), float(h),
                                             float(skip)))

    # ---- tracing
    def trace(self, camera, rule, pixels=None, nthreads=0):
        """Trace the given pixel indices (row-major j*W+i; all if None).
        Returns dict hit[n,3], t[n], dir[n,3], id[n], steps[n], rejected[n]."""
        W, H = camera["width"], camera["height"]
        if pixels is None:
            pixels = np.arange(W * H, dtype=np.int64)
        pixels = np.ascontiguousarray(pixels, np.int64)
        n = pixels.shape[0]
        out = np.zeros((n, 8))
        ids = np.zeros(n, np.int32)
        steps = np.zeros(n, np.int32)
        rej = np.zeros(n, np.int32)
        cam = camera_struct(camera)
        r = _rule(rule)
        i32 = C.POINTER(C.c_int32)
        lib().orc_trace_pixels(C.byref(self.m), C.byref(self.s), C.byref(cam), C.byref(r), n,
                               pixels.ctypes.data_as(C.POINTER(C.c_int64)), _dptr(out),
                               ids.ctypes.data_as(i32), steps.ctypes.data_as(i32),
                               rej.ctypes.data_as(i32), int(nthreads))
        return dict(hit=out[:, 0:3].copy(), t=out[:, 3].copy(), dir=out[:, 4:7].copy(),
                    id=ids, steps=steps, rejected=rej)

    def camera_dir(self, camera, i, j):
        d = np.zeros(3)
        cam = camera_struct(camera)
        lib().orc_camera_dir(C.byref(cam), int(i), int(j), _dptr(d))
        return d


def camera_struct(c):
    f = lambda v: (C.c_double * 3)(*[float(np.float32(x)) for x in v])
    return _Camera(f(c["eye"]), f(c["forward"]), f(c["up"]), float(np.float32(c["vfov_deg"])),
                   int(c["width"]), int(c["height"]))


def _rule(r):
    g = lambda k: float(np.float32(r[k]))
    return _Rule(int(r["kind"]), g("h"), g("rtol"), g("atol"), g("h_min"), g("h_max"),
                 g("t_max"), int(r["max_steps"]), 60)


# --------------------------------------------------------------------------
# Differentiation reference: the masked L2 loss between a hit map and a
# target map, and its central finite-difference gradient with respect to
# every bump parameter (a, cx, cy, cz, sigma).  This is the definition of
# the derivative the GPU adjoint must reproduce; it uses nothing but the
# traced hit points above.
def l2_loss(hit, target_hit, mask):
    """L = sum over masked pixels of |hit - target|^2 (FP64)."""
    d = (np.asarray(hit, np.float64) - np.asarray(target_hit, np.float64))[mask]
    return float((d * d).sum())


def fd_gradient(metric, scene, camera, rule, pixels, target_hit, target_id, set_index=0, eps=1e-4,
                nthreads=0):
    """Central differences (L(theta + eps e_i) - L(theta - eps e_i)) / (2 eps)
    over all n_bumps x 5 parameters of one set.

    Pixels count only where the traced id equals the target id at theta and
    at every perturbed theta (a common mask: FD across a change of the hit
    object is meaningless).  Returns (grad [n_bumps, 5], loss at theta,
    mask)."""
    b0 = np.asarray(metric["bumps"], np.float32)
    if b0.ndim == 3:
        b0 = b0[set_index]
    base = b0.astype(np.float64)
    nb = base.shape[0]

    def run(bumps64):
        return Oracle(metric, scene, bumps64=bumps64).trace(camera, rule, pixels, nthreads=nthreads)

    r0 = run(base)
    target_id = np.asarray(target_id)
    mask = (r0["id"] == target_id) & (r0["id"] >= 0)
    plus, minus = {}, {}
    for i in range(nb):
        for j in range(5):
            bp = base.copy()
            bp[i, j] += eps
            bm = base.copy()
            bm[i, j] -= eps
            plus[i, j] = run(bp)
            minus[i, j] = run(bm)
            mask &= (plus[i, j]["id"] == r0["id"]) & (minus[i, j]["id"] == r0["id"])
    grad = np.zeros((nb, 5))
    for (i, j), rp in plus.items():
        grad[i, j] = (l2_loss(rp["hit"], target_hit, mask) - l2_loss(minus[i, j]["hit"], target_hit, mask)) / (2 * eps)
    return grad, l2_loss(r0["hit"], target_hit, mask), mask
