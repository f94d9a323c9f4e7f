"""Closed forms and independent references used to pin the oracle.

Nothing here calls the oracle or the GPU library.  These are the facts the
paper and the mathematics fix:

  * camera directions (the convention the paper leaves open, written out);
  * straight rays in flat space against spheres, planes (closed form) and a
    torus (roots of the quartic, numpy.roots);
  * the graph metric of Eq. 5.2 and the pullback metric of Eq. 5.6 built
    from f / phi by complex-step differentiation, and the generic
    Levi-Civita Christoffel symbols of Eq. 3.4 (read with the standard
    index order) from central differences of g;
  * the exact geodesics of one isotropic bump: the metric is spherically
    symmetric about the bump centre, so each geodesic is planar, conserves
    the Euclidean angular momentum L = (x - c) x y, and with r = b cosh(u)
    (b = |L| for unit g-speed) its polar angle and arc length are the 1-D
    integrals  dphi = sqrt(1 + F'(r)^2) / cosh(u) du,
               dt   = sqrt(1 + F'(r)^2) b cosh(u) du;
  * pullback geodesics are preimages of straight lines: phi(x(t)) =
    phi(p) + t J(p) v, and the z-twist of Sec. 5.2 has a closed-form inverse.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------- camera
def camera_dirs(cam, pixels):
    f = np.asarray(cam["forward"], np.float64)
    f = f / np.linalg.norm(f)
    up = np.asarray(cam["up"], np.float64)
    r = np.cross(up, f)
    r /= np.linalg.norm(r)
    u = np.cross(f, r)
    W, H = cam["width"], cam["height"]
    i = (pixels % W).astype(np.float64)
    j = (pixels // W).astype(np.float64)
    th = np.tan(0.5 * np.deg2rad(np.float64(np.float32(cam["vfov_deg"]))))
    su = (2.0 * (i + 0.5) / W - 1.0) * th * W / H
    sv = (1.0 - 2.0 * (j + 0.5) / H) * th
    d = su[:, None] * r + sv[:, None] * u + f
    return d / np.linalg.norm(d, axis=1, keepdims=True)


# ------------------------------------------------------- flat-space hits
def line_hits(eye, dirs, scene, t_max):
    """First intersection of x(t) = eye + t d (|d| = 1) with the scene.
    Returns (t, id); id -1 and t inf for a miss."""
    eye = np.asarray(eye, np.float64)
    n = dirs.shape[0]
    best_t = np.full(n, np.inf)
    best_id = np.full(n, -1, np.int64)
    oid = 0
    for s in np.asarray(scene["spheres"], np.float64).reshape(-1, 4):
        oc = eye - s[:3]
        b = dirs @ oc
        c = oc @ oc - s[3] ** 2
        disc = b * b - c
        with np.errstate(invalid="ignore"):
            t1 = -b - np.sqrt(disc)
        ok = (disc >= 0) & (t1 >= 0) & (t1 < best_t)
        best_t[ok] = t1[ok]
        best_id[ok] = oid
        oid += 1
    for p in np.asarray(scene["planes"], np.float64).reshape(-1, 4):
        dn = dirs @ p[:3]
        with np.errstate(divide="ignore", invalid="ignore"):
            t1 = (p[3] - eye @ p[:3]) / dn
        ok = np.isfinite(t1) & (t1 >= 0) & (t1 < best_t)
        best_t[ok] = t1[ok]
        best_id[ok] = oid
        oid += 1
    for tor in np.asarray(scene["tori"], np.float64).reshape(-1, 8):
        c, a, R, r = tor[:3], tor[3:6], tor[6], tor[7]
        # local frame with the axis as z
        e1 = np.cross(a, [1.0, 0, 0] if abs(a[0]) < 0.9 else [0, 1.0, 0])
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(a, e1)
        Bm = np.stack([e1, e2, a])
        o = Bm @ (eye - c)
        for q in range(n):
            d = Bm @ dirs[q]
            # (|p|^2 + R^2 - r^2)^2 = 4 R^2 (px^2 + py^2), p = o + t d
            bb = o @ d
            K = o @ o + R * R - r * r
            # (t^2 + 2 bb t + K)^2 - 4R^2 ((ox + t dx)^2 + (oy + t dy)^2)
            c4 = 1.0
            c3 = 4.0 * bb
            c2 = 4.0 * bb * bb + 2.0 * K - 4.0 * R * R * (d[0] ** 2 + d[1] ** 2)
            c1 = 4.0 * bb * K - 8.0 * R * R * (o[0] * d[0] + o[1] * d[1])
            c0 = K * K - 4.0 * R * R * (o[0] ** 2 + o[1] ** 2)
            roots = np.roots([c4, c3, c2, c1, c0])
            real = roots[np.abs(roots.imag) < 1e-9].real
            real = real[real >= 0]
            if real.size and real.min() < best_t[q]:
                best_t[q] = real.min()
                best_id[q] = oid
        oid += 1
    miss = best_t > t_max
    best_id[miss] = -1
    return best_t, best_id


# --------------------------------------------------- metrics, generically
def gauss_f(bumps, x):
    """f = sum a exp(-|x-c|^2/(2 s^2)) (Eq. 6.1, isotropic), complex-safe."""
    f = 0.0
    for a, cx, cy, cz, s in np.asarray(bumps, np.float64).reshape(-1, 5):
        d2 = (x[0] - cx) ** 2 + (x[1] - cy) ** 2 + (x[2] - cz) ** 2
        f = f + a * np.exp(-d2 / (2 * s * s))
    return f


def gauss_aniso_f(abumps, x):
    """f = sum a exp(-sum_i (x_i - c_i)^2 / (2 s_i^2)) (Eq. 6.1), complex-safe."""
    f = 0.0
    for a, cx, cy, cz, sx, sy, sz in np.asarray(abumps, np.float64).reshape(-1, 7):
        f = f + a * np.exp(-0.5 * (((x[0] - cx) / sx) ** 2 + ((x[1] - cy) / sy) ** 2 + ((x[2] - cz) / sz) ** 2))
    return f


def quadric_f(q, x):
    """f = q0 x^2 + q1 y^2 + q2 z^2 (the example of Sec. 5.1 is (1, 1, -1))."""
    return q[0] * x[0] ** 2 + q[1] * x[1] ** 2 + q[2] * x[2] ** 2


def twist_phi(x, amp=float(np.float32(0.4)), th0=float(np.float32(1.2))):
    """phi(x) = x + amp tanh|x| R_z(th0 exp(-|x|^2)) x (complex-safe)."""
    r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2]
    A = amp * np.tanh(np.sqrt(r2))
    th = th0 * np.exp(-r2)
    c, s = np.cos(th), np.sin(th)
    return np.array([x[0] + A * (c * x[0] - s * x[1]),
                     x[1] + A * (s * x[0] + c * x[1]),
                     x[2] + A * x[2]])


def ztwist_phi(x):
    """Sec. 5.2 example: Phi(x,y,z) = (cos z x - sin z y, sin z x + cos z y, z)."""
    c, s = np.cos(x[2]), np.sin(x[2])
    return np.array([c * x[0] - s * x[1], s * x[0] + c * x[1], x[2] + 0 * x[0]])


def ztwist_inv(X):
    c, s = np.cos(X[..., 2]), np.sin(X[..., 2])
    return np.stack([c * X[..., 0] + s * X[..., 1], -s * X[..., 0] + c * X[..., 1], X[..., 2]], axis=-1)


def deform_phi(x, deforms):
    """Phi = Phi_1 o ... o Phi_k, Phi_i(p) = p + f_i(p) V_i(p) (Sec. 6.2,
    Eqs. 6.1-6.2) with V_i(p) = v + w x (p - c); rows (a, cx, cy, cz, sx,
    sy, sz, vx, vy, vz[, wx, wy, wz]), Phi_k applied first (complex-safe)."""
    d = np.asarray(deforms, np.float64)
    d = d.reshape(-1, d.shape[-1])
    if d.shape[1] == 10:
        d = np.concatenate([d, np.zeros((d.shape[0], 3))], axis=1)
    q = [x[0], x[1], x[2]]
    for a, cx, cy, cz, sx, sy, sz, vx, vy, vz, wx, wy, wz in d[::-1]:
        dx, dy, dz = q[0] - cx, q[1] - cy, q[2] - cz
        f = a * np.exp(-0.5 * ((dx / sx) ** 2 + (dy / sy) ** 2 + (dz / sz) ** 2))
        V = (vx + (wy * dz - wz * dy), vy + (wz * dx - wx * dz), vz + (wx * dy - wy * dx))
        q = [q[0] + f * V[0], q[1] + f * V[1], q[2] + f * V[2]]
    return np.array(q)


def cs_grad(fun, x, h=1e-30):
    """Complex-step gradient of a scalar function (exact to rounding)."""
    g = np.zeros(3)
    for i in range(3):
        xc = np.array(x, dtype=np.complex128)
        xc[i] += 1j * h
        g[i] = np.imag(fun(xc)) / h
    return g


def cs_jac(fun, x, h=1e-30):
    """Complex-step Jacobian J[s, i] = d fun_s / d x_i."""
    J = np.zeros((3, 3))
    for i in range(3):
        xc = np.array(x, dtype=np.complex128)
        xc[i] += 1j * h
        J[:, i] = np.imag(fun(xc)) / h
    return J


def graph_g(bumps, x, f=None):
    """Eq. 5.2: g = I + grad f grad f^T (f: the isotropic bump sum unless given)."""
    gr = cs_grad(f if f is not None else (lambda z: gauss_f(bumps, z)), x)
    return np.eye(3) + np.outer(gr, gr)


def pullback_g(phi, x):
    """Eq. 5.6: g = J^T J."""
    J = cs_jac(phi, x)
    return J.T @ J


def generic_accel(gfun, x, y, h=1e-5):
    """-Gamma^m_ij y_i y_j with Gamma^m_ij = 1/2 g^{mk}(d_i g_jk + d_j g_ik -
    d_k g_ij) (Eq. 3.4 in the standard index order), dg by central
    differences of g."""
    dg = np.zeros((3, 3, 3))  # dg[k] = d g / d x_k
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        dg[k] = (gfun(x + e) - gfun(x - e)) / (2 * h)
    ginv = np.linalg.inv(gfun(x))
    gam = np.zeros((3, 3, 3))
    for m in range(3):
        for i in range(3):
            for j in range(3):
                s = 0.0
                for k in range(3):
                    s += ginv[m, k] * (dg[i][j, k] + dg[j][i, k] - dg[k][i, j])
                gam[m, i, j] = 0.5 * s
    return -np.einsum("mij,i,j->m", gam, y, y)


# ------------------------------------------------ exact single-bump rays
_GL_X, _GL_W = np.polynomial.legendre.leggauss(20)


def _gl(fun, a, b):
    """20-point Gauss-Legendre on each panel [a_k, b_k] (vectorised)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    mid = 0.5 * (a + b)
    hw = 0.5 * (b - a)
    u = mid[..., None] + hw[..., None] * _GL_X
    return hw * (fun(u) @ _GL_W)


class SingleBumpRay:
    """Exact continuous geodesic of g = I + grad f grad f^T for one bump
    f = amp exp(-|x-c|^2/(2 sig^2)), started at x0 with unit g-speed
    Euclidean-direction d, where grad f(x0) is negligible (x0 far away)."""

    def __init__(self, amp, centre, sig, x0, d, du=0.004):
        self.amp, self.sig = float(amp), float(sig)
        self.c = np.asarray(centre, np.float64)
        x0 = np.asarray(x0, np.float64) - self.c
        d = np.asarray(d, np.float64)
        d = d / np.linalg.norm(d)
        L = np.cross(x0, d)
        self.b = np.linalg.norm(L)
        self.r0 = np.linalg.norm(x0)
        self.e1 = x0 / self.r0
        e2 = d - (d @ self.e1) * self.e1
        self.e2 = e2 / np.linalg.norm(e2)
        assert d @ x0 < 0, "ray must start inbound"
        self.u0 = np.arccosh(self.r0 / self.b)
        # path parameter tau in [-u0, +umax]; r = b cosh(tau)
        self.du = du

    def Fp(self, r):
        return -(r / self.sig ** 2) * self.amp * np.exp(-r * r / (2 * self.sig ** 2))

    def _dphi(self, u):
        r = self.b * np.cosh(u)
        return np.sqrt(1.0 + self.Fp(r) ** 2) / np.cosh(u)

    def _dt(self, u):
        r = self.b * np.cosh(u)
        return np.sqrt(1.0 + self.Fp(r) ** 2) * r

    def tabulate(self, t_max):
        """phi(tau) and t(tau) on a grid tau = -u0 .. umax, where |tau| = u
        and tau < 0 is the inbound branch, tau > 0 the outbound one."""
        tau_in = np.linspace(-self.u0, 0.0, int(np.ceil(self.u0 / self.du)) + 1)
        umax = max(self.u0, 1.0)
        while True:
            tau_out = np.linspace(0.0, umax, int(np.ceil(umax / self.du)) + 1)[1:]
            tau = np.concatenate([tau_in, tau_out])
            t = self._t_of(tau)
            if t[-1] > t_max + 1.0:
                break
            umax *= 1.5
        u = np.abs(tau)
        lo, hi = np.minimum(u[:-1], u[1:]), np.maximum(u[:-1], u[1:])
        self.tau = tau
        self.phi = np.concatenate([[0.0], np.cumsum(_gl(self._dphi, lo, hi))])
        self.t = t
        return self

    def _t_of(self, tau):
        u = np.abs(np.asarray(tau))
        lo, hi = np.minimum(u[:-1], u[1:]), np.maximum(u[:-1], u[1:])
        return np.concatenate([[0.0], np.cumsum(_gl(self._dt, lo, hi))])

    def at(self, tau):
        """phi, t, position at a single tau (interpolation-free: integrates
        from the nearest grid node)."""
        k = int(np.clip(np.searchsorted(self.tau, tau) - 1, 0, len(self.tau) - 2))
        a = self.tau[k]
        lo, hi = sorted([abs(a), abs(tau)])
        if a < 0 <= tau:
            dphi = _gl(self._dphi, 0.0, abs(a)) + _gl(self._dphi, 0.0, abs(tau))
            dt = _gl(self._dt, 0.0, abs(a)) + _gl(self._dt, 0.0, abs(tau))
        else:
            dphi = _gl(self._dphi, lo, hi)
            dt = _gl(self._dt, lo, hi)
        phi = self.phi[k] + float(dphi)
        t = self.t[k] + float(dt)
        r = self.b * np.cosh(tau)
        x = self.c + r * (np.cos(phi) * self.e1 + np.sin(phi) * self.e2)
        return phi, t, x

    def first_hit(self, objects, t_max):
        """objects: list of callables F(x) (>0 outside).  Returns (t, id, x)
        of the first sign change along the path with t <= t_max."""
        xs = np.array([self._pos_node(k) for k in range(len(self.tau))])
        best = (np.inf, -1, None)
        from scipy.optimize import brentq
        for oid, F in enumerate(objects):
            vals = np.array([F(x) for x in xs])
            pos = vals > 0
            ch = np.nonzero(pos[:-1] != pos[1:])[0]
            if ch.size == 0:
                continue
            k = ch[0]
            fun = lambda tau: F(self.at(tau)[2])
            tau_s = brentq(fun, self.tau[k], self.tau[k + 1], xtol=1e-15, rtol=1e-15, maxiter=200)
            _, t, x = self.at(tau_s)
            if t < best[0] and t <= t_max:
                best = (t, oid, x)
        return best

    def _pos_node(self, k):
        r = self.b * np.cosh(self.tau[k])
        phi = self.phi[k]
        return self.c + r * (np.cos(phi) * self.e1 + np.sin(phi) * self.e2)


def crossing_exact(kappa, c):
    """Exact crossing of the support sphere (radius 3) of the canonical bump
    F(r) = kappa exp(-r^2/2) (sigma = 1), entered at (3, 0, 0) with Euclidean
    direction (-c, s, 0), s = sqrt(1 - c^2).  Returns the swept polar angle of
    the exit point and the g-length of the arc inside the sphere.

    Rotation invariance keeps J = |x x x'| constant and g(x', x') = 1 gives
    r'^2 (1 + F'^2) + J^2 / r^2 = 1; with r = J cosh(u) the swept angle is
    2 int_0^u1 sqrt(1 + F'^2) / cosh(u) du and the length
    2 int_0^u1 r sqrt(1 + F'^2) du, with J cosh(u1) = 3.  At the entry the
    g-unit speed has Euclidean size v = 1 / sqrt(1 + F'(3)^2 c^2), so
    J = 3 v s."""
    kappa = abs(float(kappa))
    c = float(c)
    s = np.sqrt(max(0.0, 1.0 - c * c))

    def Fp(r):
        return -kappa * r * np.exp(-0.5 * r * r)

    if s < 1e-12:      # head-on: straight through the centre
        edges = np.linspace(0.0, 3.0, 257)
        half = float(np.sum(_gl(lambda r: np.sqrt(1.0 + Fp(r) ** 2), edges[:-1], edges[1:])))
        return np.pi, 2.0 * half
    v = 1.0 / np.sqrt(1.0 + (Fp(3.0) * c) ** 2)
    J = 3.0 * v * s
    u1 = np.arccosh(3.0 / J) if J < 3.0 else 0.0
    if u1 == 0.0:
        return 0.0, 0.0
    edges = np.linspace(0.0, u1, 513)
    dphi = _gl(lambda u: np.sqrt(1.0 + Fp(J * np.cosh(u)) ** 2) / np.cosh(u), edges[:-1], edges[1:])
    dt = _gl(lambda u: J * np.cosh(u) * np.sqrt(1.0 + Fp(J * np.cosh(u)) ** 2), edges[:-1], edges[1:])
    return 2.0 * float(np.sum(dphi)), 2.0 * float(np.sum(dt))
