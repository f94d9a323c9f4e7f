/* FP64 CPU oracle of the Riemannian ray tracer -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code with the GPU path.  Everything is
 * double precision, scalar, with no culling and no reordering of the
 * method's arithmetic beyond what the paper's formulas state.
 *
 * What it computes, following the paper (Novello, da Silva, Velho 2020):
 *   - the observer field of directions at p and the exponential map exp_p
 *     (Sec. 3.4 and Sec. 4, "Riemannian shading"): one geodesic per pixel
 *     direction, launched with unit speed in the metric g at p;
 *   - the geodesic flow x' = y, y' = -Gamma(y, y) (Eq. 3.3);
 *   - Gamma for graph metrics (Sec. 5.1, Eqs. 5.2-5.4) with f a sum of
 *     isotropic Gaussians (Eq. 6.1 and "Summing functions", Sec. 6.2);
 *   - Gamma for diffeomorphism pullbacks (Sec. 5.2, Thm 5.1 / Eq. 5.7,
 *     flow Eq. 5.8 read with index k on the left and right), the Jacobian
 *     and second derivatives of the map taken with hyper-dual numbers;
 *     the maps include compositions of local deformations (Sec. 6.2,
 *     Eqs. 6.1 and 6.2), differentiated as one map;
 *   - ray marching: the integration polygon, each segment tested against
 *     the scene (Sec. 4.1).  Integrators: the paper's explicit Euler
 *     (Eq. 4.1), classical RK4 and Dormand-Prince 5(4) (the Runge-Kutta
 *     alternative named at the end of Sec. 4.1);
 *   - the hit refined by bisection on the step fraction of the last step.
 */
#include "rt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- vectors */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static void normalize3(double *a)
{
    double n = sqrt(dot3(a, a));
    a[0] /= n; a[1] /= n; a[2] /= n;
}

/* ------------------------------------------------------------------ camera
 * The paper leaves the camera model open (Sec. 4 only says each direction of
 * the observer field V of S^2_p gets a ray).  Reading: pinhole, vertical
 * field of view, pixel centres, column i to the right, row 0 at the top,
 * right = up x forward. */
void orc_camera_dir(const orc_camera *cam, int i, int j, double d[3])
{
    double f[3] = {cam->fwd[0], cam->fwd[1], cam->fwd[2]};
    normalize3(f);
    double r[3];
    cross3(cam->up, f, r);
    normalize3(r);
    double u[3];
    cross3(f, r, u);
    double th = tan(0.5 * cam->vfov_deg * M_PI / 180.0);
    double W = cam->width, H = cam->height;
    double su = (2.0 * (i + 0.5) / W - 1.0) * th * W / H;
    double sv = (1.0 - 2.0 * (j + 0.5) / H) * th;
    for (int k = 0; k < 3; k++) d[k] = su * r[k] + sv * u[k] + f[k];
    normalize3(d);
}

/* ------------------------------------------------------------ graph metric
 * f = sum_b a_b exp(-|x - c_b|^2 / (2 sigma_b^2))  (Eq. 6.1, isotropic;
 * the sum follows "Summing functions": derivatives of f are sums of the
 * derivatives of the f_b).  Returns grad f and the Hessian f_ij. */
static void graph_derivs(const orc_metric *m, const double x[3], double grad[3], double hess[9])
{
    memset(grad, 0, 3 * sizeof(double));
    memset(hess, 0, 9 * sizeof(double));
    if (m->kind == ORC_GRAPH_QUADRIC) {
        /* f = sum_i q_i x_i^2: f_i = 2 q_i x_i, f_ij = 2 q_i delta_ij (Sec. 5.1 example) */
        for (int i = 0; i < 3; i++) {
            grad[i] = 2.0 * m->quadric[i] * x[i];
            hess[3 * i + i] = 2.0 * m->quadric[i];
        }
        return;
    }
    if (m->kind == ORC_GRAPH_ANISO) {
        /* f = sum_b a_b exp(-sum_i (x_i - c_i)^2 / (2 s_i^2)) (Eq. 6.1, three spreads):
         * f_i = -(d_i / s_i^2) f_b, f_ij = (d_i d_j / (s_i^2 s_j^2) - delta_ij / s_i^2) f_b */
        for (int b = 0; b < m->n_abumps; b++) {
            const double *p = m->abumps + 7 * b;
            double d[3] = {x[0] - p[1], x[1] - p[2], x[2] - p[3]};
            double s2[3] = {p[4] * p[4], p[5] * p[5], p[6] * p[6]};
            double e = 0.0;
            for (int i = 0; i < 3; i++) e += d[i] * d[i] / s2[i];
            double fb = p[0] * exp(-0.5 * e);
            for (int i = 0; i < 3; i++) {
                grad[i] += -d[i] / s2[i] * fb;
                for (int j = 0; j < 3; j++)
                    hess[3 * i + j] += (d[i] * d[j] / (s2[i] * s2[j]) - (i == j ? 1.0 / s2[i] : 0.0)) * fb;
            }
        }
        return;
    }
    for (int b = 0; b < m->n_bumps; b++) {
        const double *p = m->bumps + 5 * b;
        double a = p[0], sg = p[4];
        double d[3] = {x[0] - p[1], x[1] - p[2], x[2] - p[3]};
        double s2 = sg * sg;
        double fb = a * exp(-dot3(d, d) / (2.0 * s2));
        for (int i = 0; i < 3; i++) {
            grad[i] += -d[i] / s2 * fb;
            for (int j = 0; j < 3; j++)
                hess[3 * i + j] += (d[i] * d[j] / (s2 * s2) - (i == j ? 1.0 / s2 : 0.0)) * fb;
        }
    }
}

/* Eq. 5.4: y'_k = - sum_ij f_k f_ij y_i y_j / (1 + |grad f|^2). */
static void graph_accel(const orc_metric *m, const double x[3], const double y[3], double a[3])
{
    double g[3], H[9];
    graph_derivs(m, x, g, H);
    double den = 1.0 + dot3(g, g);
    for (int k = 0; k < 3; k++) {
        double s = 0.0;
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) s += g[k] * H[3 * i + j] * y[i] * y[j];
        a[k] = -s / den;
    }
}

/* ------------------------------------------------------- hyper-dual numbers
 * v + e1 E1 + e2 E2 + e12 E1E2 with E1^2 = E2^2 = 0.  Evaluating a map at
 * p + E1 u + E2 w yields its value, the directional derivatives along u and
 * w, and the mixed second derivative D^2(u, w), all exact to rounding. */
typedef struct { double v, e1, e2, e12; } hd;
static hd hd_c(double v) { hd r = {v, 0, 0, 0}; return r; }
static hd hd_add(hd a, hd b) { hd r = {a.v + b.v, a.e1 + b.e1, a.e2 + b.e2, a.e12 + b.e12}; return r; }
static hd hd_sub(hd a, hd b) { hd r = {a.v - b.v, a.e1 - b.e1, a.e2 - b.e2, a.e12 - b.e12}; return r; }
static hd hd_mul(hd a, hd b)
{
    hd r = {a.v * b.v, a.v * b.e1 + a.e1 * b.v, a.v * b.e2 + a.e2 * b.v,
            a.v * b.e12 + a.e1 * b.e2 + a.e2 * b.e1 + a.e12 * b.v};
    return r;
}
static hd hd_scale(hd a, double s) { hd r = {a.v * s, a.e1 * s, a.e2 * s, a.e12 * s}; return r; }
/* chain rule for a scalar function with value f0, first and second derivative f1, f2 */
static hd hd_fun(hd a, double f0, double f1, double f2)
{
    hd r = {f0, f1 * a.e1, f1 * a.e2, f1 * a.e12 + f2 * a.e1 * a.e2};
    return r;
}
static hd hd_exp(hd a) { double e = exp(a.v); return hd_fun(a, e, e, e); }
static hd hd_sin(hd a) { return hd_fun(a, sin(a.v), cos(a.v), -sin(a.v)); }
static hd hd_cos(hd a) { return hd_fun(a, cos(a.v), -sin(a.v), -cos(a.v)); }
static hd hd_tanh(hd a)
{
    double t = tanh(a.v);
    double s = 1.0 - t * t;
    return hd_fun(a, t, s, -2.0 * t * s);
}
static hd hd_sqrt(hd a)
{
    double s = sqrt(a.v);
    return hd_fun(a, s, 0.5 / s, -0.25 / (s * a.v));
}

/* The diffeomorphisms, written from their definitions.
 * twist (a radial twist about z):  phi(x) = x + amp*tanh|x| * R_z(theta) x,
 *                                   theta = theta0 * exp(-|x|^2);
 * z-twist (Sec. 5.2 example):      Phi(x,y,z) = (cos z x - sin z y,
 *                                                sin z x + cos z y, z). */
static void phi_hd(const orc_metric *m, const hd x[3], hd out[3])
{
    if (m->kind == ORC_PULLBACK_DEFORM) {
        /* Phi = Phi_1 o Phi_2 o ... o Phi_k (Sec. 6.2): Phi_k acts first.
         * Phi_i(p) = p + f_i(p) V_i(p) (Eq. 6.2), f_i the Gaussian of
         * Eq. 6.1 with amplitude a, centre c and spreads sx, sy, sz, and the
         * field V_i(p) = v + w x (p - c). */
        hd q[3] = {x[0], x[1], x[2]};
        for (int i = m->n_deforms - 1; i >= 0; i--) {
            const double *P = m->deforms + 13 * i;
            hd e = hd_c(0.0), d[3];
            for (int k = 0; k < 3; k++) {
                d[k] = hd_sub(q[k], hd_c(P[1 + k]));
                e = hd_add(e, hd_scale(hd_mul(d[k], d[k]), -1.0 / (2.0 * P[4 + k] * P[4 + k])));
            }
            hd f = hd_scale(hd_exp(e), P[0]);
            const double *w = P + 10;
            hd V[3] = {hd_add(hd_c(P[7]), hd_sub(hd_scale(d[2], w[1]), hd_scale(d[1], w[2]))),
                       hd_add(hd_c(P[8]), hd_sub(hd_scale(d[0], w[2]), hd_scale(d[2], w[0]))),
                       hd_add(hd_c(P[9]), hd_sub(hd_scale(d[1], w[0]), hd_scale(d[0], w[1])))};
            for (int k = 0; k < 3; k++) q[k] = hd_add(q[k], hd_mul(f, V[k]));
        }
        for (int k = 0; k < 3; k++) out[k] = q[k];
        return;
    }
    if (m->kind == ORC_PULLBACK_ZTWIST) {
        hd c = hd_cos(x[2]), s = hd_sin(x[2]);
        out[0] = hd_sub(hd_mul(c, x[0]), hd_mul(s, x[1]));
        out[1] = hd_add(hd_mul(s, x[0]), hd_mul(c, x[1]));
        out[2] = x[2];
        return;
    }
    hd r2 = hd_add(hd_add(hd_mul(x[0], x[0]), hd_mul(x[1], x[1])), hd_mul(x[2], x[2]));
    hd rho = hd_sqrt(r2);
    hd A = hd_scale(hd_tanh(rho), m->twist_amp);
    hd th = hd_scale(hd_exp(hd_scale(r2, -1.0)), m->twist_theta0);
    hd c = hd_cos(th), s = hd_sin(th);
    hd rx = hd_sub(hd_mul(c, x[0]), hd_mul(s, x[1]));
    hd ry = hd_add(hd_mul(s, x[0]), hd_mul(c, x[1]));
    out[0] = hd_add(x[0], hd_mul(A, rx));
    out[1] = hd_add(x[1], hd_mul(A, ry));
    out[2] = hd_add(x[2], hd_mul(A, x[2]));
}

/* Jacobian J[s][i] = d phi_s / d x_i at p. */
static void pullback_jacobian(const orc_metric *m, const double p[3], double J[9])
{
    for (int i = 0; i < 3; i++) {
        hd x[3], o[3];
        for (int k = 0; k < 3; k++) x[k] = hd_c(p[k]);
        x[i].e1 = 1.0;
        phi_hd(m, x, o);
        for (int s = 0; s < 3; s++) J[3 * s + i] = o[s].e1;
    }
}

/* 3x3 solve by Gaussian elimination with partial pivoting. Returns det. */
static double solve3(const double Ain[9], const double bin[3], double xo[3])
{
    double A[9], b[3];
    memcpy(A, Ain, sizeof A);
    memcpy(b, bin, sizeof b);
    double det = 1.0;
    for (int c = 0; c < 3; c++) {
        int piv = c;
        for (int r = c + 1; r < 3; r++)
            if (fabs(A[3 * r + c]) > fabs(A[3 * piv + c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < 3; k++) {
                double t = A[3 * c + k]; A[3 * c + k] = A[3 * piv + k]; A[3 * piv + k] = t;
            }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
            det = -det;
        }
        det *= A[3 * c + c];
        if (A[3 * c + c] == 0.0) return 0.0;
        for (int r = c + 1; r < 3; r++) {
            double f = A[3 * r + c] / A[3 * c + c];
            for (int k = c; k < 3; k++) A[3 * r + k] -= f * A[3 * c + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = 2; r >= 0; r--) {
        double s = b[r];
        for (int k = r + 1; k < 3; k++) s -= A[3 * r + k] * xo[k];
        xo[r] = s / A[3 * r + r];
    }
    return det;
}

/* Thm 5.1 / Eq. 5.8: y'_k = - sum_s [J^-1]_ks (sum_ij d_ij phi_s y_i y_j),
 * i.e. solve J a = -w with w = D^2 phi[y, y].  Returns 0 if J is singular. */
static int pullback_accel(const orc_metric *m, const double p[3], const double y[3], double a[3])
{
    double J[9];
    pullback_jacobian(m, p, J);
    hd x[3], o[3];
    for (int k = 0; k < 3; k++) {
        x[k] = hd_c(p[k]);
        x[k].e1 = y[k];
        x[k].e2 = y[k];
    }
    phi_hd(m, x, o);
    double w[3] = {-o[0].e12, -o[1].e12, -o[2].e12};
    double det = solve3(J, w, a);
    return det > 0.0;
}

int orc_accel(const orc_metric *m, const double x[3], const double y[3], double a[3])
{
    switch (m->kind) {
    case ORC_EUCLID:
        a[0] = a[1] = a[2] = 0.0;
        return 1;
    case ORC_GRAPH_GAUSS:
    case ORC_GRAPH_ANISO:
    case ORC_GRAPH_QUADRIC:
        graph_accel(m, x, y, a);
        return 1;
    case ORC_PULLBACK_TWIST:
    case ORC_PULLBACK_ZTWIST:
    case ORC_PULLBACK_DEFORM:
        return pullback_accel(m, x, y, a);
    }
    return 0;
}

/* Metric tensor: Eq. 5.2 for graphs (g = I + grad f grad f^T), Eq. 5.6 for
 * pullbacks (g_ij = sum_k d_i x_k d_j x_k). */
void orc_metric_tensor(const orc_metric *m, const double x[3], double g[9])
{
    if (m->kind == ORC_GRAPH_GAUSS || m->kind == ORC_GRAPH_ANISO || m->kind == ORC_GRAPH_QUADRIC) {
        double gr[3], H[9];
        graph_derivs(m, x, gr, H);
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) g[3 * i + j] = (i == j ? 1.0 : 0.0) + gr[i] * gr[j];
    } else if (m->kind == ORC_PULLBACK_TWIST || m->kind == ORC_PULLBACK_ZTWIST || m->kind == ORC_PULLBACK_DEFORM) {
        double J[9];
        pullback_jacobian(m, x, J);
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                double s = 0.0;
                for (int k = 0; k < 3; k++) s += J[3 * k + i] * J[3 * k + j];
                g[3 * i + j] = s;
            }
    } else {
        for (int i = 0; i < 9; i++) g[i] = (i % 4 == 0) ? 1.0 : 0.0;
    }
}

/* --------------------------------------------------------------- the flow */
/* Eq. 3.3 on the state z = (x, y): z' = (y, -Gamma(y, y)). */
static int flow(const orc_metric *m, const double z[6], double dz[6])
{
    dz[0] = z[3]; dz[1] = z[4]; dz[2] = z[5];
    return orc_accel(m, z, z + 3, dz + 3);
}

/* Dormand-Prince 5(4) coefficients (Dormand & Prince 1980). */
static const double DP_C[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
static const double DP_A[7][6] = {
    {0},
    {1.0 / 5},
    {3.0 / 40, 9.0 / 40},
    {44.0 / 45, -56.0 / 15, 32.0 / 9},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656},
    {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
static const double DP_B[7] = {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0.0};
static const double DP_BH[7] = {5179.0 / 57600, 0.0, 7571.0 / 16695, 393.0 / 640,
                                -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};

/* One step of size h.  Euler: Eq. 4.1.  RK4: the classical four stages.
 * RK45: Dormand-Prince, out = 5th-order solution, err = h sum (b - bhat) k.
 * Returns 0 on a numerical failure (singular Jacobian). */
int orc_step(const orc_metric *m, int kind, const double z[6], double h, double out[6], double err[6])
{
    int ok = 1;
    if (err) memset(err, 0, 6 * sizeof(double));
    if (kind == ORC_EULER) {
        double k[6];
        ok &= flow(m, z, k);
        for (int i = 0; i < 6; i++) out[i] = z[i] + h * k[i];
        return ok;
    }
    if (kind == ORC_RK4) {
        double k1[6], k2[6], k3[6], k4[6], t[6];
        ok &= flow(m, z, k1);
        for (int i = 0; i < 6; i++) t[i] = z[i] + 0.5 * h * k1[i];
        ok &= flow(m, t, k2);
        for (int i = 0; i < 6; i++) t[i] = z[i] + 0.5 * h * k2[i];
        ok &= flow(m, t, k3);
        for (int i = 0; i < 6; i++) t[i] = z[i] + h * k3[i];
        ok &= flow(m, t, k4);
        for (int i = 0; i < 6; i++) out[i] = z[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        return ok;
    }
    double k[7][6], t[6];
    ok &= flow(m, z, k[0]);
    for (int s = 1; s < 7; s++) {
        for (int i = 0; i < 6; i++) {
            double acc = 0.0;
            for (int j = 0; j < s; j++) acc += DP_A[s][j] * k[j][i];
            t[i] = z[i] + h * acc;
        }
        ok &= flow(m, t, k[s]);
    }
    for (int i = 0; i < 6; i++) {
        double acc = 0.0, e = 0.0;
        for (int s = 0; s < 7; s++) {
            acc += DP_B[s] * k[s][i];
            e += (DP_B[s] - DP_BH[s]) * k[s][i];
        }
        out[i] = z[i] + h * acc;
        if (err) err[i] = h * e;
    }
    return ok;
}

static int finite6(const double z[6])
{
    for (int i = 0; i < 6; i++)
        if (!isfinite(z[i])) return 0;
    return 1;
}

/* ------------------------------------------------------------ the scene */
/* Implicit functions whose sign separates outside (>0) and inside (<=0). */
static double obj_F(const orc_scene *s, int id, const double x[3])
{
    if (id < s->n_spheres) {
        const double *p = s->spheres + 4 * id;
        double d[3] = {x[0] - p[0], x[1] - p[1], x[2] - p[2]};
        return dot3(d, d) - p[3] * p[3];
    }
    id -= s->n_spheres;
    if (id < s->n_planes) {
        const double *p = s->planes + 4 * id;
        return dot3(p, x) - p[3];
    }
    id -= s->n_planes;
    const double *p = s->tori + 8 * id;
    double q[3] = {x[0] - p[0], x[1] - p[1], x[2] - p[2]};
    double ax = dot3(q, p + 3);
    double rad[3] = {q[0] - ax * p[3], q[1] - ax * p[4], q[2] - ax * p[5]};
    double e = sqrt(dot3(rad, rad)) - p[6];
    return sqrt(e * e + ax * ax) - p[7];
}

/* Segment-versus-scene test of the chord [x0, x1] (Sec. 4.1): the earliest
 * crossing parameter s in [0, 1] over all objects; ties keep the lower id.
 * Spheres: smallest root of the quadratic; planes and the torus SDF: a sign
 * change between the endpoints, s by linear interpolation. */
static int chord_test(const orc_scene *s, const double x0[3], const double x1[3], double *s_out)
{
    double D[3] = {x1[0] - x0[0], x1[1] - x0[1], x1[2] - x0[2]};
    int best = -1;
    double bs = 2.0;
    int nobj = s->n_spheres + s->n_planes + s->n_tori;
    for (int id = 0; id < nobj; id++) {
        double sc = 2.0;
        if (id < s->n_spheres) {
            const double *p = s->spheres + 4 * id;
            double oc[3] = {x0[0] - p[0], x0[1] - p[1], x0[2] - p[2]};
            double A = dot3(D, D), B = dot3(D, oc), C = dot3(oc, oc) - p[3] * p[3];
            if (A <= 0.0) continue;
            double disc = B * B - A * C;
            if (disc < 0.0) continue;
            double q = sqrt(disc);
            double s1 = (-B - q) / A, s2 = (-B + q) / A;
            if (s1 >= 0.0 && s1 <= 1.0) sc = s1;
            else if (s2 >= 0.0 && s2 <= 1.0) sc = s2;
        } else {
            double F0 = obj_F(s, id, x0), F1 = obj_F(s, id, x1);
            if ((F0 > 0.0) != (F1 > 0.0)) {
                sc = F0 / (F0 - F1);
                if (sc < 0.0) sc = 0.0;
                if (sc > 1.0) sc = 1.0;
            }
        }
        if (sc <= 1.0 && sc < bs) {
            bs = sc;
            best = id;
        }
    }
    *s_out = bs;
    return best;
}

/* ------------------------------------------------- direct illumination
 * The geodesic from state z0 over arc length T: ceil(T / h) classical RK4
 * steps, the last one shortened to end exactly at T. */
int orc_shoot(const orc_metric *m, const double z0[6], double T, double h, double out[6])
{
    int n = (int)ceil(T / h);
    if (n < 1) n = 1;
    double z[6];
    memcpy(z, z0, sizeof z);
    for (int i = 0; i < n; i++) {
        double hs = (i == n - 1) ? T - (n - 1) * h : h;
        double zn[6];
        if (!orc_step(m, ORC_RK4, z, hs, zn, NULL)) return 0;
        memcpy(z, zn, sizeof z);
    }
    memcpy(out, z, sizeof z);
    return 1;
}

/* Whether that geodesic crosses no object between arc length skip and T
 * (Sec. 4, Riemannian illumination: a light reaches q along a geodesic
 * that meets nothing on the way): every step's chord against every object,
 * spheres by both roots of the quadratic, planes and tori by a sign change
 * of the implicit function. */
int orc_geodesic_clear(const orc_metric *m, const orc_scene *s, const double z0[6], double T, double h,
                       double skip)
{
    int n = (int)ceil(T / h);
    if (n < 1) n = 1;
    double z[6], t = 0.0;
    memcpy(z, z0, sizeof z);
    int nobj = s->n_spheres + s->n_planes + s->n_tori;
    for (int i = 0; i < n; i++) {
        double hs = (i == n - 1) ? T - (n - 1) * h : h;
        double zn[6];
        if (!orc_step(m, ORC_RK4, z, hs, zn, NULL)) return 0;
        double D[3] = {zn[0] - z[0], zn[1] - z[1], zn[2] - z[2]};
        for (int id = 0; id < nobj; id++) {
            if (id < s->n_spheres) {
                const double *p = s->spheres + 4 * id;
                double oc[3] = {z[0] - p[0], z[1] - p[1], z[2] - p[2]};
                double A = dot3(D, D), B = dot3(D, oc), C = dot3(oc, oc) - p[3] * p[3];
                double disc = B * B - A * C;
                if (A <= 0.0 || disc < 0.0) continue;
                double q = sqrt(disc);
                double r[2] = {(-B - q) / A, (-B + q) / A};
                for (int k = 0; k < 2; k++)
                    if (r[k] >= 0.0 && r[k] <= 1.0 && t + r[k] * hs > skip) return 0;
            } else {
                double F0 = obj_F(s, id, z), F1 = obj_F(s, id, zn);
                if ((F0 > 0.0) != (F1 > 0.0)) {
                    double sc = F0 / (F0 - F1);
                    if (t + sc * hs > skip) return 0;
                }
            }
        }
        memcpy(z, zn, sizeof z);
        t += hs;
    }
    return 1;
}

/* --------------------------------------------------------------- tracing */
static void finish(orc_result *res, const double z[6], double t, int id)
{
    res->hit[0] = z[0]; res->hit[1] = z[1]; res->hit[2] = z[2];
    double n = sqrt(dot3(z + 3, z + 3));
    res->dir[0] = z[3] / n; res->dir[1] = z[4] / n; res->dir[2] = z[5] / n;
    res->t = t;
    res->id = id;
}

/* One geodesic from x0 in the Euclidean direction d: y0 = d / sqrt(g(d,d))
 * (unit speed in g, so t is Riemannian arc length: exp_p(v) = gamma(|v|),
 * Sec. 3.4).  March until the chord of an accepted step meets the scene,
 * then bisect the step fraction s on the sign of the hit object's implicit
 * function along the partial step Psi_{s h}(z_k) of the same integrator.
 * A chord hit without a sign change (a grazing sphere chord) keeps the chord
 * root.  Miss: steps == max_steps or t >= t_max (id -1, final state).
 * Non-finite state, a singular pullback Jacobian or a step below h_min:
 * id -2. */
void orc_trace_ray(const orc_metric *m, const orc_scene *s, const orc_rule *r,
                   const double x0[3], const double d[3], orc_result *res)
{
    double z[6], zn[6], err[6];
    double g[9];
    orc_metric_tensor(m, x0, g);
    double gdd = 0.0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) gdd += d[i] * g[3 * i + j] * d[j];
    double sp = sqrt(gdd);
    for (int i = 0; i < 3; i++) {
        z[i] = x0[i];
        z[3 + i] = d[i] / sp;
    }
    res->steps = 0;
    res->rejected = 0;
    double t = 0.0;
    double h = r->h;
    int steps = 0;
    int attempts = 0;
    for (;;) {
        if (steps >= r->max_steps || t >= r->t_max) {
            finish(res, z, t, -1);
            res->steps = steps;
            return;
        }
        double hs = h;
        int ok;
        if (r->kind == ORC_RK45) {
            for (;;) {
                if (t + hs > r->t_max) hs = r->t_max - t;
                ok = orc_step(m, ORC_RK45, z, hs, zn, err);
                attempts++;
                if (!ok || !finite6(zn)) break;
                double e2 = 0.0;
                for (int i = 0; i < 6; i++) {
                    double sc = r->atol + r->rtol * fmax(fabs(z[i]), fabs(zn[i]));
                    e2 += (err[i] / sc) * (err[i] / sc);
                }
                double en = sqrt(e2 / 6.0);
                double fac = en > 0.0 ? 0.9 * pow(en, -0.2) : 5.0;
                if (fac < 0.2) fac = 0.2;
                if (fac > 5.0) fac = 5.0;
                if (en <= 1.0) {
                    h = fmin(hs * fac, r->h_max);
                    break;
                }
                res->rejected++;
                hs = hs * fmin(fac, 1.0);
                if (hs < r->h_min || attempts > 8 * r->max_steps) {
                    ok = 0;
                    break;
                }
            }
        } else {
            ok = orc_step(m, r->kind, z, hs, zn, NULL);
        }
        if (!ok || !finite6(zn)) {
            finish(res, z, t, -2);
            res->steps = steps;
            return;
        }
        double sc;
        int id = chord_test(s, z, zn, &sc);
        if (id >= 0) {
            double F0 = obj_F(s, id, z), F1 = obj_F(s, id, zn);
            double sstar = sc;
            if ((F0 > 0.0) != (F1 > 0.0)) {
                double lo = 0.0, hi = 1.0;
                for (int it = 0; it < r->bisect_iters; it++) {
                    double mid = 0.5 * (lo + hi);
                    double zm[6];
                    orc_step(m, r->kind, z, mid * hs, zm, NULL);
                    if ((obj_F(s, id, zm) > 0.0) == (F0 > 0.0)) lo = mid;
                    else hi = mid;
                }
                sstar = 0.5 * (lo + hi);
            }
            double zs[6];
            orc_step(m, r->kind, z, sstar * hs, zs, NULL);
            double tk = (r->kind == ORC_RK45) ? t : steps * r->h;
            finish(res, zs, tk + sstar * hs, id);
            res->steps = steps + 1;
            return;
        }
        memcpy(z, zn, sizeof z);
        steps++;
        if (r->kind == ORC_RK45) t += hs;
        else t = steps * r->h;
    }
}

int orc_trace_pixels(const orc_metric *m, const orc_scene *s, const orc_camera *c,
                     const orc_rule *r, int64_t n, const int64_t *pix,
                     double *out8, int32_t *ids, int32_t *steps,
                     int32_t *rejected, int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t q = 0; q < n; q++) {
        int64_t p = pix[q];
        int i = (int)(p % c->width), j = (int)(p / c->width);
        double d[3];
        orc_camera_dir(c, i, j, d);
        orc_result res;
        orc_trace_ray(m, s, r, c->eye, d, &res);
        double *o = out8 + 8 * q;
        o[0] = res.hit[0]; o[1] = res.hit[1]; o[2] = res.hit[2];
        o[3] = res.t;
        o[4] = res.dir[0]; o[5] = res.dir[1]; o[6] = res.dir[2];
        o[7] = 0.0;
        ids[q] = res.id;
        steps[q] = res.steps;
        if (rejected) rejected[q] = res.rejected;
    }
    return 0;
}

/* Fixed-step trajectory z_0..z_n of the integrator (RK45 uses the fixed h
 * given, without control), for invariant checks. */
int orc_trajectory(const orc_metric *m, const orc_rule *r, const double z0[6],
                   int n_steps, double *out)
{
    memcpy(out, z0, 6 * sizeof(double));
    for (int k = 0; k < n_steps; k++)
        if (!orc_step(m, r->kind, out + 6 * k, r->h, out + 6 * (k + 1), NULL)) return k + 1;
    return 0;
}
