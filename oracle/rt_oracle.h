/* FP64 CPU oracle of the Riemannian ray tracer (test infrastructure only).
 *
 * Plain, slow, obviously-correct double-precision reference of what the
 * GPU path computes.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load it; the product library never does.  It shares no
 * code, header or constant with the GPU sources.
 *
 * Paper: Novello, da Silva, Velho, "Design and visualization of Riemannian
 * metrics" (2020).  Section/equation numbers below are the paper's.
 */
#ifndef RT_ORACLE_H
#define RT_ORACLE_H
#include <stdint.h>

#define ORC_EUCLID 0
#define ORC_GRAPH_GAUSS 1
#define ORC_PULLBACK_TWIST 2
#define ORC_PULLBACK_ZTWIST 3
#define ORC_PULLBACK_DEFORM 4
#define ORC_GRAPH_ANISO 5
#define ORC_GRAPH_QUADRIC 6

#define ORC_RK4 0
#define ORC_RK45 1
#define ORC_EULER 2

typedef struct {
    int kind;
    int n_bumps;
    const double *bumps; /* [n_bumps][5] a, cx, cy, cz, sigma */
    double twist_amp, twist_theta0;
    int n_deforms;
    const double *deforms; /* [n_deforms][13] a, cx, cy, cz, sx, sy, sz, vx, vy, vz, wx, wy, wz */
    int n_abumps;
    const double *abumps;  /* [n_abumps][7] a, cx, cy, cz, sx, sy, sz */
    double quadric[3];     /* f = q0 x^2 + q1 y^2 + q2 z^2 */
} orc_metric;

typedef struct {
    int n_spheres;
    const double *spheres; /* [n][4] cx cy cz r */
    int n_planes;
    const double *planes;  /* [n][4] nx ny nz d   (n.x = d) */
    int n_tori;
    const double *tori;    /* [n][8] cx cy cz ax ay az R r */
} orc_scene;

typedef struct {
    double eye[3], fwd[3], up[3];
    double vfov_deg;
    int width, height;
} orc_camera;

typedef struct {
    int kind;
    double h, rtol, atol, h_min, h_max, t_max;
    int max_steps;
    int bisect_iters;
} orc_rule;

/* one traced pixel: hit[3], t, dir[3] ; id ; accepted steps ; rejected */
typedef struct {
    double hit[3];
    double t;
    double dir[3];
    int id;
    int steps;
    int rejected;
} orc_result;

void orc_camera_dir(const orc_camera *cam, int i, int j, double d[3]);
int orc_accel(const orc_metric *m, const double x[3], const double y[3], double a[3]);
void orc_metric_tensor(const orc_metric *m, const double x[3], double g[9]);
int orc_step(const orc_metric *m, int kind, const double z[6], double h,
             double out[6], double err[6]);
void orc_trace_ray(const orc_metric *m, const orc_scene *s, const orc_rule *r,
                   const double x0[3], const double d[3], orc_result *res);
int orc_trace_pixels(const orc_metric *m, const orc_scene *s, const orc_camera *c,
                     const orc_rule *r, int64_t n, const int64_t *pix,
                     double *out8, int32_t *ids, int32_t *steps,
                     int32_t *rejected, int nthreads);
int orc_shoot(const orc_metric *m, const double z0[6], double T, double h, double out[6]);
int orc_geodesic_clear(const orc_metric *m, const orc_scene *s, const double z0[6], double T, double h,
                       double skip);
int orc_trajectory(const orc_metric *m, const orc_rule *r, const double z0[6],
                   int n_steps, double *out /* [n_steps+1][6] */);
#endif
