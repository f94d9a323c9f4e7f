/* rt.h -- C ABI of the MI355X Riemannian ray tracer.
 *
 * The engine answers the question of the paper's "Riemannian shading"
 * (Novello, da Silva, Velho, "Design and visualization of Riemannian
 * metrics", Sec. 4): for every direction v of the observer field at a point
 * p, follow the geodesic gamma with gamma(0) = p, gamma'(0) = v -- the
 * exponential map of Sec. 3.4 -- and report what it hits.  The geodesic is
 * the solution of the geodesic flow x' = y, y' = -Gamma(y, y) (Eq. 3.3),
 * marched with a Runge-Kutta or Euler step (Sec. 4.1, Eq. 4.1), each step's
 * segment tested against the scene (Sec. 4.1).  The hit point, the
 * parameter t at the hit, the object id and the final direction are
 * returned per pixel; colours are left to the caller (Sec. 4, last
 * paragraph: pseudo-colour from the hit coordinates).
 *
 * Conventions shared by every entry point:
 *  - All functions return rt_status (RT_OK = 0).  On any error nothing is
 *    written to caller buffers and rt_last_error() explains.
 *  - Host pointers (metric, scene, camera, rule structs and the arrays they
 *    point to) are read during the call only; the context keeps copies.
 *  - Device pointers (rt_outputs) are caller-owned device memory on the
 *    context's device; the caller keeps them alive until the stream work
 *    finishes.
 *  - hip_stream is a hipStream_t (NULL = the legacy default stream); all
 *    device work is enqueued on it asynchronously, in call order.
 *  - A context is not thread-safe; use one context per host thread.  Calls
 *    that enqueue work on one context must not overlap on two streams.
 *  - Per-pixel outcomes are encoded in the id output, never in the status:
 *    id >= 0 hit object, -1 miss (step budget or t_max reached),
 *    -2 numerical failure (non-finite state, singular Jacobian, step size
 *    below h_min).
 */
#ifndef RT_H
#define RT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RT_ABI_VERSION 6

typedef enum rt_status {
    RT_OK = 0,
    RT_EINVAL = -1,       /* bad argument (null pointer, bad size, non-finite value) */
    RT_ENOMEM = -2,       /* device or host allocation failed */
    RT_EDEVICE = -3,      /* HIP runtime error, no device, or an asynchronous fault */
    RT_EUNSUPPORTED = -4, /* combination not implemented (kind x step rule) */
    RT_ESTATE = -5        /* metric or scene not set, or host-only context */
} rt_status;

typedef struct rt_ctx rt_ctx;

/* Library ABI version (RT_ABI_VERSION of the build). */
int rt_abi_version(void);

/* Create a context on HIP device `hip_device`.  hip_device = -1 creates a
 * host-only context: every argument check runs, nothing is launched, and
 * rt_trace returns RT_ESTATE after validation.  *out is set to NULL on
 * failure; the message is then available from rt_last_error(NULL). */
rt_status rt_create(int hip_device, rt_ctx **out);

/* Release the context and its device memory (waits for its streams' work
 * to finish first).  NULL is ignored. */
void rt_destroy(rt_ctx *ctx);

/* Human-readable message for the last failing call on ctx (NULL ctx: the
 * last failing rt_create on this thread).  Empty string if none.  The
 * pointer stays valid until the next call on the same context. */
const char *rt_last_error(const rt_ctx *ctx);

/* ------------------------------------------------------------------ metric
 * RT_METRIC_EUCLID           flat R^3 (Gamma = 0).
 * RT_METRIC_GRAPH_GAUSS      pull-back of the graph of f: R^3 -> R
 *                            (Sec. 5.1): g = I + grad f grad f^T (Eq. 5.2),
 *                            Gamma^m_ij = f_m f_ij / (1 + |grad f|^2)
 *                            (Eq. 5.3), flow Eq. 5.4; f is a sum of
 *                            isotropic Gaussians a exp(-|x-c|^2/(2 sigma^2))
 *                            (Eq. 6.1 with equal spreads; sums as in
 *                            Sec. 6.2, "Summing functions").
 * RT_METRIC_PULLBACK_TWIST   pull-back g = J^T J (Eq. 5.6) of the radial
 *                            twist phi(x) = x + amp tanh|x| R_z(theta) x,
 *                            theta = theta0 exp(-|x|^2); Gamma from Thm 5.1
 *                            (Eq. 5.7), flow Eq. 5.8.
 * RT_METRIC_PULLBACK_ZTWIST  pull-back of the z-twist of Sec. 5.2,
 *                            Phi(x,y,z) = (cos z x - sin z y,
 *                                          sin z x + cos z y, z).
 * RT_METRIC_GRAPH_ANISO      as RT_METRIC_GRAPH_GAUSS, with the Gaussians of
 *                            Eq. 6.1 in full: three spreads per bump,
 *                            a exp(-sum_j (x_j - c_j)^2 / (2 s_j^2)).
 * RT_METRIC_GRAPH_QUADRIC    the graph metric of the quadratic
 *                            f = qx x^2 + qy y^2 + qz z^2; the paper's
 *                            example of Sec. 5.1 is (qx, qy, qz) = (1, 1, -1).
 *                            One parameter set.
 * RT_METRIC_PULLBACK_DEFORM  pull-back g = J^T J (Eq. 5.6) of a composition
 *                            Phi = Phi_1 o Phi_2 o ... o Phi_k of local
 *                            deformations (Sec. 6.2, "Composing
 *                            diffeomorphisms"; Phi_k acts first), each
 *                            Phi_i(p) = p + f_i(p) V_i(p) (Eq. 6.2) with f_i
 *                            the anisotropic Gaussian of Eq. 6.1 and the
 *                            affine field V_i(p) = v_i + w_i x (p - c_i): a
 *                            constant direction (w_i = 0) or, with w_i, a
 *                            local rotation about the axis w_i through c_i.
 *                            The Jacobian is the chain-rule product and
 *                            D^2 Phi[y, y] is propagated through the chain
 *                            with the pushed-forward velocity (the Hessian
 *                            composition formula of Sec. 6.2 contracted
 *                            with y); flow Eq. 5.8.  Each Phi_i must be a
 *                            diffeomorphism.  With w_i = 0 that holds iff
 *                            |a| |(vx/sx, vy/sy, vz/sz)| exp(-1/2) < 1;
 *                            otherwise it holds when the Lipschitz bound
 *                            |a| (exp(-1/2) |v| / s_min
 *                                 + |w| (2/e s_max / s_min + 1)) < 1.
 *                            rt_set_metric requires the bound <= 0.95.
 */
typedef enum rt_metric_kind {
    RT_METRIC_EUCLID = 0,
    RT_METRIC_GRAPH_GAUSS = 1,
    RT_METRIC_PULLBACK_TWIST = 2,
    RT_METRIC_PULLBACK_ZTWIST = 3,
    RT_METRIC_PULLBACK_DEFORM = 4,
    RT_METRIC_GRAPH_ANISO = 5,
    RT_METRIC_GRAPH_QUADRIC = 6
} rt_metric_kind;

typedef struct rt_bump {
    float a;          /* amplitude */
    float cx, cy, cz; /* centre */
    float sigma;      /* spread, > 0 */
} rt_bump;

typedef struct rt_deform {
    float a;          /* amplitude of f_i */
    float cx, cy, cz; /* centre */
    float sx, sy, sz; /* spreads along x, y, z, > 0 */
    float vx, vy, vz; /* constant part v_i of the field (its length scales the displacement) */
    float wx, wy, wz; /* rotation part w_i of the field, V_i(p) = v_i + w_i x (p - c_i) */
} rt_deform;

typedef struct rt_abump {
    float a;          /* amplitude */
    float cx, cy, cz; /* centre */
    float sx, sy, sz; /* spreads along x, y, z, > 0 */
} rt_abump;

typedef struct rt_metric {
    int kind;            /* rt_metric_kind */
    int n_sets;          /* independent parameter sets traced side by side, 1..64 */
    int n_bumps;         /* bumps per set, 0..64 (GRAPH_GAUSS only) */
    const rt_bump *bumps;/* host, [n_sets][n_bumps], row-major */
    float twist_amp;     /* PULLBACK_TWIST amplitude (0.4 in the 4K workload), 0 <= amp <= 1 */
    float twist_theta0;  /* PULLBACK_TWIST peak angle (1.2), |theta0| <= 1.5 */
    float cull_sigmas;   /* a bump is ignored where |x - c| > cull_sigmas * sigma;
                            >= 4, 6 recommended (exp(-18) is below FP32 resolution);
                            for a deformation or an anisotropic bump, where
                            sum_j ((x_j - c_j) / s_j)^2 > cull_sigmas^2 (there
                            Phi_i is the identity and the bump is zero) */
    int n_deforms;              /* deformations per set, 1..64 (PULLBACK_DEFORM only) */
    const rt_deform *deforms;   /* host, [n_sets][n_deforms], row-major, Phi_1 first */
    int n_abumps;               /* anisotropic bumps per set, 0..64 (GRAPH_ANISO only) */
    const rt_abump *abumps;     /* host, [n_sets][n_abumps], row-major */
    float quadric[3];           /* GRAPH_QUADRIC coefficients (qx, qy, qz), |q| <= 100 */
} rt_metric;

/* Copy and validate the metric: finite values, sigma > 0, sizes in range.
 * Replaces any previous metric. */
rt_status rt_set_metric(rt_ctx *ctx, const rt_metric *metric);

/* ------------------------------------------------------------------- scene
 * Object ids: spheres 0..n_spheres-1, then planes, then tori.  Each object
 * has an implicit function, > 0 outside, <= 0 inside:
 *   sphere |x - c|^2 - r^2 ; plane n.x - d ; torus (axis a, |a| = 1) the
 *   signed distance sqrt((|x_perp| - R)^2 + x_par^2) - r.                  */
typedef struct rt_sphere { float cx, cy, cz, r; } rt_sphere;
typedef struct rt_plane { float nx, ny, nz, d; } rt_plane;
typedef struct rt_torus { float cx, cy, cz, ax, ay, az, R, r; } rt_torus;

typedef struct rt_scene {
    int n_spheres;             /* 0..256 */
    const rt_sphere *spheres;  /* host */
    int n_planes;              /* 0..8 */
    const rt_plane *planes;    /* host; |n| = 1 */
    int n_tori;                /* 0..8 */
    const rt_torus *tori;      /* host; |a| = 1, 0 < r < R */
} rt_scene;

/* Copy and validate the scene.  Replaces any previous scene. */
rt_status rt_set_scene(rt_ctx *ctx, const rt_scene *scene);

/* ------------------------------------------------------------------ camera
 * Pinhole at eye.  The paper leaves the observer field open (Sec. 4); this
 * ABI uses: vertical field of view vfov_deg, pixel centres, column i to
 * the right, row 0 at the top, right = up x forward.  The initial velocity
 * is the pixel direction scaled to unit length in the metric g at the eye,
 * so t is Riemannian arc length (exp_p(v) = gamma(|v|), Sec. 3.4). */
typedef struct rt_camera {
    float eye[3], forward[3], up[3];
    float vfov_deg; /* (0, 180) */
    int width, height; /* >= 1, width * height * n_sets <= 2^31 - 1 */
} rt_camera;

/* --------------------------------------------------------------- step rule
 * RT_STEP_RK4    classical fixed-step Runge-Kutta, step h.
 * RT_STEP_RK45   Dormand-Prince 5(4), first trial step h, error control on
 *                the RMS of h*sum(b - bhat)k over the 6 state components
 *                scaled by atol + rtol*max(|z|, |z_new|); step factor
 *                clamp(0.9 err^(-1/5), 0.2, 5), h <= h_max, the last step
 *                clipped to t_max; a step below h_min fails the ray (id -2).
 * RT_STEP_EULER  the paper's explicit Euler march (Eq. 4.1), step h.
 * A ray stops at the first accepted step whose segment meets the scene; the
 * hit is then refined in double precision: the step fraction s where the
 * object's implicit function changes sign along the partial step of the same
 * integrator is bracketed to a width of 2^-bisect_iters (the precision of
 * that many bisection halvings), by regula falsi with the Illinois
 * modification started at the segment's root and a halving whenever two
 * probes have not halved the bracket; s is the bracket's midpoint.  A
 * grazing sphere segment with no sign change keeps the segment's root.
 * Otherwise it stops after max_steps accepted steps or when t reaches t_max
 * (miss). */
typedef enum rt_step_kind { RT_STEP_RK4 = 0, RT_STEP_RK45 = 1, RT_STEP_EULER = 2 } rt_step_kind;

typedef struct rt_step_rule {
    int kind;          /* rt_step_kind */
    float h;           /* step (RK4/Euler) or first trial step (RK45), > 0 */
    float rtol, atol;  /* RK45 tolerances, > 0 */
    float h_min, h_max;/* RK45 step bounds, 0 < h_min <= h_max */
    float t_max;       /* > 0; RK4/Euler rays also stop at max_steps */
    int cull_every;    /* K: steps between per-wave re-culls of bumps/objects, 1..256 (16) */
    int pass_steps;    /* S: steps per launch before surviving rays are compacted, >= 16 (256) */
    int bisect_iters;  /* hit refinement: bracket the step fraction to 2^-bisect_iters, 0..60 (24: h 2^-24 is below the
                          float spacing of the hit; 0: no refinement, s = 1/2 when the sign changes) */
    int flags;         /* RT_FLAG_* bits, 0 for a plain trace */
} rt_step_rule;

/* RT_FLAG_TIMING: record HIP events on the stream around every kernel of the
 *   trace; rt_get_stats then reports their durations.
 * RT_FLAG_COUNT_WORK: run the instrumented kernel variant that also counts,
 *   per lane, the work the method needs (acceleration evaluations, bumps
 *   inside their cut sphere, objects inside the lane's own window); same
 *   outputs, slower.  Used to compute algorithmic FLOP counts. */
#define RT_FLAG_TIMING 1
#define RT_FLAG_COUNT_WORK 2
/* RT_FLAG_SURROGATE: use the networks given to rt_surrogate_load for the
 *   support spheres of eligible bumps (graph metric, RT_STEP_RK4, one
 *   parameter set; RT_EUNSUPPORTED otherwise, RT_ESTATE if none loaded). */
#define RT_FLAG_SURROGATE 4
/* RT_FLAG_BATCH_SEGMENTS: batched multi-segment intersection (the batching
 *   of polygon segments Sec. 4.1 proposes).  Each wave marches a culling
 *   window of cull_every steps with no scene test, each lane keeping the
 *   bounding box of its polygon; the boxes are then tested against the
 *   window's objects, and only the lanes whose box meets one march the window
 *   again with the per-step chord tests.  Outputs equal the plain trace's bit
 *   for bit.  RT_STEP_RK4 and RT_STEP_EULER; not with RT_FLAG_COUNT_WORK,
 *   RT_FLAG_SURROGATE or a tape (RT_EUNSUPPORTED). */
#define RT_FLAG_BATCH_SEGMENTS 8

/* ----------------------------------------------------------------- outputs
 * Caller-owned device arrays, indexed [set][row][column] (pixel index
 * p = (set*height + j)*width + i):
 *   hit   float[.][3]  hit point (miss/failure: final position)
 *   t     float[.]     geodesic parameter at the hit / at termination
 *   id    int32[.]     object id, -1 miss, -2 numerical failure
 *   dir   float[.][3]  unit Euclidean direction of the velocity there
 *   steps int32[.]     accepted steps taken, including the hit step
 *                      (optional: NULL skips it)                        */
typedef struct rt_outputs {
    float *hit;
    float *t;
    int32_t *id;
    float *dir;
    int32_t *steps;
} rt_outputs;

/* Trace every pixel of every parameter set.  Requires rt_set_metric and
 * rt_set_scene.  Asynchronous on hip_stream; scratch memory sized for the
 * largest frame seen so far is kept by the context.  max_steps in
 * 1..1000000.  RT_EUNSUPPORTED if the step kind is unknown. */
rt_status rt_trace(rt_ctx *ctx, const rt_camera *camera, const rt_step_rule *rule,
                   int max_steps, const rt_outputs *out, void *hip_stream);

/* rt_trace without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, kernels and results as rt_trace
 * (bitwise), but the trace's workspace (ray state, survivor lists, chunk
 * scans, refine records, counters) lives in one static device array of
 * RT_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from the first
 * rt_create on that GPU until the process ends.  The workspace needs about
 * 149 bytes per ray id (ids: 8x8 pixel tiles x 64 x n_sets) plus 1 KB per
 * pass: up to about 450,000 ray ids, e.g. a 640x640 frame of one set.
 * Larger frames return RT_EINVAL before any launch.  Also RT_EUNSUPPORTED
 * for RT_FLAG_TIMING (event creation) and RT_FLAG_SURROGATE (crossing
 * queues).  Every call on one GPU shares the array: calls whose work
 * overlaps on that GPU (other streams, other contexts, other host threads)
 * race and give undefined results; serialise them.  The counters the
 * trace needs zeroed are cleared by its first kernel.  rt_get_stats reads
 * the counters of the last trace, whichever entry point ran it. */
#define RT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
rt_status rt_trace_noalloc(rt_ctx *ctx, const rt_camera *camera, const rt_step_rule *rule,
                           int max_steps, const rt_outputs *out, void *hip_stream);

/* Wait for the context's work on hip_stream and report any asynchronous
 * device error as RT_EDEVICE. */
rt_status rt_sync(rt_ctx *ctx, void *hip_stream);

/* Counters of the last rt_trace (read after its work finished; this call
 * waits for the context's last stream). */
typedef struct rt_stats {
    uint64_t rays;          /* rays launched */
    uint64_t ray_steps;     /* accepted integration steps, all rays */
    uint64_t attempts;      /* RK45 trial steps incl. rejected; = ray_steps otherwise */
    uint64_t wave_iters;    /* COUNT_WORK: wave-wide step iterations */
    uint64_t lane_iters;    /* COUNT_WORK: active lanes summed over wave iterations */
    uint64_t bump_list_sum; /* COUNT_WORK: culled bump-list length summed over wave iterations */
    uint64_t obj_list_sum;  /* COUNT_WORK: culled object-list length summed over wave iterations */
    uint64_t refined;       /* hits refined in FP64 */
    uint64_t acc_evals;     /* COUNT_WORK: lane acceleration evaluations */
    uint64_t bump_evals;    /* COUNT_WORK: lane bump terms with |x - c| inside the cut */
    uint64_t obj_tests;     /* COUNT_WORK: lane segment tests against objects in the lane's own window */
    int passes;             /* kernel passes launched */
    float pass_ms;          /* TIMING: summed duration of the integration passes */
    float refine_ms;        /* TIMING: duration of the FP64 refinement kernel */
    float compact_ms;       /* TIMING: summed duration of the survivor compaction between passes */
    float total_ms;         /* TIMING: reset + passes + refinement */
    uint64_t crossings;     /* SURROGATE: rays parked on an eligible support sphere */
    uint64_t accepted;      /* SURROGATE: crossings replaced by the network's prediction */
    float surr_ms;          /* SURROGATE + TIMING: summed duration of the crossing stages */
    int eligible;           /* SURROGATE: bumps whose support sphere the networks may replace */
    uint64_t adj_steps;     /* rt_trace_bwd since the last trace: full RK4 steps reversed */
    uint64_t adj_bump_terms; /* rt_trace_bwd: bump terms inside their cut at those steps' stages */
    uint64_t adj_recomputed; /* rt_trace_bwd: full RK4 steps recomputed from the checkpoints */
    uint64_t batch_windows; /* BATCH_SEGMENTS: culling windows marched (one per wave and window) */
    uint64_t batch_replays; /* BATCH_SEGMENTS: windows marched again because a lane's box met an object */
    uint64_t refine_evals;      /* COUNT_WORK: FP64 acceleration evaluations of the hit refinement */
    uint64_t refine_bump_terms; /* COUNT_WORK: bumps inside their cut at those evaluations (graph metric) */
    uint64_t refine_steps;      /* COUNT_WORK: FP64 integrator steps of the refinement (full and partial) */
} rt_stats;

rt_status rt_get_stats(rt_ctx *ctx, rt_stats *out);

/* ---------------------------------------------------- direct illumination
 * Riemannian illumination (Sec. 4): a surface point q is lit by a point
 * light L through the geodesics joining q to L, with a Lambertian
 * intensity that depends on the metric.  For every pixel of a trace that
 * hit an object (traced->id >= 0), rt_illuminate finds a geodesic from the
 * hit point q to L by shooting -- the g-unit direction v at q and the arc
 * length T with gamma_{q,v}(T) = L, Newton's method from the straight
 * segment, each shot an RK4 integration with step h -- then marches it
 * against the scene's objects (crossings within 1e-3 of q ignored) and
 * writes
 *   shade  = grad F . v / sqrt(grad F^T g^-1 grad F) when lit, else 0:
 *            the cosine between v and the metric normal g^-1 grad F of the
 *            surface F = 0, both measured in g at q;
 *   status = 1 lit, 0 the geodesic is blocked, 2 the surface faces away
 *            (cosine <= 0), -1 no geodesic found: not within max_iters,
 *            Newton stalled (from the fifth iteration on, a residual above
 *            half the previous one), the length grew past four times the
 *            straight segment's length in g at q plus one, or a shot
 *            overran max_steps; -3 the pixel did not hit;
 *   dir    = v (optional), len = T (optional).
 * A pixel left without a geodesic then retries from the converged
 * direction and length of a neighbouring pixel (the one of its 8 neighbours
 * with the nearest hit point), in up to 3 rounds of max(max_iters / 2, 1)
 * iterations, each round seeded from everything converged so far; the
 * pixels still without one then follow a continuation in the light
 * position, aiming at q + lambda (L - q) for lambda = 1/8, 2/8, ..., 1,
 * each stage from the previous one's solution (max(max_iters / 2, 1)
 * iterations per stage).
 * Several geodesics may join q and L; the one found is the one reached
 * from the straight segment or from a neighbour's.  The paper describes this illumination but
 * not how to compute it.  camera must be the traced camera; the metric and
 * scene of the context are used.  Outputs are device arrays of
 * n_sets * height * width entries (dir: 3 per entry).  Asynchronous on
 * hip_stream; the context keeps a device workspace of 52 bytes per entry,
 * sized for the largest frame seen so far. */
typedef struct rt_light {
    float pos[3];   /* point light */
    float h;        /* RK4 step of the shots, (0, 0.1] */
    float tol;      /* convergence: max-norm distance of gamma(T) to the light, > 0 */
    int max_iters;  /* Newton iterations, 1..64 */
    int max_steps;  /* steps per shot, 1..100000 */
} rt_light;

typedef struct rt_shading {
    float *shade;     /* device, required */
    int32_t *status;  /* device, required */
    float *dir;       /* device, optional */
    float *len;       /* device, optional */
} rt_shading;

rt_status rt_illuminate(rt_ctx *ctx, const rt_camera *camera, const rt_outputs *traced, const rt_light *light,
                        const rt_shading *out, void *hip_stream);

/* ------------------------------------------------------- differentiation
 * Gradients of a loss on the hit map with respect to every bump parameter
 * (a, cx, cy, cz, sigma) of every set: the discrete adjoint of the RK4
 * trace of the graph metric (RT_METRIC_GRAPH_GAUSS, 1..16 bumps per set,
 * RT_STEP_RK4).  For a hitting pixel, the hit is the position of the
 * partial RK4 step of fraction s* from the last state before the hit,
 * where s* zeroes the object's implicit function; its derivative follows
 * the implicit function theorem.  Pixels that miss carry no gradient.
 *
 * Tape: caller-owned device memory of rt_tape_bytes() bytes holding the
 * state (x_hi, x_lo, y) every ckpt_every accepted steps of every ray and,
 * per pixel, the state before the hit step with s*, the step index and the
 * object.  rt_trace_bwd recomputes each ckpt_every-step segment from its
 * checkpoint into context-owned scratch, then runs the per-step
 * vector-Jacobian products backwards.  Gradient sums are reduced in a fixed
 * order: results are bitwise reproducible for a given input.            */

/* Bytes of tape for a trace of n_sets sets of the camera's frame
 * (0 on invalid arguments). */
size_t rt_tape_bytes(const rt_camera *camera, int n_sets, int max_steps, int ckpt_every);

/* rt_trace plus the tape.  ckpt_every in 1..max_steps.  RT_EUNSUPPORTED
 * unless the metric is GRAPH_GAUSS with 1..16 bumps and the rule is RK4;
 * RT_EINVAL if tape_bytes < rt_tape_bytes(...).  The context remembers the
 * call (camera, rule, tape) for rt_trace_bwd. */
rt_status rt_trace_fwd_ckpt(rt_ctx *ctx, const rt_camera *camera, const rt_step_rule *rule, int max_steps,
                            int ckpt_every, const rt_outputs *out, void *tape, size_t tape_bytes,
                            void *hip_stream);

/* Masked L2 loss per set, loss[set] = sum_p m_p |hit_p - target_p|^2 with
 * m_p = (id_p >= 0) && (id_p == target_id_p) && (mask == NULL || mask[p]),
 * and grad_hit_p = 2 m_p (hit_p - target_p) (grad_hit may be NULL).  All
 * arrays are device arrays indexed like rt_outputs ([set][row][column]);
 * loss has n_sets floats. */
rt_status rt_loss_l2(rt_ctx *ctx, const rt_camera *camera, const float *hit, const int32_t *id,
                     const float *target_hit, const int32_t *target_id, const uint8_t *mask, float *loss,
                     float *grad_hit, void *hip_stream);

/* Gradient of sum_p grad_hit_p . hit_p with respect to the bump parameters,
 * written to grad_params [n_sets][n_bumps][5] (device).  tape must be the
 * tape of the last rt_trace_fwd_ckpt on this context, with the metric and
 * the scene unchanged since (RT_ESTATE otherwise, before any launch). */
rt_status rt_trace_bwd(rt_ctx *ctx, const void *tape, const float *grad_hit, float *grad_params, void *hip_stream);

/* ------------------------------------------------------------- surrogate
 * Learned crossing map of one bump's support sphere: an MLP
 * 6 -> 256 -> 256 -> 256 -> 6 with SiLU hidden activations.  The two
 * 256x256 products run on the BF16 matrix cores with FP32 accumulation
 * (W2, W3 from a bf16 copy of the parameters, uint16 bit patterns in the
 * same layout; their inputs h1, h2 rounded to bf16); the first layer
 * (K = 6) and the output layer (N = 6) run in FP32 from the FP32 master,
 * as do all biases.  Parameters of one network, in this order
 * (RT_MLP_PARAMS floats): W1[256][6], b1[256], W2[256][256], b2[256],
 * W3[256][256], b3[256], W4[6][256], b4[6]  (h = silu(W x + b)).
 * Several networks (n_nets) are processed in one launch, each on its own
 * batch rows: x [n_nets][batch][6]. */
#define RT_MLP_PARAMS 134918

/* Bytes of device workspace for rt_mlp_fwd/rt_mlp_bwd at this size. */
size_t rt_mlp_work_bytes(int n_nets, int batch);

/* y = MLP(x) per network; the workspace keeps the activations for a
 * following rt_mlp_bwd with the same sizes and workspace. */
rt_status rt_mlp_fwd(rt_ctx *ctx, int n_nets, int batch, const uint16_t *w_bf16, const float *params,
                     const float *x, float *y, void *work, size_t work_bytes, void *hip_stream);

/* Inference forward for rows grouped by network (the kernel the tracer
 * runs on its crossings): network g maps rows [off_g, off_g + rows[g]) of
 * x [sum rows][6] to y [sum rows][6], off_g = rows[0] + ... + rows[g-1].
 * rows is a host array [n_nets], n_nets <= 64; same rounding points as
 * rt_mlp_fwd. */
rt_status rt_mlp_fwd_grouped(rt_ctx *ctx, int n_nets, const int32_t *rows, const uint16_t *w_bf16,
                             const float *params, const float *x, float *y, void *hip_stream);

/* grad [n_nets][RT_MLP_PARAMS] = d/dparams of sum_rows dy . y, for the
 * activations stored in work by the last rt_mlp_fwd with the same weights.
 * Reductions over rows run in a fixed order. */
rt_status rt_mlp_bwd(rt_ctx *ctx, int n_nets, int batch, const uint16_t *w_bf16, const float *params, const float *dy,
                     float *grad, void *work, size_t work_bytes, void *hip_stream);

/* Mean-squared-error gradient for training: dy = 2 (y - t) / batch over n
 * values (device arrays), and 64 partial sums of (y - t)^2 written to
 * sq_partial[64] (their sum / batch is the loss); fixed summation order. */
rt_status rt_mse_grad(rt_ctx *ctx, const float *y, const float *t, float *dy, size_t n, int batch, float *sq_partial,
                      void *hip_stream);

/* AdamW with bias correction (step >= 1) on n FP32 parameters; refreshes
 * the bf16 copy. */
rt_status rt_adamw_step(rt_ctx *ctx, float *params, uint16_t *w_bf16, float *m, float *v, const float *grad, size_t n,
                        float lr, float beta1, float beta2, float eps, float weight_decay, int step, void *hip_stream);

/* Training data for the surrogate networks (one per bump shape kappa =
 * a / sigma; the metric depends on |kappa| only): n_per_shape single-bump
 * geodesics per shape, integrated with RK4 (step h in units of sigma, the
 * graph-metric acceleration of Eq. 5.4) from the support sphere of radius
 * 3 sigma to the exit, which is refined by bisection.  In the canonical
 * frame the entry point is (3, 0, 0) and the direction (-cos th, sin th, 0).
 * mode 0: sin^2 th uniform in [0, 1) from a counter-based generator of
 * (seed, shape, sample), i.e. entry points uniform over the disc of impact
 * parameters; mode 1: cos th = i / (n_per_shape - 1); mode 2: sin th
 * uniform in [0, 1) (impact parameters uniform); mode 4 or 6: as 0 or 2
 * with stratified draws, sample i in stratum i of n_per_shape equal strata
 * of the uniform variable (the training loop's draws).  kappa and scale
 * are host arrays [n_shapes]; outputs are device arrays:
 *   x   [n_shapes][n_per_shape][6]  network input (1, 0, 0, -cos th, sin th, 0)
 *   y   [n_shapes][n_per_shape][6]  target: (exit point / 3 - (-cos 2th, sin 2th, 0),
 *                                   unit exit direction - input direction) / scale[shape]
 *   aux [n_shapes][n_per_shape][4]  impact parameter 3 sin th, arc length inside
 *                                   the sphere (units of sigma; -1 if the
 *                                   ray did not exit), exit / 3 (x, y) */
rt_status rt_surrogate_gen(rt_ctx *ctx, int n_shapes, const float *kappa, const float *scale, int n_per_shape,
                           float h, int mode, uint64_t seed, float *x, float *y, float *aux, void *hip_stream);

/* The whole training loop of the surrogate networks in one call (the
 * sequence rt_surrogate_gen -> rt_mlp_fwd -> rt_mse_grad -> rt_mlp_bwd ->
 * rt_adamw_step, n_steps times, enqueued from the host without
 * synchronising).  Every step uses batch fresh crossings per shape (mode 0
 * or 2 of rt_surrogate_gen, step h), drawn 16 steps at a time with seed
 * seed + 1000003 (c + 1) for the c-th group of 16 steps, stratified: the
 * 16 batch draws of a group split [0, 1) into 16 batch equal strata of the
 * uniform variable, one draw in each, and step j of the group takes the
 * strata congruent to j modulo 16; step s (1-based) uses the
 * learning rate lr s / warmup for s <= warmup, then a cosine decay from lr
 * to lr_min.  kappa, scale: host [n_nets].  params (FP32 master), w_bf16,
 * adam_m, adam_v: device [n_nets][RT_MLP_PARAMS], updated in place.
 * work: at least rt_surrogate_train_bytes(n_nets, batch) bytes of device
 * memory.  loss_log: device float[n_log][64] or NULL: for every step s
 * with s % log_every == 0 (s <= n_steps), row s / log_every - 1 receives
 * the 64 partial sums of squares of that step (their sum / (batch n_nets)
 * is the mean loss per network). */
size_t rt_surrogate_train_bytes(int n_nets, int batch);
rt_status rt_surrogate_train(rt_ctx *ctx, int n_nets, const float *kappa, const float *scale, int batch, int n_steps,
                             float h, int mode, uint64_t seed, float lr, float lr_min, int warmup, float beta1,
                             float beta2, float eps, float weight_decay, float *params, uint16_t *w_bf16,
                             float *adam_m, float *adam_v, void *work, size_t work_bytes, float *loss_log,
                             int log_every, void *hip_stream);

/* Calibration of the surrogate's error bounds: for predictions `pred` and
 * targets `target` (scaled residuals as produced by rt_surrogate_gen, both
 * [n_shapes][n_per_shape][6], inputs x as produced there), the maximum over
 * samples of the decoded exit-point error and unit-direction error, per bin
 * of cos th (n_bins equal bins of [0, 1]), written to err
 * [n_shapes][n_bins][2] (device).  scale is a host array [n_shapes]. */
rt_status rt_surrogate_calibrate(rt_ctx *ctx, int n_shapes, int n_per_shape, const float *x, const float *pred,
                                 const float *target, const float *scale, int n_bins, float *err, void *hip_stream);

/* Hand trained networks to the tracer (used by traces with
 * RT_FLAG_SURROGATE).  The context copies everything:
 *   w_bf16 [n_nets][RT_MLP_PARAMS], params [n_nets][RT_MLP_PARAMS] (device)
 *   scale  [n_nets] (host)  target scale of each network
 *   arc    [n_nets][n_tab] (device)  arc length through the sphere in units
 *          of sigma at cos th = i / (n_tab - 1), n_tab >= 2
 *   err    [n_nets][n_bins][2] (device)  calibrated error bounds
 *   net_of_bump [n_bumps] (host)  network of every bump of the current
 *          metric, -1 for none; checked against the metric at trace time
 *   tol    probe tolerance on the estimated hit error (scene units).
 * A bump is eligible when its support sphere (radius 3 sigma) meets no
 * object and no other bump's cut sphere; eligibility is recomputed when the
 * metric or scene changes.  n_nets = 0 unloads.  At most 64 networks. */
rt_status rt_surrogate_load(rt_ctx *ctx, int n_nets, const uint16_t *w_bf16, const float *params, const float *scale,
                            const float *arc, int n_tab, const float *err, int n_bins, const int32_t *net_of_bump,
                            int n_bumps, float tol);

#ifdef __cplusplus
}
#endif
#endif /* RT_H */
