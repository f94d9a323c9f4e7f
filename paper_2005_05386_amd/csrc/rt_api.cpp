// C-ABI of the tracer: argument validation, device copies of the metric and
// scene, the per-context workspace, launch sizing and statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rt.h"
#include "rt_internal.hpp"

namespace {
thread_local std::string g_create_error;

constexpr int MAX_BUMPS = 64, MAX_SETS = 64, MAX_SPHERES = 256, MAX_PLANES = 8, MAX_TORI = 8;
}  // namespace

struct rt_ctx {
    int device = -1;
    bool host_only = true;
    std::string err;
    int n_cu = 256;
    // metric (host copy)
    bool has_metric = false;
    int kind = 0, n_sets = 1, n_bumps = 0;
    float amp = 0.f, th0 = 0.f, cull = 6.f;
    std::vector<rt_bump> bumps;
    // PULLBACK_DEFORM: bound on the Euclidean speed of a g-unit velocity
    // (may be infinite) and on the displacement |Phi(x) - x|
    double deform_vmax = 1.0, deform_disp = 0.0;
    bool deform_rot = false;  // some deformation's field rotates
    // scene (host copy)
    bool has_scene = false;
    std::vector<rt_sphere> sph;
    std::vector<rt_plane> pln;
    std::vector<rt_torus> tor;
    // device copies
    void *d_bump_f = nullptr, *d_bump_d = nullptr, *d_scene = nullptr;
    size_t bump_f_bytes = 0, bump_d_bytes = 0, scene_bytes = 0;
    rti::DeviceData dd{};
    // workspace (grow-only)
    float *d_st = nullptr;             // ray state, Q_NFIELDS x ws_cap
    int *d_ids[2] = {nullptr, nullptr};  // survivor lists, ws_cap + 64 * MAX_SETS each
    unsigned long long *d_cmask = nullptr;
    int *d_cscan = nullptr, *d_bscan = nullptr;
    float4 *d_rec = nullptr;           // refine records, ws_cap
    int64_t ws_cap = 0;                // ray ids the workspace holds
    int *d_ctr = nullptr;
    unsigned long long *d_stats = nullptr;
    // static workspace of rt_trace_noalloc on this device (looked up at create)
    void *d_noalloc = nullptr;
    hipError_t noalloc_err = hipErrorNotInitialized;
    hipStream_t last_stream = nullptr;
    bool traced = false;
    int last_passes = 0;
    bool last_timed = false;
    bool last_surr = false;       // the last trace ran the crossing stages
    bool last_surr_flag = false;  // it was asked for the surrogate
    std::vector<hipEvent_t> ev;  // timing events of the last trace
    // differentiation
    bool adj_valid = false;
    const void *adj_tape = nullptr;
    rti::TraceArgs adj_args{};
    float *d_adj_scr = nullptr, *d_adj_part = nullptr, *d_loss_blk = nullptr;
    int64_t adj_scr_cap = 0, adj_part_cap = 0, loss_cap = 0;
    // surrogate
    void *d_gen_ks = nullptr;
    size_t gen_ks_bytes = 0;
    int surr_nets = 0, surr_tab = 0, surr_bins = 0;
    float surr_tol = 1e-3f;
    std::vector<float> surr_scale;
    std::vector<int> surr_net_of_bump;
    void *d_surr = nullptr;            // networks and tables (context copy)
    size_t surr_bytes = 0;
    rti::SurrArgs surr{};
    void *d_surr_sb = nullptr;         // per-bump eligibility records
    size_t surr_sb_bytes = 0;
    bool surr_sb_dirty = true;
    int surr_eligible = 0;
    void *d_grp_ctl = nullptr;         // control block of rt_mlp_fwd_grouped
    size_t grp_ctl_bytes = 0;
    void *d_grp_w = nullptr;           // its aligned copy of the networks
    size_t grp_w_bytes = 0;
    void *d_xbuf = nullptr;            // crossing queues, sized for xbuf_cap rays
    int64_t xbuf_cap = 0;
    void *d_ibuf = nullptr;            // illumination workspace, sized for ibuf_cap pixels
    int64_t ibuf_cap = 0;
};

static rt_status fail(rt_ctx *c, rt_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

static rt_status hip_fail(rt_ctx *c, hipError_t e, const char *what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, e == hipErrorOutOfMemory ? RT_ENOMEM : RT_EDEVICE, m);
}

static bool finite(float v) { return std::isfinite(v); }

extern "C" {

int rt_abi_version(void) { return RT_ABI_VERSION; }

rt_status rt_create(int hip_device, rt_ctx **out) {
    if (!out) {
        g_create_error = "rt_create: out is NULL";
        return RT_EINVAL;
    }
    *out = nullptr;
    g_create_error.clear();
    if (hip_device < -1) {
        g_create_error = "rt_create: device must be >= -1";
        return RT_EINVAL;
    }
    rt_ctx *c = new (std::nothrow) rt_ctx();
    if (!c) {
        g_create_error = "rt_create: out of host memory";
        return RT_ENOMEM;
    }
    if (hip_device >= 0) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess || hip_device >= n) {
            g_create_error = std::string("rt_create: no HIP device ") + std::to_string(hip_device) + " (" +
                             (e != hipSuccess ? hipGetErrorString(e) : "index out of range") + ")";
            delete c;
            return RT_EDEVICE;
        }
        hipDeviceProp_t prop;
        if ((e = hipSetDevice(hip_device)) != hipSuccess || (e = hipGetDeviceProperties(&prop, hip_device)) != hipSuccess) {
            g_create_error = std::string("rt_create: ") + hipGetErrorString(e);
            delete c;
            return RT_EDEVICE;
        }
        c->device = hip_device;
        c->host_only = false;
        c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
        e = hipMalloc((void **)&c->d_stats, sizeof(unsigned long long) * rti::ST_N);
        if (e != hipSuccess) {
            g_create_error = std::string("rt_create: ") + hipGetErrorString(e);
            delete c;
            return RT_ENOMEM;
        }
        e = hipMemset(c->d_stats, 0, sizeof(unsigned long long) * rti::ST_N);
        if (e != hipSuccess) {
            g_create_error = std::string("rt_create: ") + hipGetErrorString(e);
            (void)hipFree(c->d_stats);
            delete c;
            return RT_EDEVICE;
        }
        // address of the allocation-free trace's workspace on this device;
        // a failure is reported by rt_trace_noalloc, the only user
        c->noalloc_err = rti::noalloc_scratch(hip_device, &c->d_noalloc);
    }
    *out = c;
    return RT_OK;
}

void rt_destroy(rt_ctx *c) {
    if (!c) return;
    if (!c->host_only) {
        // best effort: a destroy reports nothing, and frees what it can
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        (void)hipFree(c->d_bump_f);
        (void)hipFree(c->d_bump_d);
        (void)hipFree(c->d_scene);
        (void)hipFree(c->d_st);
        (void)hipFree(c->d_ids[0]);
        (void)hipFree(c->d_ids[1]);
        (void)hipFree(c->d_cmask);
        (void)hipFree(c->d_cscan);
        (void)hipFree(c->d_bscan);
        (void)hipFree(c->d_rec);
        (void)hipFree(c->d_ctr);
        (void)hipFree(c->d_stats);
        (void)hipFree(c->d_adj_scr);
        (void)hipFree(c->d_adj_part);
        (void)hipFree(c->d_loss_blk);
        (void)hipFree(c->d_gen_ks);
        (void)hipFree(c->d_surr);
        (void)hipFree(c->d_surr_sb);
        (void)hipFree(c->d_xbuf);
        (void)hipFree(c->d_ibuf);
        (void)hipFree(c->d_grp_ctl);
        (void)hipFree(c->d_grp_w);
        for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    }
    delete c;
}

const char *rt_last_error(const rt_ctx *c) {
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

static rt_status sync_last(rt_ctx *c) {
    if (c->host_only || !c->traced) return RT_OK;
    hipError_t e = hipStreamSynchronize(c->last_stream);
    if (e != hipSuccess) return hip_fail(c, e, "stream synchronize");
    return RT_OK;
}

static rt_status upload(rt_ctx *c, void **dst, size_t *cap, const void *src, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (*cap < bytes) {
        (void)hipFree(*dst);
        *dst = nullptr;
        *cap = 0;
        hipError_t e = hipMalloc(dst, bytes);
        if (e != hipSuccess) return hip_fail(c, e, "hipMalloc");
        *cap = bytes;
    }
    hipError_t e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "hipMemcpy");
    return RT_OK;
}

// Composition of local deformations (Sec. 6.2).  Device tables, per
// deformation (Phi_1 first):
//   float: (cx, cy, cz, a), (1/sx^2, 1/sy^2, 1/sz^2, 0), (vx, vy, vz, cut2),
//          ((rb - cull_sigmas * max spread) / min spread, |a| |v|, 1 / min spread, 0)
//   double: cx, cy, cz, a, 1/sx^2, 1/sy^2, 1/sz^2, cut2, vx, vy, vz, 0
// cut2 = cull_sigmas^2 bounds the spread-scaled squared distance at which
// Phi_i acts.  rb is the radius of a ball about c in the coordinates of the
// ray that contains every point p whose image under the deformations applied
// before Phi_i (Phi_{i+1} ... Phi_k) falls where Phi_i acts: Phi_j moves
// points by at most |a_j| |v_j|, and only inside its own ball, so each
// earlier deformation whose ball meets the current one widens it by that
// much.  Two bounds limit how far a ray moves in a culling window of
// duration T.  A g-unit velocity has Euclidean speed at most
// 1 / sigma_min(J), sigma_min(J_j) >= 1 - |a_j| |v_j| exp(-1/2) / min spread,
// and a point lies only in balls that meet each other, so the product of
// 1 / (1 - kappa_j) over the balls meeting one ball bounds the speed.  And a
// geodesic is the preimage of a unit-speed straight line (Sec. 5.2), so it
// moves at most T + 2 max |Phi(x) - x|, the displacement being at most the
// sum of |a_j| |v_j| over the balls meeting one ball.
// Kernel variant of the context's metric: composed deformations with a
// rotating field run the rotating chain's instantiation.
static int kernel_kind(const rt_ctx *c) {
    return c->kind == RT_METRIC_PULLBACK_DEFORM && c->deform_rot ? rti::KERNEL_KIND_DEFORM_ROT : c->kind;
}

static rt_status set_deform_metric(rt_ctx *c, const rt_metric *m) {
    const int nd = m->n_deforms;
    if (nd < 1 || nd > MAX_BUMPS) return fail(c, RT_EINVAL, "rt_set_metric: n_deforms must be in 1..64");
    if (!m->deforms) return fail(c, RT_EINVAL, "rt_set_metric: deforms is NULL");
    if (!finite(m->cull_sigmas) || m->cull_sigmas < 4.0f)
        return fail(c, RT_EINVAL, "rt_set_metric: cull_sigmas must be finite and >= 4");
    const size_t n = (size_t)m->n_sets * nd;
    const double e_half = std::exp(-0.5);
    // Lipschitz bound of f V for a field with a rotation part: with rho the
    // spread-scaled distance, |grad f| <= |a| rho exp(-rho^2/2) / s_min,
    // |d| <= s_max rho and rho^2 exp(-rho^2/2) <= 2/e, so
    // |DF| <= |grad f| (|v| + |om| |d|) + |f| |om|
    //      <= |a| (exp(-1/2) |v| / s_min + |om| (2/e s_max / s_min + 1)).
    auto lip = [&](const rt_deform &d) {
        const double smax = std::max(d.sx, std::max(d.sy, d.sz)), smin = std::min(d.sx, std::min(d.sy, d.sz));
        const double vn = std::sqrt((double)d.vx * d.vx + (double)d.vy * d.vy + (double)d.vz * d.vz);
        const double on = std::sqrt((double)d.wx * d.wx + (double)d.wy * d.wy + (double)d.wz * d.wz);
        return std::fabs((double)d.a) * (e_half * vn / smin + on * (2.0 / std::exp(1.0) * smax / smin + 1.0));
    };
    auto rotates = [](const rt_deform &d) { return d.wx != 0.f || d.wy != 0.f || d.wz != 0.f; };
    for (size_t i = 0; i < n; ++i) {
        const rt_deform &d = m->deforms[i];
        const float v[13] = {d.a, d.cx, d.cy, d.cz, d.sx, d.sy, d.sz, d.vx, d.vy, d.vz, d.wx, d.wy, d.wz};
        for (float x : v)
            if (!finite(x)) return fail(c, RT_EINVAL, "rt_set_metric: non-finite deformation parameter at " + std::to_string(i));
        if (!(d.sx > 0.f && d.sy > 0.f && d.sz > 0.f))
            return fail(c, RT_EINVAL, "rt_set_metric: spreads must be > 0 at deformation " + std::to_string(i));
        if (rotates(d)) {
            if (lip(d) > 0.95)
                return fail(c, RT_EINVAL, "rt_set_metric: deformation " + std::to_string(i) +
                                              " is not a diffeomorphism with margin (need the Lipschitz bound "
                                              "|a| (exp(-1/2) |v| / s_min + |w| (2/e s_max / s_min + 1)) <= 0.95)");
            continue;
        }
        const double q = (double)d.vx * d.vx / ((double)d.sx * d.sx) + (double)d.vy * d.vy / ((double)d.sy * d.sy) +
                         (double)d.vz * d.vz / ((double)d.sz * d.sz);
        if (std::fabs((double)d.a) * std::sqrt(q) * e_half > 0.95)
            return fail(c, RT_EINVAL, "rt_set_metric: deformation " + std::to_string(i) +
                                          " is not a diffeomorphism with margin (need |a| |v/s| exp(-1/2) <= 0.95)");
    }
    const double cut = m->cull_sigmas;
    constexpr int NF = 4 * rti::DEFORM_F4, ND = rti::DEFORM_D;
    std::vector<float> bf(n * NF, 0.f);
    std::vector<double> bd(n * ND, 0.0);
    double vmax = 1.0, disp = 0.0;
    for (int set = 0; set < m->n_sets; ++set) {
        const rt_deform *D = m->deforms + (size_t)set * nd;
        std::vector<double> R(nd), delta(nd), rb(nd), kap(nd);
        for (int i = 0; i < nd; ++i) {
            const rt_deform &d = D[i];
            const double smax = std::max(d.sx, std::max(d.sy, d.sz)), smin = std::min(d.sx, std::min(d.sy, d.sz));
            const double vn = std::sqrt((double)d.vx * d.vx + (double)d.vy * d.vy + (double)d.vz * d.vz);
            const double on = std::sqrt((double)d.wx * d.wx + (double)d.wy * d.wy + (double)d.wz * d.wz);
            R[i] = cut * smax;
            // the largest displacement |f V| <= |a| (|v| + |om| s_max rho exp(-rho^2/2))
            // <= |a| (|v| + |om| s_max exp(-1/2))
            delta[i] = std::fabs((double)d.a) * (vn + on * smax * e_half);
            // a bound on |J_i - I|
            kap[i] = rotates(d) ? lip(d) : delta[i] * e_half / smin;
        }
        auto dist = [&](int i, int j) {
            const double dx = (double)D[i].cx - D[j].cx, dy = (double)D[i].cy - D[j].cy, dz = (double)D[i].cz - D[j].cz;
            return std::sqrt(dx * dx + dy * dy + dz * dz);
        };
        for (int i = 0; i < nd; ++i) {
            double r = R[i];
            for (int j = i + 1; j < nd; ++j)
                if (dist(i, j) <= r + R[j] + delta[j]) r += delta[j];
            rb[i] = r;
        }
        for (int i = 0; i < nd; ++i) {
            double P = 1.0, S = 0.0;
            for (int j = 0; j < nd; ++j)
                if (dist(i, j) <= rb[i] + rb[j]) {
                    P = kap[j] < 1.0 ? P / (1.0 - kap[j]) : INFINITY;
                    S += delta[j];
                }
            vmax = std::max(vmax, P);
            disp = std::max(disp, S);
        }
        for (int i = 0; i < nd; ++i) {
            const rt_deform &d = D[i];
            const size_t o = ((size_t)set * nd + i);
            const double s[3] = {1.0 / ((double)d.sx * d.sx), 1.0 / ((double)d.sy * d.sy), 1.0 / ((double)d.sz * d.sz)};
            const double smin = std::min(d.sx, std::min(d.sy, d.sz));
            // slack and displacement rounded up so that the float tests stay conservative
            const double smax = std::max(d.sx, std::max(d.sy, d.sz));
            const double av = std::fabs((double)d.a) *
                              std::sqrt((double)d.vx * d.vx + (double)d.vy * d.vy + (double)d.vz * d.vz);
            const double aw = std::fabs((double)d.a) * smax *
                              std::sqrt((double)d.wx * d.wx + (double)d.wy * d.wy + (double)d.wz * d.wz);
            const float f[NF] = {d.cx, d.cy, d.cz, d.a, (float)s[0], (float)s[1], (float)s[2], 0.f,
                                 d.vx, d.vy, d.vz, (float)(cut * cut),
                                 (float)((rb[i] - R[i]) / smin * (1.0 + 1e-6)), (float)(av * (1.0 + 1e-6)),
                                 (float)(1.0 / smin * (1.0 + 1e-6)), (float)(aw * (1.0 + 1e-6)),
                                 d.wx, d.wy, d.wz, 0.f};
            const double g[ND] = {d.cx, d.cy, d.cz, d.a, s[0], s[1], s[2], cut * cut,
                                  d.vx, d.vy, d.vz, 0.0, d.wx, d.wy, d.wz, 0.0};
            std::copy(f, f + NF, bf.begin() + o * NF);
            std::copy(g, g + ND, bd.begin() + o * ND);
        }
    }
    if (!c->host_only) {
        rt_status st = sync_last(c);
        if (st != RT_OK) return st;
        if (hipError_t e = hipSetDevice(c->device); e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
        if ((st = upload(c, &c->d_bump_f, &c->bump_f_bytes, bf.data(), bf.size() * sizeof(float))) != RT_OK) return st;
        if ((st = upload(c, &c->d_bump_d, &c->bump_d_bytes, bd.data(), bd.size() * sizeof(double))) != RT_OK) return st;
        c->dd.bump_f = (const float4 *)c->d_bump_f;
        c->dd.bump_d = (const double *)c->d_bump_d;
    }
    c->kind = m->kind;
    c->n_sets = m->n_sets;
    c->n_bumps = nd;  // parameter records per set
    c->amp = 0.f;
    c->th0 = 0.f;
    c->cull = m->cull_sigmas;
    c->bumps.clear();
    c->deform_vmax = vmax;
    c->deform_disp = disp;
    c->deform_rot = std::any_of(m->deforms, m->deforms + n, rotates);
    c->has_metric = true;
    c->surr_sb_dirty = true;
    c->adj_valid = false;
    c->err.clear();
    return RT_OK;
}

// Graph metrics of anisotropic Gaussian sums and of the quadratic.  Device
// tables: anisotropic bumps as (cx, cy, cz, a), (1/sx^2, 1/sy^2, 1/sz^2,
// cull_sigmas^2) in float and the same eight values in double; the
// quadratic as (qx, qy, qz, 0) in both.
static rt_status set_graph2_metric(rt_ctx *c, const rt_metric *m) {
    if (!finite(m->cull_sigmas) || m->cull_sigmas < 4.0f)
        return fail(c, RT_EINVAL, "rt_set_metric: cull_sigmas must be finite and >= 4");
    std::vector<float> bf;
    std::vector<double> bd;
    int nb = 0;
    if (m->kind == RT_METRIC_GRAPH_ANISO) {
        nb = m->n_abumps;
        if (nb < 0 || nb > MAX_BUMPS) return fail(c, RT_EINVAL, "rt_set_metric: n_abumps must be in 0..64");
        if (nb > 0 && !m->abumps) return fail(c, RT_EINVAL, "rt_set_metric: abumps is NULL");
        const size_t n = (size_t)m->n_sets * nb;
        for (size_t i = 0; i < n; ++i) {
            const rt_abump &b = m->abumps[i];
            const float v[7] = {b.a, b.cx, b.cy, b.cz, b.sx, b.sy, b.sz};
            for (float x : v)
                if (!finite(x)) return fail(c, RT_EINVAL, "rt_set_metric: non-finite bump parameter at " + std::to_string(i));
            if (!(b.sx > 0.f && b.sy > 0.f && b.sz > 0.f))
                return fail(c, RT_EINVAL, "rt_set_metric: spreads must be > 0 at bump " + std::to_string(i));
        }
        const double cut2 = (double)m->cull_sigmas * m->cull_sigmas;
        bf.assign(std::max<size_t>(n, 1) * 8, 0.f);
        bd.assign(std::max<size_t>(n, 1) * 8, 0.0);
        for (size_t i = 0; i < n; ++i) {
            const rt_abump &b = m->abumps[i];
            const double s[3] = {1.0 / ((double)b.sx * b.sx), 1.0 / ((double)b.sy * b.sy), 1.0 / ((double)b.sz * b.sz)};
            const double g[8] = {b.cx, b.cy, b.cz, b.a, s[0], s[1], s[2], cut2};
            for (int k = 0; k < 8; ++k) {
                bf[8 * i + k] = (float)g[k];
                bd[8 * i + k] = g[k];
            }
        }
    } else {
        if (m->n_sets != 1) return fail(c, RT_EINVAL, "rt_set_metric: the quadric metric takes one parameter set");
        for (int k = 0; k < 3; ++k)
            if (!finite(m->quadric[k]) || std::fabs(m->quadric[k]) > 100.f)
                return fail(c, RT_EINVAL, "rt_set_metric: quadric coefficients must be finite with |q| <= 100");
        bf = {m->quadric[0], m->quadric[1], m->quadric[2], 0.f, 0.f, 0.f, 0.f, 0.f};
        bd = {m->quadric[0], m->quadric[1], m->quadric[2], 0.0, 0.0, 0.0, 0.0, 0.0};
    }
    if (!c->host_only) {
        rt_status st = sync_last(c);
        if (st != RT_OK) return st;
        if (hipError_t e = hipSetDevice(c->device); e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
        if ((st = upload(c, &c->d_bump_f, &c->bump_f_bytes, bf.data(), bf.size() * sizeof(float))) != RT_OK) return st;
        if ((st = upload(c, &c->d_bump_d, &c->bump_d_bytes, bd.data(), bd.size() * sizeof(double))) != RT_OK) return st;
        c->dd.bump_f = (const float4 *)c->d_bump_f;
        c->dd.bump_d = (const double *)c->d_bump_d;
    }
    c->kind = m->kind;
    c->n_sets = m->n_sets;
    c->n_bumps = nb;
    c->amp = 0.f;
    c->th0 = 0.f;
    c->cull = m->cull_sigmas;
    c->bumps.clear();
    c->has_metric = true;
    c->surr_sb_dirty = true;
    c->adj_valid = false;
    c->err.clear();
    return RT_OK;
}

rt_status rt_set_metric(rt_ctx *c, const rt_metric *m) {
    if (!c) return RT_EINVAL;
    if (!m) return fail(c, RT_EINVAL, "rt_set_metric: metric is NULL");
    if (m->kind < RT_METRIC_EUCLID || m->kind > RT_METRIC_GRAPH_QUADRIC)
        return fail(c, RT_EUNSUPPORTED, "rt_set_metric: unknown metric kind " + std::to_string(m->kind));
    if (m->n_sets < 1 || m->n_sets > MAX_SETS)
        return fail(c, RT_EINVAL, "rt_set_metric: n_sets must be in 1..64");
    if (m->kind == RT_METRIC_PULLBACK_DEFORM) return set_deform_metric(c, m);
    if (m->kind == RT_METRIC_GRAPH_ANISO || m->kind == RT_METRIC_GRAPH_QUADRIC) return set_graph2_metric(c, m);
    int nb = m->kind == RT_METRIC_GRAPH_GAUSS ? m->n_bumps : 0;
    if (nb < 0 || nb > MAX_BUMPS) return fail(c, RT_EINVAL, "rt_set_metric: n_bumps must be in 0..64");
    if (nb > 0 && !m->bumps) return fail(c, RT_EINVAL, "rt_set_metric: bumps is NULL");
    if (!finite(m->cull_sigmas) || m->cull_sigmas < 4.0f)
        return fail(c, RT_EINVAL, "rt_set_metric: cull_sigmas must be finite and >= 4");
    if (m->kind == RT_METRIC_PULLBACK_TWIST) {
        if (!finite(m->twist_amp) || m->twist_amp < 0.f || m->twist_amp > 1.f)
            return fail(c, RT_EINVAL, "rt_set_metric: twist_amp must be in [0, 1]");
        if (!finite(m->twist_theta0) || std::fabs(m->twist_theta0) > 1.5f)
            return fail(c, RT_EINVAL, "rt_set_metric: |twist_theta0| must be <= 1.5");
    }
    size_t n = (size_t)m->n_sets * nb;
    for (size_t i = 0; i < n; ++i) {
        const rt_bump &b = m->bumps[i];
        if (!finite(b.a) || !finite(b.cx) || !finite(b.cy) || !finite(b.cz) || !finite(b.sigma))
            return fail(c, RT_EINVAL, "rt_set_metric: non-finite bump parameter at " + std::to_string(i));
        if (!(b.sigma > 0.f)) return fail(c, RT_EINVAL, "rt_set_metric: sigma must be > 0 at " + std::to_string(i));
    }
    std::vector<float> bf(std::max<size_t>(n, 1) * 8, 0.f);
    std::vector<double> bd(std::max<size_t>(n, 1) * 8, 0.0);
    const double log2e = 1.4426950408889634;
    for (size_t i = 0; i < n; ++i) {
        const rt_bump &b = m->bumps[i];
        double s = b.sigma;
        double cut = (double)m->cull_sigmas * s;
        bf[8 * i + 0] = b.cx;
        bf[8 * i + 1] = b.cy;
        bf[8 * i + 2] = b.cz;
        bf[8 * i + 3] = (float)(-log2e / (2.0 * s * s));
        bf[8 * i + 4] = (float)((double)b.a / (s * s));
        bf[8 * i + 5] = (float)(1.0 / (s * s));
        bf[8 * i + 6] = (float)(cut * cut);
        bf[8 * i + 7] = b.sigma;
        bd[8 * i + 0] = b.a;
        bd[8 * i + 1] = b.cx;
        bd[8 * i + 2] = b.cy;
        bd[8 * i + 3] = b.cz;
        bd[8 * i + 4] = b.sigma;
        bd[8 * i + 5] = cut * cut;
        bd[8 * i + 6] = 1.0 / (s * s);
        bd[8 * i + 7] = (double)b.a * bd[8 * i + 6];
    }
    if (!c->host_only) {
        rt_status st = sync_last(c);
        if (st != RT_OK) return st;
        if (hipError_t e = hipSetDevice(c->device); e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
        if ((st = upload(c, &c->d_bump_f, &c->bump_f_bytes, bf.data(), bf.size() * sizeof(float))) != RT_OK) return st;
        if ((st = upload(c, &c->d_bump_d, &c->bump_d_bytes, bd.data(), bd.size() * sizeof(double))) != RT_OK) return st;
        c->dd.bump_f = (const float4 *)c->d_bump_f;
        c->dd.bump_d = (const double *)c->d_bump_d;
    }
    c->kind = m->kind;
    c->n_sets = m->n_sets;
    c->n_bumps = nb;
    c->amp = m->twist_amp;
    c->th0 = m->twist_theta0;
    c->cull = m->cull_sigmas;
    c->bumps.assign(m->bumps, m->bumps + n);
    c->has_metric = true;
    c->surr_sb_dirty = true;
    c->adj_valid = false;
    c->err.clear();
    return RT_OK;
}

rt_status rt_set_scene(rt_ctx *c, const rt_scene *s) {
    if (!c) return RT_EINVAL;
    if (!s) return fail(c, RT_EINVAL, "rt_set_scene: scene is NULL");
    if (s->n_spheres < 0 || s->n_spheres > MAX_SPHERES) return fail(c, RT_EINVAL, "rt_set_scene: n_spheres must be in 0..256");
    if (s->n_planes < 0 || s->n_planes > MAX_PLANES) return fail(c, RT_EINVAL, "rt_set_scene: n_planes must be in 0..8");
    if (s->n_tori < 0 || s->n_tori > MAX_TORI) return fail(c, RT_EINVAL, "rt_set_scene: n_tori must be in 0..8");
    if ((s->n_spheres && !s->spheres) || (s->n_planes && !s->planes) || (s->n_tori && !s->tori))
        return fail(c, RT_EINVAL, "rt_set_scene: NULL object array");
    for (int i = 0; i < s->n_spheres; ++i) {
        const rt_sphere &o = s->spheres[i];
        if (!finite(o.cx) || !finite(o.cy) || !finite(o.cz) || !finite(o.r) || !(o.r > 0.f))
            return fail(c, RT_EINVAL, "rt_set_scene: bad sphere " + std::to_string(i));
    }
    for (int i = 0; i < s->n_planes; ++i) {
        const rt_plane &o = s->planes[i];
        float n2 = o.nx * o.nx + o.ny * o.ny + o.nz * o.nz;
        if (!finite(o.nx) || !finite(o.ny) || !finite(o.nz) || !finite(o.d) || std::fabs(n2 - 1.f) > 1e-4f)
            return fail(c, RT_EINVAL, "rt_set_scene: bad plane " + std::to_string(i) + " (need |n| = 1)");
    }
    for (int i = 0; i < s->n_tori; ++i) {
        const rt_torus &o = s->tori[i];
        float a2 = o.ax * o.ax + o.ay * o.ay + o.az * o.az;
        bool ok = finite(o.cx) && finite(o.cy) && finite(o.cz) && finite(o.ax) && finite(o.ay) && finite(o.az) &&
                  finite(o.R) && finite(o.r) && std::fabs(a2 - 1.f) <= 1e-4f && o.r > 0.f && o.R > o.r;
        if (!ok) return fail(c, RT_EINVAL, "rt_set_scene: bad torus " + std::to_string(i));
    }
    if (!c->host_only) {
        // one allocation: f32 spheres | f32 planes | f32 tori | f64 spheres | f64 planes | f64 tori
        size_t ns = s->n_spheres, np = s->n_planes, nt = s->n_tori;
        size_t off_pf = ns * 16, off_tf = off_pf + np * 16, end_f = off_tf + nt * 32;
        size_t off_sd = (end_f + 255) & ~(size_t)255;
        size_t off_pd = off_sd + ns * 32, off_td = off_pd + np * 32, total = off_td + nt * 64;
        std::vector<char> buf(total + 16, 0);
        float *f = (float *)buf.data();
        for (size_t i = 0; i < ns; ++i) std::memcpy(f + 4 * i, &s->spheres[i], 16);
        std::memcpy(buf.data() + off_pf, s->planes, np * 16);
        std::memcpy(buf.data() + off_tf, s->tori, nt * 32);
        double *sd = (double *)(buf.data() + off_sd);
        for (size_t i = 0; i < ns; ++i) {
            sd[4 * i + 0] = s->spheres[i].cx;
            sd[4 * i + 1] = s->spheres[i].cy;
            sd[4 * i + 2] = s->spheres[i].cz;
            sd[4 * i + 3] = s->spheres[i].r;
        }
        double *pd = (double *)(buf.data() + off_pd);
        for (size_t i = 0; i < np; ++i) {
            pd[4 * i + 0] = s->planes[i].nx;
            pd[4 * i + 1] = s->planes[i].ny;
            pd[4 * i + 2] = s->planes[i].nz;
            pd[4 * i + 3] = s->planes[i].d;
        }
        double *td = (double *)(buf.data() + off_td);
        for (size_t i = 0; i < nt; ++i) {
            const float *t = &s->tori[i].cx;
            for (int k = 0; k < 8; ++k) td[8 * i + k] = t[k];
        }
        rt_status st = sync_last(c);
        if (st != RT_OK) return st;
        if (hipError_t e = hipSetDevice(c->device); e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
        if ((st = upload(c, &c->d_scene, &c->scene_bytes, buf.data(), buf.size())) != RT_OK) return st;
        char *b = (char *)c->d_scene;
        c->dd.sph_f = (const float4 *)b;
        c->dd.pln_f = (const float4 *)(b + off_pf);
        c->dd.tor_f = (const float *)(b + off_tf);
        c->dd.sph_d = (const double *)(b + off_sd);
        c->dd.pln_d = (const double *)(b + off_pd);
        c->dd.tor_d = (const double *)(b + off_td);
    }
    c->sph.assign(s->spheres, s->spheres + s->n_spheres);
    c->pln.assign(s->planes, s->planes + s->n_planes);
    c->tor.assign(s->tori, s->tori + s->n_tori);
    c->has_scene = true;
    c->surr_sb_dirty = true;
    // the implicit hit of a taped forward refers to objects of the old
    // scene (the table is re-laid out): the tape can no longer be reversed
    c->adj_valid = false;
    c->err.clear();
    return RT_OK;
}

// Chunks of one pass: every set's survivor list is padded to whole chunks.
static int64_t max_chunks_for(int64_t cap) { return cap / 64 + MAX_SETS; }

static void free_workspace(rt_ctx *c) {
    (void)hipFree(c->d_st);
    (void)hipFree(c->d_ids[0]);
    (void)hipFree(c->d_ids[1]);
    (void)hipFree(c->d_cmask);
    (void)hipFree(c->d_cscan);
    (void)hipFree(c->d_bscan);
    (void)hipFree(c->d_rec);
    c->d_st = nullptr;
    c->d_ids[0] = c->d_ids[1] = nullptr;
    c->d_cmask = nullptr;
    c->d_cscan = c->d_bscan = nullptr;
    c->d_rec = nullptr;
    c->ws_cap = 0;
}

// Ray state (Q_NFIELDS floats per ray id), two sorted survivor lists, the
// per-chunk compaction arrays, refine records (REC_F4 float4 per ray) and
// the counter block, sized for `cap` ray ids; grow-only.
static rt_status ensure_workspace(rt_ctx *c, int64_t cap) {
    hipError_t e;
    if (!c->d_ctr) {
        e = hipMalloc((void **)&c->d_ctr, sizeof(int) * (rti::CTR_PASS0 + rti::MAX_PASSES_API * rti::CTR_PASS_WORDS +
                                                         rti::CTR_SURR_WORDS));
        if (e != hipSuccess) return hip_fail(c, e, "hipMalloc (counters)");
    }
    if (c->ws_cap >= cap) return RT_OK;
    rt_status st = sync_last(c);
    if (st != RT_OK) return st;
    free_workspace(c);
    int64_t mch = max_chunks_for(cap);
    size_t list = (size_t)(cap + 64 * MAX_SETS);
    if ((e = hipMalloc((void **)&c->d_st, (size_t)cap * rti::Q_NFIELDS * sizeof(float))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_ids[0], list * sizeof(int))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_ids[1], list * sizeof(int))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_cmask, (size_t)mch * sizeof(unsigned long long))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_cscan, (size_t)mch * sizeof(int))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_bscan, (size_t)(mch / rti::SCAN_BLOCK + 2) * sizeof(int))) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_rec, (size_t)cap * rti::REC_F4 * sizeof(float4))) != hipSuccess) {
        free_workspace(c);
        return hip_fail(c, e, "hipMalloc (workspace)");
    }
    c->ws_cap = cap;
    return RT_OK;
}

// Buffers of one trace.
struct Workspace {
    int *ctr;
    float *st;
    int *ids[2];
    unsigned long long *cmask;
    int *cscan, *bscan;
    float4 *rec;
};

static Workspace context_workspace(rt_ctx *c) {
    return Workspace{c->d_ctr, c->d_st, {c->d_ids[0], c->d_ids[1]}, c->d_cmask, c->d_cscan, c->d_bscan, c->d_rec};
}

// The same buffers carved from one block (the allocation-free trace's static
// array): counter block for n_passes passes | ray state | two survivor lists
// | chunk masks | chunk scans | block scans | refine records, each starting
// on a 256-byte boundary.  Returns the bytes needed; fills *w if base is set.
static size_t carve_workspace(char *base, int64_t cap, int n_passes, Workspace *w) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off = (off + bytes + 255) & ~(size_t)255;
        return p;
    };
    const int64_t mch = max_chunks_for(cap);
    const size_t list = (size_t)(cap + 64 * MAX_SETS);
    char *ctr = take(sizeof(int) * (rti::CTR_PASS0 + (size_t)n_passes * rti::CTR_PASS_WORDS + rti::CTR_SURR_WORDS));
    char *st = take((size_t)cap * rti::Q_NFIELDS * sizeof(float));
    char *i0 = take(list * sizeof(int));
    char *i1 = take(list * sizeof(int));
    char *cm = take((size_t)mch * sizeof(unsigned long long));
    char *cs = take((size_t)mch * sizeof(int));
    char *bs = take((size_t)(mch / rti::SCAN_BLOCK + 2) * sizeof(int));
    char *rc = take((size_t)cap * rti::REC_F4 * sizeof(float4));
    if (w)
        *w = Workspace{(int *)ctr, (float *)st, {(int *)i0, (int *)i1}, (unsigned long long *)cm, (int *)cs, (int *)bs,
                       (float4 *)rc};
    return off;
}

// Eligibility of every bump for the learned crossing (one parameter set):
// its support sphere S (centre c, radius R = 3 sigma) must meet no object and
// lie outside every other bump's cut sphere, so that inside S the culled
// metric is exactly that of the bump alone.  Uploads two float4 per bump:
// (c, R^2), (sigma, network or -1, R, 0).
static rt_status surr_prepare(rt_ctx *c) {
    if (!c->surr_sb_dirty) return RT_OK;
    const int nb = c->n_bumps;
    std::vector<float> sb(std::max(nb, 1) * 8, 0.f);
    int n_el = 0;
    for (int b = 0; b < nb; ++b) {
        const rt_bump &B = c->bumps[b];
        const double R = 3.0 * (double)B.sigma;
        int net = c->surr_net_of_bump[b];
        auto dist = [&](double x, double y, double z) {
            return std::sqrt((B.cx - x) * (B.cx - x) + (B.cy - y) * (B.cy - y) + (B.cz - z) * (B.cz - z));
        };
        if (!(B.a != 0.f)) net = -1;
        for (int j = 0; j < nb && net >= 0; ++j) {
            if (j == b) continue;
            const rt_bump &O = c->bumps[j];
            if (dist(O.cx, O.cy, O.cz) < R + (double)c->cull * O.sigma) net = -1;
        }
        for (const rt_sphere &o : c->sph)
            if (net >= 0 && dist(o.cx, o.cy, o.cz) < R + o.r) net = -1;
        for (const rt_plane &o : c->pln)
            if (net >= 0 && std::fabs(o.nx * B.cx + o.ny * B.cy + o.nz * B.cz - o.d) < R) net = -1;
        for (const rt_torus &o : c->tor) {
            if (net < 0) break;
            // exact distance from the centre to the torus surface
            double px = B.cx - o.cx, py = B.cy - o.cy, pz = B.cz - o.cz;
            double along = px * o.ax + py * o.ay + pz * o.az;
            double qx = px - along * o.ax, qy = py - along * o.ay, qz = pz - along * o.az;
            double rad = std::sqrt(qx * qx + qy * qy + qz * qz) - o.R;
            if (std::sqrt(rad * rad + along * along) - o.r < R) net = -1;
        }
        if (net >= 0) n_el++;
        sb[8 * b + 0] = B.cx;
        sb[8 * b + 1] = B.cy;
        sb[8 * b + 2] = B.cz;
        sb[8 * b + 3] = (float)(R * R);
        sb[8 * b + 4] = B.sigma;
        int32_t nv = net;
        std::memcpy(&sb[8 * b + 5], &nv, 4);
        sb[8 * b + 6] = (float)R;
        sb[8 * b + 7] = 0.f;
    }
    rt_status st = upload(c, &c->d_surr_sb, &c->surr_sb_bytes, sb.data(), sb.size() * sizeof(float));
    if (st != RT_OK) return st;
    c->surr_eligible = n_el;
    c->surr_sb_dirty = false;
    return RT_OK;
}

// Crossing queue (int4), slots (int2), network inputs and outputs (6 floats
// each) for `cap` rays; grow-only.
static rt_status ensure_xbuf(rt_ctx *c, int64_t cap) {
    if (c->xbuf_cap >= cap) return RT_OK;
    rt_status st = sync_last(c);
    if (st != RT_OK) return st;
    (void)hipFree(c->d_xbuf);
    c->d_xbuf = nullptr;
    c->xbuf_cap = 0;
    hipError_t e = hipMalloc(&c->d_xbuf, (size_t)cap * (16 + 8 + 24 + 24) + 1024);
    if (e != hipSuccess) return hip_fail(c, e, "hipMalloc (crossing queues)");
    c->xbuf_cap = cap;
    return RT_OK;
}

// Shared body of rt_trace and rt_trace_fwd_ckpt (tape != NULL).
static rt_status trace_impl(rt_ctx *c, const rt_camera *cam, const rt_step_rule *r, int max_steps, const rt_outputs *o,
                            void *stream, void *tape, size_t tape_bytes, int ckpt_every, bool noalloc = false) {
    if (!c) return RT_EINVAL;
    if (!cam || !r || !o) return fail(c, RT_EINVAL, "rt_trace: NULL camera, rule or outputs");
    if (!c->has_metric || !c->has_scene) return fail(c, RT_ESTATE, "rt_trace: set the metric and the scene first");
    for (int k = 0; k < 3; ++k)
        if (!finite(cam->eye[k]) || !finite(cam->forward[k]) || !finite(cam->up[k]))
            return fail(c, RT_EINVAL, "rt_trace: non-finite camera vector");
    if (!finite(cam->vfov_deg) || cam->vfov_deg <= 0.f || cam->vfov_deg >= 180.f)
        return fail(c, RT_EINVAL, "rt_trace: vfov_deg must be in (0, 180)");
    if (cam->width < 1 || cam->height < 1) return fail(c, RT_EINVAL, "rt_trace: width and height must be >= 1");
    int64_t hw = (int64_t)cam->width * cam->height;
    if (hw * c->n_sets > 2147483647LL) return fail(c, RT_EINVAL, "rt_trace: width*height*n_sets exceeds 2^31-1");
    // camera basis: right = up x forward, up' = forward x right
    double f[3] = {cam->forward[0], cam->forward[1], cam->forward[2]};
    double fn = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(fn > 0)) return fail(c, RT_EINVAL, "rt_trace: zero forward vector");
    for (double &v : f) v /= fn;
    const float *u = cam->up;
    double rt[3] = {u[1] * f[2] - u[2] * f[1], u[2] * f[0] - u[0] * f[2], u[0] * f[1] - u[1] * f[0]};
    double rn = std::sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
    if (!(rn > 1e-12)) return fail(c, RT_EINVAL, "rt_trace: up is parallel to forward");
    for (double &v : rt) v /= rn;
    double up[3] = {f[1] * rt[2] - f[2] * rt[1], f[2] * rt[0] - f[0] * rt[2], f[0] * rt[1] - f[1] * rt[0]};

    if (r->kind < RT_STEP_RK4 || r->kind > RT_STEP_EULER)
        return fail(c, RT_EUNSUPPORTED, "rt_trace: unknown step kind " + std::to_string(r->kind));
    if (!finite(r->h) || !(r->h > 0.f)) return fail(c, RT_EINVAL, "rt_trace: h must be finite and > 0");
    if (!finite(r->t_max) || !(r->t_max > 0.f)) return fail(c, RT_EINVAL, "rt_trace: t_max must be finite and > 0");
    if (r->kind == RT_STEP_RK45) {
        if (!(r->rtol > 0.f) || !(r->atol > 0.f) || !finite(r->rtol) || !finite(r->atol))
            return fail(c, RT_EINVAL, "rt_trace: rtol and atol must be finite and > 0");
        if (!(r->h_min > 0.f) || !(r->h_max >= r->h_min) || !finite(r->h_max))
            return fail(c, RT_EINVAL, "rt_trace: need 0 < h_min <= h_max");
    }
    if (r->cull_every < 1 || r->cull_every > 256) return fail(c, RT_EINVAL, "rt_trace: cull_every must be in 1..256");
    if (r->pass_steps < 16) return fail(c, RT_EINVAL, "rt_trace: pass_steps must be >= 16");
    if (r->bisect_iters < 0 || r->bisect_iters > 60) return fail(c, RT_EINVAL, "rt_trace: bisect_iters must be in 0..60");
    if (r->flags & ~(RT_FLAG_TIMING | RT_FLAG_COUNT_WORK | RT_FLAG_SURROGATE | RT_FLAG_BATCH_SEGMENTS))
        return fail(c, RT_EINVAL, "rt_trace: unknown flag bits");
    const bool batch = (r->flags & RT_FLAG_BATCH_SEGMENTS) != 0;
    if (batch && (r->kind == RT_STEP_RK45 || (r->flags & (RT_FLAG_COUNT_WORK | RT_FLAG_SURROGATE)) || tape))
        return fail(c, RT_EUNSUPPORTED, "rt_trace: batched segments need RK4 or Euler, a plain trace and no tape");
    if (noalloc && (r->flags & (RT_FLAG_TIMING | RT_FLAG_SURROGATE)))
        return fail(c, RT_EUNSUPPORTED, "rt_trace_noalloc: RT_FLAG_TIMING and RT_FLAG_SURROGATE need allocations");
    if (max_steps < 1 || max_steps > 1000000) return fail(c, RT_EINVAL, "rt_trace: max_steps must be in 1..1000000");
    const bool surr = (r->flags & RT_FLAG_SURROGATE) != 0;
    if (surr) {
        if (c->kind != RT_METRIC_GRAPH_GAUSS || r->kind != RT_STEP_RK4 || c->n_sets != 1 || tape)
            return fail(c, RT_EUNSUPPORTED, "rt_trace: the surrogate needs the graph metric, RK4, one parameter set "
                                            "and no tape");
        if (c->surr_nets < 1) return fail(c, RT_ESTATE, "rt_trace: no surrogate networks loaded");
        if ((int)c->surr_net_of_bump.size() != c->n_bumps)
            return fail(c, RT_ESTATE, "rt_trace: surrogate net_of_bump does not match the metric's bump count");
    }
    int n_passes = (max_steps + r->pass_steps - 1) / r->pass_steps;
    if (n_passes > rti::MAX_PASSES_API)
        return fail(c, RT_EINVAL, "rt_trace: max_steps / pass_steps must be <= " + std::to_string(rti::MAX_PASSES_API));
    if (!o->hit || !o->t || !o->id || !o->dir) return fail(c, RT_EINVAL, "rt_trace: NULL output pointer");
    if (c->host_only) return fail(c, RT_ESTATE, "rt_trace: host-only context (created with device -1)");

    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    bool use_surr = surr;
    if (surr) {
        rt_status st0 = surr_prepare(c);
        if (st0 != RT_OK) return st0;
        // no eligible bump: no ray can park, the plain kernels give the same frame
        if (c->surr_eligible == 0) use_surr = false;
    }
    // each learned crossing ends a ray's pass early: allow extra passes
    if (use_surr) n_passes = std::min(n_passes + 1 + std::max(16, 2 * c->n_bumps), rti::MAX_PASSES_API);
    const int tiles_x = (cam->width + 7) / 8, tiles_y = (cam->height + 7) / 8;
    const int64_t T = (int64_t)tiles_x * tiles_y * 64;
    int64_t cap = T * c->n_sets;
    if (cap > 2147483647LL - 4096) return fail(c, RT_EINVAL, "rt_trace: frame too large");
    Workspace ws{};
    rt_status st = RT_OK;
    if (noalloc) {
        size_t need = carve_workspace(nullptr, cap, n_passes, nullptr);
        if (need > RT_NOALLOC_SCRATCH_BYTES)
            return fail(c, RT_EINVAL, "rt_trace_noalloc: the frame needs " + std::to_string(need) +
                                          " bytes of workspace, more than RT_NOALLOC_SCRATCH_BYTES (" +
                                          std::to_string(RT_NOALLOC_SCRATCH_BYTES) + ")");
        if (c->noalloc_err != hipSuccess || !c->d_noalloc)
            return hip_fail(c, c->noalloc_err != hipSuccess ? c->noalloc_err : hipErrorInvalidSymbol,
                            "rt_trace_noalloc: static workspace address");
        carve_workspace((char *)c->d_noalloc, cap, n_passes, &ws);
    } else {
        if ((st = ensure_workspace(c, cap)) != RT_OK) return st;
        ws = context_workspace(c);
    }

    rti::TraceArgs a{};
    a.kind = kernel_kind(c);
    a.n_sets = c->n_sets;
    a.n_bumps = c->n_bumps;
    a.twist_amp = c->amp;
    a.twist_theta0 = c->th0;
    a.n_spheres = (int)c->sph.size();
    a.n_planes = (int)c->pln.size();
    a.n_tori = (int)c->tor.size();
    for (int k = 0; k < 3; ++k) {
        a.eye[k] = cam->eye[k];
        a.right[k] = (float)rt[k];
        a.up[k] = (float)up[k];
        a.fwd[k] = (float)f[k];
    }
    a.tan_half = (float)std::tan(0.5 * (double)cam->vfov_deg * M_PI / 180.0);
    a.aspect = (float)((double)cam->width / (double)cam->height);
    a.width = cam->width;
    a.height = cam->height;
    a.tiles_x = tiles_x;
    a.tiles_y = tiles_y;
    a.T = (int)T;
    a.step_kind = r->kind;
    a.h = r->h;
    a.rtol = r->rtol;
    a.atol = r->atol;
    a.h_min = r->h_min;
    a.h_max = r->kind == RT_STEP_RK45 ? r->h_max : r->h;
    a.t_max = r->t_max;
    a.max_steps = max_steps;
    a.K = r->cull_every;
    a.S = r->pass_steps;
    a.bisect_iters = r->bisect_iters;
    a.count = (r->flags & RT_FLAG_COUNT_WORK) ? 1 : 0;
    a.batch = batch ? 1 : 0;
    // Culling window: before the next re-cull a lane moves at most K+1 steps
    // of Euclidean length <= h_max * vmax.  A g-unit velocity has Euclidean
    // speed <= 1 wherever g >= I: always for the graph metric
    // (g = I + grad f grad f^T), and for the twist, whose Jacobian has
    // smallest singular value >= 1 (vmax carries a 5% safety factor there).
    // The z-twist has g < I away from its axis and is not culled.
    // A composition of local deformations takes the smaller of its two
    // bounds (see set_deform_metric).
    double vmax = c->kind == RT_METRIC_PULLBACK_TWIST ? 1.05 : 1.0;
    double margin = (r->cull_every + 1) * (double)a.h_max * vmax * 1.02 + 1e-4;
    if (c->kind == RT_METRIC_PULLBACK_DEFORM)
        margin = std::min((r->cull_every + 1) * (double)a.h_max * c->deform_vmax * 1.02,
                          (r->cull_every + 1) * (double)a.h_max * 1.02 + 2.0 * c->deform_disp) + 1e-4;
    a.cull_margin = c->kind == RT_METRIC_PULLBACK_ZTWIST ? -1.0f : (float)margin;
    a.cull_base = (float)((r->cull_every + 1) * (double)a.h_max * 1.02 + 1e-4);
    a.cull_disp = (float)(c->deform_disp * (1.0 + 1e-6));
    a.st = ws.st;
    a.ids[0] = ws.ids[0];
    a.ids[1] = ws.ids[1];
    a.cmask = ws.cmask;
    a.cscan = ws.cscan;
    a.bscan = ws.bscan;
    a.max_chunks = (int)max_chunks_for(cap);
    a.cap = cap;
    a.ctr = ws.ctr;
    a.stats = c->d_stats;
    a.rec = ws.rec;
    a.out_hit = o->hit;
    a.out_t = o->t;
    a.out_dir = o->dir;
    a.out_id = o->id;
    a.out_steps = o->steps;
    a.tape_ck = nullptr;
    a.tape_hit = nullptr;
    a.ckpt_every = 1;
    a.n_ckpt = 1;
    if (tape) {
        size_t need = rt_tape_bytes(cam, c->n_sets, max_steps, ckpt_every);
        if (tape_bytes < need)
            return fail(c, RT_EINVAL, "rt_trace_fwd_ckpt: tape_bytes " + std::to_string(tape_bytes) + " < " +
                                          std::to_string(need));
        a.ckpt_every = ckpt_every;
        a.n_ckpt = (max_steps + ckpt_every - 1) / ckpt_every;
        a.tape_ck = (float *)tape;
        a.tape_hit = (float *)tape + (size_t)cap * a.n_ckpt * 9;
    }

    a.surr = use_surr ? 1 : 0;
    a.n_passes = n_passes;
    a.xctl = ws.ctr + rti::CTR_PASS0 + n_passes * rti::CTR_PASS_WORDS;
    rti::SurrArgs S = c->surr;
    if (use_surr) {
        if ((st = ensure_xbuf(c, cap)) != RT_OK) return st;
        char *xb = (char *)c->d_xbuf;
        a.surr_sb = (const float4 *)c->d_surr_sb;
        a.xq = (int4 *)xb;
        S.sorted = (int2 *)(xb + (size_t)cap * 16);
        S.xin = (float *)(xb + (size_t)cap * 24);
        S.xout = (float *)(xb + (size_t)cap * 48);
    }

    int bpc = rti::trace_blocks_per_cu(a.kind, a.step_kind);
    int64_t chunks = cap / 64 + 1;
    int64_t grid = (int64_t)c->n_cu * bpc;
    if (grid * 4 > chunks) grid = (chunks + 3) / 4;
    if (grid < 1) grid = 1;
    int rgrid = (int)std::min<int64_t>((cap + 255) / 256, (int64_t)c->n_cu * 8);
    if (rgrid < 1) rgrid = 1;
    if (const char *g = std::getenv("RT_GRID_BLOCKS")) {
        int v = std::atoi(g);
        if (v >= 1) grid = v;
    }
    hipStream_t s = (hipStream_t)stream;
    bool timed = (r->flags & RT_FLAG_TIMING) != 0;
    if (timed) {
        while ((int)c->ev.size() < 4 * n_passes + 3) {
            hipEvent_t ev;
            if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_fail(c, e, "hipEventCreate");
            c->ev.push_back(ev);
        }
    }
    e = rti::launch_trace(a, c->dd, n_passes, (int)grid, rgrid, s, timed ? c->ev.data() : nullptr,
                          use_surr ? &S : nullptr, 2 * c->n_cu);
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
    c->last_stream = s;
    c->traced = true;
    c->last_passes = n_passes;
    c->last_timed = timed;
    c->last_surr = use_surr;
    c->last_surr_flag = surr;
    if (tape) {
        c->adj_args = a;
        c->adj_tape = tape;
        c->adj_valid = true;
    }
    c->err.clear();
    return RT_OK;
}

rt_status rt_illuminate(rt_ctx *c, const rt_camera *cam, const rt_outputs *traced, const rt_light *L,
                        const rt_shading *out, void *stream) {
    if (!c) return RT_EINVAL;
    if (!cam || !traced || !L || !out) return fail(c, RT_EINVAL, "rt_illuminate: NULL camera, traced outputs, light or output");
    if (!c->has_metric || !c->has_scene) return fail(c, RT_ESTATE, "rt_illuminate: set the metric and the scene first");
    if (cam->width < 1 || cam->height < 1) return fail(c, RT_EINVAL, "rt_illuminate: width and height must be >= 1");
    if ((int64_t)cam->width * cam->height * c->n_sets > 2147483647LL)
        return fail(c, RT_EINVAL, "rt_illuminate: width*height*n_sets exceeds 2^31-1");
    if (!traced->hit || !traced->id) return fail(c, RT_EINVAL, "rt_illuminate: traced hit and id are required");
    if (!out->shade || !out->status) return fail(c, RT_EINVAL, "rt_illuminate: shade and status are required");
    for (int k = 0; k < 3; ++k)
        if (!finite(L->pos[k])) return fail(c, RT_EINVAL, "rt_illuminate: non-finite light position");
    if (!finite(L->h) || !(L->h > 0.f) || L->h > 0.1f) return fail(c, RT_EINVAL, "rt_illuminate: h must be in (0, 0.1]");
    if (!finite(L->tol) || !(L->tol > 0.f)) return fail(c, RT_EINVAL, "rt_illuminate: tol must be finite and > 0");
    if (L->max_iters < 1 || L->max_iters > 64) return fail(c, RT_EINVAL, "rt_illuminate: max_iters must be in 1..64");
    if (L->max_steps < 1 || L->max_steps > 100000)
        return fail(c, RT_EINVAL, "rt_illuminate: max_steps must be in 1..100000");
    if (c->host_only) return fail(c, RT_ESTATE, "rt_illuminate: host-only context (created with device -1)");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    rti::IllumArgs a{};
    a.kind = kernel_kind(c);
    a.n_sets = c->n_sets;
    a.n_bumps = c->n_bumps;
    a.twist_amp = c->amp;
    a.twist_theta0 = c->th0;
    a.n_spheres = (int)c->sph.size();
    a.n_planes = (int)c->pln.size();
    a.n_tori = (int)c->tor.size();
    a.width = cam->width;
    a.height = cam->height;
    a.hit = traced->hit;
    a.id = traced->id;
    for (int k = 0; k < 3; ++k) a.light[k] = L->pos[k];
    a.h = L->h;
    a.tol = L->tol;
    a.max_iters = L->max_iters;
    a.max_steps = L->max_steps;
    {
        // culling windows of the shots, as for a trace with step h: a
        // g-unit geodesic covers at most (K+1) h vmax of Euclidean length
        // before the next window (no bound for the z-twist)
        const double K1 = rti::ILLUM_CULL_EVERY + 1;
        double m = K1 * L->h * (c->kind == RT_METRIC_PULLBACK_TWIST ? 1.05 : 1.0) * 1.02 + 1e-4;
        if (c->kind == RT_METRIC_PULLBACK_DEFORM)
            m = std::min(K1 * L->h * c->deform_vmax * 1.02, K1 * L->h * 1.02 + 2.0 * c->deform_disp) + 1e-4;
        a.cull_margin = c->kind == RT_METRIC_PULLBACK_ZTWIST ? -1.0f : (float)m;
    }
    a.shade = out->shade;
    a.status = out->status;
    a.dir = out->dir;
    a.len = out->len;
    const int64_t n = (int64_t)cam->width * cam->height * c->n_sets;
    // workspace: Newton state (4 floats), the base shot (6 floats), three
    // pixel lists, the list counters of the first round and the retries
    if (c->ibuf_cap < n) {
        rt_status st = sync_last(c);
        if (st != RT_OK) return st;
        (void)hipFree(c->d_ibuf);
        c->d_ibuf = nullptr;
        c->ibuf_cap = 0;
        e = hipMalloc(&c->d_ibuf, (size_t)n * 52 +
                                      (1 + rti::ILLUM_RETRY_ROUNDS + rti::ILLUM_CONT_STAGES) * 130 * sizeof(int) + 256);
        if (e != hipSuccess) return hip_fail(c, e, "hipMalloc (illumination workspace)");
        c->ibuf_cap = n;
    }
    char *ib = (char *)c->d_ibuf;
    a.w_al = (float *)ib;
    a.w_be = (float *)(ib + (size_t)n * 4);
    a.w_T = (float *)(ib + (size_t)n * 8);
    a.w_F = (float *)(ib + (size_t)n * 12);
    a.w_X = (float *)(ib + (size_t)n * 16);
    a.w_Y = (float *)(ib + (size_t)n * 28);
    a.list[0] = (int *)(ib + (size_t)n * 40);
    a.list[1] = (int *)(ib + (size_t)n * 44);
    a.list[2] = (int *)(ib + (size_t)n * 48);
    a.ctr = (int *)(ib + (size_t)n * 52);
    a.cont = 1.0f;
    a.conv_code = 3;  // converged, awaiting the finish
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, (int64_t)c->n_cu * 8));
    hipStream_t s = (hipStream_t)stream;
    e = rti::launch_illum(a, c->dd, grid, s);
    if (e != hipSuccess) return hip_fail(c, e, "rt_illuminate launch");
    c->last_stream = s;
    c->err.clear();
    return RT_OK;
}

rt_status rt_trace(rt_ctx *c, const rt_camera *cam, const rt_step_rule *r, int max_steps, const rt_outputs *o,
                   void *stream) {
    return trace_impl(c, cam, r, max_steps, o, stream, nullptr, 0, 0);
}

rt_status rt_trace_noalloc(rt_ctx *c, const rt_camera *cam, const rt_step_rule *r, int max_steps, const rt_outputs *o,
                           void *stream) {
    return trace_impl(c, cam, r, max_steps, o, stream, nullptr, 0, 0, true);
}

size_t rt_tape_bytes(const rt_camera *cam, int n_sets, int max_steps, int ckpt_every) {
    if (!cam || cam->width < 1 || cam->height < 1 || n_sets < 1 || max_steps < 1 || ckpt_every < 1) return 0;
    size_t tiles = (size_t)((cam->width + 7) / 8) * ((cam->height + 7) / 8);
    size_t cap = tiles * 64 * (size_t)n_sets;
    size_t n_ckpt = ((size_t)max_steps + ckpt_every - 1) / ckpt_every;
    return (cap * n_ckpt * 9 + (size_t)n_sets * cam->width * cam->height * rti::TAPE_REC) * sizeof(float);
}

rt_status rt_trace_fwd_ckpt(rt_ctx *c, const rt_camera *cam, const rt_step_rule *r, int max_steps, int ckpt_every,
                            const rt_outputs *o, void *tape, size_t tape_bytes, void *stream) {
    if (!c) return RT_EINVAL;
    if (!tape) return fail(c, RT_EINVAL, "rt_trace_fwd_ckpt: tape is NULL");
    if (ckpt_every < 1 || ckpt_every > max_steps)
        return fail(c, RT_EINVAL, "rt_trace_fwd_ckpt: ckpt_every must be in 1..max_steps");
    if (!c->has_metric || c->kind != RT_METRIC_GRAPH_GAUSS)
        return fail(c, RT_EUNSUPPORTED, "rt_trace_fwd_ckpt: differentiation needs the graph metric");
    if (c->n_bumps < 1 || c->n_bumps > rti::adjoint_max_bumps())
        return fail(c, RT_EUNSUPPORTED, "rt_trace_fwd_ckpt: differentiation supports 1..16 bumps per set");
    if (r && r->kind != RT_STEP_RK4) return fail(c, RT_EUNSUPPORTED, "rt_trace_fwd_ckpt: the adjoint is RK4 only");
    c->adj_valid = false;
    return trace_impl(c, cam, r, max_steps, o, stream, tape, tape_bytes, ckpt_every);
}

rt_status rt_loss_l2(rt_ctx *c, const rt_camera *cam, const float *hit, const int32_t *id, const float *target_hit,
                     const int32_t *target_id, const uint8_t *mask, float *loss, float *grad_hit, void *stream) {
    if (!c) return RT_EINVAL;
    if (!cam || !hit || !id || !target_hit || !target_id || !loss)
        return fail(c, RT_EINVAL, "rt_loss_l2: NULL argument");
    if (cam->width < 1 || cam->height < 1) return fail(c, RT_EINVAL, "rt_loss_l2: bad frame size");
    if (c->host_only) return fail(c, RT_ESTATE, "rt_loss_l2: host-only context");
    int HW = cam->width * cam->height;
    int64_t nblk = ((int64_t)HW + 255) / 256;
    int64_t need = nblk * c->n_sets;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    if (c->loss_cap < need) {
        rt_status st = sync_last(c);
        if (st != RT_OK) return st;
        (void)hipFree(c->d_loss_blk);
        c->d_loss_blk = nullptr;
        c->loss_cap = 0;
        if ((e = hipMalloc((void **)&c->d_loss_blk, need * sizeof(float))) != hipSuccess)
            return hip_fail(c, e, "hipMalloc (loss)");
        c->loss_cap = need;
    }
    hipStream_t s = (hipStream_t)stream;
    e = rti::launch_loss(hit, id, target_hit, target_id, mask, c->n_sets, HW, grad_hit, c->d_loss_blk, loss, s);
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch (loss)");
    c->last_stream = s;
    c->traced = true;
    return RT_OK;
}

rt_status rt_trace_bwd(rt_ctx *c, const void *tape, const float *grad_hit, float *grad_params, void *stream) {
    if (!c) return RT_EINVAL;
    if (!tape || !grad_hit || !grad_params) return fail(c, RT_EINVAL, "rt_trace_bwd: NULL argument");
    if (!c->adj_valid || c->adj_tape != tape)
        return fail(c, RT_ESTATE, "rt_trace_bwd: no rt_trace_fwd_ckpt recorded this tape on this context");
    rti::TraceArgs a = c->adj_args;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    int64_t chunks = (int64_t)a.n_sets * a.tiles_x * a.tiles_y;
    // persistent one-wave blocks, as many as stay resident (more would wait
    // for a slot and finish their chunk share late)
    int blocks = (int)std::min<int64_t>(chunks, (int64_t)c->n_cu * rti::adjoint_blocks_per_cu(a.n_bumps));
    if (blocks < 1) blocks = 1;
    int64_t scr = (int64_t)blocks * a.ckpt_every * 6 * 64;
    int64_t part = chunks * a.n_bumps * 5 + 64;  // + the chunk queue counter
    if (c->adj_scr_cap < scr || c->adj_part_cap < part) {
        rt_status st = sync_last(c);
        if (st != RT_OK) return st;
        (void)hipFree(c->d_adj_scr);
        (void)hipFree(c->d_adj_part);
        c->d_adj_scr = c->d_adj_part = nullptr;
        c->adj_scr_cap = c->adj_part_cap = 0;
        if ((e = hipMalloc((void **)&c->d_adj_scr, scr * sizeof(float))) != hipSuccess ||
            (e = hipMalloc((void **)&c->d_adj_part, part * sizeof(float))) != hipSuccess)
            return hip_fail(c, e, "hipMalloc (adjoint scratch)");
        c->adj_scr_cap = scr;
        c->adj_part_cap = part;
    }
    hipStream_t s = (hipStream_t)stream;
    e = rti::launch_adjoint(a, c->dd, grad_hit, c->d_adj_part, grad_params, c->d_adj_scr,
                            (int *)(c->d_adj_part + chunks * a.n_bumps * 5), c->d_stats, blocks, s);
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch (adjoint)");
    c->last_stream = s;
    return RT_OK;
}

size_t rt_mlp_work_bytes(int n_nets, int batch) {
    if (n_nets < 1 || batch < 1) return 0;
    return rti::mlp_work_bytes(n_nets, batch);
}

static rt_status mlp_check(rt_ctx *c, int n_nets, int batch, const void *w, void *work, size_t work_bytes,
                           const char *who) {
    if (!c) return RT_EINVAL;
    if (n_nets < 1 || n_nets > 4096 || batch < 1 || (int64_t)n_nets * batch > (1LL << 28))
        return fail(c, RT_EINVAL, std::string(who) + ": bad n_nets or batch");
    if (!w || !work) return fail(c, RT_EINVAL, std::string(who) + ": NULL argument");
    if (work_bytes < rti::mlp_work_bytes(n_nets, batch))
        return fail(c, RT_EINVAL, std::string(who) + ": workspace too small");
    if (c->host_only) return fail(c, RT_ESTATE, std::string(who) + ": host-only context");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    return RT_OK;
}

rt_status rt_mlp_fwd(rt_ctx *c, int n_nets, int batch, const uint16_t *w_bf16, const float *params, const float *x,
                     float *y, void *work, size_t work_bytes, void *stream) {
    if (c && (!params || !x || !y)) return fail(c, RT_EINVAL, "rt_mlp_fwd: NULL argument");
    rt_status st = mlp_check(c, n_nets, batch, w_bf16, work, work_bytes, "rt_mlp_fwd");
    if (st != RT_OK) return st;
    rti::MlpWork w;
    rti::mlp_work_carve(work, n_nets, batch, w);
    hipError_t e = rti::mlp_forward(n_nets, batch, (const __bf16 *)w_bf16, params, x, y, w, true, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch (mlp forward)");
    return RT_OK;
}

rt_status rt_mlp_fwd_grouped(rt_ctx *c, int n_nets, const int32_t *rows, const uint16_t *w_bf16,
                             const float *params, const float *x, float *y, void *stream) {
    if (!c) return RT_EINVAL;
    if (n_nets < 1 || n_nets > rti::MAX_NETS) return fail(c, RT_EINVAL, "rt_mlp_fwd_grouped: n_nets must be in 1..64");
    if (!rows || !w_bf16 || !params || !x || !y) return fail(c, RT_EINVAL, "rt_mlp_fwd_grouped: NULL argument");
    std::vector<int> ctl(rti::CTR_SURR_WORDS, 0);
    int64_t tot = 0, tiles = 0;
    for (int g = 0; g < n_nets; ++g) {
        if (rows[g] < 0) return fail(c, RT_EINVAL, "rt_mlp_fwd_grouped: negative row count");
        ctl[rti::XC_ROW + g] = (int)tot;
        ctl[rti::XC_TILE + g] = (int)tiles;
        tot += rows[g];
        tiles += (rows[g] + 63) / 64;
        if (tot > (1LL << 30)) return fail(c, RT_EINVAL, "rt_mlp_fwd_grouped: too many rows");
    }
    for (int g = n_nets; g <= 64; ++g) {
        ctl[rti::XC_ROW + g] = (int)tot;
        ctl[rti::XC_TILE + g] = (int)tiles;
    }
    if (c->host_only) return fail(c, RT_ESTATE, "rt_mlp_fwd_grouped: host-only context");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    rt_status st = sync_last(c);
    if (st != RT_OK) return st;
    if ((st = upload(c, &c->d_grp_ctl, &c->grp_ctl_bytes, ctl.data(), ctl.size() * sizeof(int))) != RT_OK) return st;
    if (tiles == 0) return RT_OK;
    // the kernel reads weight rows with 128-bit loads: copy them to 16-byte
    // aligned rows of MLP_P_PAD values
    const size_t P = RT_MLP_PARAMS, PP = rti::MLP_P_PAD;
    const size_t need = (size_t)n_nets * PP * 6;
    if (c->grp_w_bytes < need) {
        (void)hipFree(c->d_grp_w);
        c->d_grp_w = nullptr;
        c->grp_w_bytes = 0;
        if ((e = hipMalloc(&c->d_grp_w, need)) != hipSuccess) return hip_fail(c, e, "hipMalloc (grouped mlp)");
        c->grp_w_bytes = need;
    }
    char *gw = (char *)c->d_grp_w;
    hipStream_t hs = (hipStream_t)stream;
    if ((e = hipMemcpy2DAsync(gw, PP * 2, w_bf16, P * 2, P * 2, n_nets, hipMemcpyDeviceToDevice, hs)) != hipSuccess ||
        (e = hipMemcpy2DAsync(gw + (size_t)n_nets * PP * 2, PP * 4, params, P * 4, P * 4, n_nets,
                              hipMemcpyDeviceToDevice, hs)) != hipSuccess)
        return hip_fail(c, e, "hipMemcpy2DAsync (grouped mlp)");
    rti::SurrArgs S{};
    S.n_nets = n_nets;
    S.stride = (int64_t)PP;
    S.wb = (const __bf16 *)gw;
    S.params = (const float *)(gw + (size_t)n_nets * PP * 2);
    S.xin = (float *)x;
    S.xout = y;
    int blocks = (int)std::min<int64_t>(tiles, 2 * (int64_t)c->n_cu);
    e = rti::launch_mlp_grouped((const int *)c->d_grp_ctl, S, blocks, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch (grouped mlp)");
    c->last_stream = (hipStream_t)stream;
    c->traced = true;
    return RT_OK;
}

rt_status rt_mlp_bwd(rt_ctx *c, int n_nets, int batch, const uint16_t *w_bf16, const float *params, const float *dy,
                     float *grad, void *work, size_t work_bytes, void *stream) {
    if (c && (!params || !dy || !grad)) return fail(c, RT_EINVAL, "rt_mlp_bwd: NULL argument");
    rt_status st = mlp_check(c, n_nets, batch, w_bf16, work, work_bytes, "rt_mlp_bwd");
    if (st != RT_OK) return st;
    rti::MlpWork w;
    rti::mlp_work_carve(work, n_nets, batch, w);
    hipError_t e =
        rti::mlp_backward(n_nets, batch, (const __bf16 *)w_bf16, params, dy, grad, w, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch (mlp backward)");
    return RT_OK;
}

rt_status rt_mse_grad(rt_ctx *c, const float *y, const float *t, float *dy, size_t n, int batch, float *part,
                      void *stream) {
    if (!c) return RT_EINVAL;
    if (!y || !t || !dy || !part || batch < 1) return fail(c, RT_EINVAL, "rt_mse_grad: bad argument");
    if (c->host_only) return fail(c, RT_ESTATE, "rt_mse_grad: host-only context");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    e = rti::launch_mse_grad(y, t, dy, (int64_t)n, batch, part, 64, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch (mse)");
    return RT_OK;
}

rt_status rt_adamw_step(rt_ctx *c, float *params, uint16_t *w_bf16, float *m, float *v, const float *grad, size_t n,
                        float lr, float beta1, float beta2, float eps, float wd, int step, void *stream) {
    if (!c) return RT_EINVAL;
    if (!params || !w_bf16 || !m || !v || !grad) return fail(c, RT_EINVAL, "rt_adamw_step: NULL argument");
    if (step < 1 || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f) ||
        !finite(lr) || !finite(wd))
        return fail(c, RT_EINVAL, "rt_adamw_step: bad hyper-parameters");
    if (c->host_only) return fail(c, RT_ESTATE, "rt_adamw_step: host-only context");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    e = rti::launch_adamw(params, (__bf16 *)w_bf16, m, v, grad, (int64_t)n, lr, beta1, beta2, eps, wd, step,
                          (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch (adamw)");
    return RT_OK;
}

rt_status rt_surrogate_gen(rt_ctx *c, int n_shapes, const float *kappa, const float *scale, int n_per, float h,
                           int mode, uint64_t seed, float *x, float *y, float *aux, void *stream) {
    if (!c) return RT_EINVAL;
    if (n_shapes < 1 || n_shapes > 4096 || n_per < 1 || (int64_t)n_shapes * n_per > (1LL << 31) - 1)
        return fail(c, RT_EINVAL, "rt_surrogate_gen: bad sizes");
    if (!kappa || !scale || !x || !y || !aux) return fail(c, RT_EINVAL, "rt_surrogate_gen: NULL argument");
    if (!(h >= 1e-3f && h <= 0.5f) || !(mode == 0 || mode == 1 || mode == 2 || mode == 4 || mode == 6))
        return fail(c, RT_EINVAL, "rt_surrogate_gen: need 1e-3 <= h <= 0.5 and mode in {0, 1, 2, 4, 6}");
    for (int i = 0; i < n_shapes; ++i)
        if (!finite(kappa[i]) || std::fabs(kappa[i]) > 100.f || !(scale[i] > 0.f) || !finite(scale[i]))
            return fail(c, RT_EINVAL, "rt_surrogate_gen: bad kappa or scale");
    if (c->host_only) return fail(c, RT_ESTATE, "rt_surrogate_gen: host-only context");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    std::vector<float> ks(2 * (size_t)n_shapes);
    float kmax = 0.f;
    for (int i = 0; i < n_shapes; ++i) {
        ks[i] = kappa[i];
        ks[n_shapes + i] = scale[i];
        kmax = std::max(kmax, std::fabs(kappa[i]));
    }
    rt_status st = upload(c, &c->d_gen_ks, &c->gen_ks_bytes, ks.data(), ks.size() * sizeof(float));
    if (st != RT_OK) return st;
    const float *dk = (const float *)c->d_gen_ks;
    e = rti::launch_cross_gen(dk, dk + n_shapes, n_shapes, n_per, h, mode, seed, x, y, aux, kmax,
                              (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch (surrogate data)");
    c->last_stream = (hipStream_t)stream;
    c->traced = true;
    return RT_OK;
}

// Training batches are generated TRAIN_CHUNK steps at a time (one launch
// with enough crossings to fill the GPU).
static constexpr int TRAIN_CHUNK = 16;

size_t rt_surrogate_train_bytes(int n_nets, int batch) {
    if (n_nets < 1 || batch < 1) return 0;
    const size_t nb = (size_t)n_nets * batch;
    const size_t nc = nb * TRAIN_CHUNK;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    // x, y, aux of a chunk, pred, dy, grad, loss partials, then the MLP workspace
    return al(nc * 6 * 4) * 2 + al(nc * 4 * 4) + al(nb * 6 * 4) * 2 + al((size_t)n_nets * RT_MLP_PARAMS * 4) +
           al(64 * 4) + al(rti::mlp_work_bytes(n_nets, batch));
}

rt_status rt_surrogate_train(rt_ctx *c, int n_nets, const float *kappa, const float *scale, int batch, int n_steps,
                             float h, int mode, uint64_t seed, float lr, float lr_min, int warmup, float b1, float b2,
                             float eps, float wd, float *params, uint16_t *w_bf16, float *adam_m, float *adam_v,
                             void *work, size_t work_bytes, float *loss_log, int log_every, void *stream) {
    if (!c) return RT_EINVAL;
    if (n_nets < 1 || n_nets > 4096 || batch < 1 || (int64_t)n_nets * batch > (1LL << 26) || n_steps < 1)
        return fail(c, RT_EINVAL, "rt_surrogate_train: bad sizes");
    if (!kappa || !scale || !params || !w_bf16 || !adam_m || !adam_v || !work)
        return fail(c, RT_EINVAL, "rt_surrogate_train: NULL argument");
    if (!(h >= 1e-3f && h <= 0.5f) || (mode != 0 && mode != 2) || warmup < 0 || !(lr > 0.f) || !(lr_min >= 0.f) ||
        !finite(lr) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f) || !finite(wd))
        return fail(c, RT_EINVAL, "rt_surrogate_train: bad hyper-parameters");
    if (loss_log && log_every < 1) return fail(c, RT_EINVAL, "rt_surrogate_train: log_every must be >= 1");
    if (work_bytes < rt_surrogate_train_bytes(n_nets, batch))
        return fail(c, RT_EINVAL, "rt_surrogate_train: workspace too small");
    float kmax = 0.f;
    for (int i = 0; i < n_nets; ++i) {
        if (!finite(kappa[i]) || std::fabs(kappa[i]) > 100.f || !(scale[i] > 0.f) || !finite(scale[i]))
            return fail(c, RT_EINVAL, "rt_surrogate_train: bad kappa or scale");
        kmax = std::max(kmax, std::fabs(kappa[i]));
    }
    if (c->host_only) return fail(c, RT_ESTATE, "rt_surrogate_train: host-only context");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    rt_status st = sync_last(c);
    if (st != RT_OK) return st;
    std::vector<float> ks(2 * (size_t)n_nets);
    for (int i = 0; i < n_nets; ++i) {
        ks[i] = kappa[i];
        ks[n_nets + i] = scale[i];
    }
    if ((st = upload(c, &c->d_gen_ks, &c->gen_ks_bytes, ks.data(), ks.size() * sizeof(float))) != RT_OK) return st;
    const float *dk = (const float *)c->d_gen_ks;
    const size_t nb = (size_t)n_nets * batch;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *p = (char *)work;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += al(bytes);
        return r;
    };
    const size_t nc = nb * TRAIN_CHUNK;
    float *X = (float *)take(nc * 6 * 4), *Y = (float *)take(nc * 6 * 4), *AUX = (float *)take(nc * 4 * 4);
    float *PRED = (float *)take(nb * 6 * 4), *DY = (float *)take(nb * 6 * 4);
    float *G = (float *)take((size_t)n_nets * RT_MLP_PARAMS * 4), *PART = (float *)take(64 * 4);
    rti::MlpWork w;
    rti::mlp_work_carve(take(rti::mlp_work_bytes(n_nets, batch)), n_nets, batch, w);
    hipStream_t s = (hipStream_t)stream;
    const size_t np = (size_t)n_nets * RT_MLP_PARAMS;
    for (int step = 1; step <= n_steps; ++step) {
        float lr_t;
        if (step <= warmup) {
            lr_t = lr * (float)step / (float)warmup;
        } else {
            const double q = (double)(step - warmup) / (double)std::max(1, n_steps - warmup);
            lr_t = (float)(lr_min + 0.5 * (lr - lr_min) * (1.0 + std::cos(M_PI * q)));
        }
        float *part = (loss_log && step % log_every == 0) ? loss_log + (size_t)(step / log_every - 1) * 64 : PART;
        const int j = (step - 1) % TRAIN_CHUNK;
        if (j == 0) {
            // crossings of the next TRAIN_CHUNK steps, step-major
            const uint64_t chunk = (uint64_t)(step - 1) / TRAIN_CHUNK;
            if ((e = rti::launch_cross_gen(dk, dk + n_nets, n_nets, batch * TRAIN_CHUNK, h, mode,
                                           seed + 1000003ull * (chunk + 1), X, Y, AUX, kmax, s, batch)) != hipSuccess)
                return hip_fail(c, e, "kernel launch (surrogate training data)");
        }
        const float *Xs = X + (size_t)j * nb * 6, *Ys = Y + (size_t)j * nb * 6;
        if ((e = rti::mlp_forward(n_nets, batch, (const __bf16 *)w_bf16, params, Xs, PRED, w, true, s)) !=
                hipSuccess ||
            (e = rti::launch_mse_grad(PRED, Ys, DY, (int64_t)nb * 6, batch, part, 64, s)) != hipSuccess ||
            (e = rti::mlp_backward(n_nets, batch, (const __bf16 *)w_bf16, params, DY, G, w, s)) != hipSuccess ||
            (e = rti::launch_adamw(params, (__bf16 *)w_bf16, adam_m, adam_v, G, (int64_t)np, lr_t, b1, b2, eps, wd,
                                   step, s)) != hipSuccess)
            return hip_fail(c, e, "kernel launch (surrogate training)");
    }
    c->last_stream = s;
    c->traced = true;
    return RT_OK;
}

rt_status rt_surrogate_calibrate(rt_ctx *c, int n_shapes, int n_per, const float *x, const float *pred,
                                 const float *target, const float *scale, int n_bins, float *err, void *stream) {
    if (!c) return RT_EINVAL;
    if (n_shapes < 1 || n_shapes > 4096 || n_per < 1 || (int64_t)n_shapes * n_per > (1LL << 31) - 1 || n_bins < 1 ||
        n_bins > 4096)
        return fail(c, RT_EINVAL, "rt_surrogate_calibrate: bad sizes");
    if (!x || !pred || !target || !scale || !err) return fail(c, RT_EINVAL, "rt_surrogate_calibrate: NULL argument");
    for (int i = 0; i < n_shapes; ++i)
        if (!(scale[i] > 0.f) || !finite(scale[i])) return fail(c, RT_EINVAL, "rt_surrogate_calibrate: bad scale");
    if (c->host_only) return fail(c, RT_ESTATE, "rt_surrogate_calibrate: host-only context");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    rt_status st = upload(c, &c->d_gen_ks, &c->gen_ks_bytes, scale, (size_t)n_shapes * sizeof(float));
    if (st != RT_OK) return st;
    e = rti::launch_cross_cal(x, pred, target, (const float *)c->d_gen_ks, n_shapes, n_per, n_bins, err,
                              (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "kernel launch (surrogate calibration)");
    c->last_stream = (hipStream_t)stream;
    c->traced = true;
    return RT_OK;
}

rt_status rt_surrogate_load(rt_ctx *c, int n_nets, const uint16_t *w_bf16, const float *params, const float *scale,
                            const float *arc, int n_tab, const float *err, int n_bins, const int32_t *net_of_bump,
                            int n_bumps, float tol) {
    if (!c) return RT_EINVAL;
    if (n_nets == 0) {
        c->surr_nets = 0;
        c->err.clear();
        return RT_OK;
    }
    if (n_nets < 0 || n_nets > rti::MAX_NETS) return fail(c, RT_EINVAL, "rt_surrogate_load: n_nets must be in 0..64");
    if (!w_bf16 || !params || !scale || !arc || !err || (n_bumps > 0 && !net_of_bump))
        return fail(c, RT_EINVAL, "rt_surrogate_load: NULL argument");
    if (n_tab < 2 || n_tab > 1 << 20 || n_bins < 1 || n_bins > 4096 || n_bumps < 0 || n_bumps > MAX_BUMPS)
        return fail(c, RT_EINVAL, "rt_surrogate_load: bad table sizes or bump count");
    if (!(tol > 0.f) || !finite(tol)) return fail(c, RT_EINVAL, "rt_surrogate_load: tol must be finite and > 0");
    for (int i = 0; i < n_nets; ++i)
        if (!(scale[i] > 0.f) || !finite(scale[i])) return fail(c, RT_EINVAL, "rt_surrogate_load: bad scale");
    for (int b = 0; b < n_bumps; ++b)
        if (net_of_bump[b] < -1 || net_of_bump[b] >= n_nets)
            return fail(c, RT_EINVAL, "rt_surrogate_load: net_of_bump out of range");
    if (c->host_only) return fail(c, RT_ESTATE, "rt_surrogate_load: host-only context");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    rt_status st = sync_last(c);
    if (st != RT_OK) return st;
    const size_t P = RT_MLP_PARAMS, PP = rti::MLP_P_PAD;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_w = 0, o_p = al(n_nets * PP * 2), o_s = o_p + al(n_nets * PP * 4), o_a = o_s + al(n_nets * 4),
                 o_e = o_a + al((size_t)n_nets * n_tab * 4), total = o_e + al((size_t)n_nets * n_bins * 8);
    if (c->surr_bytes < total) {
        (void)hipFree(c->d_surr);
        c->d_surr = nullptr;
        c->surr_bytes = 0;
        if ((e = hipMalloc(&c->d_surr, total)) != hipSuccess) return hip_fail(c, e, "hipMalloc (surrogate)");
        c->surr_bytes = total;
    }
    char *d = (char *)c->d_surr;
    if ((e = hipMemcpy2D(d + o_w, PP * 2, w_bf16, P * 2, P * 2, n_nets, hipMemcpyDeviceToDevice)) != hipSuccess ||
        (e = hipMemcpy2D(d + o_p, PP * 4, params, P * 4, P * 4, n_nets, hipMemcpyDeviceToDevice)) != hipSuccess ||
        (e = hipMemcpy(d + o_s, scale, n_nets * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(d + o_a, arc, (size_t)n_nets * n_tab * 4, hipMemcpyDeviceToDevice)) != hipSuccess ||
        (e = hipMemcpy(d + o_e, err, (size_t)n_nets * n_bins * 8, hipMemcpyDeviceToDevice)) != hipSuccess)
        return hip_fail(c, e, "hipMemcpy (surrogate)");
    rti::SurrArgs S{};
    S.n_nets = n_nets;
    S.stride = (int64_t)PP;
    S.n_tab = n_tab;
    S.n_bins = n_bins;
    S.tol = tol;
    S.wb = (const __bf16 *)(d + o_w);
    S.params = (const float *)(d + o_p);
    S.scale = (const float *)(d + o_s);
    S.arc = (const float *)(d + o_a);
    S.err = (const float *)(d + o_e);
    c->surr = S;
    c->surr_nets = n_nets;
    c->surr_tab = n_tab;
    c->surr_bins = n_bins;
    c->surr_tol = tol;
    c->surr_scale.assign(scale, scale + n_nets);
    c->surr_net_of_bump.assign(net_of_bump, net_of_bump + n_bumps);
    c->surr_sb_dirty = true;
    c->err.clear();
    return RT_OK;
}

rt_status rt_sync(rt_ctx *c, void *stream) {
    if (!c) return RT_EINVAL;
    if (c->host_only) return RT_OK;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "rt_sync");
    return RT_OK;
}

rt_status rt_get_stats(rt_ctx *c, rt_stats *out) {
    if (!c || !out) return c ? fail(c, RT_EINVAL, "rt_get_stats: out is NULL") : RT_EINVAL;
    std::memset(out, 0, sizeof(*out));
    if (c->host_only || !c->traced) return RT_OK;
    rt_status st = sync_last(c);
    if (st != RT_OK) return st;
    unsigned long long v[rti::ST_N];
    hipError_t e = hipMemcpy(v, c->d_stats, sizeof(v), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "rt_get_stats");
    out->rays = v[rti::ST_RAYS];
    out->ray_steps = v[rti::ST_STEPS];
    out->attempts = v[rti::ST_ATTEMPTS];
    out->wave_iters = v[rti::ST_WAVE_ITERS];
    out->lane_iters = v[rti::ST_LANE_ITERS];
    out->bump_list_sum = v[rti::ST_BUMP_LIST];
    out->obj_list_sum = v[rti::ST_OBJ_LIST];
    out->refined = v[rti::ST_REFINED];
    out->acc_evals = v[rti::ST_ACC_EVALS];
    out->bump_evals = v[rti::ST_BUMP_EVALS];
    out->obj_tests = v[rti::ST_OBJ_TESTS];
    out->passes = c->last_passes;
    out->crossings = v[rti::ST_XING];
    out->accepted = v[rti::ST_XACC];
    out->adj_steps = v[rti::ST_ADJ_STEPS];
    out->adj_bump_terms = v[rti::ST_ADJ_TERMS];
    out->adj_recomputed = v[rti::ST_ADJ_RECOMP];
    out->batch_windows = v[rti::ST_BATCH_WIN];
    out->batch_replays = v[rti::ST_BATCH_REPLAY];
    out->refine_evals = v[rti::ST_REF_EVALS];
    out->refine_bump_terms = v[rti::ST_REF_BUMPS];
    out->refine_steps = v[rti::ST_REF_STEPS];
    out->eligible = c->last_surr_flag ? c->surr_eligible : 0;
    if (c->last_timed) {
        // events: 0 before reset, 1 after reset, 2+p after pass p, 2+np after
        // refine, 2np+2+p after the compaction that precedes pass p (p >= 1),
        // 3np+3+p after the crossing stage that follows pass p
        float ms = 0.f, pass = 0.f, comp = 0.f, xs = 0.f;
        int np = c->last_passes;
        for (int p = 0; p < np; ++p) {
            hipEvent_t start = p == 0 ? c->ev[1] : c->ev[2 * np + 2 + p];
            if ((e = hipEventElapsedTime(&ms, start, c->ev[2 + p])) != hipSuccess) return hip_fail(c, e, "timing");
            pass += ms;
            if (p > 0) {
                hipEvent_t prev = c->last_surr ? c->ev[3 * np + 3 + p - 1] : c->ev[1 + p];
                if ((e = hipEventElapsedTime(&ms, prev, start)) != hipSuccess) return hip_fail(c, e, "timing");
                comp += ms;
            }
            if (c->last_surr) {
                if ((e = hipEventElapsedTime(&ms, c->ev[2 + p], c->ev[3 * np + 3 + p])) != hipSuccess)
                    return hip_fail(c, e, "timing");
                xs += ms;
            }
        }
        out->pass_ms = pass;
        out->compact_ms = comp;
        out->surr_ms = xs;
        hipEvent_t rstart = c->last_surr ? c->ev[4 * np + 2] : c->ev[1 + np];
        if ((e = hipEventElapsedTime(&ms, rstart, c->ev[2 + np])) != hipSuccess) return hip_fail(c, e, "timing");
        out->refine_ms = ms;
        if ((e = hipEventElapsedTime(&ms, c->ev[0], c->ev[2 + np])) != hipSuccess) return hip_fail(c, e, "timing");
        out->total_ms = ms;
    }
    return RT_OK;
}

}  // extern "C"
