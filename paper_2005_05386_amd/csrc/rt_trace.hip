// Geodesic trace kernels for gfx950.
//
// A trace is a short sequence of launches on one stream:
//   reset    zero the counter block and statistics (a fill kernel, so the
//            sequence stays valid inside a captured graph);
//   pass p   persistent waves pull 64-ray chunks from per-XCD atomic
//            counters and integrate each lane's ray for at most S accepted
//            steps; rays that neither hit nor terminated are compacted into
//            the other ray queue (per parameter set) for pass p+1, so every
//            pass starts with full waves;
//   refine   one lane per chord hit, in double precision: bisection of the
//            step fraction on the sign of the hit object's implicit function
//            along the partial step of the same integrator, then the output.
//
// Inside a pass, every K steps each wave computes the bounding box of its
// lanes' positions, grows it by the distance a unit-speed ray can cover in
// K+1 steps (g >= I for the graph metric and the 4K twist, so the Euclidean
// speed of a g-unit velocity is at most 1), and culls bumps (cut sphere
// cull_sigmas*sigma) and objects against it: lane i tests bump i / sphere
// 64w+i and a ballot turns the answers into wave-uniform masks.  Bump
// parameters for the masked bumps are then read with scalar loads.
#include "rt_device.hpp"
#include "rt_internal.hpp"

using namespace rtd;
using rti::TraceArgs;

namespace {

// ------------------------------------------------ Dormand-Prince 5(4) table
// Coefficients of Dormand & Prince (1980).  The flow is second order
// (x' = y, y' = a(x, y)), so with A_l = a(X_l, Y_l) the stage states are
//   Y_i = y + h sum_l a_il A_l,  X_i = x + h c_i y + h^2 sum_l (a a)_il A_l
// and the step and its error estimate need only the A_l.
constexpr double DPA[7][7] = {
    {0, 0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0}};
constexpr double DPB[7] = {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0};
constexpr double DPBH[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};

constexpr double dp_c(int i) {
    double s = 0;
    for (int j = 0; j < 7; ++j) s += DPA[i][j];
    return s;
}
constexpr double dp_aa(int i, int l) {
    double s = 0;
    for (int j = 0; j < 7; ++j) s += DPA[i][j] * DPA[j][l];
    return s;
}
constexpr double dp_ba(int l) {
    double s = 0;
    for (int i = 0; i < 7; ++i) s += DPB[i] * DPA[i][l];
    return s;
}
constexpr double dp_ea(int l) {
    double s = 0;
    for (int i = 0; i < 7; ++i) s += (DPB[i] - DPBH[i]) * DPA[i][l];
    return s;
}

// --------------------------------------------------------------- steppers
// Each stepper returns the increments (dx, dv) of one step of size h from
// (p, y); acc(p, y, a) evaluates the acceleration and reports failure.
template <class T, class F>
__device__ __forceinline__ bool step_euler(F &acc, V3<T> p, V3<T> y, T h, V3<T> &dx, V3<T> &dv) {
    V3<T> a;
    bool ok = acc(p, y, a);
    dx = h * y;
    dv = h * a;
    return ok;
}

template <class T, class F>
__device__ __forceinline__ bool step_rk4(F &acc, V3<T> p, V3<T> y, T h, V3<T> &dx, V3<T> &dv) {
    V3<T> k1, k2, k3, k4;
    T hh = T(0.5) * h;
    bool ok = acc(p, y, k1);
    V3<T> y2 = axpy(hh, k1, y);
    ok &= acc(axpy(hh, y, p), y2, k2);
    V3<T> y3 = axpy(hh, k2, y);
    ok &= acc(axpy(hh, y2, p), y3, k3);
    V3<T> y4 = axpy(h, k3, y);
    ok &= acc(axpy(h, y3, p), y4, k4);
    T h6 = h * T(1.0 / 6.0);
    dx = h6 * (y + T(2) * (y2 + y3) + y4);
    dv = h6 * (k1 + T(2) * (k2 + k3) + k4);
    return ok;
}

// Dormand-Prince 5(4).  On entry A0 = a(p, y); on exit A0 = a at the new
// state (first-same-as-last).  ex, ev: embedded error h*sum(b - bhat)k.
template <class T, class F>
__device__ __forceinline__ bool step_dp5(F &acc, V3<T> p, V3<T> y, T h, V3<T> &A0, V3<T> &dx, V3<T> &dv,
                                         V3<T> &ex, V3<T> &ev) {
    V3<T> Ak[7];
    Ak[0] = A0;
    bool ok = true;
    T h2 = h * h;
#pragma unroll
    for (int i = 1; i < 7; ++i) {
        V3<T> X = axpy(h * T(dp_c(i)), y, p);
        V3<T> Y = y;
#pragma unroll
        for (int l = 0; l < i; ++l) {
            if (DPA[i][l] != 0.0) Y = axpy(h * T(DPA[i][l]), Ak[l], Y);
            if (dp_aa(i, l) != 0.0) X = axpy(h2 * T(dp_aa(i, l)), Ak[l], X);
        }
        ok &= acc(X, Y, Ak[i]);
    }
    dx = h * y;
    dv = mk(T(0), T(0), T(0));
    ex = mk(T(0), T(0), T(0));
    ev = mk(T(0), T(0), T(0));
#pragma unroll
    for (int l = 0; l < 7; ++l) {
        if (dp_ba(l) != 0.0) dx = axpy(h2 * T(dp_ba(l)), Ak[l], dx);
        if (DPB[l] != 0.0) dv = axpy(h * T(DPB[l]), Ak[l], dv);
        if (dp_ea(l) != 0.0) ex = axpy(h2 * T(dp_ea(l)), Ak[l], ex);
        if (DPB[l] - DPBH[l] != 0.0) ev = axpy(h * T(DPB[l] - DPBH[l]), Ak[l], ev);
    }
    A0 = Ak[6];
    return ok;
}

// Knuth's TwoSum followed by a fast renormalisation: (hi, lo) += d.
__device__ __forceinline__ void two_sum_add(float &hi, float &lo, float d) {
    float s = hi + d;
    float bp = s - hi;
    float e = (hi - (s - bp)) + (d - bp);
    float l = lo + e;
    float hn = s + l;
    lo = l - (hn - s);
    hi = hn;
}

__device__ __forceinline__ float box_dist2(float cx, float cy, float cz, const float lo[3], const float hi[3]) {
    float dx = fmaxf(fmaxf(lo[0] - cx, cx - hi[0]), 0.0f);
    float dy = fmaxf(fmaxf(lo[1] - cy, cy - hi[1]), 0.0f);
    float dz = fmaxf(fmaxf(lo[2] - cz, cz - hi[2]), 0.0f);
    return dx * dx + dy * dy + dz * dz;
}

__device__ __forceinline__ bool finite3(V3<float> v) {
    return __builtin_isfinite(v.x) && __builtin_isfinite(v.y) && __builtin_isfinite(v.z);
}

template <int KIND, bool COUNT> struct Acc32 {
    const float4 *__restrict__ B;
    uint64_t mask;
    float amp, th0;
    unsigned *n_eval, *n_bump;  // COUNT only
    __device__ __forceinline__ bool operator()(V3<float> p, V3<float> y, V3<float> &a) const {
        if (COUNT) *n_eval += 1;
        if constexpr (KIND == KIND_GRAPH) {
            a = graph_accel_f32<COUNT>(B, mask, p, y, n_bump);
            return true;
        } else if constexpr (KIND == KIND_TWIST) {
            return twist_accel<float>(amp, th0, p, y, a);
        } else if constexpr (KIND == KIND_ZTWIST) {
            a = ztwist_accel<float>(p, y);
            return true;
        } else {
            a = mk(0.f, 0.f, 0.f);
            return true;
        }
    }
};

__device__ __forceinline__ void write_out(const TraceArgs &A, int64_t oi, V3<float> x, float t, V3<float> y, int id,
                                          int steps) {
    A.out_hit[3 * oi + 0] = x.x;
    A.out_hit[3 * oi + 1] = x.y;
    A.out_hit[3 * oi + 2] = x.z;
    A.out_t[oi] = t;
    A.out_id[oi] = id;
    float n = rsqrt_(dot(y, y));
    A.out_dir[3 * oi + 0] = y.x * n;
    A.out_dir[3 * oi + 1] = y.y * n;
    A.out_dir[3 * oi + 2] = y.z * n;
    if (A.out_steps) A.out_steps[oi] = steps;
}

// ================================================================ the pass
template <int KIND, int STEP, bool COUNT>
__global__ __launch_bounds__(256) void k_trace_pass(TraceArgs A, int pass, const float4 *__restrict__ BF,
                                                    const float4 *__restrict__ SPH,
                                                    const float4 *__restrict__ PLN,
                                                    const float *__restrict__ TOR) {
    const int lane = lane_id();
    const int xcd0 = blockIdx.x % N_XCD;
    int *pass_ctr = A.ctr + rti::CTR_PASS0 + pass * rti::CTR_PASS_WORDS;
    const int HW = A.width * A.height;
    const int tiles = A.tiles_x * A.tiles_y;
    const int n_bumps = A.n_bumps, ns = A.n_spheres, np = A.n_planes, nt = A.n_tori;
    const int nsw = (ns + 63) >> 6;

    // chunk table of this pass
    int total_chunks, pre = 0, cnt = 0;
    if (pass == 0) {
        total_chunks = A.n_sets * tiles;
    } else {
        const int *surv = A.ctr + rti::CTR_PASS0 + (pass - 1) * rti::CTR_PASS_WORDS + rti::CTR_SURV;
        cnt = lane < A.n_sets ? surv[lane] : 0;
        pre = wave_incl_scan((cnt + 63) >> 6);
        total_chunks = uniform_i(__shfl(pre, 63));
    }
    const float *__restrict__ qin = A.q[(pass + 1) & 1];
    float *__restrict__ qout = A.q[pass & 1];
    const int64_t cap = A.cap;

    unsigned long long st_wave = 0, st_lane = 0, st_bl = 0, st_ol = 0, st_steps = 0, st_rays = 0;
    unsigned long long st_ev = 0, st_be = 0, st_ot = 0;  // COUNT only

    for (int xi = 0; xi < N_XCD; ++xi) {
        const int xp = (xcd0 + xi) & (N_XCD - 1);
        int *ctr = pass_ctr + xp * rti::CTR_CHUNK_STRIDE;
        for (;;) {
            int k = 0;
            if (lane == 0) k = atomicAdd(ctr, 1);
            k = uniform_i(__shfl(k, 0));
            const int chunk = k * N_XCD + xp;
            if (chunk >= total_chunks) break;

            // ---- resolve the set and this lane's ray
            int set, slot = 0, pix = 0;
            bool valid;
            if (pass == 0) {
                set = chunk / tiles;
                int tile = chunk - set * tiles;
                int ty = tile / A.tiles_x, tx = tile - ty * A.tiles_x;
                int i = tx * 8 + (lane & 7), j = ty * 8 + (lane >> 3);
                valid = i < A.width && j < A.height;
                pix = j * A.width + i;
            } else {
                set = __popcll(ballot(pre <= chunk));
                int base_chunk = set > 0 ? __shfl(pre, set - 1) : 0;
                int cnt_s = __shfl(cnt, set);
                slot = (chunk - base_chunk) * 64 + lane;
                valid = slot < cnt_s;
            }
            set = uniform_i(set);
            const float4 *__restrict__ Bs = BF + (int64_t)set * n_bumps * 2;
            const int64_t qbase = (int64_t)set * HW;

            V3<float> xh, xl, y;
            float th = 0.f, tl = 0.f, hc = A.h;
            int steps = 0, att = 0;
            if (pass == 0) {
                int i = pix % A.width, j = pix / A.width;
                float su = (2.0f * ((float)i + 0.5f) / (float)A.width - 1.0f) * A.tan_half * A.aspect;
                float sv = (1.0f - 2.0f * ((float)j + 0.5f) / (float)A.height) * A.tan_half;
                V3<float> d = mk(su * A.right[0] + sv * A.up[0] + A.fwd[0], su * A.right[1] + sv * A.up[1] + A.fwd[1],
                                 su * A.right[2] + sv * A.up[2] + A.fwd[2]);
                d = rsqrt_(dot(d, d)) * d;
                xh = mk(A.eye[0], A.eye[1], A.eye[2]);
                xl = mk(0.f, 0.f, 0.f);
                float gdd;
                if constexpr (KIND == KIND_GRAPH) {
                    GraphAccum G{0.f, 0.f, 0.f, 0.f};
                    for (int b = 0; b < n_bumps; ++b) graph_bump_f32(Bs[2 * b], Bs[2 * b + 1], xh, d, 1.0f, G);
                    float gd = G.gx * d.x + G.gy * d.y + G.gz * d.z;
                    gdd = dot(d, d) + gd * gd;
                } else if constexpr (KIND == KIND_TWIST) {
                    gdd = twist_gdd<float>(A.twist_amp, A.twist_theta0, xh, d);
                } else if constexpr (KIND == KIND_ZTWIST) {
                    gdd = ztwist_gdd<float>(xh, d);
                } else {
                    gdd = dot(d, d);
                }
                y = rsqrt_(gdd) * d;
            } else if (valid) {
                const float *src = qin + qbase + slot;
                xh = mk(src[rti::Q_XH * cap], src[(rti::Q_XH + 1) * cap], src[(rti::Q_XH + 2) * cap]);
                xl = mk(src[rti::Q_XL * cap], src[(rti::Q_XL + 1) * cap], src[(rti::Q_XL + 2) * cap]);
                y = mk(src[rti::Q_Y * cap], src[(rti::Q_Y + 1) * cap], src[(rti::Q_Y + 2) * cap]);
                th = src[rti::Q_TH * cap];
                tl = src[rti::Q_TL * cap];
                hc = src[rti::Q_H * cap];
                steps = __float_as_int(src[rti::Q_STEPS * cap]);
                pix = __float_as_int(src[rti::Q_PIX * cap]);
                att = __float_as_int(src[rti::Q_ATT * cap]);
            } else {
                xh = xl = y = mk(0.f, 0.f, 0.f);
            }
            if (pass == 0) st_rays += __popcll(ballot(valid));

            bool alive = valid;
            int acc_pass = 0;
            int it = 0;
            uint64_t bmask = 0, omask = 0;
            uint64_t sm[4] = {0, 0, 0, 0};
            V3<float> A0 = mk(0.f, 0.f, 0.f);
            bool need_a0 = true;
            unsigned c_eval = 0, c_bump = 0, c_obj = 0, lane_objs = 0;  // COUNT only

            for (;;) {
                bool act = alive && (STEP == STEP_RK45 ? acc_pass < A.S : it < A.S);
                uint64_t am = ballot(act);
                if (am == 0) break;

                // ---- per-wave culling window
                if (it % A.K == 0) {
                    V3<float> p = xh + xl;
                    if (A.cull_margin < 0.f) {
                        bmask = n_bumps >= 64 ? ~0ull : ((1ull << n_bumps) - 1ull);
#pragma unroll
                        for (int w = 0; w < 4; ++w) {
                            int rem = ns - 64 * w;
                            sm[w] = rem >= 64 ? ~0ull : (rem > 0 ? ((1ull << rem) - 1ull) : 0ull);
                        }
                        omask = ((1ull << np) - 1ull) | (((1ull << nt) - 1ull) << 8);
                    } else {
                        const float inf = __builtin_huge_valf();
                        float lo[3], hi[3];
                        lo[0] = wave_min(act ? p.x : inf) - A.cull_margin;
                        lo[1] = wave_min(act ? p.y : inf) - A.cull_margin;
                        lo[2] = wave_min(act ? p.z : inf) - A.cull_margin;
                        hi[0] = wave_max(act ? p.x : -inf) + A.cull_margin;
                        hi[1] = wave_max(act ? p.y : -inf) + A.cull_margin;
                        hi[2] = wave_max(act ? p.z : -inf) + A.cull_margin;
                        bool need = false;
                        if (KIND == KIND_GRAPH && lane < n_bumps) {
                            float4 b0 = Bs[2 * lane], b1 = Bs[2 * lane + 1];
                            need = box_dist2(b0.x, b0.y, b0.z, lo, hi) <= b1.z;
                        }
                        bmask = ballot(need);
#pragma unroll
                        for (int w = 0; w < 4; ++w) {
                            bool ns_need = false;
                            int idx = 64 * w + lane;
                            if (w < nsw && idx < ns) {
                                float4 s = SPH[idx];
                                ns_need = box_dist2(s.x, s.y, s.z, lo, hi) <= s.w * s.w;
                            }
                            sm[w] = w < nsw ? ballot(ns_need) : 0ull;
                        }
                        bool on = false;
                        if (lane < np) {
                            float4 pl = PLN[lane];
                            float cx = 0.5f * (lo[0] + hi[0]), cy = 0.5f * (lo[1] + hi[1]), cz = 0.5f * (lo[2] + hi[2]);
                            float ex = 0.5f * (hi[0] - lo[0]), ey = 0.5f * (hi[1] - lo[1]), ez = 0.5f * (hi[2] - lo[2]);
                            float c = pl.x * cx + pl.y * cy + pl.z * cz - pl.w;
                            float r = fabsf(pl.x) * ex + fabsf(pl.y) * ey + fabsf(pl.z) * ez;
                            on = fabsf(c) <= r;
                        } else if (lane >= 8 && lane < 8 + nt) {
                            const float *tp = TOR + 8 * (lane - 8);
                            float rr = tp[6] + tp[7];
                            on = box_dist2(tp[0], tp[1], tp[2], lo, hi) <= rr * rr;
                        }
                        omask = ballot(on);
                    }
                    if (COUNT && act) {
                        // objects inside this lane's own window (what one ray alone would need)
                        float m = A.cull_margin < 0.f ? 1e30f : A.cull_margin;
                        float llo[3] = {p.x - m, p.y - m, p.z - m}, lhi[3] = {p.x + m, p.y + m, p.z + m};
                        lane_objs = 0;
                        for (int i = 0; i < ns; ++i) {
                            float4 s = SPH[i];
                            lane_objs += box_dist2(s.x, s.y, s.z, llo, lhi) <= s.w * s.w ? 1u : 0u;
                        }
                        for (int i = 0; i < np; ++i) {
                            float4 pl = PLN[i];
                            float c = pl.x * p.x + pl.y * p.y + pl.z * p.z - pl.w;
                            lane_objs += fabsf(c) <= m * (fabsf(pl.x) + fabsf(pl.y) + fabsf(pl.z)) ? 1u : 0u;
                        }
                        for (int i = 0; i < nt; ++i) {
                            const float *tp = TOR + 8 * i;
                            float rr = tp[6] + tp[7];
                            lane_objs += box_dist2(tp[0], tp[1], tp[2], llo, lhi) <= rr * rr ? 1u : 0u;
                        }
                    }
                }
                st_wave++;
                st_lane += __popcll(am);
                st_bl += __popcll(bmask);
                st_ol += __popcll(sm[0]) + __popcll(sm[1]) + __popcll(sm[2]) + __popcll(sm[3]) + __popcll(omask);

                Acc32<KIND, COUNT> acc{Bs, bmask, A.twist_amp, A.twist_theta0, &c_eval, &c_bump};
                bool hit = false, done_miss = false, done_fail = false;
                int hit_id = -1;
                float hit_s = 2.f, hstep = A.h;
                V3<float> xh0 = xh, xl0 = xl, y0 = y;
                float th0 = th, tl0 = tl;
                int steps0 = steps;
                if (act) {
                    V3<float> p = xh + xl;
                    V3<float> dx, dv;
                    bool ok, accepted = true;
                    if constexpr (STEP == STEP_RK45) {
                        bool ok0 = true;
                        if (need_a0) {
                            ok0 = acc(p, y, A0);
                            need_a0 = false;
                        }
                        hstep = fminf(hc, A.t_max - (th + tl));
                        V3<float> Anew = A0, ex, ev;
                        ok = step_dp5<float>(acc, p, y, hstep, Anew, dx, dv, ex, ev) && ok0;
                        att++;
                        V3<float> pn = p + dx, yn = y + dv;
                        auto sc = [&](float a, float b) { return A.atol + A.rtol * fmaxf(fabsf(a), fabsf(b)); };
                        float e2 = 0.f, r;
                        r = ex.x / sc(p.x, pn.x); e2 = fmaf(r, r, e2);
                        r = ex.y / sc(p.y, pn.y); e2 = fmaf(r, r, e2);
                        r = ex.z / sc(p.z, pn.z); e2 = fmaf(r, r, e2);
                        r = ev.x / sc(y.x, yn.x); e2 = fmaf(r, r, e2);
                        r = ev.y / sc(y.y, yn.y); e2 = fmaf(r, r, e2);
                        r = ev.z / sc(y.z, yn.z); e2 = fmaf(r, r, e2);
                        float en = sqrtf(e2 * (1.0f / 6.0f));
                        float fac = en > 0.f ? 0.9f * exp2f(-0.2f * __log2f(en)) : 5.0f;
                        fac = fminf(fmaxf(fac, 0.2f), 5.0f);
                        if (en <= 1.0f) {
                            hc = fminf(hstep * fac, A.h_max);
                            A0 = Anew;
                        } else {
                            accepted = false;
                            hc = hstep * fminf(fac, 1.0f);
                            if (hc < A.h_min || att > 8 * A.max_steps) ok = false;
                        }
                    } else if constexpr (STEP == STEP_RK4) {
                        ok = step_rk4<float>(acc, p, y, A.h, dx, dv);
                    } else {
                        ok = step_euler<float>(acc, p, y, A.h, dx, dv);
                    }
                    if (!ok) {
                        done_fail = true;
                    } else if (accepted) {
                        if (COUNT) c_obj += lane_objs;
                        two_sum_add(xh.x, xl.x, dx.x);
                        two_sum_add(xh.y, xl.y, dx.y);
                        two_sum_add(xh.z, xl.z, dx.z);
                        y = y + dv;
                        steps++;
                        acc_pass++;
                        if (STEP == STEP_RK45) two_sum_add(th, tl, hstep);
                        if (!finite3(xh) || !finite3(y)) {
                            done_fail = true;
                        } else {
                            // ---- segment versus scene
                            float DD = dot(dx, dx);
#pragma unroll
                            for (int w = 0; w < 4; ++w) {
                                uint64_t m = sm[w];
                                while (m) {
                                    int b = __builtin_ctzll(m);
                                    m &= m - 1;
                                    int idx = 64 * w + b;
                                    float4 s = SPH[idx];
                                    V3<float> o = mk((xh0.x - s.x) + xl0.x, (xh0.y - s.y) + xl0.y, (xh0.z - s.z) + xl0.z);
                                    float sc = sphere_chord(s, o, dx, DD);
                                    if (sc < hit_s) {
                                        hit_s = sc;
                                        hit_id = idx;
                                    }
                                }
                            }
                            uint64_t m = omask;
                            while (m) {
                                int b = __builtin_ctzll(m);
                                m &= m - 1;
                                float F0, F1;
                                int id;
                                V3<float> x0 = xh0 + xl0;
                                if (b < 8) {
                                    float4 pl = PLN[b];
                                    F0 = pl.x * x0.x + pl.y * x0.y + pl.z * x0.z - pl.w;
                                    F1 = F0 + (pl.x * dx.x + pl.y * dx.y + pl.z * dx.z);
                                    id = ns + b;
                                } else {
                                    const float *tp = TOR + 8 * (b - 8);
                                    F0 = torus_sdf<float>(tp, x0);
                                    F1 = torus_sdf<float>(tp, x0 + dx);
                                    id = ns + np + (b - 8);
                                }
                                if ((F0 > 0.f) != (F1 > 0.f)) {
                                    float sc = fminf(fmaxf(F0 / (F0 - F1), 0.f), 1.f);
                                    if (sc < hit_s) {
                                        hit_s = sc;
                                        hit_id = id;
                                    }
                                }
                            }
                            if (hit_id >= 0) {
                                hit = true;
                            } else {
                                // RK45 lands on t_max up to float rounding of the clipped last step
                                float t = (STEP == STEP_RK45) ? th + tl : (float)steps * A.h;
                                float t_end = (STEP == STEP_RK45) ? A.t_max * (1.0f - 1e-6f) : A.t_max;
                                if (steps >= A.max_steps || t >= t_end) done_miss = true;
                            }
                        }
                    }
                    if (done_fail) {
                        write_out(A, qbase + pix, xh0 + xl0,
                                  STEP == STEP_RK45 ? th0 + tl0 : (float)steps0 * A.h, y0, -2, steps0);
                    } else if (done_miss) {
                        write_out(A, qbase + pix, xh + xl, STEP == STEP_RK45 ? th + tl : (float)steps * A.h, y, -1,
                                  steps);
                    }
                    if (done_fail || done_miss || hit) alive = false;
                }
                // ---- push chord hits to the refine queue (wave-aggregated)
                uint64_t hm = ballot(hit);
                if (hm) {
                    int base = 0;
                    if (lane == 0) base = atomicAdd(A.ctr + rti::CTR_REFINE, __popcll(hm));
                    base = uniform_i(__shfl(base, 0));
                    if (hit) {
                        int64_t r = base + mbcnt64(hm);
                        float4 *rec = A.rec + rti::REC_F4 * r;
                        rec[0] = make_float4(xh0.x, xh0.y, xh0.z, xl0.x);
                        rec[1] = make_float4(xl0.y, xl0.z, y0.x, y0.y);
                        rec[2] = make_float4(y0.z, th0, hstep, hit_s);
                        rec[3] = make_float4(__int_as_float(hit_id), __int_as_float((int)(qbase + pix)),
                                             __int_as_float(steps0), tl0);
                        rec[4] = make_float4(__int_as_float((int)(uint32_t)bmask), __int_as_float((int)(bmask >> 32)),
                                             0.f, 0.f);
                    }
                }
                it++;
            }

            // ---- compact survivors into the next queue
            uint64_t sv = ballot(alive);
            if (sv) {
                int base = 0;
                if (lane == 0) base = atomicAdd(pass_ctr + rti::CTR_SURV + set, __popcll(sv));
                base = uniform_i(__shfl(base, 0));
                if (alive) {
                    float *dst = qout + qbase + base + mbcnt64(sv);
                    dst[rti::Q_XH * cap] = xh.x;
                    dst[(rti::Q_XH + 1) * cap] = xh.y;
                    dst[(rti::Q_XH + 2) * cap] = xh.z;
                    dst[rti::Q_XL * cap] = xl.x;
                    dst[(rti::Q_XL + 1) * cap] = xl.y;
                    dst[(rti::Q_XL + 2) * cap] = xl.z;
                    dst[rti::Q_Y * cap] = y.x;
                    dst[(rti::Q_Y + 1) * cap] = y.y;
                    dst[(rti::Q_Y + 2) * cap] = y.z;
                    dst[rti::Q_TH * cap] = th;
                    dst[rti::Q_TL * cap] = tl;
                    dst[rti::Q_H * cap] = hc;
                    dst[rti::Q_STEPS * cap] = __int_as_float(steps);
                    dst[rti::Q_PIX * cap] = __int_as_float(pix);
                    dst[rti::Q_ATT * cap] = __int_as_float(att);
                }
            }
            // accepted steps of this chunk
            int acc_l = acc_pass;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) acc_l += __shfl_xor(acc_l, o);
            st_steps += (unsigned)uniform_i(acc_l);
            if (COUNT) {
                unsigned v[3] = {c_eval, c_bump, c_obj};
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    unsigned x = v[q];
#pragma unroll
                    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
                    v[q] = (unsigned)uniform_i((int)x);
                }
                st_ev += v[0];
                st_be += v[1];
                st_ot += v[2];
            }
        }
    }
    if (lane == 0) {
        if (st_rays) atomicAdd(A.stats + rti::ST_RAYS, st_rays);
        atomicAdd(A.stats + rti::ST_STEPS, st_steps);
        atomicAdd(A.stats + rti::ST_WAVE_ITERS, st_wave);
        atomicAdd(A.stats + rti::ST_LANE_ITERS, st_lane);
        atomicAdd(A.stats + rti::ST_BUMP_LIST, st_bl);
        atomicAdd(A.stats + rti::ST_OBJ_LIST, st_ol);
        atomicAdd(A.stats + rti::ST_ATTEMPTS, STEP == STEP_RK45 ? st_lane : st_steps);
        if (COUNT) {
            atomicAdd(A.stats + rti::ST_ACC_EVALS, st_ev);
            atomicAdd(A.stats + rti::ST_BUMP_EVALS, st_be);
            atomicAdd(A.stats + rti::ST_OBJ_TESTS, st_ot);
        }
    }
}

// =============================================================== refinement
__device__ __forceinline__ double obj_F64(int id, V3<double> x, int ns, int np, const double *__restrict__ SPD,
                                          const double *__restrict__ PLD, const double *__restrict__ TOD) {
    if (id < ns) {
        const double *s = SPD + 4 * id;
        V3<double> d = mk(x.x - s[0], x.y - s[1], x.z - s[2]);
        return dot(d, d) - s[3] * s[3];
    }
    id -= ns;
    if (id < np) {
        const double *p = PLD + 4 * id;
        return p[0] * x.x + p[1] * x.y + p[2] * x.z - p[3];
    }
    return torus_sdf<double>(TOD + 8 * (id - np), x);
}

template <int KIND, int STEP>
__global__ __launch_bounds__(256) void k_refine(TraceArgs A, const double *__restrict__ BD,
                                                const double *__restrict__ SPD, const double *__restrict__ PLD,
                                                const double *__restrict__ TOD) {
    const int n = A.ctr[rti::CTR_REFINE];
    const int HW = A.width * A.height;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const float4 *rec = A.rec + rti::REC_F4 * (int64_t)r;
        float4 r0 = rec[0], r1 = rec[1], r2 = rec[2], r3 = rec[3], r4 = rec[4];
        V3<double> x = mk((double)r0.x + (double)r0.w, (double)r0.y + (double)r1.x, (double)r0.z + (double)r1.y);
        V3<double> y = mk((double)r1.z, (double)r1.w, (double)r2.x);
        double tk_hi = r2.y, h = r2.z;
        double sc = r2.w;
        int obj = __float_as_int(r3.x), oi = __float_as_int(r3.y), k = __float_as_int(r3.z);
        double tk_lo = r3.w;
        uint64_t mask = (uint64_t)(uint32_t)__float_as_int(r4.x) | ((uint64_t)(uint32_t)__float_as_int(r4.y) << 32);
        int set = oi / HW;
        const double *Bs = BD + (int64_t)set * A.n_bumps * 8;
        double amp = A.twist_amp, th0 = A.twist_theta0;
        auto acc = [&](V3<double> p, V3<double> v, V3<double> &a) -> bool {
            if constexpr (KIND == KIND_GRAPH) {
                a = graph_accel_f64(Bs, mask, p, v);
                return true;
            } else if constexpr (KIND == KIND_TWIST) {
                return twist_accel<double>(amp, th0, p, v, a);
            } else if constexpr (KIND == KIND_ZTWIST) {
                a = ztwist_accel<double>(p, v);
                return true;
            } else {
                a = mk(0.0, 0.0, 0.0);
                return true;
            }
        };
        V3<double> a0;
        if (STEP == STEP_RK45) acc(x, y, a0);
        auto step = [&](double hs, V3<double> &xo, V3<double> &yo) {
            V3<double> dx, dv;
            if constexpr (STEP == STEP_RK45) {
                V3<double> A1 = a0, ex, ev;
                step_dp5<double>(acc, x, y, hs, A1, dx, dv, ex, ev);
            } else if constexpr (STEP == STEP_RK4) {
                step_rk4<double>(acc, x, y, hs, dx, dv);
            } else {
                step_euler<double>(acc, x, y, hs, dx, dv);
            }
            xo = x + dx;
            yo = y + dv;
        };
        double F0 = obj_F64(obj, x, A.n_spheres, A.n_planes, SPD, PLD, TOD);
        V3<double> x1, y1;
        step(h, x1, y1);
        double F1 = obj_F64(obj, x1, A.n_spheres, A.n_planes, SPD, PLD, TOD);
        double s = sc;
        if ((F0 > 0.0) != (F1 > 0.0)) {
            double lo = 0.0, hi = 1.0;
            for (int i = 0; i < A.bisect_iters; ++i) {
                double mid = 0.5 * (lo + hi);
                V3<double> xm, ym;
                step(mid * h, xm, ym);
                if ((obj_F64(obj, xm, A.n_spheres, A.n_planes, SPD, PLD, TOD) > 0.0) == (F0 > 0.0)) lo = mid;
                else hi = mid;
            }
            s = 0.5 * (lo + hi);
        }
        V3<double> xs, ys;
        step(s * h, xs, ys);
        double tk = STEP == STEP_RK45 ? tk_hi + tk_lo : (double)k * (double)A.h;
        A.out_hit[3 * (int64_t)oi + 0] = (float)xs.x;
        A.out_hit[3 * (int64_t)oi + 1] = (float)xs.y;
        A.out_hit[3 * (int64_t)oi + 2] = (float)xs.z;
        A.out_t[oi] = (float)(tk + s * h);
        A.out_id[oi] = obj;
        double nrm = 1.0 / sqrt(dot(ys, ys));
        A.out_dir[3 * (int64_t)oi + 0] = (float)(ys.x * nrm);
        A.out_dir[3 * (int64_t)oi + 1] = (float)(ys.y * nrm);
        A.out_dir[3 * (int64_t)oi + 2] = (float)(ys.z * nrm);
        if (A.out_steps) A.out_steps[oi] = k + 1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(A.stats + rti::ST_REFINED, (unsigned long long)n);
}

__global__ void k_reset(int *ctr, int n_words, unsigned long long *stats) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += gridDim.x * blockDim.x) ctr[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < rti::ST_N) stats[threadIdx.x] = 0;
}

template <int KIND, int STEP>
hipError_t launch_kind_step(const TraceArgs &a, const rti::DeviceData &d, int n_passes, int grid, int rgrid,
                            hipStream_t s, hipEvent_t *ev) {
    for (int p = 0; p < n_passes; ++p) {
        if (a.count)
            hipLaunchKernelGGL((k_trace_pass<KIND, STEP, true>), dim3(grid), dim3(256), 0, s, a, p, d.bump_f, d.sph_f,
                               d.pln_f, d.tor_f);
        else
            hipLaunchKernelGGL((k_trace_pass<KIND, STEP, false>), dim3(grid), dim3(256), 0, s, a, p, d.bump_f,
                               d.sph_f, d.pln_f, d.tor_f);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (ev) hipEventRecord(ev[2 + p], s);
    }
    hipLaunchKernelGGL((k_refine<KIND, STEP>), dim3(rgrid), dim3(256), 0, s, a, d.bump_d, d.sph_d, d.pln_d, d.tor_d);
    hipError_t e = hipGetLastError();
    if (ev) hipEventRecord(ev[2 + n_passes], s);
    return e;
}

template <int KIND, int STEP> int occ() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_trace_pass<KIND, STEP, false>, 256, 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

}  // namespace

namespace rti {

bool supported(int kind, int step) {
    return kind >= 0 && kind <= 3 && step >= 0 && step <= 2;
}

#define RT_DISPATCH(KIND, FN, ...)                                                 \
    switch (step) {                                                                \
    case STEP_RK4: return FN<KIND, STEP_RK4>(__VA_ARGS__);                         \
    case STEP_RK45: return FN<KIND, STEP_RK45>(__VA_ARGS__);                       \
    default: return FN<KIND, STEP_EULER>(__VA_ARGS__);                             \
    }

int trace_blocks_per_cu(int kind, int step) {
    switch (kind) {
    case KIND_EUCLID: RT_DISPATCH(KIND_EUCLID, occ)
    case KIND_GRAPH: RT_DISPATCH(KIND_GRAPH, occ)
    case KIND_TWIST: RT_DISPATCH(KIND_TWIST, occ)
    default: RT_DISPATCH(KIND_ZTWIST, occ)
    }
}

hipError_t launch_trace(const TraceArgs &a, const DeviceData &d, int n_passes, int grid, int rgrid, hipStream_t s,
                        hipEvent_t *ev) {
    int words = CTR_PASS0 + n_passes * CTR_PASS_WORDS;
    if (ev) hipEventRecord(ev[0], s);
    hipLaunchKernelGGL(k_reset, dim3(64), dim3(256), 0, s, a.ctr, words, a.stats);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev) hipEventRecord(ev[1], s);
    const int step = a.step_kind;
    switch (a.kind) {
    case KIND_EUCLID: RT_DISPATCH(KIND_EUCLID, launch_kind_step, a, d, n_passes, grid, rgrid, s, ev)
    case KIND_GRAPH: RT_DISPATCH(KIND_GRAPH, launch_kind_step, a, d, n_passes, grid, rgrid, s, ev)
    case KIND_TWIST: RT_DISPATCH(KIND_TWIST, launch_kind_step, a, d, n_passes, grid, rgrid, s, ev)
    default: RT_DISPATCH(KIND_ZTWIST, launch_kind_step, a, d, n_passes, grid, rgrid, s, ev)
    }
}

}  // namespace rti
