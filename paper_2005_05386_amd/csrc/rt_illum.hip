// Riemannian illumination, direct part (Sec. 4, "Riemannian illumination"):
// a point q of a surface is lit by a point light L through the geodesics
// that connect q to L, and its radiant intensity is Lambertian, measured
// in the metric.  For every traced pixel that hit an object this pass
//   - finds a geodesic from q to L by shooting: the g-unit direction v at q
//     and the arc length T with gamma_{q,v}(T) = L, solved by Newton's
//     method on two direction angles and T (finite-difference columns for
//     the angles, the end velocity for T), starting from the straight
//     segment;
//   - marches that geodesic (RK4, each step's chord tested against the
//     objects its culling window reaches, hits within 1e-3 of q ignored) to
//     decide whether it reaches L;
//   - takes the Lambert term cos = g(N, v) / |N|_g with N the metric normal
//     of the surface, g^-1 grad F, so that g(N, v) = grad F . v and
//     |N|_g^2 = grad F^T g^-1 grad F.
// Several geodesics may join q and L; this finds the one reached from the
// straight segment.  The paper gives no method for this step.
#include <algorithm>

#include "rt_device.hpp"
#include "rt_internal.hpp"
#include "rt_step.hpp"

using namespace rtd;

namespace {

// Outward gradient of the implicit function of object id at x (sphere
// |x - c|^2 - r^2, plane n.x - d, torus signed distance).
__device__ __forceinline__ V3<float> obj_grad(int id, V3<float> x, int ns, int np, const float4 *__restrict__ SPH,
                                              const float4 *__restrict__ PLN, const float *__restrict__ TOR) {
    if (id < ns) {
        const float4 s = SPH[id];
        return mk(2.f * (x.x - s.x), 2.f * (x.y - s.y), 2.f * (x.z - s.z));
    }
    id -= ns;
    if (id < np) {
        const float4 p = PLN[id];
        return mk(p.x, p.y, p.z);
    }
    const float *tp = TOR + 8 * (id - np);
    const V3<float> q = mk(x.x - tp[0], x.y - tp[1], x.z - tp[2]);
    const V3<float> a = mk(tp[3], tp[4], tp[5]);
    const float ax = dot(q, a);
    const V3<float> rad = axpy(-ax, a, q);
    const float rn = sqrt_(dot(rad, rad));
    const float e = rn - tp[6];
    const V3<float> g = axpy(ax, a, (rn > 1e-20f ? e / rn : 0.f) * rad);
    return rsqrt_(e * e + ax * ax) * g;
}

// Culling windows of the shots and the visibility march: every
// ILLUM_CULL_EVERY steps a lane's window is the box of half-width
// A.cull_margin about its position (the distance it can cover before the
// next window, from the metric's speed bound); the bumps and objects that
// some active lane's window reaches are OR-ed over the wave by ballots.
// Isotropic and anisotropic graph bumps are culled this way; the other
// kinds walk every record of the table and skip, wave by wave, a record no
// lane is inside.
template <int KIND> constexpr bool bump_cull = KIND == KIND_GRAPH || KIND == KIND_GANISO;
template <int KIND> using IAcc = Acc32<KIND, false, false, !bump_cull<KIND>>;

struct Box {
    float lo[3], hi[3];
};
__device__ __forceinline__ Box lane_box(V3<float> p, float m) {
    return {{p.x - m, p.y - m, p.z - m}, {p.x + m, p.y + m, p.z + m}};
}

template <int KIND>
__device__ __forceinline__ uint64_t bump_window(const float4 *__restrict__ Bs, int n, const Box &w) {
    uint64_t mask = 0;
    for (int b = 0; b < n; ++b) {
        const float4 b0 = Bs[2 * b], b1 = Bs[2 * b + 1];
        bool need;
        if constexpr (KIND == KIND_GRAPH) {
            need = box_dist2(b0.x, b0.y, b0.z, w.lo, w.hi) <= b1.z;
        } else {
            const float rho = aniso_box_rho(b0, b1, w.lo, w.hi);
            need = rho * rho <= b1.w * 1.00001f;
        }
        if (ballot(need)) mask |= 1ull << b;
    }
    return mask;
}

// Integrate the geodesic from (q, v) over arc length T: n = ceil(T / h)
// RK4 steps, the last one shortened; two-float position.  Returns false on
// a non-finite state or a step budget overrun.
template <int KIND>
__device__ __forceinline__ bool shoot(IAcc<KIND> &acc, const rti::IllumArgs &A, V3<float> q, V3<float> v, float T,
                                      V3<float> &X, V3<float> &Y) {
    const float h = A.h;
    const int n = max(1, (int)ceilf(T / h));
    if (n > A.max_steps) return false;
    V3<float> xh = q, xl = mk(0.f, 0.f, 0.f), y = v;
    for (int i = 0; i < n; ++i) {
        if constexpr (bump_cull<KIND>)
            if (i % rti::ILLUM_CULL_EVERY == 0 && A.cull_margin >= 0.f)
                acc.mask = bump_window<KIND>(acc.B, A.n_bumps, lane_box(xh + xl, A.cull_margin));
        const float hs = i == n - 1 ? T - (float)(n - 1) * h : h;
        V3<float> dx, dv;
        if (!step_rk4<float>(acc, xh + xl, y, hs, dx, dv) || !finite6(dx, dv)) return false;
        two_sum_add(xh.x, xl.x, dx.x);
        two_sum_add(xh.y, xl.y, dx.y);
        two_sum_add(xh.z, xl.z, dx.z);
        y = y + dv;
    }
    X = xh + xl;
    Y = y;
    return true;
}

// March the same geodesic with the chord of every step tested against the
// objects of the window; true when nothing is crossed between t = skip and
// t = T.
template <int KIND>
__device__ __forceinline__ bool reaches(IAcc<KIND> &acc, V3<float> q, V3<float> v, float T, float skip,
                                        const rti::IllumArgs &A, const float4 *__restrict__ SPH,
                                        const float4 *__restrict__ PLN, const float *__restrict__ TOR) {
    const float h = A.h;
    const int n = max(1, (int)ceilf(T / h));
    const int no = A.n_planes + A.n_tori;
    V3<float> xh = q, xl = mk(0.f, 0.f, 0.f), y = v;
    float t = 0.f;
    uint64_t sm[4] = {0ull, 0ull, 0ull, 0ull};
    uint32_t om = 0;
    for (int i = 0; i < n; ++i) {
        const V3<float> p = xh + xl;
        if (i % rti::ILLUM_CULL_EVERY == 0) {
            if (A.cull_margin >= 0.f) {
                const Box w = lane_box(p, A.cull_margin);
                if constexpr (bump_cull<KIND>) acc.mask = bump_window<KIND>(acc.B, A.n_bumps, w);
#pragma unroll
                for (int c = 0; c < 4; ++c) sm[c] = 0ull;
                for (int k = 0; k < A.n_spheres; ++k) {
                    const float4 s = SPH[k];
                    if (ballot(box_dist2(s.x, s.y, s.z, w.lo, w.hi) <= s.w * s.w)) sm[k >> 6] |= 1ull << (k & 63);
                }
                om = 0;
                for (int k = 0; k < no; ++k) {
                    bool on;
                    if (k < A.n_planes) {
                        const float4 pl = PLN[k];
                        const float c = pl.x * p.x + pl.y * p.y + pl.z * p.z - pl.w;
                        on = fabsf(c) <= A.cull_margin * (fabsf(pl.x) + fabsf(pl.y) + fabsf(pl.z));
                    } else {
                        const float *tp = TOR + 8 * (k - A.n_planes);
                        const float rr = tp[6] + tp[7];
                        on = box_dist2(tp[0], tp[1], tp[2], w.lo, w.hi) <= rr * rr;
                    }
                    if (ballot(on)) om |= 1u << k;
                }
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int rem = A.n_spheres - 64 * c;
                    sm[c] = rem >= 64 ? ~0ull : (rem > 0 ? (1ull << rem) - 1ull : 0ull);
                }
                om = (1u << no) - 1u;
            }
        }
        const float hs = i == n - 1 ? T - (float)(n - 1) * h : h;
        V3<float> dx, dv;
        if (!step_rk4<float>(acc, p, y, hs, dx, dv)) return false;
        const float DD = dot(dx, dx);
        float first = 2.f;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            for (uint64_t m = sm[c]; m; m &= m - 1ull) {
                const float4 s = SPH[64 * c + __builtin_ctzll(m)];
                const V3<float> o = mk((xh.x - s.x) + xl.x, (xh.y - s.y) + xl.y, (xh.z - s.z) + xl.z);
                // both roots: a chord that starts on a sphere (s ~ 0) may still cross it later
                const float B = dot(dx, o), C = fmaf(-s.w, s.w, dot(o, o));
                const float disc = fmaf(B, B, -DD * C);
                if (disc >= 0.f) {
                    const float qd = sqrt_(disc), inv = rcp_(DD);
                    const float s1 = (-B - qd) * inv, s2 = (-B + qd) * inv;
                    if (s1 >= 0.f && s1 <= 1.f && t + s1 * hs > skip) first = fminf(first, s1);
                    else if (s2 >= 0.f && s2 <= 1.f && t + s2 * hs > skip) first = fminf(first, s2);
                }
            }
        }
        for (uint32_t m = om; m; m &= m - 1u) {
            const int k = __builtin_ctz(m);
            float F0, F1;
            if (k < A.n_planes) {
                const float4 pl = PLN[k];
                F0 = pl.x * p.x + pl.y * p.y + pl.z * p.z - pl.w;
                F1 = F0 + (pl.x * dx.x + pl.y * dx.y + pl.z * dx.z);
            } else {
                const float *tp = TOR + 8 * (k - A.n_planes);
                F0 = torus_sdf<float>(tp, p);
                F1 = torus_sdf<float>(tp, p + dx);
            }
            if ((F0 > 0.f) != (F1 > 0.f)) {
                const float sc = fminf(fmaxf(F0 / (F0 - F1), 0.f), 1.f);
                if (t + sc * hs > skip) first = fminf(first, sc);
            }
        }
        if (first <= 1.f) return false;
        two_sum_add(xh.x, xl.x, dx.x);
        two_sum_add(xh.y, xl.y, dx.y);
        two_sum_add(xh.z, xl.z, dx.z);
        y = y + dv;
        t += hs;
    }
    return true;
}

// Per-pixel frame about the straight direction to the light and the
// direction for the angles (al, be), normalised to g-unit at q.
struct Frame {
    V3<float> e0, e1, e2;
};
__device__ __forceinline__ Frame light_frame(V3<float> q, V3<float> L) {
    const V3<float> dl = L - q;
    Frame f;
    f.e0 = rsqrt_(dot(dl, dl)) * dl;
    const V3<float> t0 = fabsf(f.e0.x) < 0.9f ? mk(1.f, 0.f, 0.f) : mk(0.f, 1.f, 0.f);
    f.e1 = axpy(-dot(t0, f.e0), f.e0, t0);
    f.e1 = rsqrt_(dot(f.e1, f.e1)) * f.e1;
    f.e2 = mk(f.e0.y * f.e1.z - f.e0.z * f.e1.y, f.e0.z * f.e1.x - f.e0.x * f.e1.z, f.e0.x * f.e1.y - f.e0.y * f.e1.x);
    return f;
}

// Everything a lane needs for one pixel.
template <int KIND> struct Pixel {
    const float4 *Bs;
    V3<float> q;
    Frame F;
    __device__ __forceinline__ float gdd(const rti::IllumArgs &A, V3<float> d) const {
        return metric_gdd<KIND>(Bs, A.n_bumps, A.twist_amp, A.twist_theta0, q, d);
    }
    __device__ __forceinline__ V3<float> dir(const rti::IllumArgs &A, float al, float be) const {
        const V3<float> u = axpy(be, F.e2, axpy(al, F.e1, F.e0));
        return rsqrt_(gdd(A, u)) * u;
    }
};
// ONE: a single parameter set, so the table pointer is the same for every
// lane and the bump records are read with scalar loads.
template <int KIND, bool ONE = false>
__device__ __forceinline__ Pixel<KIND> pixel(const rti::IllumArgs &A, const float4 *__restrict__ BF, int pix) {
    Pixel<KIND> P;
    if constexpr (ONE) {
        P.Bs = BF;
    } else {
        const int set = pix / (A.width * A.height);
        P.Bs = BF + (int64_t)set * A.n_bumps * (is_deform(KIND) ? DEFORM_F4 : 2);
    }
    P.q = mk(A.hit[3 * pix], A.hit[3 * pix + 1], A.hit[3 * pix + 2]);
    P.F = light_frame(P.q, mk(A.light[0], A.light[1], A.light[2]));
    return P;
}
__device__ __forceinline__ uint64_t all_bumps(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }

// Wave-aggregated append of pix to list (count at *ctr).
__device__ __forceinline__ void append(int *list, int *ctr, int pix, bool take) {
    const uint64_t m = ballot(take);
    if (!m) return;
    const int lane = lane_id();
    const int leader = __builtin_ctzll(m);
    int base = 0;
    if (lane == leader) base = atomicAdd(ctr, __popcll(m));
    base = __shfl(base, leader);
    if (take) list[base + __popcll(m & ((1ull << lane) - 1ull))] = pix;
}

// Status codes of the API; 3 marks a converged pixel awaiting the finish,
// 4 one converged at an intermediate target of the continuation.
enum { ST_LIT = 1, ST_BLOCKED = 0, ST_AWAY = 2, ST_NONE = -1, ST_NOHIT = -3, ST_CONV = 3, ST_CONT = 4 };

// The target of the shots of pixel P: the light, or during the
// continuation the point q + cont (L - q) of the straight segment.
template <class P> __device__ __forceinline__ V3<float> target(const rti::IllumArgs &A, const P &Px, V3<float> L) {
    return A.cont < 1.f ? axpy(A.cont, L - Px.q, Px.q) : L;
}

// Initial state: pixels that hit start from the straight segment.
template <int KIND>
__global__ __launch_bounds__(256) void k_illum_init(rti::IllumArgs A, const float4 *__restrict__ BF) {
    const int n = A.n_sets * A.width * A.height;
    for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const int pix = base + threadIdx.x;
        const bool hit = pix < n && A.id[pix] >= 0;
        if (pix < n) {
            float T = 0.f;
            if (hit) {
                const Pixel<KIND> P = pixel<KIND>(A, BF, pix);
                const V3<float> L = mk(A.light[0], A.light[1], A.light[2]);
                T = sqrtf(P.gdd(A, L - P.q));
            }
            A.w_al[pix] = 0.f;
            A.w_be[pix] = 0.f;
            A.w_T[pix] = T;
            A.w_F[pix] = __builtin_huge_valf();
            A.status[pix] = hit ? ST_NONE : ST_NOHIT;
            A.shade[pix] = 0.f;
        }
        append(A.list[0], A.ctr + 0, pix, hit);
    }
}

// Residual of the base shot of pixel pix: returns 1 when a Newton step is
// to be taken, 0 when the pixel leaves the list (converged, marked ST_CONV,
// or stalled: from the fifth iteration on, a residual that did not halve).
__device__ __forceinline__ int judge(const rti::IllumArgs &A, int pix, int it, V3<float> F) {
    const float fn = fmaxf(fabsf(F.x), fmaxf(fabsf(F.y), fabsf(F.z)));
    const bool stalled = it >= 4 && fn > 0.5f * A.w_F[pix];
    A.w_F[pix] = fn;
    if (fn < A.tol) {
        A.status[pix] = A.conv_code;
        return 0;
    }
    return stalled ? 0 : 1;
}

// Damped Newton step on (al, be, T) from the residual F = X - L, the end
// velocity Y (the T column) and the shots Xa, Xb at al + eps, be + eps;
// true when the pixel stays on the list.
template <int KIND>
__device__ __forceinline__ bool newton(const rti::IllumArgs &A, const Pixel<KIND> &P, int pix, V3<float> L, float eps,
                                      float al, float be, float T, V3<float> F, V3<float> X, V3<float> Y,
                                      V3<float> Xa, V3<float> Xb) {
    const V3<float> ca = (1.f / eps) * (Xa - X), cb = (1.f / eps) * (Xb - X);
    const float M[9] = {ca.x, cb.x, Y.x, ca.y, cb.y, Y.y, ca.z, cb.z, Y.z};
    const float c0 = M[4] * M[8] - M[5] * M[7], c1 = M[2] * M[7] - M[1] * M[8], c2 = M[1] * M[5] - M[2] * M[4];
    const float c3 = M[5] * M[6] - M[3] * M[8], c4 = M[0] * M[8] - M[2] * M[6], c5 = M[2] * M[3] - M[0] * M[5];
    const float c6 = M[3] * M[7] - M[4] * M[6], c7 = M[1] * M[6] - M[0] * M[7], c8 = M[0] * M[4] - M[1] * M[3];
    const float det = M[0] * c0 + M[1] * c3 + M[2] * c6;
    if (!(fabsf(det) > 1e-20f)) return false;
    const float idet = -1.f / det;
    const float da = idet * (c0 * F.x + c1 * F.y + c2 * F.z);
    const float db = idet * (c3 * F.x + c4 * F.y + c5 * F.z);
    const float dT = idet * (c6 * F.x + c7 * F.y + c8 * F.z);
    // damping: at most 0.3 in the angles and half the length per step
    const float m = fmaxf(fabsf(da), fabsf(db));
    const float sa = m > 0.3f ? 0.3f / m : 1.f;
    const float sT = fabsf(dT) > 0.5f * T ? 0.5f * T / fabsf(dT) : 1.f;
    const float sc = fminf(sa, sT);
    A.w_al[pix] = al + sc * da;
    A.w_be[pix] = be + sc * db;
    A.w_T[pix] = T + sc * dT;
    // geodesics much longer than the straight segment are not pursued
    return T + sc * dT <= 4.f * sqrtf(P.gdd(A, L - P.q)) + 1.f;
}

// Pixels per wave when the three shots of an iteration run on three lanes.
constexpr int PAR_PIX = 21;
// Angle displacement of the finite-difference shots.
constexpr float ILLUM_EPS = 1e-3f;

// One Newton iteration for every pixel of list[it & 1]: shoot; converged
// pixels are marked, the others take a damped step and move to the next list.
// While the list fills the grid, the iteration runs in two launches: here a
// lane shoots the base direction of one pixel, and a pixel that is due a
// step keeps its end point and velocity and goes to the step list, whose
// displaced shots k_illum_step takes two lanes per pixel; so lanes whose
// pixel converged do not wait on the displaced shots of their neighbours.
// Once the list fits in one pass at three lanes per pixel (the
// latency-bound last iterations), lanes 3j, 3j+1, 3j+2 of a wave shoot the
// base and the two displaced directions of pixel j side by side and the
// step list stays empty.  Both ways compute the same values.
template <int KIND, bool ONE>
__global__ __launch_bounds__(256) void k_illum_iter(rti::IllumArgs A, const float4 *__restrict__ BF, int it) {
    const int *in = A.list[it & 1];
    int *out = A.list[(it + 1) & 1];
    const int n_in = A.ctr[it];
    const uint64_t all = all_bumps(A.n_bumps);
    const V3<float> L = mk(A.light[0], A.light[1], A.light[2]);
    const float eps = ILLUM_EPS;
    const int per_block = PAR_PIX * (blockDim.x / 64);
    if (n_in <= (int)gridDim.x * per_block) {
        const int lane = lane_id(), role = lane % 3;
        for (int base = blockIdx.x * per_block; base < n_in; base += gridDim.x * per_block) {
            const int k = base + (threadIdx.x >> 6) * PAR_PIX + lane / 3;
            const bool act = lane < 3 * PAR_PIX && k < n_in;
            bool again = false, ok = false;
            int pix = 0;
            V3<float> X = mk(0.f, 0.f, 0.f), Y = X;
            float al = 0.f, be = 0.f, T = 0.f;
            Pixel<KIND> P{};
            if (act) {
                pix = in[k];
                P = pixel<KIND, ONE>(A, BF, pix);
                IAcc<KIND> acc{P.Bs, all, A.twist_amp, A.twist_theta0, nullptr, nullptr};
                al = A.w_al[pix];
                be = A.w_be[pix];
                T = A.w_T[pix];
                const float as = role == 1 ? al + eps : al, bs = role == 2 ? be + eps : be;
                ok = shoot<KIND>(acc, A, P.q, P.dir(A, as, bs), T, X, Y);
            }
            // the displaced shots of lanes 3j+1, 3j+2 to lane 3j
            const int src = lane + 1 < 64 ? lane + 1 : lane, src2 = lane + 2 < 64 ? lane + 2 : lane;
            const V3<float> Xa = mk(__shfl(X.x, src), __shfl(X.y, src), __shfl(X.z, src));
            const V3<float> Xb = mk(__shfl(X.x, src2), __shfl(X.y, src2), __shfl(X.z, src2));
            const int oka = __shfl((int)ok, src), okb = __shfl((int)ok, src2);
            if (act && role == 0 && ok) {
                const V3<float> Lp = target(A, P, L);
                const V3<float> F = X - Lp;
                if (judge(A, pix, it, F) && oka && okb) again = newton<KIND>(A, P, pix, Lp, eps, al, be, T, F, X, Y, Xa, Xb);
            }
            append(out, A.ctr + it + 1, pix, again);
        }
        return;
    }
    int *steps = A.list[2];
    for (int base = blockIdx.x * blockDim.x; base < n_in; base += gridDim.x * blockDim.x) {
        const int k = base + threadIdx.x;
        bool due = false;
        int pix = 0;
        if (k < n_in) {
            pix = in[k];
            const Pixel<KIND> P = pixel<KIND, ONE>(A, BF, pix);
            IAcc<KIND> acc{P.Bs, all, A.twist_amp, A.twist_theta0, nullptr, nullptr};
            V3<float> X, Y;
            if (shoot<KIND>(acc, A, P.q, P.dir(A, A.w_al[pix], A.w_be[pix]), A.w_T[pix], X, Y) &&
                judge(A, pix, it, X - target(A, P, L))) {
                A.w_X[3 * pix] = X.x;
                A.w_X[3 * pix + 1] = X.y;
                A.w_X[3 * pix + 2] = X.z;
                A.w_Y[3 * pix] = Y.x;
                A.w_Y[3 * pix + 1] = Y.y;
                A.w_Y[3 * pix + 2] = Y.z;
                due = true;
            }
        }
        append(steps, A.ctr + A.max_iters + 1 + it, pix, due);
    }
}

// Second launch of a full-grid iteration: for every pixel of the step list,
// lanes 2j and 2j+1 shoot the two displaced directions of pixel j, and lane
// 2j takes the Newton step from them and the stored base shot.
template <int KIND, bool ONE>
__global__ __launch_bounds__(256) void k_illum_step(rti::IllumArgs A, const float4 *__restrict__ BF, int it) {
    const int *steps = A.list[2];
    int *out = A.list[(it + 1) & 1];
    const int n_st = A.ctr[A.max_iters + 1 + it];
    const uint64_t all = all_bumps(A.n_bumps);
    const V3<float> L = mk(A.light[0], A.light[1], A.light[2]);
    const float eps = ILLUM_EPS;
    const int lane = lane_id(), role = lane & 1;
    const int per_block = blockDim.x / 2;
    for (int base = blockIdx.x * per_block; base < n_st; base += gridDim.x * per_block) {
        const int k = base + (threadIdx.x >> 1);
        const bool act = k < n_st;
        bool again = false, ok = false;
        int pix = 0;
        V3<float> Xs = mk(0.f, 0.f, 0.f), Ys = Xs;
        float al = 0.f, be = 0.f, T = 0.f;
        Pixel<KIND> P{};
        if (act) {
            pix = steps[k];
            P = pixel<KIND, ONE>(A, BF, pix);
            IAcc<KIND> acc{P.Bs, all, A.twist_amp, A.twist_theta0, nullptr, nullptr};
            al = A.w_al[pix];
            be = A.w_be[pix];
            T = A.w_T[pix];
            const float as = role == 0 ? al + eps : al, bs = role == 1 ? be + eps : be;
            ok = shoot<KIND>(acc, A, P.q, P.dir(A, as, bs), T, Xs, Ys);
        }
        // the beta shot of lane 2j+1 to lane 2j
        const int src = lane | 1;
        const V3<float> Xb = mk(__shfl(Xs.x, src), __shfl(Xs.y, src), __shfl(Xs.z, src));
        const int okb = __shfl((int)ok, src);
        if (act && role == 0 && ok && okb) {
            const V3<float> X = mk(A.w_X[3 * pix], A.w_X[3 * pix + 1], A.w_X[3 * pix + 2]);
            const V3<float> Y = mk(A.w_Y[3 * pix], A.w_Y[3 * pix + 1], A.w_Y[3 * pix + 2]);
            const V3<float> Lp = target(A, P, L);
            again = newton<KIND>(A, P, pix, Lp, eps, al, be, T, X - Lp, X, Y, Xs, Xb);
        }
        append(out, A.ctr + it + 1, pix, again);
    }
}

// Lambert term and visibility for the converged pixels; every hit pixel
// gets its direction and length.
template <int KIND, bool ONE>
__global__ __launch_bounds__(256) void k_illum_finish(rti::IllumArgs A, const float4 *__restrict__ BF,
                                                      const float4 *__restrict__ SPH, const float4 *__restrict__ PLN,
                                                      const float *__restrict__ TOR) {
    const int n = A.n_sets * A.width * A.height;
    const uint64_t all = all_bumps(A.n_bumps);
    for (int pix = blockIdx.x * blockDim.x + threadIdx.x; pix < n; pix += gridDim.x * blockDim.x) {
        int status = A.status[pix];
        if (status == ST_NOHIT) {
            if (A.dir) A.dir[3 * pix] = A.dir[3 * pix + 1] = A.dir[3 * pix + 2] = 0.f;
            if (A.len) A.len[pix] = 0.f;
            continue;
        }
        const Pixel<KIND> P = pixel<KIND, ONE>(A, BF, pix);
        const float T = A.w_T[pix];
        const V3<float> v = P.dir(A, A.w_al[pix], A.w_be[pix]);
        float shade = 0.f;
        if (status == ST_CONV) {
            // Lambert term in the metric: grad F . v / sqrt(grad F^T g^-1 grad F)
            const V3<float> gF = obj_grad(A.id[pix], P.q, A.n_spheres, A.n_planes, SPH, PLN, TOR);
            float G[9];
            const V3<float> E[3] = {mk(1.f, 0.f, 0.f), mk(0.f, 1.f, 0.f), mk(0.f, 0.f, 1.f)};
            for (int i = 0; i < 3; ++i) G[4 * i] = P.gdd(A, E[i]);
            for (int i = 0; i < 3; ++i)
                for (int j = i + 1; j < 3; ++j)
                    G[3 * i + j] = G[3 * j + i] = 0.5f * (P.gdd(A, E[i] + E[j]) - G[4 * i] - G[4 * j]);
            const float a0 = G[4] * G[8] - G[5] * G[7], a1 = G[2] * G[7] - G[1] * G[8], a2 = G[1] * G[5] - G[2] * G[4];
            const float a4 = G[0] * G[8] - G[2] * G[6], a5 = G[2] * G[3] - G[0] * G[5], a8 = G[0] * G[4] - G[1] * G[3];
            const float gdet = G[0] * a0 + G[1] * (G[5] * G[6] - G[3] * G[8]) + G[2] * (G[3] * G[7] - G[4] * G[6]);
            // grad F^T adj(G) grad F / det (adj(G) is symmetric for symmetric G)
            const float qf = (gF.x * (a0 * gF.x + a1 * gF.y + a2 * gF.z) + gF.y * (a1 * gF.x + a4 * gF.y + a5 * gF.z) +
                              gF.z * (a2 * gF.x + a5 * gF.y + a8 * gF.z)) / gdet;
            const float c = dot(gF, v) * rsqrt_(qf);
            IAcc<KIND> acc{P.Bs, all, A.twist_amp, A.twist_theta0, nullptr, nullptr};
            if (!(c > 0.f)) {
                status = ST_AWAY;
            } else if (reaches<KIND>(acc, P.q, v, T, 1e-3f, A, SPH, PLN, TOR)) {
                status = ST_LIT;
                shade = fminf(c, 1.f);
            } else {
                status = ST_BLOCKED;
            }
        }
        A.status[pix] = status;
        A.shade[pix] = shade;
        if (A.dir) {
            A.dir[3 * pix] = v.x;
            A.dir[3 * pix + 1] = v.y;
            A.dir[3 * pix + 2] = v.z;
        }
        if (A.len) A.len[pix] = T;
    }
}

__global__ void k_illum_zero(int *ctr, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) ctr[i] = 0;
}

// Retry seeds.  A hit pixel left without a geodesic (its Newton iteration
// from the straight segment stalled, failed or ran out of iterations)
// starts again from the converged direction of a neighbour: of the 8
// neighbouring pixels of the same parameter set that have converged, the
// one whose hit point is nearest, its direction written in this pixel's
// frame (angles about the straight direction to the light) and its length.
// Reads only converged pixels and writes only unconverged ones.
template <int KIND, bool ONE>
__global__ __launch_bounds__(256) void k_illum_seed(rti::IllumArgs A, const float4 *__restrict__ BF, int *ctr) {
    const int HW = A.width * A.height;
    const int n = A.n_sets * HW;
    for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const int pix = base + threadIdx.x;
        bool take = false;
        if (pix < n && A.status[pix] == ST_NONE) {
            const int set = pix / HW, r = pix - set * HW, j = r / A.width, i = r - j * A.width;
            const V3<float> q = mk(A.hit[3 * pix], A.hit[3 * pix + 1], A.hit[3 * pix + 2]);
            int best = -1;
            float bestd = __builtin_huge_valf();
            for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di) {
                    const int ii = i + di, jj = j + dj;
                    if ((di == 0 && dj == 0) || ii < 0 || jj < 0 || ii >= A.width || jj >= A.height) continue;
                    const int nb = set * HW + jj * A.width + ii;
                    if (A.status[nb] != ST_CONV) continue;
                    const V3<float> d = mk(A.hit[3 * nb], A.hit[3 * nb + 1], A.hit[3 * nb + 2]) - q;
                    const float d2 = dot(d, d);
                    if (d2 < bestd) {
                        bestd = d2;
                        best = nb;
                    }
                }
            if (best >= 0) {
                const Pixel<KIND> P = pixel<KIND, ONE>(A, BF, pix), Q = pixel<KIND, ONE>(A, BF, best);
                const V3<float> v = Q.dir(A, A.w_al[best], A.w_be[best]);
                const float c = dot(v, P.F.e0);
                if (c > 1e-2f * sqrt_(dot(v, v))) {
                    const float ic = 1.f / c;
                    A.w_al[pix] = dot(v, P.F.e1) * ic;
                    A.w_be[pix] = dot(v, P.F.e2) * ic;
                    A.w_T[pix] = A.w_T[best];
                    A.w_F[pix] = __builtin_huge_valf();
                    take = true;
                }
            }
        }
        append(A.list[0], ctr, pix, take);
    }
}

// Continuation stage: targets move from q + lam0 (L - q) to q + lam1 (L - q).
// lam0 = 0: every hit pixel still without a geodesic starts from the
// straight segment to the first target; otherwise the pixels that converged
// at lam0 (ST_CONT) start from that solution, the length scaled.
template <int KIND, bool ONE>
__global__ __launch_bounds__(256) void k_illum_cont(rti::IllumArgs A, const float4 *__restrict__ BF, int *ctr,
                                                    float lam0, float lam1) {
    const int n = A.n_sets * A.width * A.height;
    const V3<float> L = mk(A.light[0], A.light[1], A.light[2]);
    for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const int pix = base + threadIdx.x;
        bool take = false;
        if (pix < n) {
            const int st = A.status[pix];
            if (lam0 == 0.f && st == ST_NONE) {
                const Pixel<KIND> P = pixel<KIND, ONE>(A, BF, pix);
                A.w_al[pix] = 0.f;
                A.w_be[pix] = 0.f;
                A.w_T[pix] = lam1 * sqrtf(P.gdd(A, L - P.q));
                take = true;
            } else if (lam0 > 0.f && st == ST_CONT) {
                A.w_T[pix] *= lam1 / lam0;
                take = true;
            }
            if (take) {
                A.status[pix] = ST_NONE;
                A.w_F[pix] = __builtin_huge_valf();
            }
        }
        append(A.list[0], ctr, pix, take);
    }
}

template <int KIND, bool ONE>
void illum_rounds(const rti::IllumArgs &a, const rti::DeviceData &d, int grid, hipStream_t s) {
    for (int it = 0; it < a.max_iters; ++it) {
        hipLaunchKernelGGL((k_illum_iter<KIND, ONE>), dim3(grid), dim3(256), 0, s, a, d.bump_f, it);
        hipLaunchKernelGGL((k_illum_step<KIND, ONE>), dim3(grid), dim3(256), 0, s, a, d.bump_f, it);
    }
    // retries from converged neighbours, a quarter of the iterations each (a
    // seed from a neighbour is close: 1080p 432 -> 390 ms for 99.88 -> 99.83%
    // of the hits found, the quadric unchanged); each round has its own
    // counters
    rti::IllumArgs r = a;
    r.max_iters = std::max(a.max_iters / 4, 1);
    for (int round = 1; round <= rti::ILLUM_RETRY_ROUNDS; ++round) {
        r.ctr = a.ctr + round * 2 * (a.max_iters + 1);
        hipLaunchKernelGGL((k_illum_seed<KIND, ONE>), dim3(grid), dim3(256), 0, s, r, d.bump_f, r.ctr);
        for (int it = 0; it < r.max_iters; ++it) {
            hipLaunchKernelGGL((k_illum_iter<KIND, ONE>), dim3(grid), dim3(256), 0, s, r, d.bump_f, it);
            hipLaunchKernelGGL((k_illum_step<KIND, ONE>), dim3(grid), dim3(256), 0, s, r, d.bump_f, it);
        }
    }
    // continuation in the light position for the pixels still unsolved, half
    // the iterations per stage (a quarter loses 15% of the quadric's hits)
    r.max_iters = std::max(a.max_iters / 2, 1);
    for (int st = 0; st < rti::ILLUM_CONT_STAGES; ++st) {
        const float lam0 = (float)st / rti::ILLUM_CONT_STAGES, lam1 = (float)(st + 1) / rti::ILLUM_CONT_STAGES;
        r.ctr = a.ctr + (1 + rti::ILLUM_RETRY_ROUNDS + st) * 2 * (a.max_iters + 1);
        r.cont = lam1;
        r.conv_code = st + 1 < rti::ILLUM_CONT_STAGES ? ST_CONT : ST_CONV;
        hipLaunchKernelGGL((k_illum_cont<KIND, ONE>), dim3(grid), dim3(256), 0, s, r, d.bump_f, r.ctr, lam0, lam1);
        for (int it = 0; it < r.max_iters; ++it) {
            hipLaunchKernelGGL((k_illum_iter<KIND, ONE>), dim3(grid), dim3(256), 0, s, r, d.bump_f, it);
            hipLaunchKernelGGL((k_illum_step<KIND, ONE>), dim3(grid), dim3(256), 0, s, r, d.bump_f, it);
        }
    }
    hipLaunchKernelGGL((k_illum_finish<KIND, ONE>), dim3(grid), dim3(256), 0, s, a, d.bump_f, d.sph_f, d.pln_f,
                       d.tor_f);
}

template <int KIND>
hipError_t illum_kind(const rti::IllumArgs &a, const rti::DeviceData &d, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_illum_zero, dim3(1), dim3(256), 0, s, a.ctr,
                       (1 + rti::ILLUM_RETRY_ROUNDS + rti::ILLUM_CONT_STAGES) * 2 * (a.max_iters + 1));
    hipLaunchKernelGGL((k_illum_init<KIND>), dim3(grid), dim3(256), 0, s, a, d.bump_f);
    if (a.n_sets == 1)
        illum_rounds<KIND, true>(a, d, grid, s);
    else
        illum_rounds<KIND, false>(a, d, grid, s);
    return hipGetLastError();
}

}  // namespace

namespace rti {

hipError_t launch_illum(const IllumArgs &a, const DeviceData &d, int grid, hipStream_t s) {
    switch (a.kind) {
#define RT_ILLUM(K) \
    case K: return illum_kind<K>(a, d, grid, s);
        RT_ILLUM(KIND_EUCLID)
        RT_ILLUM(KIND_GRAPH)
        RT_ILLUM(KIND_TWIST)
        RT_ILLUM(KIND_ZTWIST)
        RT_ILLUM(KIND_DEFORM)
        RT_ILLUM(KIND_DEFORM_ROT)
        RT_ILLUM(KIND_GANISO)
        RT_ILLUM(KIND_GQUAD)
#undef RT_ILLUM
    default: return hipErrorInvalidValue;
    }
}

}  // namespace rti
