// Riemannian illumination, direct part (Sec. 4, "Riemannian illumination"):
// a point q of a surface is lit by a point light L through the geodesics
// that connect q to L, and its radiant intensity is Lambertian, measured
// in the metric.  For every traced pixel that hit an object this pass
//   - finds a geodesic from q to L by shooting: the g-unit direction v at q
//     and the arc length T with gamma_{q,v}(T) = L, solved by Newton's
//     method on two direction angles and T (finite-difference columns for
//     the angles, the end velocity for T), starting from the straight
//     segment;
//   - marches that geodesic (RK4, each step's chord tested against every
//     object, hits within 1e-3 of q ignored) to decide whether it reaches L;
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

// Integrate the geodesic from (q, v) over arc length T: n = ceil(T / h)
// RK4 steps, the last one shortened; two-float position.  Returns false on
// a non-finite state or a step budget overrun.
template <class Acc>
__device__ __forceinline__ bool shoot(Acc &acc, V3<float> q, V3<float> v, float T, float h, int max_steps,
                                      V3<float> &X, V3<float> &Y) {
    const int n = max(1, (int)ceilf(T / h));
    if (n > max_steps) return false;
    V3<float> xh = q, xl = mk(0.f, 0.f, 0.f), y = v;
    for (int i = 0; i < n; ++i) {
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

// March the same geodesic with the chord of every step tested against every
// object; true when nothing is crossed between t = skip and t = T.
template <class Acc>
__device__ __forceinline__ bool reaches(Acc &acc, V3<float> q, V3<float> v, float T, float h, float skip,
                                        const rti::IllumArgs &A, const float4 *__restrict__ SPH,
                                        const float4 *__restrict__ PLN, const float *__restrict__ TOR) {
    const int n = max(1, (int)ceilf(T / h));
    V3<float> xh = q, xl = mk(0.f, 0.f, 0.f), y = v;
    float t = 0.f;
    for (int i = 0; i < n; ++i) {
        const float hs = i == n - 1 ? T - (float)(n - 1) * h : h;
        V3<float> dx, dv;
        if (!step_rk4<float>(acc, xh + xl, y, hs, dx, dv)) return false;
        const V3<float> p = xh + xl;
        const float DD = dot(dx, dx);
        float first = 2.f;
        for (int k = 0; k < A.n_spheres; ++k) {
            const float4 s = SPH[k];
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
        for (int k = 0; k < A.n_planes + A.n_tori; ++k) {
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

template <int KIND>
__global__ __launch_bounds__(256) void k_illum(rti::IllumArgs A, const float4 *__restrict__ BF,
                                               const float4 *__restrict__ SPH, const float4 *__restrict__ PLN,
                                               const float *__restrict__ TOR) {
    const int64_t n = (int64_t)A.n_sets * A.width * A.height;
    const int HW = A.width * A.height;
    const int stride = KIND == KIND_DEFORM ? 4 : 2;
    const uint64_t all = A.n_bumps >= 64 ? ~0ull : ((1ull << A.n_bumps) - 1ull);
    const V3<float> L = mk(A.light[0], A.light[1], A.light[2]);
    for (int64_t pix = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; pix < n;
         pix += (int64_t)gridDim.x * blockDim.x) {
        const int obj = A.id[pix];
        int status = -3;
        float shade = 0.f, T = 0.f;
        V3<float> v = mk(0.f, 0.f, 0.f);
        if (obj >= 0) {
            const int set = (int)(pix / HW);
            const float4 *__restrict__ Bs = BF + (int64_t)set * A.n_bumps * stride;
            Acc32<KIND, false> acc{Bs, all, A.twist_amp, A.twist_theta0, nullptr, nullptr};
            const V3<float> q = mk(A.hit[3 * pix], A.hit[3 * pix + 1], A.hit[3 * pix + 2]);
            auto gdd = [&](V3<float> d) { return metric_gdd<KIND>(Bs, A.n_bumps, A.twist_amp, A.twist_theta0, q, d); };
            // orthonormal frame about the straight direction to the light
            const V3<float> dl = L - q;
            const V3<float> e0 = rsqrt_(dot(dl, dl)) * dl;
            const V3<float> t0 = fabsf(e0.x) < 0.9f ? mk(1.f, 0.f, 0.f) : mk(0.f, 1.f, 0.f);
            V3<float> e1 = axpy(-dot(t0, e0), e0, t0);
            e1 = rsqrt_(dot(e1, e1)) * e1;
            const V3<float> e2 = mk(e0.y * e1.z - e0.z * e1.y, e0.z * e1.x - e0.x * e1.z, e0.x * e1.y - e0.y * e1.x);
            auto dir = [&](float al, float be) {
                const V3<float> u = axpy(be, e2, axpy(al, e1, e0));
                return rsqrt_(gdd(u)) * u;
            };
            float al = 0.f, be = 0.f;
            T = sqrtf(gdd(dl));
            bool conv = false;
            const float eps = 1e-3f;
            for (int it = 0; it < A.max_iters; ++it) {
                v = dir(al, be);
                V3<float> X, Y, Xa, Xb, Ya, Yb;
                if (!shoot(acc, q, v, T, A.h, A.max_steps, X, Y)) break;
                const V3<float> F = X - L;
                if (fmaxf(fabsf(F.x), fmaxf(fabsf(F.y), fabsf(F.z))) < A.tol) {
                    conv = true;
                    break;
                }
                if (!shoot(acc, q, dir(al + eps, be), T, A.h, A.max_steps, Xa, Ya)) break;
                if (!shoot(acc, q, dir(al, be + eps), T, A.h, A.max_steps, Xb, Yb)) break;
                // Newton step on (al, be, T): columns dX/dal, dX/dbe, dX/dT = Y
                const V3<float> ca = (1.f / eps) * (Xa - X), cb = (1.f / eps) * (Xb - X);
                const float M[9] = {ca.x, cb.x, Y.x, ca.y, cb.y, Y.y, ca.z, cb.z, Y.z};
                const float c0 = M[4] * M[8] - M[5] * M[7], c1 = M[2] * M[7] - M[1] * M[8], c2 = M[1] * M[5] - M[2] * M[4];
                const float c3 = M[5] * M[6] - M[3] * M[8], c4 = M[0] * M[8] - M[2] * M[6], c5 = M[2] * M[3] - M[0] * M[5];
                const float c6 = M[3] * M[7] - M[4] * M[6], c7 = M[1] * M[6] - M[0] * M[7], c8 = M[0] * M[4] - M[1] * M[3];
                const float det = M[0] * c0 + M[1] * c3 + M[2] * c6;
                if (!(fabsf(det) > 1e-20f)) break;
                const float idet = -1.f / det;
                float da = idet * (c0 * F.x + c1 * F.y + c2 * F.z);
                float db = idet * (c3 * F.x + c4 * F.y + c5 * F.z);
                float dT = idet * (c6 * F.x + c7 * F.y + c8 * F.z);
                // damping: at most 0.3 in the angles and half the length per step
                const float sa = fmaxf(fabsf(da), fabsf(db)) > 0.3f ? 0.3f / fmaxf(fabsf(da), fabsf(db)) : 1.f;
                const float sT = fabsf(dT) > 0.5f * T ? 0.5f * T / fabsf(dT) : 1.f;
                const float sc = fminf(sa, sT);
                al += sc * da;
                be += sc * db;
                T += sc * dT;
            }
            if (!conv) {
                status = -1;
            } else {
                // Lambert term in the metric: grad F . v / sqrt(grad F^T g^-1 grad F)
                const V3<float> gF = obj_grad(obj, q, A.n_spheres, A.n_planes, SPH, PLN, TOR);
                float G[9];
                const V3<float> E[3] = {mk(1.f, 0.f, 0.f), mk(0.f, 1.f, 0.f), mk(0.f, 0.f, 1.f)};
                for (int i = 0; i < 3; ++i) G[4 * i] = gdd(E[i]);
                for (int i = 0; i < 3; ++i)
                    for (int j = i + 1; j < 3; ++j)
                        G[3 * i + j] = G[3 * j + i] = 0.5f * (gdd(E[i] + E[j]) - G[4 * i] - G[4 * j]);
                const float a0 = G[4] * G[8] - G[5] * G[7], a1 = G[2] * G[7] - G[1] * G[8], a2 = G[1] * G[5] - G[2] * G[4];
                const float a4 = G[0] * G[8] - G[2] * G[6], a5 = G[2] * G[3] - G[0] * G[5], a8 = G[0] * G[4] - G[1] * G[3];
                const float gdet = G[0] * a0 + G[1] * (G[5] * G[6] - G[3] * G[8]) + G[2] * (G[3] * G[7] - G[4] * G[6]);
                // grad F^T adj(G) grad F / det (adj(G) symmetric for symmetric G)
                const float qf = (gF.x * (a0 * gF.x + a1 * gF.y + a2 * gF.z) + gF.y * (a1 * gF.x + a4 * gF.y + a5 * gF.z) +
                                  gF.z * (a2 * gF.x + a5 * gF.y + a8 * gF.z)) / gdet;
                const float c = dot(gF, v) * rsqrt_(qf);
                if (!(c > 0.f)) {
                    status = 2;
                } else if (reaches(acc, q, v, T, A.h, 1e-3f, A, SPH, PLN, TOR)) {
                    status = 1;
                    shade = fminf(c, 1.f);
                } else {
                    status = 0;
                }
            }
        }
        A.shade[pix] = shade;
        A.status[pix] = status;
        if (A.dir) {
            A.dir[3 * pix] = v.x;
            A.dir[3 * pix + 1] = v.y;
            A.dir[3 * pix + 2] = v.z;
        }
        if (A.len) A.len[pix] = T;
    }
}

}  // namespace

namespace rti {

hipError_t launch_illum(const IllumArgs &a, const DeviceData &d, int grid, hipStream_t s) {
    switch (a.kind) {
#define RT_ILLUM(K)                                                                                             \
    case K: hipLaunchKernelGGL((k_illum<K>), dim3(grid), dim3(256), 0, s, a, d.bump_f, d.sph_f, d.pln_f, d.tor_f); \
        break;
        RT_ILLUM(KIND_EUCLID)
        RT_ILLUM(KIND_GRAPH)
        RT_ILLUM(KIND_TWIST)
        RT_ILLUM(KIND_ZTWIST)
        RT_ILLUM(KIND_DEFORM)
        RT_ILLUM(KIND_GANISO)
        RT_ILLUM(KIND_GQUAD)
#undef RT_ILLUM
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace rti
