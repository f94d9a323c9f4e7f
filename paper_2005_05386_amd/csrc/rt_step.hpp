// Integration steps shared by the trace and the adjoint kernels, so that
// the adjoint's recomputation of a trajectory repeats the forward
// arithmetic exactly.
#pragma once

#include "rt_device.hpp"

namespace rtd {

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
__device__ __forceinline__ bool step_euler(F &acc, V3<T> p, V3<T> y, T h, V3<T> &dx, V3<T> &dv,
                                           const V3<T> *k1 = nullptr) {
    V3<T> a;
    bool ok = true;
    if (k1)
        a = *k1;
    else
        ok = acc(p, y, a);
    dx = h * y;
    dv = h * a;
    return ok;
}

template <class T, class F>
__device__ __forceinline__ bool step_rk4(F &acc, V3<T> p, V3<T> y, T h, V3<T> &dx, V3<T> &dv,
                                         const V3<T> *k1 = nullptr) {
    // Classical RK4 on (x, y): stage s evaluates k_s = a(P_s, Y_s) with
    // (P_0, Y_0) = (p, y) and (P_s, Y_s) = (p + c_s Y_{s-1}, y + c_s k_{s-1}),
    // c = (h/2, h/2, h); the stage sums with weights (1, 2, 2, 1) are
    // accumulated as the stages are produced.
    const T hh = T(0.5) * h;
    V3<T> P = p, Y = y;
    V3<T> sx, sv;
    bool ok = true;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        V3<T> k;
        if (st == 0 && k1)
            k = *k1;  // first stage supplied by the caller
        else
            ok &= acc(P, Y, k);
        if (st == 0) {
            sx = Y;
            sv = k;
        } else {
            const T w = st == 3 ? T(1) : T(2);
            sx = axpy(w, Y, sx);
            sv = axpy(w, k, sv);
        }
        const T c = st < 2 ? hh : h;
        P = axpy(c, Y, p);
        Y = axpy(c, k, y);
    }
    const T h6 = h * T(1.0 / 6.0);
    dx = h6 * sx;
    dv = h6 * sv;
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

// (hi, lo) += d for a two-float value: Dekker's Fast2Sum of hi and d, its
// rounding error added to lo.  hi is the plain float sum of the increments
// and lo collects what that sum dropped; the value is hi + lo (exact in
// double, and hi + lo rounded for the float arithmetic).  lo is not folded
// back into hi: over n steps it grows to at most n/2 ulps of hi, and its own
// rounding then adds at most n ulps of lo, far below the steps' truncation
// error (4000 steps near |x| = 10: |lo| < 2e-3, error < 5e-7).  Fast2Sum is
// exact when hi's exponent is at least d's; otherwise (a coordinate within
// one step of zero) the error term is off by at most about half an ulp of d.
__device__ __forceinline__ void two_sum_add(float &hi, float &lo, float d) {
    const float s = hi + d;
    lo += d - (s - hi);
    hi = s;
}

__device__ __forceinline__ float box_dist2(float cx, float cy, float cz, const float lo[3], const float hi[3]) {
    float dx = fmaxf(fmaxf(lo[0] - cx, cx - hi[0]), 0.0f);
    float dy = fmaxf(fmaxf(lo[1] - cy, cy - hi[1]), 0.0f);
    float dz = fmaxf(fmaxf(lo[2] - cz, cz - hi[2]), 0.0f);
    return dx * dx + dy * dy + dz * dz;
}

// One test for six components: a NaN or infinity in any of them makes the
// sum non-finite (as does a sum beyond the float range, a failed state too).
__device__ __forceinline__ bool finite6(V3<float> a, V3<float> b) {
    return __builtin_isfinite(((a.x + a.y) + (a.z + b.x)) + (b.y + b.z));
}

// SREG: the bump mask is wave-uniform and held in scalar registers.
// WAVE: the lanes of a wave share the mask but not their region; a bump or
// deformation none of them is inside is skipped by the wave.
template <int KIND, bool COUNT, bool SREG = false, bool WAVE = false> struct Acc32 {
    const float4 *__restrict__ B;
    uint64_t mask;
    float amp, th0;
    unsigned *n_eval, *n_bump;  // COUNT only
    __device__ __forceinline__ bool operator()(V3<float> p, V3<float> y, V3<float> &a) const {
        if (COUNT) *n_eval += 1;
        if constexpr (KIND == KIND_GRAPH) {
            a = graph_accel_f32<COUNT, SREG, WAVE>(B, mask, p, y, n_bump);
            return true;
        } else if constexpr (KIND == KIND_TWIST) {
            return twist_accel<float>(amp, th0, p, y, a);
        } else if constexpr (KIND == KIND_ZTWIST) {
            a = ztwist_accel<float>(p, y);
            return true;
        } else if constexpr (is_deform(KIND)) {
            return deform_accel<float, COUNT, KIND == KIND_DEFORM_ROT>(B, mask, p, y, a, n_bump);
        } else if constexpr (KIND == KIND_GANISO) {
            a = graph_aniso_accel<float, COUNT, WAVE>(B, mask, p, y, n_bump);
            return true;
        } else if constexpr (KIND == KIND_GQUAD) {
            const float4 q = B[0];
            a = graph_quad_accel<float>(mk(q.x, q.y, q.z), p, y);
            return true;
        } else {
            a = mk(0.f, 0.f, 0.f);
            return true;
        }
    }
};

// g(d, d) at x for every metric kind, in single precision; Bs is the
// parameter set's table and n its number of records.
template <int KIND>
__device__ __forceinline__ float metric_gdd(const float4 *__restrict__ Bs, int n, float amp, float th0, V3<float> x,
                                            V3<float> d) {
    if constexpr (KIND == KIND_GRAPH) {
        GraphAccum G{0.f, 0.f, 0.f, 0.f};
        for (int b = 0; b < n; ++b) graph_bump_f32(Bs[2 * b], Bs[2 * b + 1], x, d, 1.0f, G);
        const float gd = G.gx * d.x + G.gy * d.y + G.gz * d.z;
        return dot(d, d) + gd * gd;
    } else if constexpr (KIND == KIND_TWIST) {
        return twist_gdd<float>(amp, th0, x, d);
    } else if constexpr (KIND == KIND_ZTWIST) {
        return ztwist_gdd<float>(x, d);
    } else if constexpr (is_deform(KIND)) {
        return deform_gdd<float, KIND == KIND_DEFORM_ROT>(Bs, n, x, d);
    } else if constexpr (KIND == KIND_GANISO) {
        // g(d, d) = |d|^2 + (grad f . d)^2
        float gd = 0.f;
        for (int b = 0; b < n; ++b) {
            const ABump<float> P = abump_at(Bs, b);
            const V3<float> q = mk(x.x - P.c.x, x.y - P.c.y, x.z - P.c.z);
            const V3<float> Sq = mk(P.s.x * q.x, P.s.y * q.y, P.s.z * q.z);
            const float r2 = dot(q, Sq);
            const float w = r2 <= P.cut2 ? P.a * exp2_(-0.5f * log2e_<float>() * r2) : 0.f;
            gd -= w * dot(Sq, d);
        }
        return dot(d, d) + gd * gd;
    } else if constexpr (KIND == KIND_GQUAD) {
        const float4 q = Bs[0];
        const float gd = 2.f * (q.x * x.x * d.x + q.y * x.y * d.y + q.z * x.z * d.z);
        return dot(d, d) + gd * gd;
    } else {
        return dot(d, d);
    }
}

}  // namespace rtd
