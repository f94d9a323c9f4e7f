// Device building blocks of the geodesic tracer for gfx950 (CDNA4, wave64).
//
// One lane integrates one ray.  Per-wave state that is the same for all
// lanes (culled bump and object lists, set index) lives in scalar registers:
// the bump list is a 64-bit mask walked with s_ff1 and the bump parameters
// are fetched with scalar loads, so the vector ALU consumes them directly as
// SGPR operands.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtd {

enum { KIND_EUCLID = 0, KIND_GRAPH = 1, KIND_TWIST = 2, KIND_ZTWIST = 3, KIND_DEFORM = 4, KIND_GANISO = 5, KIND_GQUAD = 6,
       // composed deformations with at least one rotating field: the same
       // metric kind, compiled separately so that the constant-field chain
       // keeps its registers
       KIND_DEFORM_ROT = 7 };
constexpr bool is_deform(int kind) { return kind == KIND_DEFORM || kind == KIND_DEFORM_ROT; }
enum { STEP_RK4 = 0, STEP_RK45 = 1, STEP_EULER = 2 };

constexpr int MAX_BUMPS = 64;
constexpr int MAX_SETS = 64;
constexpr int MAX_SPHERES = 256;
constexpr int MAX_PLANES = 8;
constexpr int MAX_TORI = 8;
constexpr int MAX_PASSES = 512;
constexpr int N_XCD = 8;

// ------------------------------------------------------------------ vectors
template <class T> struct V3 {
    T x, y, z;
};
template <class T> __device__ __forceinline__ V3<T> mk(T x, T y, T z) { return V3<T>{x, y, z}; }
template <class T> __device__ __forceinline__ V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> __device__ __forceinline__ V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> __device__ __forceinline__ V3<T> operator*(T s, V3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T> __device__ __forceinline__ T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
// a + s*b
template <class T> __device__ __forceinline__ V3<T> axpy(T s, V3<T> b, V3<T> a) { return {a.x + s * b.x, a.y + s * b.y, a.z + s * b.z}; }

// --------------------------------------------------------------- math shims
// Single precision uses the hardware transcendental units (v_exp_f32,
// v_rcp_f32, v_sqrt_f32, v_sin/cos_f32); double uses the device libm.
__device__ __forceinline__ float exp2_(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double exp2_(double x) { return exp2(x); }
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ void sincos_(float x, float *s, float *c) { *s = __sinf(x); *c = __cosf(x); }
__device__ __forceinline__ void sincos_(double x, double *s, double *c) { sincos(x, s, c); }
template <class T> __device__ __forceinline__ T log2e_() { return T(1.4426950408889634); }

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
// DPP lane movement within the wave (GFX9 encodings): quad permutations
// xor-1 and xor-2, row half-mirror, row mirror, and the row broadcasts of
// lane 15 / lane 31 into the following rows.
template <int CTRL, int ROW_MASK = 0xF> __device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}
// Wave-wide min / max (all 64 lanes must be active); result is uniform.
__device__ __forceinline__ float wave_min(float v) {
    v = fminf(v, dpp<0xB1>(v));
    v = fminf(v, dpp<0x4E>(v));
    v = fminf(v, dpp<0x141>(v));
    v = fminf(v, dpp<0x140>(v));
    v = fminf(v, dpp<0x142, 0xA>(v));
    v = fminf(v, dpp<0x143, 0xC>(v));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ float wave_max(float v) {
    v = fmaxf(v, dpp<0xB1>(v));
    v = fmaxf(v, dpp<0x4E>(v));
    v = fmaxf(v, dpp<0x141>(v));
    v = fmaxf(v, dpp<0x140>(v));
    v = fmaxf(v, dpp<0x142, 0xA>(v));
    v = fmaxf(v, dpp<0x143, 0xC>(v));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ int wave_incl_scan(int v) {
    int l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int u = __shfl_up(v, o);
        if (l >= o) v += u;
    }
    return v;
}
// rank of this lane among the set bits of m below it
__device__ __forceinline__ int mbcnt64(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

// ------------------------------------------------------ metric parameters
// Graph metric, one bump, packed for single precision (two float4):
//   B0 = (cx, cy, cz, nk)   nk = -log2(e) / (2 sigma^2)  so exp(-r^2/2s^2) = exp2(nk r^2)
//   B1 = (as, s, cut2, sigma)   as = a / sigma^2, s = 1 / sigma^2, cut2 = (cull sigma)^2
// and in double: (a, cx, cy, cz, sigma, cut2, s, as).
struct MetricArgs {
    int kind, n_sets, n_bumps;
    float twist_amp, twist_theta0;
};

// Graph metric acceleration (Eq. 5.4 regrouped):
//   grad f = -sum_b w_b d_b,           d_b = x - c_b, w_b = (a_b/s_b^2) e_b
//   y^T H y = sum_b w_b (s_b (d_b.y)^2 - |y|^2)
//   y' = - grad f (y^T H y) / (1 + |grad f|^2)
// A bump contributes only where |d_b|^2 <= cut2 (per lane), which keeps each
// lane's result independent of which superset list its wave walked.
struct GraphAccum {
    float gx, gy, gz, q;
};

// FIRST: the sums start at this bump (the same values as accumulating onto
// zeros, without the zero-initialisation).
template <bool FIRST = false>
__device__ __forceinline__ void graph_bump_f32(const float4 b0, const float4 b1, V3<float> p, V3<float> y,
                                               float yy, GraphAccum &A) {
    float dx = p.x - b0.x, dy = p.y - b0.y, dz = p.z - b0.z;
    float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    float e = exp2_(b0.w * r2);
    float w = (r2 <= b1.z) ? b1.x * e : 0.0f;
    float dv = fmaf(dz, y.z, fmaf(dy, y.y, dx * y.x));
    if constexpr (FIRST) {
        A.gx = -w * dx;
        A.gy = -w * dy;
        A.gz = -w * dz;
        A.q = w * fmaf(b1.y, dv * dv, -yy);
    } else {
        A.gx = fmaf(-w, dx, A.gx);
        A.gy = fmaf(-w, dy, A.gy);
        A.gz = fmaf(-w, dz, A.gz);
        A.q = fmaf(w, fmaf(b1.y, dv * dv, -yy), A.q);
    }
}

__device__ __forceinline__ V3<float> graph_finish(const GraphAccum &A) {
    float den = fmaf(A.gz, A.gz, fmaf(A.gy, A.gy, fmaf(A.gx, A.gx, 1.0f)));
    float c = -A.q * rcp_(den);
    return {c * A.gx, c * A.gy, c * A.gz};
}

// Walk a wave-uniform bump mask in increasing index order; bump data by
// scalar loads at a 32-bit byte offset from B, the bit cleared in place, so
// that each bump costs a handful of scalar instructions next to its vector
// work.  COUNT adds the number of bumps inside their cut sphere at p to
// *n_in.
__device__ __forceinline__ void bump_at(const float4 *__restrict__ B, int b, float4 &b0, float4 &b1) {
    const float4 *q = (const float4 *)((const char *)B + ((unsigned)b << 5));
    b0 = q[0];
    b1 = q[1];
}

// SREG: the caller's mask is held in scalar registers; a fresh scalar copy
// per evaluation keeps the emptiness test a scalar branch instead of a lane
// mask carried across the stages of a step (the compiler rejects the copy,
// at build time, for a mask it cannot keep in scalar registers).
// WAVE: lanes of a wave walk a common mask, and a bump that no active lane
// has inside its cut is skipped by the whole wave (its terms are zero).
template <bool COUNT = false, bool SREG = false, bool WAVE = false>
__device__ __forceinline__ V3<float> graph_accel_f32(const float4 *__restrict__ B, uint64_t mask, V3<float> p,
                                                     V3<float> y, unsigned *n_in = nullptr) {
    if constexpr (SREG) __asm__("" : "+s"(mask));
    if constexpr (WAVE) {
        GraphAccum A{0.f, 0.f, 0.f, 0.f};
        const float yy = dot(y, y);
        while (mask) {
            const int b = __builtin_ctzll(mask);
            mask &= ~(1ull << b);
            float4 b0, b1;
            bump_at(B, b, b0, b1);
            const float dx = p.x - b0.x, dy = p.y - b0.y, dz = p.z - b0.z;
            if (ballot(fmaf(dz, dz, fmaf(dy, dy, dx * dx)) <= b1.z) == 0) continue;
            graph_bump_f32(b0, b1, p, y, yy, A);
        }
        return graph_finish(A);
    }
    if (!mask) return mk(0.f, 0.f, 0.f);
    GraphAccum A;
    float yy = dot(y, y);
    unsigned n = 0;
    auto in_cut = [&](float4 b0, float4 b1) {
        float dx = p.x - b0.x, dy = p.y - b0.y, dz = p.z - b0.z;
        return (fmaf(dz, dz, fmaf(dy, dy, dx * dx)) <= b1.z) ? 1u : 0u;
    };
    {
        const int b = __builtin_ctzll(mask);
        mask &= ~(1ull << b);
        float4 b0, b1;
        bump_at(B, b, b0, b1);
        graph_bump_f32<true>(b0, b1, p, y, yy, A);
        if (COUNT) n += in_cut(b0, b1);
    }
    while (mask) {
        const int b = __builtin_ctzll(mask);
        mask &= ~(1ull << b);
        float4 b0, b1;
        bump_at(B, b, b0, b1);
        graph_bump_f32(b0, b1, p, y, yy, A);
        if (COUNT) n += in_cut(b0, b1);
    }
    if (COUNT) *n_in += n;
    return graph_finish(A);
}

// Graph metric of a sum of anisotropic Gaussians (Eq. 6.1 with three
// spreads): with d = x - c, S = diag(1/s^2) and w = a exp(-d^T S d / 2),
//   grad f = -sum_b w_b S d_b,   y^T H y = sum_b w_b ((S d_b . y)^2 - y^T S_b y)
// and y' = -grad f (y^T H y) / (1 + |grad f|^2) as for the isotropic kind.
// Parameters: two float4 per bump, (cx, cy, cz, a), (1/sx^2, 1/sy^2, 1/sz^2,
// cut2); double, eight values in the same order.  A bump contributes only
// where d^T S d <= cut2 (per lane).
template <class T> struct ABump {
    V3<T> c, s;
    T a, cut2;
};
__device__ __forceinline__ ABump<float> abump_at(const float4 *__restrict__ B, int i) {
    const float4 *q = (const float4 *)((const char *)B + ((unsigned)i << 5));
    const float4 b0 = q[0], b1 = q[1];
    return {mk(b0.x, b0.y, b0.z), mk(b1.x, b1.y, b1.z), b0.w, b1.w};
}
__device__ __forceinline__ ABump<double> abump_at(const double *__restrict__ B, int i) {
    const double *q = B + 8 * i;
    return {mk(q[0], q[1], q[2]), mk(q[4], q[5], q[6]), q[3], q[7]};
}

template <class T, bool COUNT = false, bool WAVE = false, class PB>
__device__ __forceinline__ V3<T> graph_aniso_accel(PB B, uint64_t mask, V3<T> p, V3<T> y, unsigned *n_in = nullptr) {
    T gx = T(0), gy = T(0), gz = T(0), q = T(0);
    unsigned n = 0;
    while (mask) {
        const int b = __builtin_ctzll(mask);
        mask &= ~(1ull << b);
        const auto P = abump_at(B, b);
        const V3<T> d = mk(p.x - P.c.x, p.y - P.c.y, p.z - P.c.z);
        const V3<T> Sd = mk(P.s.x * d.x, P.s.y * d.y, P.s.z * d.z);
        const T r2 = dot(d, Sd);
        if (WAVE && ballot(r2 <= P.cut2) == 0) continue;
        const T w = r2 <= P.cut2 ? P.a * exp2_(T(-0.5) * log2e_<T>() * r2) : T(0);
        if (COUNT) n += r2 <= P.cut2 ? 1u : 0u;
        gx -= w * Sd.x;
        gy -= w * Sd.y;
        gz -= w * Sd.z;
        const T u = dot(Sd, y);
        const T ySy = P.s.x * y.x * y.x + P.s.y * y.y * y.y + P.s.z * y.z * y.z;
        q += w * (u * u - ySy);
    }
    if (COUNT) *n_in += n;
    const T den = T(1) + gx * gx + gy * gy + gz * gz;
    const T c = -q * rcp_(den);
    return mk(c * gx, c * gy, c * gz);
}

// Graph metric of the quadratic f = qx x^2 + qy y^2 + qz z^2 (the example of
// Sec. 5.1 is (1, 1, -1)): grad f = 2 q x, y^T H y = 2 sum_j q_j y_j^2.
template <class T> __device__ __forceinline__ V3<T> graph_quad_accel(V3<T> q, V3<T> p, V3<T> y) {
    const V3<T> g = mk(T(2) * q.x * p.x, T(2) * q.y * p.y, T(2) * q.z * p.z);
    const T h = T(2) * (q.x * y.x * y.x + q.y * y.y * y.y + q.z * y.z * y.z);
    const T c = -h * rcp_(T(1) + dot(g, g));
    return c * g;
}

// Double precision version over a (per-lane) mask, same regrouping.
// n_in (optional): adds the number of bumps inside their cut at p.
__device__ __forceinline__ V3<double> graph_accel_f64(const double *__restrict__ B, uint64_t mask, V3<double> p,
                                                      V3<double> y, unsigned *n_in = nullptr) {
    double gx = 0, gy = 0, gz = 0, q = 0;
    double yy = dot(y, y);
    while (mask) {
        int b = __builtin_ctzll(mask);
        mask &= mask - 1;
        const double *pb = B + 8 * b;
        double s = pb[6];
        double dx = p.x - pb[1], dy = p.y - pb[2], dz = p.z - pb[3];
        double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 > pb[5]) continue;
        if (n_in) ++*n_in;
        double w = pb[7] * exp(-0.5 * r2 * s);
        gx -= w * dx;
        gy -= w * dy;
        gz -= w * dz;
        double dv = dx * y.x + dy * y.y + dz * y.z;
        q += w * (s * dv * dv - yy);
    }
    double den = 1.0 + gx * gx + gy * gy + gz * gz;
    double c = -q / den;
    return {c * gx, c * gy, c * gz};
}

// Twist pull-back, phi(x) = x + A(rho) R_z(theta(rho)) x, A = amp tanh rho,
// theta = theta0 exp(-rho^2), rho = |x|.  With u = x/rho:
//   J = I + A R + v u^T,        v = A' R x + A theta' R' x
//   w = D^2 phi[y,y] = (A'' rho'^2) R x + A' P R u + 2 A' rho' R y
//       + (2 A' theta' rho'^2 + A theta'' rho'^2) R' x + A theta' P R' u
//       + 2 A theta' rho' R' y + A theta'^2 rho'^2 R'' x
// where rho' = u.y and P = |y|^2 - rho'^2 (so rho'' x = P u: bounded at the
// origin, where phi is only C^1).  The flow is y' = -J^-1 w (Eq. 5.8),
// solved with Sherman-Morrison on M = I + A R (a scaled rotation in the
// xy-plane, 1 + A along z).  Returns false when the solve is singular.
template <class T>
__device__ __forceinline__ bool twist_accel(T amp, T th0, V3<T> x, V3<T> y, V3<T> &acc) {
    T r2 = dot(x, x);
    T rho = sqrt_(r2);
    T tiny = T(1e-30);
    T inv_rho = rho > tiny ? rcp_(rho) : T(0);
    V3<T> u = inv_rho * x;
    // tanh(rho) = (1 - e)/(1 + e), e = exp(-2 rho) (rho >= 0)
    T e = exp2_(T(-2) * log2e_<T>() * rho);
    T th = (T(1) - e) * rcp_(T(1) + e);
    T sech2 = T(1) - th * th;
    T A = amp * th, A1 = amp * sech2, A2 = T(-2) * th * A1;
    T ang = th0 * exp2_(-log2e_<T>() * r2);
    T t1 = T(-2) * rho * ang, t2 = (T(4) * r2 - T(2)) * ang;
    T s, c;
    sincos_(ang, &s, &c);
    auto R = [&](V3<T> a) { return mk(c * a.x - s * a.y, s * a.x + c * a.y, a.z); };
    auto Rp = [&](V3<T> a) { return mk(-s * a.x - c * a.y, c * a.x - s * a.y, T(0)); };
    auto Rpp = [&](V3<T> a) { return mk(-c * a.x + s * a.y, -s * a.x - c * a.y, T(0)); };
    T rp = dot(u, y);
    T P = dot(y, y) - rp * rp;
    V3<T> Rx = R(x), Rpx = Rp(x);
    V3<T> v = axpy(A * t1, Rpx, A1 * Rx);
    T rp2 = rp * rp;
    V3<T> w = (A2 * rp2) * Rx;
    w = axpy(A1 * P, R(u), w);
    w = axpy(T(2) * A1 * rp, R(y), w);
    w = axpy((T(2) * A1 * t1 + A * t2) * rp2, Rpx, w);
    w = axpy(A * t1 * P, Rp(u), w);
    w = axpy(T(2) * A * t1 * rp, Rp(y), w);
    w = axpy(A * t1 * t1 * rp2, Rpp(x), w);
    // M^-1 for M = I + A R:  xy block [[1+Ac, -As],[As, 1+Ac]], z: 1 + A
    T m = T(1) + A * c, n = A * s;
    T idet = rcp_(m * m + n * n), iz = rcp_(T(1) + A);
    auto Minv = [&](V3<T> a) { return mk(idet * (m * a.x + n * a.y), idet * (-n * a.x + m * a.y), iz * a.z); };
    V3<T> Mw = Minv(w), Mv = Minv(v);
    T den = T(1) + dot(u, Mv);
    if (!(den > T(1e-12))) return false;
    T coef = dot(u, Mw) * rcp_(den);
    // a = -J^-1 w = -(M^-1 w - M^-1 v (u.M^-1 w)/(1 + u.M^-1 v))
    acc = mk(-(Mw.x - coef * Mv.x), -(Mw.y - coef * Mv.y), -(Mw.z - coef * Mv.z));
    return true;
}

// |J d|^2 for the twist (initial speed normalisation).
template <class T> __device__ __forceinline__ T twist_gdd(T amp, T th0, V3<T> x, V3<T> d) {
    T r2 = dot(x, x);
    T rho = sqrt_(r2);
    T inv_rho = rho > T(1e-30) ? rcp_(rho) : T(0);
    V3<T> u = inv_rho * x;
    T e = exp2_(T(-2) * log2e_<T>() * rho);
    T th = (T(1) - e) * rcp_(T(1) + e);
    T A = amp * th, A1 = amp * (T(1) - th * th);
    T ang = th0 * exp2_(-log2e_<T>() * r2);
    T t1 = T(-2) * rho * ang;
    T s, c;
    sincos_(ang, &s, &c);
    V3<T> Rx = mk(c * x.x - s * x.y, s * x.x + c * x.y, x.z);
    V3<T> Rpx = mk(-s * x.x - c * x.y, c * x.x - s * x.y, T(0));
    V3<T> Rd = mk(c * d.x - s * d.y, s * d.x + c * d.y, d.z);
    V3<T> v = axpy(A * t1, Rpx, A1 * Rx);
    V3<T> Jd = axpy(dot(u, d), v, axpy(A, Rd, d));
    return dot(Jd, Jd);
}

// z-twist of Sec. 5.2: Phi = (cos z x - sin z y, sin z x + cos z y, z).
//   J = [[c, -s, -s x - c y], [s, c, c x - s y], [0, 0, 1]]
//   D^2 Phi[v,v] = (-v3^2 (c x - s y) - 2 v3 (s v1 + c v2),
//                   -v3^2 (s x + c y) + 2 v3 (c v1 - s v2), 0)
//   J a = -w  =>  a3 = 0, (a1, a2) = -R(z)^T (w1, w2).
template <class T> __device__ __forceinline__ V3<T> ztwist_accel(V3<T> x, V3<T> v) {
    T s, c;
    sincos_(x.z, &s, &c);
    T v3 = v.z;
    T w1 = -v3 * v3 * (c * x.x - s * x.y) - T(2) * v3 * (s * v.x + c * v.y);
    T w2 = -v3 * v3 * (s * x.x + c * x.y) + T(2) * v3 * (c * v.x - s * v.y);
    return mk(-(c * w1 + s * w2), -(-s * w1 + c * w2), T(0));
}
template <class T> __device__ __forceinline__ T ztwist_gdd(V3<T> x, V3<T> d) {
    T s, c;
    sincos_(x.z, &s, &c);
    T j1 = c * d.x - s * d.y + (-s * x.x - c * x.y) * d.z;
    T j2 = s * d.x + c * d.y + (c * x.x - s * x.y) * d.z;
    return j1 * j1 + j2 * j2 + d.z * d.z;
}

// ---------------------------------------------- composed local deformations
// Phi = Phi_1 o ... o Phi_k (Sec. 6.2, "Composing diffeomorphisms"),
// Phi_i(q) = q + f_i(q) V_i(q) (Eq. 6.2), f_i = a exp(-d^T S d / 2) with
// d = q - c and S = diag(1/sx^2, 1/sy^2, 1/sz^2) (Eq. 6.1), and the affine
// field V_i(q) = v + om x d (om = 0: a constant direction).  With
// grad f = -f S d and u^T H(f) u = f ((S d . u)^2 - u^T S u), Phi_i has
//   J_i = I + V grad f^T + f [om]x,
//   D^2 Phi_i[u, u] = V (u^T H(f) u) + 2 (grad f . u) (om x u).
// Walking the chain from Phi_k (applied first) to Phi_1 with the point q,
// the pushed-forward velocity u = J(Phi_[i+1,k]) y and w = D^2 Phi_[i+1,k][y, y]:
//   w <- J_i w + D^2 Phi_i[u, u],   u <- J_i u,   q <- q + f V,   M <- J_i M
// leaves M = J(Phi) (the chain rule product) and w = D^2 Phi[y, y]: the
// Hessian composition formula of Sec. 6.2 contracted with y on both sides.
// Then y' = -M^-1 w (Eq. 5.8).  Where the spread-scaled squared distance
// exceeds cut2, Phi_i is the identity (f = 0), so every lane's result is
// the same for any superset mask.  Bit i of the mask is Phi_{i+1}.
// Parameters: float, DEFORM_F4 = 5 float4 per deformation
// (cx, cy, cz, a), (1/sx^2, 1/sy^2, 1/sz^2, 0), (vx, vy, vz, cut2),
// (slack / min spread, |a| |v|, 1 / min spread, |a| |om| s_max),
// (omx, omy, omz, 0) with slack the largest displacement of a point by the
// deformations applied before this one where they can bring it into this
// one's region; at spread-scaled distance >= rho,
// |f V| <= (|a| |v| + |a| |om| s_max max(rho, 1)) exp(-rho^2 / 2);
// double, DEFORM_D = 16 values (cx, cy, cz, a, 1/sx^2, 1/sy^2, 1/sz^2, cut2,
// vx, vy, vz, 0, omx, omy, omz, 0).
constexpr int DEFORM_F4 = 5, DEFORM_D = 16;
template <class T> struct Deform {
    V3<T> c, s, v, om;
    T a, cut2;
};
__device__ __forceinline__ Deform<float> deform_at(const float4 *__restrict__ B, int i) {
    const float4 *q = B + (unsigned)i * (unsigned)DEFORM_F4;
    const float4 d0 = q[0], d1 = q[1], d2 = q[2], d4 = q[4];
    return {mk(d0.x, d0.y, d0.z), mk(d1.x, d1.y, d1.z), mk(d2.x, d2.y, d2.z), mk(d4.x, d4.y, d4.z), d0.w, d2.w};
}
__device__ __forceinline__ Deform<double> deform_at(const double *__restrict__ B, int i) {
    const double *q = B + DEFORM_D * i;
    return {mk(q[0], q[1], q[2]), mk(q[4], q[5], q[6]), mk(q[8], q[9], q[10]), mk(q[12], q[13], q[14]), q[3], q[7]};
}

// Spread-scaled distance from the box [lo, hi] to the centre of an
// anisotropic bump (c, 1/s^2 as the first three values of the float4 pair),
// rounded down by 1e-5.
__device__ __forceinline__ float aniso_box_rho(float4 b0, float4 b1, const float lo[3], const float hi[3]) {
    const float ex = fmaxf(fmaxf(lo[0] - b0.x, b0.x - hi[0]), 0.0f);
    const float ey = fmaxf(fmaxf(lo[1] - b0.y, b0.y - hi[1]), 0.0f);
    const float ez = fmaxf(fmaxf(lo[2] - b0.z, b0.z - hi[2]), 0.0f);
    return sqrt_(ex * ex * b1.x + ey * ey * b1.y + ez * ez * b1.z) * 0.99999f;
}

// Lower bound on the spread-scaled distance rho from the points where the
// deformation at P (four float4) is evaluated, for ray points in the box
// [lo, hi], to its centre: the box distance along each axis scaled by
// 1/spread (rounded down by 1e-5), less the displacement of the earlier
// deformations in spread units: the smaller of the static slack and disp.
__device__ __forceinline__ float deform_box_rho(const float4 *__restrict__ P, const float lo[3], const float hi[3],
                                                float disp) {
    const float4 d0 = P[0], d1 = P[1], d3 = P[3];
    const float ex = fmaxf(fmaxf(lo[0] - d0.x, d0.x - hi[0]), 0.0f);
    const float ey = fmaxf(fmaxf(lo[1] - d0.y, d0.y - hi[1]), 0.0f);
    const float ez = fmaxf(fmaxf(lo[2] - d0.z, d0.z - hi[2]), 0.0f);
    const float sd2 = ex * ex * d1.x + ey * ey * d1.y + ez * ez * d1.z;
    return fmaxf(sqrt_(sd2) * 0.99999f - fminf(d3.x, disp * d3.z), 0.0f);
}

// One deformation of the chain; returns f (0 outside the cut).  WAVE: when
// no active lane of the wave is inside the cut, the whole wave skips the
// update, which is the identity there.
template <class T> __device__ __forceinline__ V3<T> cross(V3<T> a, V3<T> b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

template <class T, bool WAVE = false, bool ROT = false>
__device__ __forceinline__ T deform_apply(const Deform<T> &D, V3<T> &q, V3<T> &u, V3<T> &w, T M[9]) {
    const V3<T> d = mk(q.x - D.c.x, q.y - D.c.y, q.z - D.c.z);
    const V3<T> Sd = mk(D.s.x * d.x, D.s.y * d.y, D.s.z * d.z);
    const T r2 = dot(d, Sd);
    if (WAVE && ballot(r2 <= D.cut2) == 0) return T(0);
    const T f = r2 <= D.cut2 ? D.a * exp2_(T(-0.5) * log2e_<T>() * r2) : T(0);
    const V3<T> g = (-f) * Sd;
    const T su = dot(Sd, u);
    const T uSu = D.s.x * u.x * u.x + D.s.y * u.y * u.y + D.s.z * u.z * u.z;
    const T cw = dot(g, w) + f * (su * su - uSu);
    const T cu = dot(g, u);
    const T m0 = g.x * M[0] + g.y * M[3] + g.z * M[6];
    const T m1 = g.x * M[1] + g.y * M[4] + g.z * M[7];
    const T m2 = g.x * M[2] + g.y * M[5] + g.z * M[8];
    // ROT: the rotation part, from the old u, w, M before they are updated
    V3<T> V = D.v;
    if constexpr (ROT) {
        const V3<T> ou = cross(D.om, u), ow = cross(D.om, w);
        const V3<T> oc0 = cross(D.om, mk(M[0], M[3], M[6]));
        const V3<T> oc1 = cross(D.om, mk(M[1], M[4], M[7]));
        const V3<T> oc2 = cross(D.om, mk(M[2], M[5], M[8]));
        V = V + cross(D.om, d);
        w = w + (T(2) * cu) * ou + f * ow;
        u = u + f * ou;
        M[0] += f * oc0.x; M[1] += f * oc1.x; M[2] += f * oc2.x;
        M[3] += f * oc0.y; M[4] += f * oc1.y; M[5] += f * oc2.y;
        M[6] += f * oc0.z; M[7] += f * oc1.z; M[8] += f * oc2.z;
    }
    w = axpy(cw, V, w);
    u = axpy(cu, V, u);
    q = axpy(f, V, q);
    M[0] += V.x * m0; M[1] += V.x * m1; M[2] += V.x * m2;
    M[3] += V.y * m0; M[4] += V.y * m1; M[5] += V.y * m2;
    M[6] += V.z * m0; M[7] += V.z * m1; M[8] += V.z * m2;
    return f;
}

template <class T, bool COUNT = false, bool ROT = false, class PB>
__device__ __forceinline__ bool deform_accel(PB B, uint64_t mask, V3<T> p, V3<T> y, V3<T> &acc,
                                             unsigned *n_in = nullptr) {
    V3<T> q = p, u = y, w = mk(T(0), T(0), T(0));
    T M[9] = {T(1), T(0), T(0), T(0), T(1), T(0), T(0), T(0), T(1)};
    unsigned n = 0;
    while (mask) {
        const int i = 63 - __builtin_clzll(mask);
        mask &= ~(1ull << i);
        const T f = deform_apply<T, sizeof(T) == 4, ROT>(deform_at(B, i), q, u, w, M);
        if (COUNT) n += f != T(0) ? 1u : 0u;
    }
    if (COUNT) *n_in += n;
    // M a = -w by the adjugate
    const T c0 = M[4] * M[8] - M[5] * M[7], c1 = M[2] * M[7] - M[1] * M[8], c2 = M[1] * M[5] - M[2] * M[4];
    const T c3 = M[5] * M[6] - M[3] * M[8], c4 = M[0] * M[8] - M[2] * M[6], c5 = M[2] * M[3] - M[0] * M[5];
    const T c6 = M[3] * M[7] - M[4] * M[6], c7 = M[1] * M[6] - M[0] * M[7], c8 = M[0] * M[4] - M[1] * M[3];
    const T det = M[0] * c0 + M[1] * c3 + M[2] * c6;
    if (!(det > T(1e-12))) return false;
    const T id = -rcp_(det);
    acc = mk(id * (c0 * w.x + c1 * w.y + c2 * w.z), id * (c3 * w.x + c4 * w.y + c5 * w.z),
             id * (c6 * w.x + c7 * w.y + c8 * w.z));
    return true;
}

// |J d|^2 for the chain of the first n deformations (initial speed normalisation).
template <class T, bool ROT = false, class PB> __device__ __forceinline__ T deform_gdd(PB B, int n, V3<T> p, V3<T> d) {
    V3<T> q = p, u = d, w = mk(T(0), T(0), T(0));
    T M[9] = {T(1), T(0), T(0), T(0), T(1), T(0), T(0), T(0), T(1)};
    for (int i = n - 1; i >= 0; --i) (void)deform_apply<T, false, ROT>(deform_at(B, i), q, u, w, M);
    return dot(u, u);
}

// ------------------------------------------------------------------- scene
// Segment-vs-object tests on the chord [x0, x0 + D] in single precision.
// Return the crossing parameter s in [0,1], or 2 for none.
__device__ __forceinline__ float sphere_chord(float4 sp, V3<float> o, V3<float> D, float DD) {
    // o = x0 - c
    float B = dot(D, o);
    float Cq = fmaf(-sp.w, sp.w, dot(o, o));
    float disc = fmaf(B, B, -DD * Cq);
    if (!(disc >= 0.0f)) return 2.0f;
    float q = sqrt_(disc);
    float inv = rcp_(DD);
    float s1 = (-B - q) * inv, s2 = (-B + q) * inv;
    if (s1 >= 0.0f && s1 <= 1.0f) return s1;
    if (s2 >= 0.0f && s2 <= 1.0f) return s2;
    return 2.0f;
}

template <class T> __device__ __forceinline__ T torus_sdf(const T *tp, V3<T> x) {
    V3<T> q = mk(x.x - tp[0], x.y - tp[1], x.z - tp[2]);
    V3<T> a = mk(tp[3], tp[4], tp[5]);
    T ax = dot(q, a);
    V3<T> rad = axpy(-ax, a, q);
    T e = sqrt_(dot(rad, rad)) - tp[6];
    return sqrt_(e * e + ax * ax) - tp[7];
}

}  // namespace rtd
