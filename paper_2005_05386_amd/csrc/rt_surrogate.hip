// Learned crossing surrogate for graph metrics built from Gaussian bumps.
//
// Canonical frame.  In units of sigma centred on a bump, the graph metric of
// a exp(-|x-c|^2 / 2 sigma^2) becomes that of kappa exp(-|u|^2 / 2) with
// kappa = a / sigma (lengths scale by sigma, which does not change the
// geodesics as point sets), and f -> -f leaves g = I + grad f grad f^T
// unchanged, so one network per |kappa| serves every bump of that shape.
// The support sphere has radius 3.  The metric is rotation invariant about
// the centre, so a crossing is fixed by the angle th between the incoming
// direction and the inward normal: in the frame where the entry point is
// (3, 0, 0) and the direction (-cos th, sin th, 0) the exit lies in the
// plane z = 0.
//
// Network input (unit-sphere entry point, direction): (1, 0, 0, -c, s, 0)
// with c = cos th, s = sin th.  Target: residual against the straight chord,
//   (u_exit - (-cos 2th, sin 2th, 0), w_exit - (-c, s, 0)) / scale,
// u_exit the exit point on the unit sphere, w_exit the unit exit direction.
//
// This file holds the training-data generator, the calibration of per-bin
// error bounds, and the crossing stage of a trace: group the crossings that
// a pass parked by network, run a fused MLP forward on the matrix cores,
// then decode, probe and either move each ray to the predicted exit or mark
// the sphere to be integrated through.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rt_device.hpp"
#include "rt_internal.hpp"
#include "rt_step.hpp"

using namespace rtd;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// SplitMix64 finaliser (Steele, Lea, Flood 2014) as a counter-based generator.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }

// Canonical chord baseline of a crossing with cos th = c, sin th = s.
__device__ __forceinline__ void chord_baseline(float c, float s, V3<float> &uc, V3<float> &vin) {
    uc = mk(-(c * c - s * s), 2.f * s * c, 0.f);
    vin = mk(-c, s, 0.f);
}

// ===================================================== training crossings
// Sample i of shape sh: sin^2 th uniform in [0, 1) (mode 0: entry points
// uniform over the disc of impact parameters), cos th = i / (n - 1) (mode 1,
// a grid), or sin th uniform in [0, 1) (mode 2: impact parameters uniform).  RK4 with step h from (3, 0, 0) until a step leaves the
// sphere, then bisection of that step's fraction on |u|^2 - 9.
__global__ __launch_bounds__(256) void k_cross_gen(const float *__restrict__ kappa, const float *__restrict__ scale,
                                                   int n_per, float h, int mode, uint64_t seed,
                                                   float *__restrict__ X, float *__restrict__ Y,
                                                   float *__restrict__ AUX, int max_steps, int step_batch) {
    const int sh = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_per) return;
    const float k = fabsf(kappa[sh]);
    // stratified draws: the training loop's (step_batch > 0), or on request
    const bool strat = step_batch > 0 || (mode & 4) != 0;
    mode &= 3;
    // one bump at the origin with sigma = 1, no cut: (cx, cy, cz, -log2(e)/2), (kappa, 1, cut^2, 1)
    __shared__ float4 bump[2];
    if (threadIdx.x == 0) {
        bump[0] = make_float4(0.f, 0.f, 0.f, -0.72134752044448170f);
        bump[1] = make_float4(k, 1.0f, 1e30f, 1.0f);
    }
    __syncthreads();
    float ct, st;
    if (mode == 1) {
        ct = n_per > 1 ? (float)i / (float)(n_per - 1) : 1.0f;
        st = sqrtf(fmaxf(0.f, 1.f - ct * ct));
    } else {
        const uint64_t r = splitmix64(seed ^ splitmix64(((uint64_t)sh << 40) ^ (uint64_t)i));
        float u = (float)((r >> 11) * (1.0 / 9007199254740992.0));
        // training draws are stratified: sample i lies in stratum i of n_per,
        // so the lanes of a wave take neighbouring strata (chords of nearly
        // equal length, little divergence) and each step's batch takes every
        // (n_per / step_batch)-th stratum (see the output index below)
        if (strat) u = (float)(((double)i + (double)u) / (double)n_per);
        // mode 0: sin^2 th uniform (area-uniform impact parameters); mode 2: sin th uniform
        const float s2 = mode == 2 ? u * u : u;
        st = sqrtf(s2);
        ct = sqrtf(fmaxf(0.f, 1.f - s2));
    }
    V3<float> xh = mk(3.0f, 0.f, 0.f), xl = mk(0.f, 0.f, 0.f);
    V3<float> uc, vin;
    chord_baseline(ct, st, uc, vin);
    // unit speed in the metric at the entry point
    GraphAccum G{0.f, 0.f, 0.f, 0.f};
    graph_bump_f32(bump[0], bump[1], xh, vin, 1.0f, G);
    const float gd = G.gx * vin.x + G.gy * vin.y + G.gz * vin.z;
    V3<float> y = rsqrt_(1.0f + gd * gd) * vin;
    Acc32<KIND_GRAPH, false> acc{bump, 1ull, 0.f, 0.f, nullptr, nullptr};
    int steps = 0;
    V3<float> ue = xh, ye = y;
    float sfrac = 0.f;
    bool done = false;
    while (steps < max_steps) {
        V3<float> p = xh + xl, dx, dv;
        step_rk4<float>(acc, p, y, h, dx, dv);
        V3<float> pn = p + dx;
        if (dot(pn, pn) > 9.0f) {
            float lo = 0.f, hi = 1.f;
            for (int it = 0; it < 30; ++it) {
                float mid = 0.5f * (lo + hi);
                V3<float> d2, w2;
                step_rk4<float>(acc, p, y, mid * h, d2, w2);
                V3<float> q = p + d2;
                if (dot(q, q) > 9.0f) hi = mid;
                else lo = mid;
            }
            sfrac = 0.5f * (lo + hi);
            V3<float> d2, w2;
            step_rk4<float>(acc, p, y, sfrac * h, d2, w2);
            ue = p + d2;
            ye = y + w2;
            done = true;
            break;
        }
        two_sum_add(xh.x, xl.x, dx.x);
        two_sum_add(xh.y, xl.y, dx.y);
        two_sum_add(xh.z, xl.z, dx.z);
        y = y + dv;
        steps++;
    }
    const float arc = ((float)steps + sfrac) * h;
    const V3<float> uo = (1.0f / 3.0f) * ue;
    const V3<float> vo = rsqrt_(dot(ye, ye)) * ye;
    const float inv = 1.0f / scale[sh];
    // layout [shape][sample], or step-major [step][shape][position] with
    // step i % (n_per / step_batch) and position i / (n_per / step_batch)
    const int nst = step_batch > 0 ? n_per / step_batch : 1;
    const int64_t o = step_batch > 0 ? ((int64_t)(i % nst) * gridDim.y + sh) * step_batch + i / nst
                                     : (int64_t)sh * n_per + i;
    float *x = X + 6 * o, *yv = Y + 6 * o, *aux = AUX + 4 * o;
    x[0] = 1.f;
    x[1] = 0.f;
    x[2] = 0.f;
    x[3] = vin.x;
    x[4] = vin.y;
    x[5] = 0.f;
    yv[0] = (uo.x - uc.x) * inv;
    yv[1] = (uo.y - uc.y) * inv;
    yv[2] = (uo.z - uc.z) * inv;
    yv[3] = (vo.x - vin.x) * inv;
    yv[4] = (vo.y - vin.y) * inv;
    yv[5] = (vo.z - vin.z) * inv;
    aux[0] = 3.0f * st;
    aux[1] = done ? arc : -1.0f;
    aux[2] = uo.x;
    aux[3] = uo.y;
}

// ============================================================ calibration
// Decoded errors of predictions P against targets Y (both scaled residuals)
// in the canonical frame: |u_p - u_t| and |w_p/|w_p| - w_t/|w_t||, maxed per
// bin of cos th into err[shape][bin][2] (non-negative floats compare as
// their bit patterns, so the maximum is an integer atomic max).
__global__ void k_fill_u32(unsigned *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ __launch_bounds__(256) void k_cross_cal(const float *__restrict__ X, const float *__restrict__ P,
                                                   const float *__restrict__ Yt, const float *__restrict__ scale,
                                                   int n_per, int n_shapes, int n_bins, unsigned *__restrict__ err) {
    const int64_t n = (int64_t)n_shapes * n_per;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int sh = (int)(i / n_per);
        const float sc = scale[sh];
        const float c = -X[6 * i + 3], s = X[6 * i + 4];
        V3<float> uc, vin;
        chord_baseline(c, s, uc, vin);
        const float *p = P + 6 * i, *t = Yt + 6 * i;
        V3<float> up = mk(uc.x + sc * p[0], uc.y + sc * p[1], uc.z + sc * p[2]);
        V3<float> ut = mk(uc.x + sc * t[0], uc.y + sc * t[1], uc.z + sc * t[2]);
        V3<float> wp = mk(vin.x + sc * p[3], vin.y + sc * p[4], vin.z + sc * p[5]);
        V3<float> wt = mk(vin.x + sc * t[3], vin.y + sc * t[4], vin.z + sc * t[5]);
        wp = rsqrt_(dot(wp, wp)) * wp;
        wt = rsqrt_(dot(wt, wt)) * wt;
        V3<float> du = up - ut, dw = wp - wt;
        const float ep = sqrtf(dot(du, du)), ed = sqrtf(dot(dw, dw));
        const int bin = min(n_bins - 1, max(0, (int)(c * (float)n_bins)));
        unsigned *e = err + ((int64_t)sh * n_bins + bin) * 2;
        atomicMax(e + 0, __float_as_uint(isfinite(ep) ? ep : 3.0e38f));
        atomicMax(e + 1, __float_as_uint(isfinite(ed) ? ed : 3.0e38f));
    }
}

// ===================================================== crossing stage
// Canonical frame of a parked ray: e1 = unit entry point about the centre,
// e2 = in-plane unit vector with direction = -c e1 + s e2, e3 = e1 x e2.
struct Frame {
    V3<float> e1, e2, e3;
    float c, s;
};

__device__ __forceinline__ Frame crossing_frame(V3<float> o, V3<float> y) {
    Frame F;
    F.e1 = rsqrt_(dot(o, o)) * o;
    V3<float> v = rsqrt_(dot(y, y)) * y;
    F.c = fminf(fmaxf(-dot(F.e1, v), 0.f), 1.f);
    V3<float> perp = v + F.c * F.e1;
    float pn = dot(perp, perp);
    if (pn > 1e-12f) {
        F.e2 = rsqrt_(pn) * perp;
    } else {
        // head-on: any unit vector orthogonal to e1
        V3<float> a = fabsf(F.e1.x) < 0.9f ? mk(1.f, 0.f, 0.f) : mk(0.f, 1.f, 0.f);
        V3<float> q = a - dot(a, F.e1) * F.e1;
        F.e2 = rsqrt_(dot(q, q)) * q;
    }
    F.s = sqrtf(fmaxf(0.f, 1.f - F.c * F.c));
    F.e3 = mk(F.e1.y * F.e2.z - F.e1.z * F.e2.y, F.e1.z * F.e2.x - F.e1.x * F.e2.z,
              F.e1.x * F.e2.y - F.e1.y * F.e2.x);
    return F;
}

__device__ __forceinline__ float *state_ptr(float *st, int id) {
    return st + ((int64_t)(id >> 6) * rti::Q_NFIELDS * 64 + (id & 63));
}

// Per-network row and tile offsets of this pass's crossings (one wave).
__global__ void k_xoff(const rti::TraceArgs A, int pass) {
    const int lane = threadIdx.x;
    int *ctl = A.xctl;
    const int n = ctl[rti::XC_CNT + lane];
    const int incl = wave_incl_scan(n);
    const int tiles = (n + 63) >> 6;
    const int tincl = wave_incl_scan(tiles);
    ctl[rti::XC_ROW + lane] = incl - n;
    ctl[rti::XC_TILE + lane] = tincl - tiles;
    if (lane == 63) {
        ctl[rti::XC_ROW + 64] = incl;
        ctl[rti::XC_TILE + 64] = tincl;
        if (incl) atomicAdd(A.stats + rti::ST_XING, (unsigned long long)incl);
    }
    ctl[rti::XC_CNT + lane] = 0;  // ready for the next pass
    (void)pass;
}

// Slot of every crossing; network input in the canonical frame.
__global__ __launch_bounds__(256) void k_xprep(const rti::TraceArgs A, const rti::SurrArgs S, int pass) {
    const int n = A.ctr[rti::CTR_PASS0 + pass * rti::CTR_PASS_WORDS + rti::CTR_XQ];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int4 q = A.xq[i];
        const int net = __float_as_int(A.surr_sb[2 * q.y + 1].y);
        const int slot = A.xctl[rti::XC_ROW + net] + q.z;
        S.sorted[slot] = make_int2(q.x, q.y);
        const float *src = state_ptr(A.st, q.x);
        const float4 c0 = A.surr_sb[2 * q.y];
        V3<float> o = mk((src[rti::Q_XH * 64] - c0.x) + src[rti::Q_XL * 64],
                         (src[(rti::Q_XH + 1) * 64] - c0.y) + src[(rti::Q_XL + 1) * 64],
                         (src[(rti::Q_XH + 2) * 64] - c0.z) + src[(rti::Q_XL + 2) * 64]);
        V3<float> y = mk(src[rti::Q_Y * 64], src[(rti::Q_Y + 1) * 64], src[(rti::Q_Y + 2) * 64]);
        Frame F = crossing_frame(o, y);
        float *x = S.xin + 6 * (int64_t)slot;
        x[0] = 1.f;
        x[1] = 0.f;
        x[2] = 0.f;
        x[3] = -F.c;
        x[4] = F.s;
        x[5] = 0.f;
    }
}

// Fused grouped MLP forward.  A workgroup takes 64-row tiles of one network
// (persistent over the pass's tile list) and keeps the tile's activations
// in LDS as FP32: the first layer in FP32, the two 256x256 products on
// v_mfma_f32_16x16x32_bf16 in three-term split bf16 (Ah Bh + Ah Bl + Al Bh,
// both operands split as they are read: activations from LDS, weights from
// the FP32 master through L2), the output layer in FP32.  Rounding points
// and summation orders are those of the training forward pass.
__device__ __forceinline__ void split8(const float *v, bf16x8 &hi, bf16x8 &lo) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const __bf16 h = (__bf16)v[e];
        hi[e] = h;
        lo[e] = (__bf16)(v[e] - (float)h);
    }
}

__global__ __launch_bounds__(256) void k_mlp_infer(const int *__restrict__ ctl, const rti::SurrArgs S) {
    // FP32 rows of 260 (1040 bytes, 16-byte aligned for 128-bit reads)
    __shared__ __attribute__((aligned(16))) float Hf[64][260];
    __shared__ float Xs[64][6];
    const int total_tiles = ctl[rti::XC_TILE + 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int t = blockIdx.x; t < total_tiles; t += gridDim.x) {
        // network of tile t: the last one whose first tile is <= t
        const int toff = lane < S.n_nets ? ctl[rti::XC_TILE + lane] : 0x7fffffff;
        const int g = uniform_i(__popcll(ballot(toff <= t)) - 1);
        const int off = ctl[rti::XC_ROW + g], cnt = ctl[rti::XC_ROW + g + 1] - off;
        const int m0 = off + (t - ctl[rti::XC_TILE + g]) * 64;
        const int M = min(64, off + cnt - m0);
        const float *__restrict__ Pg = S.params + (int64_t)g * S.stride;
        for (int e = tid; e < 64 * 6; e += 256) {
            const int r = e / 6, k = e - r * 6;
            Xs[r][k] = r < M ? S.xin[6 * (int64_t)(m0 + r) + k] : 0.f;
        }
        __syncthreads();
        {   // layer 1, FP32: thread = unit
            const float *W = Pg + rti::OFF_W1 + tid * 6;
            const float w0 = W[0], w1 = W[1], w2 = W[2], w3 = W[3], w4 = W[4], w5 = W[5];
            const float b = Pg[rti::OFF_B1 + tid];
            for (int r = 0; r < 64; ++r) {
                float z = b;
                z = fmaf(w0, Xs[r][0], z);
                z = fmaf(w1, Xs[r][1], z);
                z = fmaf(w2, Xs[r][2], z);
                z = fmaf(w3, Xs[r][3], z);
                z = fmaf(w4, Xs[r][4], z);
                z = fmaf(w5, Xs[r][5], z);
                Hf[r][tid] = silu_f(z);
            }
        }
        __syncthreads();
        const int kq = (lane >> 4) * 8;
        // layers 2 and 3: wave w owns output columns [64 w, 64 w + 64)
        for (int l = 0; l < 2; ++l) {
            const float *__restrict__ W = Pg + (l == 0 ? rti::OFF_W2 : rti::OFF_W3);
            const float *__restrict__ bias = Pg + (l == 0 ? rti::OFF_B2 : rti::OFF_B3);
            f32x4 acc[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
            for (int k0 = 0; k0 < 256; k0 += 32) {
                bf16x8 bh[4], bl[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int n = wave * 64 + 16 * j + (lane & 15);
                    const float4 *src = reinterpret_cast<const float4 *>(W + (int64_t)n * 256 + k0 + kq);
                    const float4 u0 = src[0], u1 = src[1];
                    const float v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
                    split8(v, bh[j], bl[j]);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float4 *src = reinterpret_cast<const float4 *>(&Hf[16 * i + (lane & 15)][k0 + kq]);
                    const float4 u0 = src[0], u1 = src[1];
                    const float v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
                    bf16x8 ah, al;
                    split8(v, ah, al);
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int n = wave * 64 + 16 * j + (lane & 15);
                    const float bn = bias[n];
#pragma unroll
                    for (int e = 0; e < 4; ++e) Hf[16 * i + (lane >> 4) * 4 + e][n] = silu_f(acc[i][j][e] + bn);
                }
            __syncthreads();
        }
        // output layer, FP32, in the training forward's order: one wave per
        // row, lane l taking k = l + 64 q in order of q, then a butterfly sum
        // over the lanes, then the bias
        {
            float w4[6][4];
#pragma unroll
            for (int o = 0; o < 6; ++o)
#pragma unroll
                for (int q = 0; q < 4; ++q) w4[o][q] = Pg[rti::OFF_W4 + o * 256 + lane + 64 * q];
            for (int m = wave; m < M; m += 4) {
                float a[6];
#pragma unroll
                for (int o = 0; o < 6; ++o) {
                    float t = w4[o][0] * Hf[m][lane];
#pragma unroll
                    for (int q = 1; q < 4; ++q) t = fmaf(w4[o][q], Hf[m][lane + 64 * q], t);
                    a[o] = t;
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
                    for (int o = 0; o < 6; ++o) a[o] += __shfl_xor(a[o], off);
                if (lane < 6) {
                    float v = a[0];
#pragma unroll
                    for (int o = 1; o < 6; ++o) v = lane == o ? a[o] : v;
                    S.xout[6 * (int64_t)(m0 + m) + lane] = Pg[rti::OFF_B4 + lane] + v;
                }
            }
        }
        __syncthreads();
    }
}

// Decode, probe and apply.  The error estimate of a jump, in scene units:
//   R (e_pos + | |u| - 1 | + plane) + L (e_dir + angle + plane)
// with e_pos, e_dir the calibrated bounds of the bin of cos th (the larger
// of the neighbouring bins, doubled), the residuals of two symmetries the
// exact map satisfies (exit on the sphere, motion in the plane z = 0, exit
// direction at polar angle phi + th for an exit point at polar angle phi),
// and L the Euclidean length still to travel (t_max - t, since g >= I).
// Accepted rays move to the predicted exit with a g-unit velocity; others
// integrate through the sphere.
__global__ __launch_bounds__(256) void k_xapply(const rti::TraceArgs A, const rti::SurrArgs S,
                                                const float4 *__restrict__ BF) {
    const int n = A.xctl[rti::XC_ROW + 64];
    unsigned long long n_acc = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int2 q = S.sorted[i];
        const int id = q.x, b = q.y;
        const float4 c0 = A.surr_sb[2 * b], c1 = A.surr_sb[2 * b + 1];
        const float sigma = c1.x, R = c1.z;
        const int net = __float_as_int(c1.y);
        float *dst = state_ptr(A.st, id);
        V3<float> xh = mk(dst[rti::Q_XH * 64], dst[(rti::Q_XH + 1) * 64], dst[(rti::Q_XH + 2) * 64]);
        V3<float> xl = mk(dst[rti::Q_XL * 64], dst[(rti::Q_XL + 1) * 64], dst[(rti::Q_XL + 2) * 64]);
        V3<float> y = mk(dst[rti::Q_Y * 64], dst[(rti::Q_Y + 1) * 64], dst[(rti::Q_Y + 2) * 64]);
        float th = dst[rti::Q_TH * 64], tl = dst[rti::Q_TL * 64];
        const int steps = __float_as_int(dst[rti::Q_STEPS * 64]);
        V3<float> o = mk((xh.x - c0.x) + xl.x, (xh.y - c0.y) + xl.y, (xh.z - c0.z) + xl.z);
        Frame F = crossing_frame(o, y);
        const float sc = S.scale[net];
        const float *p = S.xout + 6 * (int64_t)i;
        V3<float> uc, vin;
        chord_baseline(F.c, F.s, uc, vin);
        V3<float> u = mk(uc.x + sc * p[0], uc.y + sc * p[1], uc.z + sc * p[2]);
        V3<float> w = mk(vin.x + sc * p[3], vin.y + sc * p[4], vin.z + sc * p[5]);
        w = rsqrt_(dot(w, w)) * w;
        // symmetry residuals
        const float r_err = fabsf(sqrtf(dot(u, u)) - 1.f);
        const float z_err = fabsf(u.z) + fabsf(w.z);
        const float phi = atan2f(u.y, u.x), psi = atan2f(w.y, w.x), thc = atan2f(F.s, F.c);
        float da = psi - phi - thc;
        da -= 6.28318530717958648f * rintf(da * 0.159154943091895336f);
        const float a_err = fabsf(da);
        // calibrated bounds
        const int bin = min(S.n_bins - 1, (int)(F.c * (float)S.n_bins));
        const float *E = S.err + (int64_t)net * S.n_bins * 2;
        float ep = E[2 * bin], ed = E[2 * bin + 1];
        if (bin > 0) {
            ep = fmaxf(ep, E[2 * bin - 2]);
            ed = fmaxf(ed, E[2 * bin - 1]);
        }
        if (bin + 1 < S.n_bins) {
            ep = fmaxf(ep, E[2 * bin + 2]);
            ed = fmaxf(ed, E[2 * bin + 3]);
        }
        // arc length through the sphere from the table in cos th
        const float fi = F.c * (float)(S.n_tab - 1);
        const int i0 = min(S.n_tab - 2, (int)fi);
        const float fr = fi - (float)i0;
        const float *T = S.arc + (int64_t)net * S.n_tab;
        const float arc = sigma * fmaf(fr, T[i0 + 1] - T[i0], T[i0]);
        // the ray ends at t_lim (t_max, or max_steps h if that comes first)
        const float t_lim = fminf(A.t_max, (float)A.max_steps * A.h);
        const float t_exit = (float)steps * A.h + (th + tl) + arc;
        const float L = fmaxf(0.f, t_lim - t_exit);
        const float est = R * (2.f * ep + r_err + z_err) + L * (2.f * ed + a_err + z_err);
        const bool ok = est <= S.tol && t_exit < t_lim && T[i0] >= 0.f && T[i0 + 1] >= 0.f && isfinite(est);
        if (ok) {
            V3<float> xe = mk(c0.x + R * (u.x * F.e1.x + u.y * F.e2.x + u.z * F.e3.x),
                              c0.y + R * (u.x * F.e1.y + u.y * F.e2.y + u.z * F.e3.y),
                              c0.z + R * (u.x * F.e1.z + u.y * F.e2.z + u.z * F.e3.z));
            V3<float> we = mk(w.x * F.e1.x + w.y * F.e2.x + w.z * F.e3.x, w.x * F.e1.y + w.y * F.e2.y + w.z * F.e3.y,
                              w.x * F.e1.z + w.y * F.e2.z + w.z * F.e3.z);
            we = rsqrt_(dot(we, we)) * we;
            // g-unit speed at the exit: only this bump reaches its support sphere
            GraphAccum G{0.f, 0.f, 0.f, 0.f};
            graph_bump_f32(BF[2 * b], BF[2 * b + 1], xe, we, 1.0f, G);
            const float gd = G.gx * we.x + G.gy * we.y + G.gz * we.z;
            const V3<float> yn = rsqrt_(1.0f + gd * gd) * we;
            two_sum_add(th, tl, arc);
            dst[rti::Q_XH * 64] = xe.x;
            dst[(rti::Q_XH + 1) * 64] = xe.y;
            dst[(rti::Q_XH + 2) * 64] = xe.z;
            dst[rti::Q_XL * 64] = 0.f;
            dst[(rti::Q_XL + 1) * 64] = 0.f;
            dst[(rti::Q_XL + 2) * 64] = 0.f;
            dst[rti::Q_Y * 64] = yn.x;
            dst[(rti::Q_Y + 1) * 64] = yn.y;
            dst[(rti::Q_Y + 2) * 64] = yn.z;
            dst[rti::Q_TH * 64] = th;
            dst[rti::Q_TL * 64] = tl;
            n_acc++;
        }
        // do not park again on this sphere (after a jump the ray sits on it)
        dst[rti::Q_SKIP * 64] = __int_as_float(b);
    }
    // per-wave sum, one atomic per wave
    unsigned long long v = n_acc;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(A.stats + rti::ST_XACC, v);
}

}  // namespace

namespace rti {

hipError_t launch_cross_gen(const float *kappa, const float *scale, int n_shapes, int n_per, float h, int mode,
                            uint64_t seed, float *X, float *Y, float *AUX, float kappa_max, hipStream_t s,
                            int step_batch) {
    dim3 g((n_per + 255) / 256, n_shapes);
    // arc lengths inside the sphere grow with kappa (about 11 units at
    // kappa = 4, where rays wind around the bump): a generous bound; every
    // ray stops at its exit
    const int max_steps = (int)((20.0f + 10.0f * kappa_max) / h) + 16;
    hipLaunchKernelGGL(k_cross_gen, g, dim3(256), 0, s, kappa, scale, n_per, h, mode, seed, X, Y, AUX, max_steps,
                       step_batch);
    return hipGetLastError();
}

hipError_t launch_cross_cal(const float *X, const float *P, const float *Y, const float *scale, int n_shapes,
                            int n_per, int n_bins, float *err, hipStream_t s) {
    const int64_t ne = (int64_t)n_shapes * n_bins * 2;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>((ne + 255) / 256, 1024)), dim3(256), 0, s,
                       (unsigned *)err, ne);
    const int64_t n = (int64_t)n_shapes * n_per;
    hipLaunchKernelGGL(k_cross_cal, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, s, X, P,
                       Y, scale, n_per, n_shapes, n_bins, (unsigned *)err);
    return hipGetLastError();
}

hipError_t launch_surr_stage(const TraceArgs &a, const SurrArgs &S, const float4 *bump_f, int pass, int mlp_blocks,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_xoff, dim3(1), dim3(64), 0, s, a, pass);
    hipLaunchKernelGGL(k_xprep, dim3(1024), dim3(256), 0, s, a, S, pass);
    hipLaunchKernelGGL(k_mlp_infer, dim3(mlp_blocks), dim3(256), 0, s, (const int *)a.xctl, S);
    hipLaunchKernelGGL(k_xapply, dim3(1024), dim3(256), 0, s, a, S, bump_f);
    return hipGetLastError();
}

hipError_t launch_mlp_grouped(const int *ctl, const SurrArgs &S, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_infer, dim3(blocks), dim3(256), 0, s, ctl, S);
    return hipGetLastError();
}

}  // namespace rti
