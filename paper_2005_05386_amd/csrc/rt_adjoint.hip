// Discrete adjoint of the RK4 trace for the graph metric (gradients of a
// loss on the hit map with respect to every bump's amplitude, centre and
// sigma), the masked L2 loss, and their deterministic reductions.
//
// For a hitting ray, the forward pass stored the state z_k before the hit
// step and the refined step fraction s*: the hit is X(s* h; z_k, theta),
// the position part of a partial RK4 step, where s* solves F(X) = 0 for the
// hit object's implicit function F.  By the implicit function theorem the
// cotangent of (z_k, theta) is the vector-Jacobian product of X with
//   lambda' = lambda - c grad F(hit),   c = (lambda . dX/ds) / (grad F . dX/ds),
// both dot products being the step-size cotangents of two reverse passes.
// Then each full step is reversed from k* - 1 down to 0, recomputing the
// states of each checkpoint segment into per-wave scratch first.  Finally
// the initial velocity y0 = d / sqrt(g(d, d)) at the eye depends on theta
// through g and contributes too.
#include <algorithm>

#include "rt_device.hpp"
#include "rt_internal.hpp"
#include "rt_step.hpp"

using namespace rtd;
using rti::TraceArgs;

namespace {

constexpr int ADJ_MAX_BUMPS = 16;

// ---------------------------------------------------------- per-lane sums
// Gradient accumulators of one lane live in LDS: tb[(b * 5 + j) * 64 + lane]
// for bump b, parameter j in (a, cx, cy, cz, sigma).  (A read-modify-write:
// non-returning LDS atomic adds measured twice as slow here.)
struct ThetaBar {
    float *tb;
    int lane;
    unsigned terms;  // bump terms inside their cut seen by the parameter VJPs
    __device__ __forceinline__ void add(int b, int j, float v) { tb[(b * 5 + j) * 64 + lane] += v; }
};

// Wave-uniform mask of the bumps whose cut sphere meets the box of the
// active lanes' positions grown by margin (same test as the trace's
// culling).  Must be called by the whole wave.  Bumps outside the mask
// contribute exactly zero at every point in the box, so walking the mask
// gives the same sums as walking every bump.
__device__ __forceinline__ uint64_t cull_mask(const float4 *__restrict__ B, int nb, V3<float> p, bool active,
                                              float margin) {
    const float inf = __builtin_huge_valf();
    const float lo[3] = {wave_min(active ? p.x : inf) - margin, wave_min(active ? p.y : inf) - margin,
                         wave_min(active ? p.z : inf) - margin};
    const float hi[3] = {wave_max(active ? p.x : -inf) + margin, wave_max(active ? p.y : -inf) + margin,
                         wave_max(active ? p.z : -inf) + margin};
    bool need = false;
    const int lane = lane_id();
    if (lane < nb) {
        const float4 b0 = B[2 * lane], b1 = B[2 * lane + 1];
        need = box_dist2(b0.x, b0.y, b0.z, lo, hi) <= b1.z;
    }
    return ballot(need);
}

// VJP of the graph acceleration a(p, y) = -grad f (y^T H y) / (1 + |grad f|^2)
// with the bumps of a wave-uniform mask, in increasing index order (per-lane
// cut as in the forward).  Adds the cotangents of p and y to pb, yb and
// those of the bump parameters to T when ACC is set.
// The sums grad f and q of the acceleration at (p, y), bumps of the mask in
// increasing index order (the order of the trace's walk).
__device__ __forceinline__ GraphAccum graph_sums(const float4 *__restrict__ B, uint64_t mask, V3<float> p,
                                                 V3<float> y) {
    GraphAccum G{0.f, 0.f, 0.f, 0.f};
    if (!mask) return G;
    const float yy = dot(y, y);
    float4 c0, c1;
    int b = __builtin_ctzll(mask);
    mask &= ~(1ull << b);
    bump_at(B, b, c0, c1);
    graph_bump_f32<true>(c0, c1, p, y, yy, G);
    while (mask) {
        b = __builtin_ctzll(mask);
        mask &= ~(1ull << b);
        bump_at(B, b, c0, c1);
        graph_bump_f32(c0, c1, p, y, yy, G);
    }
    return G;
}

// S: the sums at (p, y) from graph_sums.
template <bool ACC>
__device__ __forceinline__ void graph_vjp(const float4 *__restrict__ B, uint64_t mask, V3<float> p, V3<float> y,
                                          const GraphAccum &S, V3<float> ab, V3<float> &pb, V3<float> &yb,
                                          ThetaBar &T) {
    const float yy = dot(y, y);
    const float q = S.q;
    const V3<float> g = mk(S.gx, S.gy, S.gz);
    const float invD = rcp_(1.0f + dot(g, g));
    const float ga = dot(g, ab);
    // a = -(q / D) g:  gbar = -(q/D) abar + (2 q / D^2)(g . abar) g,  qbar = -(g . abar)/D
    const float qbar = -ga * invD;
    const V3<float> gbar = axpy(2.0f * q * ga * invD * invD, g, (-q * invD) * ab);
    for (uint64_t m = mask; m;) {
        const int b = __builtin_ctzll(m);
        m &= ~(1ull << b);
        float4 b0, b1;
        bump_at(B, b, b0, b1);
        const V3<float> d = mk(p.x - b0.x, p.y - b0.y, p.z - b0.z);
        const float r2 = dot(d, d);
        if (!(r2 <= b1.z)) continue;
        const float s = b1.y;                 // 1 / sigma^2
        const float e = exp2_(b0.w * r2);     // exp(-s r2 / 2)
        const float w = b1.x * e;             // (a s) e
        const float u = dot(d, y);
        const float Cw = -dot(gbar, d) + qbar * (s * u * u - yy);
        // d(loss)/d(d_b): -w gbar + 2 qbar w s u y - Cw w s d
        V3<float> Cd = axpy(2.0f * qbar * w * s * u, y, (-w) * gbar);
        Cd = axpy(-Cw * w * s, d, Cd);
        pb = pb + Cd;
        yb = axpy(2.0f * qbar * w, axpy(-1.0f, y, s * u * d), yb);
        if (ACC) {
            T.terms++;
            const float sig = b1.w;
            const float Cs = qbar * w * u * u + Cw * (w * sig * sig) * (1.0f - 0.5f * s * r2);
            T.add(b, 0, Cw * s * e);
            T.add(b, 1, -Cd.x);
            T.add(b, 2, -Cd.y);
            T.add(b, 3, -Cd.z);
            T.add(b, 4, -2.0f * Cs * s * rcp_(sig));
        }
    }
}

// Reverse of one RK4 step of size sg from (p, y) (the same stage formulas as
// the forward step): cotangents (Xb, Vb) of the new position and velocity
// become cotangents of p and y (returned in Xb, Vb), of the bump
// parameters (ACC) and of the step size (returned).
template <bool ACC>
__device__ __forceinline__ float rk4_vjp(const float4 *__restrict__ B, uint64_t mask, V3<float> p, V3<float> y,
                                         float sg, V3<float> &Xb, V3<float> &Vb, ThetaBar &T) {
    // stage sums kept for the VJPs (the accelerations are finished from the
    // same sums as in the trace, so the stages are the forward's bit for bit)
    const float c1 = 0.5f * sg;
    V3<float> P[4], Y[4], K[4];
    GraphAccum G[4];
    P[0] = p;
    Y[0] = y;
    G[0] = graph_sums(B, mask, P[0], Y[0]);
    K[0] = graph_finish(G[0]);
    P[1] = axpy(c1, Y[0], p);
    Y[1] = axpy(c1, K[0], y);
    G[1] = graph_sums(B, mask, P[1], Y[1]);
    K[1] = graph_finish(G[1]);
    P[2] = axpy(c1, Y[1], p);
    Y[2] = axpy(c1, K[1], y);
    G[2] = graph_sums(B, mask, P[2], Y[2]);
    K[2] = graph_finish(G[2]);
    P[3] = axpy(sg, Y[2], p);
    Y[3] = axpy(sg, K[2], y);
    G[3] = graph_sums(B, mask, P[3], Y[3]);
    K[3] = graph_finish(G[3]);
    const float h6 = sg * (1.0f / 6.0f);
    const V3<float> sx = Y[0] + 2.0f * (Y[1] + Y[2]) + Y[3];
    const V3<float> sv = K[0] + 2.0f * (K[1] + K[2]) + K[3];
    float sb = (dot(Xb, sx) + dot(Vb, sv)) * (1.0f / 6.0f);
    V3<float> pb = Xb, yb = Vb;
    V3<float> Yb[4], Kb[4];
    const float wgt[4] = {1.f, 2.f, 2.f, 1.f};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        Yb[i] = (wgt[i] * h6) * Xb;
        Kb[i] = (wgt[i] * h6) * Vb;
    }
#pragma unroll
    for (int i = 3; i >= 0; --i) {
        V3<float> Pb = mk(0.f, 0.f, 0.f), Ybi = mk(0.f, 0.f, 0.f);
        graph_vjp<ACC>(B, mask, P[i], Y[i], G[i], Kb[i], Pb, Ybi, T);
        Yb[i] = Yb[i] + Ybi;
        pb = pb + Pb;
        if (i > 0) {
            // P_i = p + c Y_{i-1}, Y_i = y + c K_{i-1}, c = sg/2 (i < 3) or sg
            const float c = i < 3 ? c1 : sg;
            const float dc = i < 3 ? 0.5f : 1.0f;
            Yb[i - 1] = axpy(c, Pb, Yb[i - 1]);
            sb += dc * dot(Pb, Y[i - 1]);
            yb = yb + Yb[i];
            Kb[i - 1] = axpy(c, Yb[i], Kb[i - 1]);
            sb += dc * dot(Yb[i], K[i - 1]);
        } else {
            yb = yb + Yb[0];
        }
    }
    Xb = pb;
    Vb = yb;
    return sb;
}

// Gradient of the implicit function of object id at x.
__device__ __forceinline__ V3<float> obj_grad(const TraceArgs &A, const float4 *__restrict__ SPH,
                                              const float4 *__restrict__ PLN, const float *__restrict__ TOR, int id,
                                              V3<float> x) {
    if (id < A.n_spheres) {
        float4 s = SPH[id];
        return mk(2.f * (x.x - s.x), 2.f * (x.y - s.y), 2.f * (x.z - s.z));
    }
    id -= A.n_spheres;
    if (id < A.n_planes) {
        float4 pl = PLN[id];
        return mk(pl.x, pl.y, pl.z);
    }
    const float *tp = TOR + 8 * (id - A.n_planes);
    V3<float> q = mk(x.x - tp[0], x.y - tp[1], x.z - tp[2]);
    V3<float> a = mk(tp[3], tp[4], tp[5]);
    float ax = dot(q, a);
    V3<float> rad = axpy(-ax, a, q);
    float rn = sqrt_(dot(rad, rad));
    float e = rn - tp[6];
    float sd = sqrt_(e * e + ax * ax);
    // grad = ((|q_perp| - R) q_perp / |q_perp| + q_par a) / sdf_inner
    V3<float> gr = axpy(ax, a, (e * rcp_(fmaxf(rn, 1e-30f))) * rad);
    return rcp_(fmaxf(sd, 1e-30f)) * gr;
}

__device__ __forceinline__ V3<float> pixel_dir(const TraceArgs &A, int pi, int pj) {
    float su = (2.0f * ((float)pi + 0.5f) / (float)A.width - 1.0f) * A.tan_half * A.aspect;
    float sv = (1.0f - 2.0f * ((float)pj + 0.5f) / (float)A.height) * A.tan_half;
    V3<float> d = mk(su * A.right[0] + sv * A.up[0] + A.fwd[0], su * A.right[1] + sv * A.up[1] + A.fwd[1],
                     su * A.right[2] + sv * A.up[2] + A.fwd[2]);
    return rsqrt_(dot(d, d)) * d;
}

struct AdjArgs {
    const float *grad_hit;   // [n_sets * H * W][3]
    float *partial;          // [chunks][n_bumps * 5] per-chunk gradient sums
    float *scratch;          // [grid blocks][ckpt_every][6][64] recomputed positions and velocities
    int *next;               // chunk queue (zeroed by k_adj_reset)
    unsigned long long *stats;  // ST_ADJ_STEPS, ST_ADJ_TERMS (zeroed by k_adj_reset)
};

__global__ void k_adj_reset(int *next, unsigned long long *stats) {
    if (threadIdx.x == 0) *next = 0;
    if (threadIdx.x == 1) stats[rti::ST_ADJ_STEPS] = 0;
    if (threadIdx.x == 2) stats[rti::ST_ADJ_TERMS] = 0;
    if (threadIdx.x == 3) stats[rti::ST_ADJ_RECOMP] = 0;
}

// One wave (one block of 64 threads) per chunk of 64 ray ids; persistent
// blocks take chunks from an atomic queue (ray costs vary: misses and hits
// that carry no gradient cost nothing, early hits little).
// Compiled for 4 waves per SIMD (128 VGPRs, 124 B of spills): 8% faster
// than 3 waves at 162 VGPRs with no spills, 5 waves spill 260 B and are
// slower.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_adjoint(TraceArgs A, AdjArgs J, const float4 *__restrict__ BF,
                                                const float4 *__restrict__ SPH, const float4 *__restrict__ PLN,
                                                const float *__restrict__ TOR) {
    extern __shared__ float tb_mem[];
    const int lane = threadIdx.x;
    const int nb = A.n_bumps;
    const int np5 = nb * 5;
    const int tiles = A.tiles_x * A.tiles_y;
    const int HW = A.width * A.height;
    const int n_chunks = A.n_sets * tiles;
    const int ck = A.ckpt_every;
    float *scr = J.scratch + (int64_t)blockIdx.x * ck * 6 * 64 + lane;
    ThetaBar T{tb_mem, lane, 0u};
    unsigned n_rev = 0, n_rec = 0;  // full steps this lane reversed and recomputed
    // culling window: CULL steps (plus the stages of one more) of Euclidean
    // length <= h each, since g >= I keeps a g-unit velocity at |y| <= 1
    constexpr int CULL = 16;
    const float margin = (float)(CULL + 1) * A.h * 1.02f + 1e-4f;

    for (;;) {
        int chunk = 0;
        if (lane == 0) chunk = atomicAdd(J.next, 1);
        chunk = uniform_i(__shfl(chunk, 0));
        if (chunk >= n_chunks) break;
        const int set = chunk / tiles;
        const int tile = chunk - set * tiles;
        const int ty = tile / A.tiles_x, tx = tile - ty * A.tiles_x;
        const int pi = tx * 8 + (lane & 7), pj = ty * 8 + (lane >> 3);
        const int id = chunk * 64 + lane;
        const bool valid = pi < A.width && pj < A.height;
        const int oi = set * HW + pj * A.width + pi;
        const float4 *__restrict__ Bs = BF + (int64_t)set * nb * 2;
        for (int j = 0; j < np5; ++j) tb_mem[j * 64 + lane] = 0.f;

        int kstar = 0, obj = -1;
        V3<float> lam = mk(0.f, 0.f, 0.f);
        float sstar = 0.f;
        V3<float> xh = mk(0.f, 0.f, 0.f), xl = xh, y = xh;
        if (valid) {
            const float *tr = A.tape_hit + (int64_t)oi * rti::TAPE_REC;
            obj = __float_as_int(tr[11]);
            if (obj >= 0) {
                xh = mk(tr[0], tr[1], tr[2]);
                xl = mk(tr[3], tr[4], tr[5]);
                y = mk(tr[6], tr[7], tr[8]);
                sstar = tr[9];
                kstar = __float_as_int(tr[10]);
                lam = mk(J.grad_hit[3 * (int64_t)oi], J.grad_hit[3 * (int64_t)oi + 1], J.grad_hit[3 * (int64_t)oi + 2]);
            }
        }
        bool act = obj >= 0 && (lam.x != 0.f || lam.y != 0.f || lam.z != 0.f);
        V3<float> xb = mk(0.f, 0.f, 0.f), yb = xb;
        // bumps a partial step from the hit records can reach (a g-unit
        // velocity moves at most h per step, g >= I)
        const uint64_t mask_hit = cull_mask(Bs, nb, xh + xl, act, margin);
        if (act) {
            // ---- terminal condition through the implicit hit
            const V3<float> p = xh + xl;
            const float sg = sstar * A.h;
            V3<float> dx, dv;
            Acc32<KIND_GRAPH, false> acch{Bs, mask_hit, 0.f, 0.f, nullptr, nullptr};
            step_rk4<float>(acch, p, y, sg, dx, dv);
            const V3<float> hit = p + dx;
            const V3<float> gF = obj_grad(A, SPH, PLN, TOR, obj, hit);
            V3<float> Xa = lam, Va = mk(0.f, 0.f, 0.f);
            const float sa = rk4_vjp<false>(Bs, mask_hit, p, y, sg, Xa, Va, T);
            V3<float> Xf = gF, Vf = mk(0.f, 0.f, 0.f);
            const float sf = rk4_vjp<false>(Bs, mask_hit, p, y, sg, Xf, Vf, T);
            if (fabsf(sf) > 1e-20f) {
                const float c = sa / sf;
                xb = axpy(-c, gF, lam);
                yb = mk(0.f, 0.f, 0.f);
                (void)rk4_vjp<true>(Bs, mask_hit, p, y, sg, xb, yb, T);
            } else {
                act = false;  // tangential hit: the hit point does not vary smoothly
            }
        }
        // ---- reverse over the full steps k* - 1 .. 0, one checkpoint segment at a time
        int kmax = act ? kstar : 0;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o));
        for (int seg = (kmax - 1) / ck; kmax > 0 && seg >= 0; --seg) {
            const int k0 = seg * ck;
            const int len = act ? max(0, min(ck, kstar - k0)) : 0;
            int lmax = len;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) lmax = max(lmax, __shfl_xor(lmax, o));
            // recompute the segment's states into scratch (the forward's own
            // step code; bumps culled per window of CULL steps, exact)
            V3<float> h0 = mk(0.f, 0.f, 0.f), l0 = h0, y0 = h0;
            if (len > 0) {
                const float *cp = A.tape_ck + (((int64_t)(id >> 6) * A.n_ckpt + seg) * 9) * 64 + (id & 63);
                h0 = mk(cp[0], cp[64], cp[128]);
                l0 = mk(cp[192], cp[256], cp[320]);
                y0 = mk(cp[384], cp[448], cp[512]);
            }
            uint64_t wm = 0;
            for (int j = 0; j < lmax; ++j) {
                if (j < len) {
                    // the reverse step needs only the rounded position x_hi + x_lo
                    const V3<float> x = h0 + l0;
                    float *sp = scr + (int64_t)j * 6 * 64;
                    sp[0] = x.x;
                    sp[64] = x.y;
                    sp[128] = x.z;
                    sp[192] = y0.x;
                    sp[256] = y0.y;
                    sp[320] = y0.z;
                }
                if (j + 1 < lmax) {
                    if (j % CULL == 0) wm = cull_mask(Bs, nb, h0 + l0, j + 1 < len, margin);
                    if (j + 1 < len) {
                        Acc32<KIND_GRAPH, false> accw{Bs, wm, 0.f, 0.f, nullptr, nullptr};
                        V3<float> dx, dv;
                        step_rk4<float>(accw, h0 + l0, y0, A.h, dx, dv);
                        n_rec++;
                        two_sum_add(h0.x, l0.x, dx.x);
                        two_sum_add(h0.y, l0.y, dx.y);
                        two_sum_add(h0.z, l0.z, dx.z);
                        y0 = y0 + dv;
                    }
                }
            }
            // reverse the segment's steps; a window of at most CULL steps
            // ending at j (going backward) stays within CULL steps of x_j.
            // A window starts at every multiple of CULL and wherever a lane's
            // steps begin (j = len - 1), so every lane is in the box of the
            // window it is reversed under.
            for (int j = lmax - 1; j >= 0; --j) {
                const bool has = j < len;
                V3<float> px = mk(0.f, 0.f, 0.f), vy = px;
                if (has) {
                    const float *sp = scr + (int64_t)j * 6 * 64;
                    px = mk(sp[0], sp[64], sp[128]);
                    vy = mk(sp[192], sp[256], sp[320]);
                }
                if (j % CULL == CULL - 1 || ballot(j == len - 1)) wm = cull_mask(Bs, nb, px, has, margin);
                if (has) {
                    (void)rk4_vjp<true>(Bs, wm, px, vy, A.h, xb, yb, T);
                    n_rev++;
                }
            }
        }
        // ---- the initial velocity y0 = d / sqrt(|d|^2 + (grad f . d)^2) at the eye
        if (act) {
            const V3<float> d = pixel_dir(A, pi, pj);
            const V3<float> e = mk(A.eye[0], A.eye[1], A.eye[2]);
            GraphAccum G{0.f, 0.f, 0.f, 0.f};
            for (int b = 0; b < nb; ++b) graph_bump_f32(Bs[2 * b], Bs[2 * b + 1], e, d, 1.0f, G);
            const float gd = G.gx * d.x + G.gy * d.y + G.gz * d.z;
            const float Gn = dot(d, d) + gd * gd;
            // dy0 = -d gd G^{-3/2} d(gd)
            const float coef = -dot(yb, d) * gd * rsqrt_(Gn) / Gn;
            for (int b = 0; b < nb; ++b) {
                const float4 b0 = Bs[2 * b], b1 = Bs[2 * b + 1];
                const V3<float> r = mk(e.x - b0.x, e.y - b0.y, e.z - b0.z);
                const float r2 = dot(r, r);
                if (!(r2 <= b1.z)) continue;
                const float s = b1.y, sig = b1.w;
                const float ee = exp2_(b0.w * r2);
                const float w = b1.x * ee;
                const float rd = dot(r, d);
                // gd_b = -w (r . d)
                T.add(b, 0, coef * (-s * ee * rd));
                const V3<float> dc = axpy(-w * s * rd, r, w * d);
                T.add(b, 1, coef * dc.x);
                T.add(b, 2, coef * dc.y);
                T.add(b, 3, coef * dc.z);
                const float dw_dsig = -2.0f * (w / sig) * (1.0f - 0.5f * s * r2);
                T.add(b, 4, coef * (-rd * dw_dsig));
            }
        }
        // ---- fixed-order reduction over the 64 lanes -> chunk partial
        __syncthreads();
        for (int j = 0; j < np5; ++j) {
            float v = tb_mem[j * 64 + lane];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0) J.partial[(int64_t)chunk * np5 + j] = v;
        }
        __syncthreads();
    }
    // work counters of this wave (integers: the sums are exact in any order)
    unsigned long long steps = n_rev, terms = T.terms, rec = n_rec;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        steps += __shfl_xor(steps, o);
        terms += __shfl_xor(terms, o);
        rec += __shfl_xor(rec, o);
    }
    if (lane == 0) {
        atomicAdd(J.stats + rti::ST_ADJ_STEPS, steps);
        atomicAdd(J.stats + rti::ST_ADJ_TERMS, terms);
        atomicAdd(J.stats + rti::ST_ADJ_RECOMP, rec);
    }
}

// Compensated FP32 sum in a fixed order: the rounding error of every
// addition (Knuth's TwoSum, exact in binary floating point) is carried in a
// second float, so the result is the sum to about one FP32 rounding,
// independent of the number of terms, and bitwise reproducible.
struct TwoSumAcc {
    float s = 0.f, c = 0.f;
    __device__ void add(float v) {
        float t = s + v;
        float bp = t - s;
        c += (s - (t - bp)) + (v - bp);
        s = t;
    }
    __device__ float value() const { return s + c; }
};

// grad[set][param] = sum over the set's chunks: one wave per output; lane l
// sums chunks l, l + 64, ... with a compensated sum, then the 64 partial
// (sum, error) pairs are combined in a fixed butterfly order.  The result
// does not depend on the launch.
__global__ __launch_bounds__(64) void k_grad_reduce(const float *__restrict__ partial, int n_sets, int tiles,
                                                    int np5, float *__restrict__ grad) {
    const int t = blockIdx.x;
    if (t >= n_sets * np5) return;
    const int set = t / np5, j = t - set * np5, lane = threadIdx.x;
    TwoSumAcc acc;
    for (int c = lane; c < tiles; c += 64) acc.add(partial[((int64_t)set * tiles + c) * np5 + j]);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const float s2 = __shfl_xor(acc.s, o), c2 = __shfl_xor(acc.c, o);
        // both lanes of a pair form the same sum: combine the lower lane's
        // pair first so the two agree bit for bit
        const bool low = (lane & o) == 0;
        TwoSumAcc m;
        m.s = low ? acc.s : s2;
        m.c = low ? acc.c : c2;
        m.add(low ? s2 : acc.s);
        m.c += low ? c2 : acc.c;
        acc = m;
    }
    if (lane == 0) grad[t] = acc.value();
}

// Masked L2 loss: pixel p counts if mask[p] (when given), id[p] >= 0 and
// id[p] == target_id[p]; grad_hit = 2 m (hit - target).  Per-block sums in
// a fixed tree order, then per-set sums in block order.
__global__ __launch_bounds__(256) void k_loss(const float *__restrict__ hit, const int *__restrict__ id,
                                              const float *__restrict__ thit, const int *__restrict__ tid,
                                              const unsigned char *__restrict__ mask, int HW,
                                              float *__restrict__ grad_hit, float *__restrict__ block_sum) {
    __shared__ float sh[256];
    const int set = blockIdx.y;
    const int p = blockIdx.x * 256 + threadIdx.x;
    float v = 0.f;
    if (p < HW) {
        const int64_t q = (int64_t)set * HW + p;
        bool m = id[q] >= 0 && id[q] == tid[q] && (!mask || mask[q]);
        float dx = m ? hit[3 * q] - thit[3 * q] : 0.f;
        float dy = m ? hit[3 * q + 1] - thit[3 * q + 1] : 0.f;
        float dz = m ? hit[3 * q + 2] - thit[3 * q + 2] : 0.f;
        v = dx * dx + dy * dy + dz * dz;
        if (grad_hit) {
            grad_hit[3 * q] = 2.f * dx;
            grad_hit[3 * q + 1] = 2.f * dy;
            grad_hit[3 * q + 2] = 2.f * dz;
        }
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_sum[(int64_t)set * gridDim.x + blockIdx.x] = sh[0];
}

__global__ void k_loss_reduce(const float *__restrict__ block_sum, int nblk, int n_sets, float *__restrict__ loss) {
    int set = blockIdx.x * blockDim.x + threadIdx.x;
    if (set >= n_sets) return;
    TwoSumAcc acc;
    for (int b = 0; b < nblk; ++b) acc.add(block_sum[(int64_t)set * nblk + b]);
    loss[set] = acc.value();
}

}  // namespace

namespace rti {

hipError_t launch_adjoint(const TraceArgs &a, const DeviceData &d, const float *grad_hit, float *partial,
                          float *grad, float *scratch, int *next, unsigned long long *stats, int blocks,
                          hipStream_t s) {
    AdjArgs J{grad_hit, partial, scratch, next, stats};
    size_t lds = (size_t)a.n_bumps * 5 * 64 * sizeof(float);
    hipLaunchKernelGGL(k_adj_reset, dim3(1), dim3(64), 0, s, next, stats);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adjoint, dim3(blocks), dim3(64), lds, s, a, J, d.bump_f, d.sph_f, d.pln_f, d.tor_f);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    int np5 = a.n_bumps * 5;
    int n = a.n_sets * np5;
    hipLaunchKernelGGL(k_grad_reduce, dim3(n), dim3(64), 0, s, (const float *)partial, a.n_sets,
                       a.tiles_x * a.tiles_y, np5, grad);
    return hipGetLastError();
}

hipError_t launch_loss(const float *hit, const int *id, const float *thit, const int *tid, const unsigned char *mask,
                       int n_sets, int HW, float *grad_hit, float *block_sum, float *loss, hipStream_t s) {
    int nblk = (HW + 255) / 256;
    hipLaunchKernelGGL(k_loss, dim3(nblk, n_sets), dim3(256), 0, s, hit, id, thit, tid, mask, HW, grad_hit,
                       block_sum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_loss_reduce, dim3((n_sets + 63) / 64), dim3(64), 0, s, (const float *)block_sum, nblk,
                       n_sets, loss);
    return hipGetLastError();
}

int adjoint_max_bumps() { return ADJ_MAX_BUMPS; }

int adjoint_blocks_per_cu(int n_bumps) {
    int n = 0;
    size_t lds = (size_t)n_bumps * 5 * 64 * sizeof(float);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_adjoint, 64, lds) != hipSuccess) return 1;
    return n > 0 ? n : 1;
}

}  // namespace rti
