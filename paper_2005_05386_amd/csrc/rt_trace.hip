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
#include <algorithm>
#include <mutex>

#include "rt.h"
#include "rt_device.hpp"
#include "rt_internal.hpp"
#include "rt_step.hpp"

using namespace rtd;
using rti::TraceArgs;

static_assert(rtd::DEFORM_F4 == rti::DEFORM_F4 && rtd::DEFORM_D == rti::DEFORM_D,
              "device and host deformation table strides differ");
static_assert(rtd::KIND_DEFORM_ROT == rti::KERNEL_KIND_DEFORM_ROT, "rotating deformation kind differs");

namespace {

// The output index is made opaque where it is used: otherwise the compiler
// hoists the nine per-lane output addresses (18 registers, loop invariant)
// out of the step loop, where they stay live through every step for a
// store that happens once per ray.
__device__ __forceinline__ void write_out(const TraceArgs &A, unsigned oi, V3<float> x, float t, V3<float> y, int id,
                                          int steps) {
    __asm__ volatile("" : "+v"(oi));
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

// Refine record of a chord hit: 4 float4 (64 B) where t is steps * h and
// the hit step is h (RK4 and Euler without learned crossings), else 5
// (80 B: also t as two floats and the step size).
constexpr bool compact_record(int step, bool surr) { return step != STEP_RK45 && !surr; }

// ========================================================= ray generation
// Initial state of a ray: x = eye, y = the pixel direction d scaled to unit
// length in the metric at the eye (y = d / sqrt(g(d, d))).  Computed by the
// first pass in registers, so the state makes no trip through memory.
template <int KIND>
__device__ __forceinline__ V3<float> initial_velocity(const TraceArgs &A, const float4 *__restrict__ Bs, int pi,
                                                      int pj) {
    float su = (2.0f * ((float)pi + 0.5f) / (float)A.width - 1.0f) * A.tan_half * A.aspect;
    float sv = (1.0f - 2.0f * ((float)pj + 0.5f) / (float)A.height) * A.tan_half;
    V3<float> d = mk(su * A.right[0] + sv * A.up[0] + A.fwd[0], su * A.right[1] + sv * A.up[1] + A.fwd[1],
                     su * A.right[2] + sv * A.up[2] + A.fwd[2]);
    d = rsqrt_(dot(d, d)) * d;
    const V3<float> e = mk(A.eye[0], A.eye[1], A.eye[2]);
    const float gdd = metric_gdd<KIND>(Bs, A.n_bumps, A.twist_amp, A.twist_theta0, e, d);
    return rsqrt_(gdd) * d;
}

// Batched segments: each lane's state at the start of a culling window, in
// LDS (read back only when the lane marches the window again).
__device__ __forceinline__ float4 *batch_save() {
    __shared__ float4 save[3 * 256];
    return save;
}

// ================================================================ the pass
// Occupancy: 7 waves per SIMD (at most 72 VGPRs) measured fastest for the
// RK4 graph and twist kernels, 6 for DP5(4) and for rotating deformations
// (77.5 -> 72.2 ms per 1080p frame), although long-lived values spill (the
// spills are a small share of the instructions).
// SURR: learned crossings (graph metric, RK4, one parameter set): a ray whose
// step chord enters the support sphere of an eligible bump stops on the
// sphere (the partial step is committed, its fraction of h added to t) and
// is queued for the crossing stage that runs after the pass.
// TAPE: differentiation forward (graph metric, RK4): checkpoints of the
// state every ckpt_every steps; a separate instantiation, so that the plain
// trace carries no per-step checkpoint test.
#ifndef RT_PASS_WAVES
#define RT_PASS_WAVES 7  // waves per SIMD the RK4 and Euler pass kernels are compiled for
#endif
#ifndef RT_GRAPH_WAVES
#define RT_GRAPH_WAVES 8  // the same for the isotropic graph metric, plain and taped (64 registers, no spill in the step loop)
#endif
#ifndef RT_BATCH_WAVES
#define RT_BATCH_WAVES 6  // the same for the batched-segment variant
#endif
// BATCH: batched multi-segment intersection (Sec. 4.1 proposes testing many
// segments of the polygon at once).  A culling window's K steps are first
// marched with no scene test while each lane keeps the bounding box of its
// polygon; the boxes, grown by a rounding margin, are then tested against
// the window's object lists.  If no lane's box meets an object the K steps
// stand; otherwise the lanes whose box does return to the window's start and
// march it again with the per-step chord tests, while the other lanes wait.
// A lane that ends by a miss or a failure while marching writes its output
// only once its box is cleared.  Windows and object lists only bound the
// work, so the outputs equal the plain kernel's bit for bit.
template <int KIND, int STEP, bool COUNT, bool SURR = false, bool TAPE = false, bool BATCH = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(STEP == STEP_RK45 || KIND == KIND_DEFORM_ROT ? 6 : (BATCH ? RT_BATCH_WAVES : (KIND == KIND_GRAPH && !SURR ? RT_GRAPH_WAVES : RT_PASS_WAVES)), 8))) void k_trace_pass(TraceArgs A, int pass, const float4 *__restrict__ BF,
                                                    const float4 *__restrict__ SPH,
                                                    const float4 *__restrict__ PLN,
                                                    const float *__restrict__ TOR) {
    static_assert(!BATCH || (STEP != STEP_RK45 && !COUNT && !SURR && !TAPE),
                  "batched segments: fixed-step integrators, plain trace");
    // t as two floats, the trial step and the attempt count change only
    // under DP5(4) and learned crossings; fixed-step traces derive t from the
    // step count and neither read nor keep them
    constexpr bool CARRY_T = STEP == STEP_RK45 || SURR;
    const int lane = lane_id();
    const int xcd0 = blockIdx.x % N_XCD;
    int *pass_ctr = A.ctr + rti::CTR_PASS0 + pass * rti::CTR_PASS_WORDS;
    const int HW = A.width * A.height;
    const int tiles = A.tiles_x * A.tiles_y;
    const int n_bumps = A.n_bumps, ns = A.n_spheres, np = A.n_planes, nt = A.n_tori;
    const int nsw = (ns + 63) >> 6;

    // chunk table of this pass: pass 0 walks every tile of every set; pass
    // p > 0 walks the sorted survivor list, each set padded to whole chunks
    int total_chunks, pre = 0, cnt = 0;
    if (pass == 0) {
        total_chunks = A.n_sets * tiles;
    } else {
        const int *surv = A.ctr + rti::CTR_PASS0 + (pass - 1) * rti::CTR_PASS_WORDS + rti::CTR_SURV;
        cnt = lane < A.n_sets ? surv[lane] : 0;
        pre = wave_incl_scan((cnt + 63) >> 6);
        total_chunks = uniform_i(__shfl(pre, 63));
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) pass_ctr[rti::CTR_NCH] = total_chunks;
    // no survivors (the late passes of a surrogate trace): nothing to pull,
    // count or write
    if (total_chunks == 0) return;
    const int *__restrict__ ids_in = A.ids[pass & 1];
    float *__restrict__ st = A.st;
    const int64_t cap = A.cap;

    unsigned long long st_wave = 0, st_lane = 0, st_bl = 0, st_ol = 0, st_steps = 0, st_rays = 0;
    unsigned long long st_ev = 0, st_be = 0, st_ot = 0;  // COUNT only
    unsigned long long st_bw = 0, st_br = 0;             // BATCH only: windows, replayed windows

    for (int xi = 0; xi < N_XCD; ++xi) {
        const int xp = (xcd0 + xi) & (N_XCD - 1);
        int *ctr = pass_ctr + xp * rti::CTR_CHUNK_STRIDE;
        for (;;) {
            int k = 0;
            if (lane == 0) k = atomicAdd(ctr, 1);
            k = uniform_i(__shfl(k, 0));
            const int chunk = k * N_XCD + xp;
            if (chunk >= total_chunks) break;

            // ---- resolve the set and this lane's ray id
            int set, id;
            bool valid;
            if (pass == 0) {
                set = chunk / tiles;
                id = chunk * 64 + lane;
                valid = true;
            } else {
                set = __popcll(ballot(pre <= chunk));
                int base_chunk = set > 0 ? __shfl(pre, set - 1) : 0;
                int cnt_s = __shfl(cnt, set);
                valid = (chunk - base_chunk) * 64 + lane < cnt_s;
                id = valid ? ids_in[chunk * 64 + lane] : 0;
            }
            set = uniform_i(set);
            // pixel of the ray: id = (set * tiles + tile) * 64 + lane-in-tile
            const int r = id - set * A.T;
            const int tile = r >> 6, tl_lane = r & 63;
            const int ty = tile / A.tiles_x, tx = tile - ty * A.tiles_x;
            const int pi = tx * 8 + (tl_lane & 7), pj = ty * 8 + (tl_lane >> 3);
            if (pass == 0) valid = pi < A.width && pj < A.height;
            const int pix = pj * A.width + pi;
            const float4 *__restrict__ Bs = BF + (int64_t)set * n_bumps * (is_deform(KIND) ? DEFORM_F4 : 2);
            const unsigned qbase = (unsigned)set * (unsigned)HW;

            V3<float> xh, xl, y;
            float th = 0.f, tl = 0.f, hc = A.h;
            int steps = 0, att = 0;
            int skip = -1;  // SURR only
            if (valid && pass == 0) {
                xh = mk(A.eye[0], A.eye[1], A.eye[2]);
                xl = mk(0.f, 0.f, 0.f);
                y = initial_velocity<KIND>(A, Bs, pi, pj);
            } else if (valid) {
                const float *__restrict__ src = st + ((int64_t)(id >> 6) * rti::Q_NFIELDS * 64 + (id & 63));
                auto F = [&](int f) { return src[f * 64]; };
                xh = mk(F(rti::Q_XH), F(rti::Q_XH + 1), F(rti::Q_XH + 2));
                xl = mk(F(rti::Q_XL), F(rti::Q_XL + 1), F(rti::Q_XL + 2));
                y = mk(F(rti::Q_Y), F(rti::Q_Y + 1), F(rti::Q_Y + 2));
                if constexpr (CARRY_T) {
                    th = F(rti::Q_TH);
                    tl = F(rti::Q_TL);
                    hc = F(rti::Q_H);
                    att = __float_as_int(F(rti::Q_ATT));
                }
                steps = __float_as_int(F(rti::Q_STEPS));
                if constexpr (SURR) skip = __float_as_int(F(rti::Q_SKIP));
            } else {
                xh = xl = y = mk(0.f, 0.f, 0.f);
            }
            if (pass == 0) st_rays += __popcll(ballot(valid));

            bool alive = valid;
            bool parked = false;  // SURR only
            int acc_pass = 0;
            int it = 0;
            uint64_t bmask = 0, omask = 0, emask = 0;
            uint64_t sm[4] = {0, 0, 0, 0};
            V3<float> A0 = mk(0.f, 0.f, 0.f);
            bool need_a0 = true;
            unsigned c_eval = 0, c_bump = 0, c_obj = 0, lane_objs = 0;  // COUNT only
            // BATCH only: the window's marching or replaying state (wave-uniform
            // replay, wi, wlen), the lane's state at the window start, its
            // polygon box, and whether it waits or has an output pending
            bool replay = false, hold = false, inb = false;
            int wi = 0, wlen = 0, fin = 0, it_m = 0;
            V3<float> bmin = mk(0.f, 0.f, 0.f), bmax = bmin;

            for (;;) {
                bool act = alive && (STEP == STEP_RK45 ? acc_pass < A.S : it < A.S) && !(SURR && parked);
                // batched: the pass length counts first marches only
                if constexpr (BATCH) act = alive && (replay ? (!hold && wi < wlen) : it_m < A.S);
                uint64_t am = ballot(act);
                if (am == 0) {
                    if constexpr (BATCH) {
                        // every replaying lane ended before the window did
                        if (replay) {
                            replay = false;
                            hold = false;
                            wi = 0;
                            continue;
                        }
                    }
                    break;
                }

                // ---- per-wave culling window
                if (BATCH ? (!replay && wi == 0) : it % A.K == 0) {
                    // the lane id taken afresh: the table offsets derived from it
                    // are then formed in this block, once per window, instead of
                    // being hoisted out of the step loop and spilled (not in the
                    // batched variant, whose twist kernel then spilled inside its
                    // step loop and ran 1.6x slower)
                    int lane = lane_id();
                    if constexpr (!BATCH) __asm__ volatile("" : "+v"(lane));
                    V3<float> p = xh + xl;
                    if (A.cull_margin < 0.f) {
                        bmask = n_bumps >= 64 ? ~0ull : ((1ull << n_bumps) - 1ull);
#pragma unroll
                        for (int w = 0; w < 4; ++w) {
                            int rem = ns - 64 * w;
                            sm[w] = rem >= 64 ? ~0ull : (rem > 0 ? ((1ull << rem) - 1ull) : 0ull);
                        }
                        omask = ((1ull << np) - 1ull) | (((1ull << nt) - 1ull) << 8);
                        if constexpr (SURR)
                            emask = ballot(lane < n_bumps && __float_as_int(A.surr_sb[2 * lane + 1].y) >= 0);
                    } else {
                        const float inf = __builtin_huge_valf();
                        const float pmn[3] = {wave_min(act ? p.x : inf), wave_min(act ? p.y : inf),
                                              wave_min(act ? p.z : inf)};
                        const float pmx[3] = {wave_max(act ? p.x : -inf), wave_max(act ? p.y : -inf),
                                              wave_max(act ? p.z : -inf)};
                        float m = A.cull_margin;
                        float disp = A.cull_disp;  // DEFORM: bound on |Phi(x) - x| in the window
                        if constexpr (is_deform(KIND)) {
                            // A geodesic is the preimage of a unit-speed line, so in the
                            // window it moves at most T + 2 max |Phi(x) - x|.  Deformation i
                            // moves a point q by |f_i(q)| |v_i| <= |a_i| |v_i| exp(-rho^2 / 2),
                            // rho the spread-scaled distance from q to c_i, and q is within
                            // the chain's displacement of the ray's point.  So a margin and
                            // a displacement bound that hold give, through the deformations
                            // near the box, a displacement bound and a margin that hold too;
                            // two rounds tighten both.
#pragma unroll
                            for (int round = 0; round < 2; ++round) {
                                const float lo0[3] = {pmn[0] - m, pmn[1] - m, pmn[2] - m};
                                const float hi0[3] = {pmx[0] + m, pmx[1] + m, pmx[2] + m};
                                float dl = 0.f;
                                if (lane < n_bumps) {
                                    const float rho = deform_box_rho(Bs + DEFORM_F4 * lane, lo0, hi0, disp);
                                    if (rho * rho <= Bs[DEFORM_F4 * lane + 2].w * 1.00001f) {
                                        // |f V| <= (|a||v| + |a||om| s_max max(rho, 1)) exp(-rho^2 / 2)
                                        // beyond spread-scaled distance rho
                                        const float4 d3 = Bs[DEFORM_F4 * lane + 3];
                                        dl = fmaf(d3.w, fmaxf(rho, 1.0f), d3.y) *
                                             exp2_(-0.5f * 1.44269504f * rho * rho);
                                    }
                                }
#pragma unroll
                                for (int o = 32; o >= 1; o >>= 1) dl += __shfl_xor(dl, o);
                                dl = __builtin_bit_cast(float, uniform_i(__builtin_bit_cast(int, dl))) * 1.001f;
                                disp = fminf(disp, dl);
                                m = fminf(m, A.cull_base + 2.0f * disp);
                            }
                        }
                        float lo[3], hi[3];
                        lo[0] = pmn[0] - m;
                        lo[1] = pmn[1] - m;
                        lo[2] = pmn[2] - m;
                        hi[0] = pmx[0] + m;
                        hi[1] = pmx[1] + m;
                        hi[2] = pmx[2] + m;
                        bool need = false;
                        if (KIND == KIND_GRAPH && lane < n_bumps) {
                            float4 b0 = Bs[2 * lane], b1 = Bs[2 * lane + 1];
                            need = box_dist2(b0.x, b0.y, b0.z, lo, hi) <= b1.z;
                        } else if (KIND == KIND_GANISO && lane < n_bumps) {
                            const float4 b0 = Bs[2 * lane], b1 = Bs[2 * lane + 1];
                            const float rho = aniso_box_rho(b0, b1, lo, hi);
                            need = rho * rho <= b1.w * 1.00001f;
                        } else if (is_deform(KIND) && lane < n_bumps) {
                            // the ball (in ray coordinates) where the deformation can act
                            const float rho = deform_box_rho(Bs + DEFORM_F4 * lane, lo, hi, disp);
                            need = rho * rho <= Bs[DEFORM_F4 * lane + 2].w * 1.00001f;
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
                        if constexpr (SURR) {
                            // eligible support spheres this wave can reach in the window
                            bool en = false;
                            if (lane < n_bumps) {
                                const float4 c0 = A.surr_sb[2 * lane];
                                en = __float_as_int(A.surr_sb[2 * lane + 1].y) >= 0 &&
                                     box_dist2(c0.x, c0.y, c0.z, lo, hi) <= c0.w;
                            }
                            emask = ballot(en);
                        }
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
                    if constexpr (BATCH) {
                        inb = act;
                        if (act) {
                            float4 *sv = batch_save();
                            sv[threadIdx.x] = make_float4(xh.x, xh.y, xh.z, xl.x);
                            sv[256 + threadIdx.x] = make_float4(xl.y, xl.z, y.x, y.y);
                            sv[512 + threadIdx.x] = make_float4(y.z, __int_as_float(steps), __int_as_float(acc_pass), 0.f);
                            bmin = bmax = p;
                        }
                        st_bw++;
                    }
                }
                // wave statistics (work counting only; the lane count is also DP5's attempt count)
                if (COUNT || STEP == STEP_RK45) st_lane += __popcll(am);
                if (COUNT) {
                    st_wave++;
                    st_bl += __popcll(bmask);
                    st_ol += __popcll(sm[0]) + __popcll(sm[1]) + __popcll(sm[2]) + __popcll(sm[3]) + __popcll(omask);
                }

                if (TAPE && act && steps % A.ckpt_every == 0) {
                    float *ck = A.tape_ck + ((((int64_t)(id >> 6) * A.n_ckpt + steps / A.ckpt_every) * 9) * 64 + (id & 63));
                    ck[0 * 64] = xh.x;
                    ck[1 * 64] = xh.y;
                    ck[2 * 64] = xh.z;
                    ck[3 * 64] = xl.x;
                    ck[4 * 64] = xl.y;
                    ck[5 * 64] = xl.z;
                    ck[6 * 64] = y.x;
                    ck[7 * 64] = y.y;
                    ck[8 * 64] = y.z;
                }
                Acc32<KIND, COUNT, true> acc{Bs, bmask, A.twist_amp, A.twist_theta0, &c_eval, &c_bump};
                // The step is computed, its chord tested against the scene on
                // the state before the step, and only then committed: a hit
                // records that pre-step state without keeping copies of it.
                bool hit = false;
                int hit_id = -1;
                int park_b = -1;  // SURR: sphere the lane parked on in this step
                float hit_s = 2.f, hstep = A.h;
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
                        if constexpr (SURR) {
                            // jumps and partial entry steps shift the step grid: the
                            // last step is clipped to land on min(t_max, max_steps h)
                            const float t_lim = fminf(A.t_max, (float)A.max_steps * A.h);
                            // (a remainder within rounding of h is a full step, so a ray
                            // that never parked takes exactly the plain trace's steps)
                            const float rem = t_lim - ((float)steps * A.h + (th + tl));
                            hstep = rem < A.h * (1.0f - 1e-5f) ? fmaxf(rem, 0.f) : A.h;
                        }
                        ok = step_rk4<float>(acc, p, y, hstep, dx, dv);
                    } else {
                        ok = step_euler<float>(acc, p, y, A.h, dx, dv);
                    }
                    bool done_fail = !ok || !finite6(dx, dv);
                    bool done_miss = false;
                    if (!done_fail && accepted) {
                        if (COUNT) c_obj += lane_objs;
                        // ---- segment versus scene, chord [x, x + dx] (a scalar branch:
                        // most wave iterations list no object)
                        if ((!BATCH || replay) && (sm[0] | sm[1] | sm[2] | sm[3] | omask) != 0) {
                            const float DD = dot(dx, dx);
#pragma unroll
                            for (int w = 0; w < 4; ++w) {
                                uint64_t m = sm[w];
                                while (m) {
                                    int b = __builtin_ctzll(m);
                                    m &= m - 1;
                                    int idx = 64 * w + b;
                                    float4 s = SPH[idx];
                                    V3<float> o = mk((xh.x - s.x) + xl.x, (xh.y - s.y) + xl.y, (xh.z - s.z) + xl.z);
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
                                int oid;
                                if (b < 8) {
                                    float4 pl = PLN[b];
                                    F0 = pl.x * p.x + pl.y * p.y + pl.z * p.z - pl.w;
                                    F1 = F0 + (pl.x * dx.x + pl.y * dx.y + pl.z * dx.z);
                                    oid = ns + b;
                                } else {
                                    const float *tp = TOR + 8 * (b - 8);
                                    F0 = torus_sdf<float>(tp, p);
                                    F1 = torus_sdf<float>(tp, p + dx);
                                    oid = ns + np + (b - 8);
                                }
                                if ((F0 > 0.f) != (F1 > 0.f)) {
                                    float sc = fminf(fmaxf(F0 / (F0 - F1), 0.f), 1.f);
                                    if (sc < hit_s) {
                                        hit_s = sc;
                                        hit_id = oid;
                                    }
                                }
                            }
                        }
                        // ---- chord entering an eligible support sphere (SURR)
                        float ent_s = 2.f;
                        int ent_b = -1;
                        if constexpr (SURR) {
                            uint64_t em = emask;
                            while (em) {
                                const int b = __builtin_ctzll(em);
                                em &= em - 1;
                                const float4 c0 = A.surr_sb[2 * b];
                                V3<float> o = mk((xh.x - c0.x) + xl.x, (xh.y - c0.y) + xl.y, (xh.z - c0.z) + xl.z);
                                const float o2 = dot(o, o);
                                const V3<float> on = o + dx;
                                if (b != skip && o2 >= c0.w && dot(on, on) < c0.w) {
                                    // smaller root of |o + s dx|^2 = R^2
                                    const float B = dot(o, dx), C = o2 - c0.w, DD = dot(dx, dx);
                                    const float disc = fmaxf(B * B - DD * C, 0.f);
                                    const float sr = fminf(fmaxf((-B - sqrtf(disc)) / DD, 0.f), 1.f);
                                    if (sr < ent_s) {
                                        ent_s = sr;
                                        ent_b = b;
                                    }
                                }
                            }
                            // park only while enough passes remain to finish the ray afterwards
                            if (ent_b >= 0 && (A.n_passes - 1 - pass) * A.S < A.max_steps - steps) ent_b = -1;
                        }
                        if (SURR && ent_b >= 0 && !(hit_id >= 0 && hit_s < ent_s)) {
                            two_sum_add(xh.x, xl.x, ent_s * dx.x);
                            two_sum_add(xh.y, xl.y, ent_s * dx.y);
                            two_sum_add(xh.z, xl.z, ent_s * dx.z);
                            y = y + ent_s * dv;
                            two_sum_add(th, tl, ent_s * hstep);
                            parked = true;
                            park_b = ent_b;
                            hit_id = -1;
                        } else if (hit_id >= 0) {
                            hit = true;
                            acc_pass++;  // the hit step was integrated: count it
                        } else {
                            // commit the step
                            two_sum_add(xh.x, xl.x, dx.x);
                            two_sum_add(xh.y, xl.y, dx.y);
                            two_sum_add(xh.z, xl.z, dx.z);
                            y = y + dv;
                            acc_pass++;
                            bool clipped = false;
                            if (STEP == STEP_RK45) {
                                two_sum_add(th, tl, hstep);
                                steps++;
                            } else if (SURR && hstep < A.h) {
                                // clipped last step: its length goes to t, not to the step count
                                two_sum_add(th, tl, hstep);
                                clipped = true;
                            } else {
                                steps++;
                            }
                            // RK45 lands on t_max up to float rounding of the clipped last step
                            float t = (STEP == STEP_RK45) ? th + tl : (float)steps * A.h + (SURR ? th + tl : 0.f);
                            float t_end = (STEP == STEP_RK45) ? A.t_max * (1.0f - 1e-6f) : A.t_max;
                            done_miss = steps >= A.max_steps || t >= t_end || clipped;
                            if constexpr (BATCH) {
                                if (!replay) {
                                    const V3<float> q = xh + xl;
                                    bmin = mk(fminf(bmin.x, q.x), fminf(bmin.y, q.y), fminf(bmin.z, q.z));
                                    bmax = mk(fmaxf(bmax.x, q.x), fmaxf(bmax.y, q.y), fmaxf(bmax.z, q.z));
                                }
                            }
                        }
                    }
                    if (BATCH && !replay && (done_fail || done_miss)) {
                        // the output waits until the window's box test clears this lane
                        fin = done_fail ? 2 : 1;
                    } else if (done_fail || done_miss) {
                        write_out(A, qbase + pix, xh + xl,
                                  STEP == STEP_RK45 ? th + tl : (float)steps * A.h + (SURR ? th + tl : 0.f), y,
                                  done_fail ? -2 : -1, steps);
                        if (TAPE) A.tape_hit[(int64_t)(qbase + pix) * rti::TAPE_REC + 11] = __int_as_float(-1);
                    }
                    if (done_fail || done_miss || hit) alive = false;
                }
                // ---- push chord hits to the refine queue (wave-aggregated);
                // the lane's registers still hold the state before the step
                uint64_t hm = ballot(hit);
                if (hm) {
                    int base = 0;
                    if (lane == 0) base = atomicAdd(A.ctr + rti::CTR_REFINE, __popcll(hm));
                    base = uniform_i(__shfl(base, 0));
                    if (hit) {
                        int64_t r = base + mbcnt64(hm);
                        if constexpr (compact_record(STEP, SURR)) {
                            // t = steps h and the step is h: 4 float4
                            float4 *rec = A.rec + 4 * r;
                            rec[0] = make_float4(xh.x, xh.y, xh.z, xl.x);
                            rec[1] = make_float4(xl.y, xl.z, y.x, y.y);
                            rec[2] = make_float4(y.z, hit_s, __int_as_float(hit_id), __int_as_float((int)(qbase + pix)));
                            rec[3] = make_float4(__int_as_float(steps), __int_as_float((int)(uint32_t)bmask),
                                                 __int_as_float((int)(bmask >> 32)), 0.f);
                        } else {
                            float4 *rec = A.rec + rti::REC_F4 * r;
                            rec[0] = make_float4(xh.x, xh.y, xh.z, xl.x);
                            rec[1] = make_float4(xl.y, xl.z, y.x, y.y);
                            rec[2] = make_float4(y.z, th, hstep, hit_s);
                            rec[3] = make_float4(__int_as_float(hit_id), __int_as_float((int)(qbase + pix)),
                                                 __int_as_float(steps), tl);
                            rec[4] = make_float4(__int_as_float((int)(uint32_t)bmask),
                                                 __int_as_float((int)(bmask >> 32)), 0.f, 0.f);
                        }
                    }
                }
                if constexpr (SURR) {
                    // ---- queue the rays that parked on a support sphere in this step
                    const bool now = park_b >= 0;
                    const uint64_t pm = ballot(now);
                    if (pm) {
                        int base = 0;
                        if (lane == 0) base = atomicAdd(pass_ctr + rti::CTR_XQ, __popcll(pm));
                        base = uniform_i(__shfl(base, 0));
                        if (now) {
                            const int net = __float_as_int(A.surr_sb[2 * park_b + 1].y);
                            const int rank = atomicAdd(A.xctl + net, 1);
                            A.xq[base + mbcnt64(pm)] = make_int4(id, park_b, rank, 0);
                        }
                    }
                }
                if constexpr (BATCH) {
                    wi++;
                    if (!replay) it_m++;
                    if (replay) {
                        if (wi >= wlen) {
                            replay = false;
                            hold = false;
                            wi = 0;
                        }
                    } else if (wi == A.K || ballot(alive && it_m < A.S) == 0) {
                        // ---- end of the march: the lanes' polygon boxes against
                        // the window's objects
                        bool cand = false;
                        if (inb) {
                            // margin: FP32 rounding of the positions and of the
                            // chord tests, far below it
                            const float eps = 1e-3f + 1e-5f * fmaxf(fmaxf(fabsf(bmin.x), fabsf(bmax.x)),
                                                                   fmaxf(fmaxf(fabsf(bmin.y), fabsf(bmax.y)),
                                                                         fmaxf(fabsf(bmin.z), fabsf(bmax.z))));
                            const float lo[3] = {bmin.x - eps, bmin.y - eps, bmin.z - eps};
                            const float hi[3] = {bmax.x + eps, bmax.y + eps, bmax.z + eps};
#pragma unroll
                            for (int w = 0; w < 4; ++w) {
                                uint64_t m = sm[w];
                                while (m) {
                                    const int b = __builtin_ctzll(m);
                                    m &= m - 1;
                                    const float4 sp = SPH[64 * w + b];
                                    cand |= box_dist2(sp.x, sp.y, sp.z, lo, hi) <= sp.w * sp.w;
                                }
                            }
                            uint64_t m = omask;
                            while (m) {
                                const int b = __builtin_ctzll(m);
                                m &= m - 1;
                                if (b < 8) {
                                    const float4 pl = PLN[b];
                                    const float cx = 0.5f * (lo[0] + hi[0]), cy = 0.5f * (lo[1] + hi[1]),
                                                cz = 0.5f * (lo[2] + hi[2]);
                                    const float ex = 0.5f * (hi[0] - lo[0]), ey = 0.5f * (hi[1] - lo[1]),
                                                ez = 0.5f * (hi[2] - lo[2]);
                                    const float c = pl.x * cx + pl.y * cy + pl.z * cz - pl.w;
                                    cand |= fabsf(c) <= fabsf(pl.x) * ex + fabsf(pl.y) * ey + fabsf(pl.z) * ez;
                                } else {
                                    const float *tp = TOR + 8 * (b - 8);
                                    const float rr = tp[6] + tp[7];
                                    cand |= box_dist2(tp[0], tp[1], tp[2], lo, hi) <= rr * rr;
                                }
                            }
                        }
                        if (fin && !cand) {
                            write_out(A, qbase + pix, xh + xl, (float)steps * A.h, y, fin == 2 ? -2 : -1, steps);
                            fin = 0;
                        }
                        if (ballot(cand)) {
                            if (cand) {
                                const float4 *sv = batch_save();
                                const float4 a = sv[threadIdx.x], b = sv[256 + threadIdx.x], c = sv[512 + threadIdx.x];
                                xh = mk(a.x, a.y, a.z);
                                xl = mk(a.w, b.x, b.y);
                                y = mk(b.z, b.w, c.x);
                                steps = __float_as_int(c.y);
                                acc_pass = __float_as_int(c.z);
                                alive = true;
                                fin = 0;
                            }
                            hold = !cand;
                            replay = true;
                            wlen = wi;
                            st_br++;
                        }
                        wi = 0;
                        inb = false;
                    }
                }
                it++;
            }

            // ---- survivors keep their state in place; the chunk's alive mask
            // and the per-set counts feed the ordered compaction after the pass
            uint64_t sv = ballot(alive);
            if (lane == 0) A.cmask[chunk] = sv;
            if (sv) {
                if (lane == 0) atomicAdd(pass_ctr + rti::CTR_SURV + set, __popcll(sv));
                if (alive) {
                    float *__restrict__ dst = st + ((int64_t)(id >> 6) * rti::Q_NFIELDS * 64 + (id & 63));
                    auto P = [&](int f, float v) { dst[f * 64] = v; };
                    P(rti::Q_XH, xh.x);
                    P(rti::Q_XH + 1, xh.y);
                    P(rti::Q_XH + 2, xh.z);
                    P(rti::Q_XL, xl.x);
                    P(rti::Q_XL + 1, xl.y);
                    P(rti::Q_XL + 2, xl.z);
                    P(rti::Q_Y, y.x);
                    P(rti::Q_Y + 1, y.y);
                    P(rti::Q_Y + 2, y.z);
                    if constexpr (CARRY_T) {
                        P(rti::Q_TH, th);
                        P(rti::Q_TL, tl);
                        P(rti::Q_H, hc);
                        P(rti::Q_ATT, __int_as_float(att));
                    }
                    P(rti::Q_STEPS, __int_as_float(steps));
                    if constexpr (SURR) P(rti::Q_SKIP, __int_as_float(skip));
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
        if (BATCH) {
            atomicAdd(A.stats + rti::ST_BATCH_WIN, st_bw);
            atomicAdd(A.stats + rti::ST_BATCH_REPLAY, st_br);
        }
        if (st_rays) atomicAdd(A.stats + rti::ST_RAYS, st_rays);
        atomicAdd(A.stats + rti::ST_STEPS, st_steps);
        atomicAdd(A.stats + rti::ST_ATTEMPTS, STEP == STEP_RK45 ? st_lane : st_steps);
        if (COUNT) {
            atomicAdd(A.stats + rti::ST_WAVE_ITERS, st_wave);
            atomicAdd(A.stats + rti::ST_LANE_ITERS, st_lane);
            atomicAdd(A.stats + rti::ST_BUMP_LIST, st_bl);
            atomicAdd(A.stats + rti::ST_OBJ_LIST, st_ol);
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

// COUNT: also counts the acceleration evaluations, the bumps inside their
// cut at them (graph metric) and the integrator steps (work statistics).
// Occupancy: the graph-metric RK4 refine is compiled for 4 waves per SIMD
// (128 VGPRs, 36 B of spills; 3.5% faster than 3 waves at 156 VGPRs); the
// other kinds need 144-204 VGPRs, and 3 or 4 waves measured no faster.
template <int KIND, int STEP, bool COUNT = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KIND == KIND_GRAPH && STEP == STEP_RK4 ? 4 : 1, 8))) void k_refine(TraceArgs A, const double *__restrict__ BD,
                                                const double *__restrict__ SPD, const double *__restrict__ PLD,
                                                const double *__restrict__ TOD) {
    const int n = A.ctr[rti::CTR_REFINE];
    const int HW = A.width * A.height;
    unsigned c_eval = 0, c_bump = 0, c_step = 0;  // COUNT only
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        float4 r0, r1, r2, r3, r4;
        double tk_hi, tk_lo, h, sc;
        int obj, oi, k;
        uint64_t mask;
        if (!A.surr && compact_record(STEP, false)) {
            const float4 *rec = A.rec + 4 * (int64_t)r;
            r0 = rec[0], r1 = rec[1], r2 = rec[2], r3 = rec[3];
            tk_hi = tk_lo = 0.0;
            h = A.h;
            sc = r2.y;
            obj = __float_as_int(r2.z), oi = __float_as_int(r2.w), k = __float_as_int(r3.x);
            mask = (uint64_t)(uint32_t)__float_as_int(r3.y) | ((uint64_t)(uint32_t)__float_as_int(r3.z) << 32);
        } else {
            const float4 *rec = A.rec + rti::REC_F4 * (int64_t)r;
            r0 = rec[0], r1 = rec[1], r2 = rec[2], r3 = rec[3], r4 = rec[4];
            tk_hi = r2.y, h = r2.z;
            sc = r2.w;
            obj = __float_as_int(r3.x), oi = __float_as_int(r3.y), k = __float_as_int(r3.z);
            tk_lo = r3.w;
            mask = (uint64_t)(uint32_t)__float_as_int(r4.x) | ((uint64_t)(uint32_t)__float_as_int(r4.y) << 32);
        }
        V3<double> x = mk((double)r0.x + (double)r0.w, (double)r0.y + (double)r1.x, (double)r0.z + (double)r1.y);
        V3<double> y = mk((double)r1.z, (double)r1.w, (double)r2.x);
        int set = oi / HW;
        const double *Bs = BD + (int64_t)set * A.n_bumps * (is_deform(KIND) ? DEFORM_D : 8);
        double amp = A.twist_amp, th0 = A.twist_theta0;
        auto acc = [&](V3<double> p, V3<double> v, V3<double> &a) -> bool {
            if constexpr (COUNT) c_eval++;
            if constexpr (KIND == KIND_GRAPH) {
                a = graph_accel_f64(Bs, mask, p, v, COUNT ? &c_bump : nullptr);
                return true;
            } else if constexpr (KIND == KIND_TWIST) {
                return twist_accel<double>(amp, th0, p, v, a);
            } else if constexpr (KIND == KIND_ZTWIST) {
                a = ztwist_accel<double>(p, v);
                return true;
            } else if constexpr (is_deform(KIND)) {
                return deform_accel<double, false, KIND == KIND_DEFORM_ROT>(Bs, mask, p, v, a);
            } else if constexpr (KIND == KIND_GANISO) {
                a = graph_aniso_accel<double>(Bs, mask, p, v);
                return true;
            } else if constexpr (KIND == KIND_GQUAD) {
                a = graph_quad_accel<double>(mk(Bs[0], Bs[1], Bs[2]), p, v);
                return true;
            } else {
                a = mk(0.0, 0.0, 0.0);
                return true;
            }
        };
        // every probe of the bisection restarts from the same state, so the
        // first stage a(x_k, y_k) is evaluated once
        V3<double> a0;
        acc(x, y, a0);
        auto step = [&](double hs, V3<double> &xo, V3<double> &yo) {
            if constexpr (COUNT) c_step++;
            V3<double> dx, dv;
            if constexpr (STEP == STEP_RK45) {
                V3<double> A1 = a0, ex, ev;
                step_dp5<double>(acc, x, y, hs, A1, dx, dv, ex, ev);
            } else if constexpr (STEP == STEP_RK4) {
                step_rk4<double>(acc, x, y, hs, dx, dv, &a0);
            } else {
                step_euler<double>(acc, x, y, hs, dx, dv, &a0);
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
            // The bracket [lo, hi] of the sign change is narrowed to a width
            // of 2^-bisect_iters, as bisection would, but by regula falsi with
            // the Illinois modification (the value at an end kept twice in a
            // row is halved), the first probe at the segment's FP32 root: a
            // handful of probes instead of one per halving, since the implicit
            // function is nearly linear across one step.  When two probes
            // have not halved the bracket the next one is a plain halving, so
            // the bracket halves at least every third probe.
            const bool pos0 = F0 > 0.0;
            const double tol = ldexp(1.0, -A.bisect_iters);
            double lo = 0.0, hi = 1.0, flo = F0, fhi = F1;
            double w_ref = 1.0;
            int kept = 0, since = 0;  // end kept by the last probe (-1 lo, +1 hi); probes since the last check
            bool halve = false;
            for (int i = 0; i < 3 * A.bisect_iters + 2 && hi - lo > tol; ++i) {
                double m = i == 0 ? sc : (halve ? 0.5 * (lo + hi) : lo + (hi - lo) * (flo / (flo - fhi)));
                if (!(m > lo && m < hi)) m = 0.5 * (lo + hi);
                V3<double> xm, ym;
                step(m * h, xm, ym);
                const double fm = obj_F64(obj, xm, A.n_spheres, A.n_planes, SPD, PLD, TOD);
                if (fm == 0.0) {
                    lo = hi = m;
                    break;
                }
                if ((fm > 0.0) == pos0) {
                    lo = m;
                    flo = fm;
                    if (kept == 1) fhi *= 0.5;
                    kept = 1;
                } else {
                    hi = m;
                    fhi = fm;
                    if (kept == -1) flo *= 0.5;
                    kept = -1;
                }
                halve = false;
                if (++since == 2) {
                    halve = hi - lo > 0.5 * w_ref;
                    w_ref = hi - lo;
                    since = 0;
                }
            }
            s = 0.5 * (lo + hi);
        }
        V3<double> xs, ys;
        step(s * h, xs, ys);
        // RK4 and Euler: k steps of h, plus (surrogate) jumps and partial steps
        double tk = STEP == STEP_RK45 ? tk_hi + tk_lo : (double)k * (double)A.h + (tk_hi + tk_lo);
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
        if (A.tape_hit) {
            float *tr = A.tape_hit + (int64_t)oi * rti::TAPE_REC;
            tr[0] = r0.x;
            tr[1] = r0.y;
            tr[2] = r0.z;
            tr[3] = r0.w;
            tr[4] = r1.x;
            tr[5] = r1.y;
            tr[6] = r1.z;
            tr[7] = r1.w;
            tr[8] = r2.x;
            tr[9] = (float)s;
            tr[10] = __int_as_float(k);
            tr[11] = __int_as_float(obj);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(A.stats + rti::ST_REFINED, (unsigned long long)n);
    if constexpr (COUNT) {
        unsigned v[3] = {c_eval, c_bump, c_step};
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) v[q] += __shfl_xor(v[q], o);
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(A.stats + rti::ST_REF_EVALS, (unsigned long long)v[0]);
            atomicAdd(A.stats + rti::ST_REF_BUMPS, (unsigned long long)v[1]);
            atomicAdd(A.stats + rti::ST_REF_STEPS, (unsigned long long)v[2]);
        }
    }
}

// ====================================================== ordered compaction
// After pass p: survivors of chunk c (alive mask cmask[c]) move to the
// sorted list of pass p+1 at
//   pad_base[set] + (survivors in chunks < c) + (rank in chunk) - (survivors in sets < set)
// where pad_base[set] rounds every earlier set up to whole chunks.  Sorted
// ids keep 64 consecutive survivors spatially close (same or adjacent
// tiles), which keeps the per-wave culling windows tight.
__global__ __launch_bounds__(1024) void k_chunk_scan(TraceArgs A, int pass) {
    __shared__ int sh[1024];
    const int nch = A.ctr[rti::CTR_PASS0 + pass * rti::CTR_PASS_WORDS + rti::CTR_NCH];
    const int nblk = (nch + rti::SCAN_BLOCK - 1) / rti::SCAN_BLOCK;
    for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
        int c = b * rti::SCAN_BLOCK + threadIdx.x;
        int v = c < nch ? __popcll(A.cmask[c]) : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            int u = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += u;
            __syncthreads();
        }
        if (c < nch) A.cscan[c] = sh[threadIdx.x] - v;
        if (threadIdx.x == 1023) A.bscan[b] = sh[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void k_block_scan(TraceArgs A, int pass) {
    __shared__ int sh[1024];
    __shared__ int carry;
    const int nch = A.ctr[rti::CTR_PASS0 + pass * rti::CTR_PASS_WORDS + rti::CTR_NCH];
    const int nblk = (nch + rti::SCAN_BLOCK - 1) / rti::SCAN_BLOCK;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nblk; base += 1024) {
        int i = base + threadIdx.x;
        int v = i < nblk ? A.bscan[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            int u = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += u;
            __syncthreads();
        }
        if (i < nblk) A.bscan[i] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += sh[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_scatter(TraceArgs A, int pass) {
    const int lane = lane_id();
    const int *pc = A.ctr + rti::CTR_PASS0 + pass * rti::CTR_PASS_WORDS;
    const int nch = pc[rti::CTR_NCH];
    // per-set survivor counts of this pass: unpadded and chunk-padded prefixes
    int cnt = lane < A.n_sets ? pc[rti::CTR_SURV + lane] : 0;
    int excl = wave_incl_scan(cnt) - cnt;
    int pad = (cnt + 63) & ~63;
    int pexcl = wave_incl_scan(pad) - pad;
    const int *__restrict__ ids_in = A.ids[pass & 1];
    int *__restrict__ ids_out = A.ids[(pass + 1) & 1];
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int c = wave; c < nch; c += nwaves) {
        uint64_t m = A.cmask[c];
        if (!m) continue;
        bool alive = (m >> lane) & 1ull;
        int id = alive ? (pass == 0 ? c * 64 + lane : ids_in[c * 64 + lane]) : 0;
        int s = id / A.T;
        int rank = A.bscan[c / rti::SCAN_BLOCK] + A.cscan[c] + mbcnt64(m);
        int pos = __shfl(pexcl, s) + rank - __shfl(excl, s);
        if (alive) ids_out[pos] = id;
    }
}

__global__ void k_reset(int *ctr, int n_words, unsigned long long *stats) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += gridDim.x * blockDim.x) ctr[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < rti::ST_N) stats[threadIdx.x] = 0;
}

template <int KIND, int STEP, bool SURR, bool TAPE = false>
hipError_t launch_pass(const TraceArgs &a, const rti::DeviceData &d, int p, int grid, hipStream_t s) {
    if constexpr (STEP != STEP_RK45 && !SURR && !TAPE) {
        if (a.batch) {
            hipLaunchKernelGGL((k_trace_pass<KIND, STEP, false, false, false, true>), dim3(grid), dim3(256), 0, s, a,
                               p, d.bump_f, d.sph_f, d.pln_f, d.tor_f);
            return hipGetLastError();
        }
    }
    if (a.count)
        hipLaunchKernelGGL((k_trace_pass<KIND, STEP, true, SURR, TAPE>), dim3(grid), dim3(256), 0, s, a, p,
                           d.bump_f, d.sph_f, d.pln_f, d.tor_f);
    else
        hipLaunchKernelGGL((k_trace_pass<KIND, STEP, false, SURR, TAPE>), dim3(grid), dim3(256), 0, s, a, p,
                           d.bump_f, d.sph_f, d.pln_f, d.tor_f);
    return hipGetLastError();
}

template <int KIND, int STEP>
hipError_t launch_kind_step(const TraceArgs &a, const rti::DeviceData &d, int n_passes, int grid, int rgrid,
                            hipStream_t s, hipEvent_t *ev, const rti::SurrArgs *S, int mlp_blocks) {
    const int scan_blocks = std::min((a.max_chunks + rti::SCAN_BLOCK - 1) / rti::SCAN_BLOCK, 1024);
    const int scatter_blocks = std::max(1, std::min((a.max_chunks + 3) / 4, 4096));
    for (int p = 0; p < n_passes; ++p) {
        if (p > 0) {
            // ordered compaction of the survivors of pass p-1 (not timed as a pass)
            hipLaunchKernelGGL(k_chunk_scan, dim3(scan_blocks), dim3(1024), 0, s, a, p - 1);
            hipLaunchKernelGGL(k_block_scan, dim3(1), dim3(1024), 0, s, a, p - 1);
            hipLaunchKernelGGL(k_scatter, dim3(scatter_blocks), dim3(256), 0, s, a, p - 1);
            if (ev) (void)hipEventRecord(ev[2 * n_passes + 2 + p], s);
        }
        hipError_t e;
        if constexpr (KIND == KIND_GRAPH && STEP == STEP_RK4) {
            if (a.tape_ck) {
                e = launch_pass<KIND, STEP, false, true>(a, d, p, grid, s);
                if (e != hipSuccess) return e;
                if (ev) (void)hipEventRecord(ev[2 + p], s);
                continue;
            }
            if (a.surr) {
                e = launch_pass<KIND, STEP, true>(a, d, p, grid, s);
                if (e != hipSuccess) return e;
                if (ev) (void)hipEventRecord(ev[2 + p], s);
                // crossings parked in pass p (not timed as a pass)
                e = rti::launch_surr_stage(a, *S, d.bump_f, p, mlp_blocks, s);
                if (e != hipSuccess) return e;
                if (ev) (void)hipEventRecord(ev[3 * n_passes + 3 + p], s);
                continue;
            }
        }
        e = launch_pass<KIND, STEP, false>(a, d, p, grid, s);
        if (e != hipSuccess) return e;
        if (ev) (void)hipEventRecord(ev[2 + p], s);
    }
    if (a.count)
        hipLaunchKernelGGL((k_refine<KIND, STEP, true>), dim3(rgrid), dim3(256), 0, s, a, d.bump_d, d.sph_d, d.pln_d,
                           d.tor_d);
    else
        hipLaunchKernelGGL((k_refine<KIND, STEP>), dim3(rgrid), dim3(256), 0, s, a, d.bump_d, d.sph_d, d.pln_d,
                           d.tor_d);
    hipError_t e = hipGetLastError();
    if (ev) (void)hipEventRecord(ev[2 + n_passes], s);
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
    return kind >= 0 && kind <= 7 && step >= 0 && step <= 2;
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
    case KIND_ZTWIST: RT_DISPATCH(KIND_ZTWIST, occ)
    case KIND_DEFORM: RT_DISPATCH(KIND_DEFORM, occ)
    case KIND_DEFORM_ROT: RT_DISPATCH(KIND_DEFORM_ROT, occ)
    case KIND_GANISO: RT_DISPATCH(KIND_GANISO, occ)
    default: RT_DISPATCH(KIND_GQUAD, occ)
    }
}

// Workspace of the allocation-free trace: one array per GPU, held by the
// code object until the process ends.  Host code never passes `scratch`
// itself to a kernel (on the host it names a stand-in, not device memory):
// it uses the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[RT_NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(int device, void **ptr) {
    constexpr int MAX_DEV = 64;
    static std::mutex mu;
    static void *addr[MAX_DEV] = {};
    if (!ptr || device < 0 || device >= MAX_DEV) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int prev = -1;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != device) (void)hipSetDevice(prev);  // restore the caller's device, best effort
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

hipError_t launch_trace(const TraceArgs &a, const DeviceData &d, int n_passes, int grid, int rgrid, hipStream_t s,
                        hipEvent_t *ev, const SurrArgs *S, int mlp_blocks) {
    int words = CTR_PASS0 + n_passes * CTR_PASS_WORDS + CTR_SURR_WORDS;
    if (ev) (void)hipEventRecord(ev[0], s);
    hipLaunchKernelGGL(k_reset, dim3(64), dim3(256), 0, s, a.ctr, words, a.stats);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev) (void)hipEventRecord(ev[1], s);
    const int step = a.step_kind;
    // checkpoint tapes and learned crossings exist for the graph metric with RK4 only
    if ((a.tape_ck || a.surr) && !(a.kind == KIND_GRAPH && step == STEP_RK4)) return hipErrorInvalidValue;
    switch (a.kind) {
    case KIND_EUCLID: RT_DISPATCH(KIND_EUCLID, launch_kind_step, a, d, n_passes, grid, rgrid, s, ev, S, mlp_blocks)
    case KIND_GRAPH: RT_DISPATCH(KIND_GRAPH, launch_kind_step, a, d, n_passes, grid, rgrid, s, ev, S, mlp_blocks)
    case KIND_TWIST: RT_DISPATCH(KIND_TWIST, launch_kind_step, a, d, n_passes, grid, rgrid, s, ev, S, mlp_blocks)
    case KIND_ZTWIST: RT_DISPATCH(KIND_ZTWIST, launch_kind_step, a, d, n_passes, grid, rgrid, s, ev, S, mlp_blocks)
    case KIND_DEFORM: RT_DISPATCH(KIND_DEFORM, launch_kind_step, a, d, n_passes, grid, rgrid, s, ev, S, mlp_blocks)
    case KIND_DEFORM_ROT: RT_DISPATCH(KIND_DEFORM_ROT, launch_kind_step, a, d, n_passes, grid, rgrid, s, ev, S, mlp_blocks)
    case KIND_GANISO: RT_DISPATCH(KIND_GANISO, launch_kind_step, a, d, n_passes, grid, rgrid, s, ev, S, mlp_blocks)
    default: RT_DISPATCH(KIND_GQUAD, launch_kind_step, a, d, n_passes, grid, rgrid, s, ev, S, mlp_blocks)
    }
}

}  // namespace rti
