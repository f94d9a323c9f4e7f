// Host-side launch description shared by the C-ABI layer and the kernels'
// launchers.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rti {

// Ray-state fields.  Ray ids enumerate 8x8 pixel tiles, set-major:
// id = (set * tiles + tile) * 64 + lane, so 64 consecutive ids are one tile.
// Layout is blocked by 64 ids: field f of ray id lives at float index
// ((id / 64) * Q_NFIELDS + f) * 64 + id % 64, so a wave touches 256
// contiguous bytes per field and all fields of a lane are reachable from
// one base address with small immediate offsets.
enum QField {
    Q_XH = 0,   // 0..2 position, high part
    Q_XL = 3,   // 3..5 position, low part
    Q_Y = 6,    // 6..8 velocity
    Q_TH = 9,   // t, high part (RK45)
    Q_TL = 10,  // t, low part (RK45)
    Q_H = 11,   // current trial step (RK45)
    Q_STEPS = 12,  // accepted steps (int bits)
    Q_ATT = 13,    // trial steps incl. rejected (int bits)
    Q_SKIP = 14,   // surrogate: bump whose support sphere is integrated through (int bits, -1 none)
    Q_NFIELDS = 15
};

// Counter block layout (int32 words).
constexpr int CTR_REFINE = 0;        // number of refine records
constexpr int CTR_PASS0 = 64;        // first pass block
constexpr int CTR_PASS_WORDS = 256;  // per pass: 8 chunk counters (16 words apart), 64 per-set survivors, chunk count
constexpr int CTR_CHUNK_STRIDE = 16;
constexpr int CTR_SURV = 128;        // offset of the survivor counts inside a pass block
constexpr int CTR_NCH = 192;         // offset of the pass's chunk count
constexpr int CTR_XQ = 193;          // offset of the pass's crossing count (surrogate)
// Surrogate control block after the last pass block: per-network crossing
// counts [64] at XC_CNT, row offsets [65] at XC_ROW, tile offsets [65] at
// XC_TILE (entry 64 of each: the totals).
constexpr int CTR_SURR_WORDS = 256;
constexpr int MAX_NETS = 64;
constexpr int XC_CNT = 0, XC_ROW = 64, XC_TILE = 136;
// Per-network parameter stride of the networks the tracer holds (16-byte
// aligned rows for vector loads of bf16 weights).
constexpr int64_t MLP_P_PAD = 134920;

constexpr int MAX_PASSES_API = 512;
constexpr int SCAN_BLOCK = 1024;     // chunks per block of the survivor scan

// Refine record: at most 5 float4 (80 bytes; 4 for RK4 and Euler traces
// without learned crossings).
constexpr int REC_F4 = 5;

enum Stat {
    ST_RAYS = 0,
    ST_STEPS,
    ST_ATTEMPTS,
    ST_WAVE_ITERS,
    ST_LANE_ITERS,
    ST_BUMP_LIST,
    ST_OBJ_LIST,
    ST_REFINED,
    ST_ACC_EVALS,
    ST_BUMP_EVALS,
    ST_OBJ_TESTS,
    ST_XING,  // surrogate crossings queued
    ST_XACC,  // surrogate crossings accepted
    ST_ADJ_STEPS,  // adjoint: full RK4 steps reversed
    ST_ADJ_TERMS,  // adjoint: bump terms inside their cut at the reversed steps' stages
    ST_ADJ_RECOMP, // adjoint: full RK4 steps recomputed from the checkpoints
    ST_BATCH_WIN,     // batched segments: windows marched
    ST_BATCH_REPLAY,  // batched segments: windows marched again with per-step tests
    ST_REF_EVALS,     // COUNT: FP64 refinement acceleration evaluations
    ST_REF_BUMPS,     // COUNT: bumps inside their cut at those evaluations
    ST_REF_STEPS,     // COUNT: FP64 refinement integrator steps
    ST_N
};

struct TraceArgs {
    // metric
    int kind, n_sets, n_bumps;
    float twist_amp, twist_theta0;
    // scene
    int n_spheres, n_planes, n_tori;
    // camera (basis computed on the host)
    float eye[3], right[3], up[3], fwd[3];
    float tan_half, aspect;
    int width, height, tiles_x, tiles_y;
    // rule
    int step_kind;
    float h, rtol, atol, h_min, h_max, t_max;
    int max_steps, K, S, bisect_iters;
    float cull_margin;  // < 0: no culling
    float cull_base;    // composed deformations: window motion without displacement, (K+1) h_max 1.02 + 1e-4
    float cull_disp;    // composed deformations: bound on |Phi(x) - x| over all x
    int count;          // instrumented variant
    int batch;          // batched multi-segment intersection
    // buffers
    float *st;             // ray state, Q_NFIELDS x cap
    int *ids[2];           // sorted survivor-id lists (pass p reads ids[p & 1])
    unsigned long long *cmask;  // per chunk: survivors of the current pass
    int *cscan;            // per chunk: survivors before it inside its scan block
    int *bscan;            // per scan block: survivors before it
    int64_t cap;           // ray ids = n_sets * T
    int T;                 // ray ids per set = tiles * 64
    int max_chunks;        // capacity of the per-chunk arrays
    int *ctr;
    unsigned long long *stats;
    float4 *rec;
    // outputs
    float *out_hit, *out_t, *out_dir;
    int *out_id, *out_steps;
    // adjoint tape (NULL for a plain trace): checkpoints of (x_hi, x_lo, y)
    // every ckpt_every accepted steps, blocked by 64 ray ids:
    //   tape_ck[(((id / 64) * n_ckpt + c) * 9 + f) * 64 + id % 64]
    // and one hit record per output pixel (TAPE_REC floats):
    //   x_hi[3], x_lo[3], y[3] before the hit step, s*, step index, object id
    //   (object -1: no hit, the pixel carries no gradient)
    float *tape_ck;
    float *tape_hit;
    int ckpt_every, n_ckpt;
    // surrogate (graph metric, RK4, one set): per bump two float4
    //   (cx, cy, cz, R^2), (sigma, network (int bits, -1: not eligible), R, 0)
    // with R = 3 sigma; rays entering an eligible support sphere park there
    // and push (ray id, bump, rank within the network's rows) to xq.
    int surr;
    int n_passes;
    const float4 *surr_sb;
    int4 *xq;
    int *xctl;  // control block: per-network counts, offsets, tile offsets
};

// Learned crossing stage run between passes.
struct SurrArgs {
    int n_nets, n_tab, n_bins;
    int64_t stride;       // parameters per network in wb / params (multiple of 8)
    float tol;
    const __bf16 *wb;     // [n_nets][stride], 16-byte aligned
    const float *params;  // [n_nets][stride]
    const float *scale;   // [n_nets]
    const float *arc;     // [n_nets][n_tab] arc in units of sigma at cos(theta) = i / (n_tab - 1)
    const float *err;     // [n_nets][n_bins][2] position / direction error bounds per bin of cos(theta)
    int2 *sorted;         // crossing slot -> (ray id, bump), grouped by network
    float *xin, *xout;    // [slots][6]
};

constexpr int TAPE_REC = 12;

struct DeviceData {
    const float4 *bump_f;   // [n_sets*n_bumps][2]
    const double *bump_d;   // [n_sets*n_bumps][8]
    const float4 *sph_f;    // [n_spheres]
    const float4 *pln_f;    // [n_planes]
    const float *tor_f;     // [n_tori][8]
    const double *sph_d;    // [n_spheres][4]
    const double *pln_d;    // [n_planes][4]
    const double *tor_d;    // [n_tori][8]
};

// Enqueue a full trace (reset, passes, refine).  Returns hipSuccess or the
// first launch error.
// ev: NULL, or 4 n_passes + 3 events: before the reset, after the reset,
// after each pass [2 + p], after the refinement [2 + n_passes], after each
// compaction [2 n_passes + 2 + p] and after each crossing stage
// [3 n_passes + 3 + p].  S: crossing stage (a.surr), else NULL; the
// control block after the pass blocks must hold CTR_SURR_WORDS words.
hipError_t launch_trace(const TraceArgs &a, const DeviceData &d, int n_passes, int grid_blocks,
                        int refine_blocks, hipStream_t s, hipEvent_t *ev, const struct SurrArgs *S, int mlp_blocks);
// Device address, on `device`, of the static workspace that rt_trace_noalloc
// carves (RT_NOALLOC_SCRATCH_BYTES).  Looked up with the device made current,
// once per device; later calls return the cached address.  Thread-safe.
hipError_t noalloc_scratch(int device, void **ptr);
// ------------------------------------------------------ direct illumination
// Table strides of a composed deformation: float4 records (FP32 table) and
// doubles (FP64 table) per deformation; the device helpers read the same
// layout.
constexpr int DEFORM_F4 = 5, DEFORM_D = 16;
// Kernel kind of composed deformations with a rotating field (the API kind
// is RT_METRIC_PULLBACK_DEFORM; the kernels compile the rotation terms
// only for this kind).
constexpr int KERNEL_KIND_DEFORM_ROT = 7;
// Steps between the culling windows of the illumination's shots.
constexpr int ILLUM_CULL_EVERY = 16;
struct IllumArgs {
    int kind, n_sets, n_bumps;
    float twist_amp, twist_theta0;
    int n_spheres, n_planes, n_tori;
    int width, height;
    const float *hit;  // traced hit points [n_sets * H * W][3]
    const int *id;     // traced object ids
    float light[3];
    float h, tol;
    int max_iters, max_steps;
    float cull_margin;  // half-width of a lane's culling window; < 0: no culling
    float *shade, *dir, *len;
    int *status;
    // workspace: Newton state per pixel, the two iteration lists and the
    // step list, two counters per iteration
    float *w_al, *w_be, *w_T, *w_F;  // angles, length, last residual
    float *w_X, *w_Y;                // base shot's end point and velocity [3 per pixel]
    int *list[3];
    int *ctr;  // 2 (max_iters + 1) words for each shooting attempt: list sizes, then step-list sizes
    // continuation rounds: the shots aim at q + cont (L - q) instead of L,
    // and a pixel that converges there is marked conv_code
    float cont;
    int conv_code;
};
// Pixels left without a geodesic retry from a converged neighbour's
// direction: ILLUM_RETRY_ROUNDS rounds (each seeded from everything converged
// so far) of max(max_iters / 2, 1) Newton iterations.
constexpr int ILLUM_RETRY_ROUNDS = 3;
// Then the pixels still without one follow a continuation in the light
// position: targets q + lambda (L - q) for the ILLUM_CONT_STAGES values
// lambda = 1/S, 2/S, ..., 1, each stage started from the previous solution.
constexpr int ILLUM_CONT_STAGES = 8;
hipError_t launch_illum(const IllumArgs &a, const DeviceData &d, int grid, hipStream_t s);
// ------------------------------------------------------------- MLP (BF16)
enum Epi { EPI_NONE = 0, EPI_HIDDEN = 1, EPI_BIAS = 2, EPI_DSILU = 3 };

// Grouped GEMM C = A B (see rt_mlp.hip).  Group g offsets every operand by
// its group stride; with rows != NULL group g has rows[g] rows starting at
// row row_off[g] of A and C (A's group stride is then normally 0).
struct GemmArgs {
    const __bf16 *A;
    int64_t a_g;
    int64_t sam, sak;
    const __bf16 *B;
    int64_t b_g;
    int64_t sbk, sbn;
    int M, N, K;
    const int *rows;
    const int *row_off;
    int epi;
    const float *bias;
    int64_t bias_g;
    float *Cf;
    int64_t cf_g, ldcf;
    __bf16 *Cb;
    int64_t cb_g, ldcb;
    const float *Z;
    int64_t z_g, ldz;
};

// Per-network parameter layout (floats / bf16 values).
constexpr int64_t MLP_H = 256, MLP_IN = 6, MLP_OUT = 6;
constexpr int64_t OFF_W1 = 0, OFF_B1 = OFF_W1 + MLP_H * MLP_IN, OFF_W2 = OFF_B1 + MLP_H, OFF_B2 = OFF_W2 + MLP_H * MLP_H,
                  OFF_W3 = OFF_B2 + MLP_H, OFF_B3 = OFF_W3 + MLP_H * MLP_H, OFF_W4 = OFF_B3 + MLP_H,
                  OFF_B4 = OFF_W4 + MLP_OUT * MLP_H, MLP_P = OFF_B4 + MLP_OUT;

// Activation workspace of a forward pass kept for the backward.
struct MlpWork {
    float *xf;        // [n][B][6] inputs (FP32 first layer)
    float *z[3];      // [n][B][256] pre-activations
    __bf16 *h[3];     // [n][B][256] activations (bf16, high part)
    __bf16 *hl[3];    // [n][B][256] low parts: h - hi, rounded to bf16
    __bf16 *dyb;      // [n][B][6]
    float *dzf[2];    // [n][B][256]
    __bf16 *dzb[2];   // [n][B][256]
    float *part;      // colsum partials [n][ceil(B/256)][256]
};
size_t mlp_work_bytes(int n_nets, int batch);
void mlp_work_carve(void *base, int n_nets, int batch, MlpWork &w);
hipError_t mlp_forward(int n_nets, int batch, const __bf16 *wb, const float *params, const float *x, float *y,
                       const MlpWork &w, bool keep, hipStream_t s);
hipError_t mlp_backward(int n_nets, int batch, const __bf16 *wb, const float *params, const float *dy, float *grad,
                        const MlpWork &w, hipStream_t s);
hipError_t launch_gemm(const GemmArgs &G, int groups, int max_rows, hipStream_t s);
hipError_t launch_colsum(const float *X, int64_t xg, int rows, int N, int groups, float *part, float *out,
                         int64_t out_g, hipStream_t s);
hipError_t launch_adamw(float *p, __bf16 *pb, float *m, float *v, const float *g, int64_t n, float lr, float b1,
                        float b2, float eps, float wd, int step, hipStream_t s);
hipError_t launch_to_bf16(const float *x, __bf16 *y, int64_t n, hipStream_t s);
hipError_t launch_mse_grad(const float *y, const float *t, float *dy, int64_t n, int batch, float *part, int nblk,
                           hipStream_t s);

// step_batch > 0: outputs laid out [n_per / step_batch][n_shapes][step_batch]
// (n_per a multiple of step_batch), one contiguous training batch per step.
hipError_t launch_cross_gen(const float *kappa, const float *scale, int n_shapes, int n_per, float h, int mode,
                            uint64_t seed, float *X, float *Y, float *AUX, float kappa_max, hipStream_t s,
                            int step_batch = 0);
hipError_t launch_cross_cal(const float *X, const float *P, const float *Y, const float *scale, int n_shapes,
                            int n_per, int n_bins, float *err, hipStream_t s);
// Crossing stage after pass `pass`: group by network, fused MLP forward,
// decode, probe, and jump or fall back.
// Fused grouped MLP forward: ctl holds per-network row offsets at XC_ROW
// and tile offsets at XC_TILE; uses S.wb, S.params, S.stride, S.n_nets,
// S.xin, S.xout.
hipError_t launch_mlp_grouped(const int *ctl, const SurrArgs &S, int blocks, hipStream_t s);
hipError_t launch_surr_stage(const TraceArgs &a, const SurrArgs &S, const float4 *bump_f, int pass, int mlp_blocks,
                             hipStream_t s);

// Adjoint of a taped RK4 trace (graph metric): per-chunk partial gradients,
// then per-set sums into grad [n_sets][n_bumps][5].
// blocks: persistent one-wave blocks (adjoint_blocks_per_cu x CUs); scratch
// holds ckpt_every x 6 x 64 floats per block; next: one int (chunk queue).
hipError_t launch_adjoint(const TraceArgs &a, const DeviceData &d, const float *grad_hit, float *partial,
                          float *grad, float *scratch, int *next, unsigned long long *stats, int blocks,
                          hipStream_t s);
int adjoint_blocks_per_cu(int n_bumps);
hipError_t launch_loss(const float *hit, const int *id, const float *thit, const int *tid, const unsigned char *mask,
                       int n_sets, int HW, float *grad_hit, float *block_sum, float *loss, hipStream_t s);
int adjoint_max_bumps();
// Blocks per CU the trace kernel can keep resident for this kind/step.
int trace_blocks_per_cu(int kind, int step);
bool supported(int kind, int step);

}  // namespace rti
