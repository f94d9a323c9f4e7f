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
    Q_NFIELDS = 14
};

// Counter block layout (int32 words).
constexpr int CTR_REFINE = 0;        // number of refine records
constexpr int CTR_PASS0 = 64;        // first pass block
constexpr int CTR_PASS_WORDS = 256;  // per pass: 8 chunk counters (16 words apart), 64 per-set survivors, chunk count
constexpr int CTR_CHUNK_STRIDE = 16;
constexpr int CTR_SURV = 128;        // offset of the survivor counts inside a pass block
constexpr int CTR_NCH = 192;         // offset of the pass's chunk count

constexpr int MAX_PASSES_API = 512;
constexpr int SCAN_BLOCK = 1024;     // chunks per block of the survivor scan

// Refine record: 5 float4 (80 bytes).
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
    int count;          // instrumented variant
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
// ev: NULL, or n_passes + 3 events recorded before the reset, after the
// reset, after each pass and after the refinement.
hipError_t launch_trace(const TraceArgs &a, const DeviceData &d, int n_passes, int grid_blocks,
                        int refine_blocks, hipStream_t s, hipEvent_t *ev);
// Adjoint of a taped RK4 trace (graph metric): per-chunk partial gradients,
// then per-set sums into grad [n_sets][n_bumps][5].
hipError_t launch_adjoint(const TraceArgs &a, const DeviceData &d, const float *grad_hit, float *partial,
                          float *grad, float *scratch, int blocks, hipStream_t s);
hipError_t launch_loss(const float *hit, const int *id, const float *thit, const int *tid, const unsigned char *mask,
                       int n_sets, int HW, float *grad_hit, float *block_sum, float *loss, hipStream_t s);
int adjoint_max_bumps();
// Blocks per CU the trace kernel can keep resident for this kind/step.
int trace_blocks_per_cu(int kind, int step);
bool supported(int kind, int step);

}  // namespace rti
