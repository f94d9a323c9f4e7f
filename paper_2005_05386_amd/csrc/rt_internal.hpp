// Host-side launch description shared by the C-ABI layer and the kernels'
// launchers.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rti {

// Ray-queue fields (structure of arrays, one float per ray per field).
enum QField {
    Q_XH = 0,   // 0..2 position, high part
    Q_XL = 3,   // 3..5 position, low part
    Q_Y = 6,    // 6..8 velocity
    Q_TH = 9,   // t, high part (RK45)
    Q_TL = 10,  // t, low part (RK45)
    Q_H = 11,   // current trial step (RK45)
    Q_STEPS = 12,  // accepted steps (int bits)
    Q_PIX = 13,    // pixel index within the set (int bits)
    Q_ATT = 14,    // trial steps incl. rejected (int bits)
    Q_NFIELDS = 15
};

// Counter block layout (int32 words).
constexpr int CTR_REFINE = 0;        // number of refine records
constexpr int CTR_PASS0 = 64;        // first pass block
constexpr int CTR_PASS_WORDS = 192;  // per pass: 8 chunk counters (16 words apart) + 64 per-set survivors
constexpr int CTR_CHUNK_STRIDE = 16;
constexpr int CTR_SURV = 128;        // offset of the survivor counts inside a pass block

constexpr int MAX_PASSES_API = 512;

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
    float *q[2];
    int64_t cap;  // rays per queue = n_sets * width * height
    int *ctr;
    unsigned long long *stats;
    float4 *rec;
    // outputs
    float *out_hit, *out_t, *out_dir;
    int *out_id, *out_steps;
};

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
// Blocks per CU the trace kernel can keep resident for this kind/step.
int trace_blocks_per_cu(int kind, int step);
bool supported(int kind, int step);

}  // namespace rti
