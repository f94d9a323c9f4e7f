// Kernels of the surrogate MLP (6 -> 256 -> 256 -> 256 -> 6, SiLU): the
// first layer (K = 6) and the output layer (N = 6) in FP32 on the vector
// units (1% of the FLOPs), the two 256x256 products on the BF16 matrix
// cores with FP32 accumulation, column sums for bias gradients, and the
// AdamW update.
//
// Forward products use three-term split bf16: a value v is carried as
// hi = bf16(v) and lo = bf16(v - hi), and A B is accumulated as
// Ah Bh + Ah Bl + Al Bh (the dropped Al Bl is ~2^-16 relative), which gives
// the network near-FP32 accuracy; plain bf16 forward products leave a
// relative error floor of about 1e-3 in the learned map.  The backward
// products (signals and weight gradients) stay single bf16.
//
// GEMM: for every group g (one network), C[m][n] = sum_k A(m,k) B(k,n) with
// A(m,k) = A[a_off(g) + m*sam + k*sak], B(k,n) = B[b_off(g) + k*sbk + n*sbn]
// (bf16), arbitrary strides so that transposed operands need no copies.
// A 256-thread workgroup computes a 64x64 tile of C: the 64x32 A slice and
// 32x64 B slice of each K step are staged in LDS (zero-filled outside the
// matrix; the next slice is read into registers during the products), then
// each wave accumulates a 32x32 block with four v_mfma_f32_16x16x32_bf16
// per step.  Lane l of a 16x16x32 MFMA supplies
// A[l%16][8(l/16) .. 8(l/16)+7] and B[8(l/16) .. +7][l%16] and receives
// D[4(l/16) + j][l%16], j = 0..3.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "rt_internal.hpp"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// XCD-aware tile order.  Workgroups go to the 8 XCDs round-robin by their
// linear id, and each XCD has its own L2.  Tiles are numbered with the
// column tile fastest, then the row tile, then the group (network), and
// XCD k takes the k-th contiguous eighth of that order: the column tiles of
// one row tile run one after another on the same XCD (the row slice of A
// is fetched from memory once), and a network's weights are read by one
// XCD only.  The grid is 1-D, 8 * ceil(tiles / 8) workgroups; returns false
// for the padding.
__device__ __forceinline__ bool xcd_tile(int nx, int ny, int nz, int &x, int &y, int &z) {
    const int T = nx * ny * nz;
    const int per = (T + 7) / 8;
    const int b = blockIdx.x;
    const int t = (b & 7) * per + (b >> 3);
    if ((b >> 3) >= per || t >= T) return false;
    x = t % nx;
    y = (t / nx) % ny;
    z = t / (nx * ny);
    return true;
}
inline unsigned xcd_grid(int nx, int ny, int nz) { return 8u * (unsigned)(((int64_t)nx * ny * nz + 7) / 8); }
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
    float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// Operand staging layouts of the backward GEMM: L_GEN reads element by
// element through both strides (any shape); L_KC has unit stride along k
// (16-byte loads of 8 consecutive k); L_MC has unit stride along the row
// index m (or n for B): 16-byte loads of 8 consecutive rows at one k,
// written transposed into LDS; L_MC4 is L_MC with four 4-byte loads for
// operands whose group stride is only even.  The vector layouts need
// 8 | M, N, K and the other stride, 8 | the group stride and 16-byte
// aligned bases (2 | and 4-byte aligned for L_MC4).
enum { L_GEN = 0, L_KC = 1, L_MC = 2, L_MC4 = 3 };

// Stage a 64 x 32 (row, k) slice of X(row, k) = X[row*srow + k*sk] into
// S[row][k]; rows >= R and k >= K are zero.
template <int L>
__device__ __forceinline__ void stage_load(const __bf16 *__restrict__ X, int64_t srow, int64_t sk, int r0, int R,
                                           int k0, int K, int tid, bf16x8 &v) {
    if constexpr (L == L_KC) {
        const int r = r0 + (tid >> 2), k = k0 + (tid & 3) * 8;
        if (r < R && k < K) {
            v = *(const bf16x8 *)(X + (int64_t)r * srow + k);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = (__bf16)0.0f;
        }
    } else if constexpr (L == L_MC || L == L_MC4) {
        const int k = k0 + (tid >> 3), r = r0 + (tid & 7) * 8;
        if (r < R && k < K) {
            if constexpr (L == L_MC) {
                v = *(const bf16x8 *)(X + (int64_t)k * sk + r);
            } else {
                const uint32_t *w = (const uint32_t *)(X + (int64_t)k * sk + r);
                typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
                const u32x4 u = {w[0], w[1], w[2], w[3]};
                v = __builtin_bit_cast(bf16x8, u);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = (__bf16)0.0f;
        }
    } else {
        const int r = r0 + (tid >> 2), kc = k0 + (tid & 3) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e)
            v[e] = (r < R && kc + e < K) ? X[(int64_t)r * srow + (int64_t)(kc + e) * sk] : (__bf16)0.0f;
    }
}

template <int L>
__device__ __forceinline__ void stage_store(__bf16 (*S)[40], int tid, const bf16x8 &v) {
    if constexpr (L == L_MC || L == L_MC4) {
        const int k = tid >> 3, r = (tid & 7) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) S[r + e][k] = v[e];
    } else {
        *(bf16x8 *)&S[tid >> 2][(tid & 3) * 8] = v;
    }
}

// VEC: every tile is whole and the outputs (and Z) are 16-byte aligned with
// row strides a multiple of 8 elements; the epilogue then goes through LDS
// and every thread stores 16 consecutive values of one row with 16-byte
// stores (EPI_NONE and EPI_DSILU).
template <int LA, int LB, bool VEC = false>
__global__ __launch_bounds__(256) void k_gemm(rti::GemmArgs G, int ntx, int nty, int ntz) {
    // one LDS block: the two staging arrays, reused for the output tile
    __shared__ __attribute__((aligned(16))) float smem[VEC ? 64 * 68 : 64 * 40];
    static_assert(sizeof(smem) >= 2 * 64 * 40 * sizeof(__bf16), "staging exceeds the LDS block");
    __bf16(*As)[40] = reinterpret_cast<__bf16(*)[40]>(&smem[0]);
    __bf16(*Bs)[40] = reinterpret_cast<__bf16(*)[40]>(&smem[0]) + 64;  // transposed: Bs[n][k]
    int tx, ty, g;
    if (!xcd_tile(ntx, nty, ntz, tx, ty, g)) return;
    int M = G.M;
    int64_t row0 = 0;
    if (G.rows) {
        M = G.rows[g];
        row0 = G.row_off[g];
    }
    const int m0 = ty * 64, n0 = tx * 64;
    if (m0 >= M) return;
    const __bf16 *__restrict__ A = G.A + g * G.a_g + row0 * G.sam;
    const __bf16 *__restrict__ B = G.B + g * G.b_g;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // the next slice is loaded into registers while the current one is
    // multiplied
    bf16x8 va, vb;
    stage_load<LA>(A, G.sam, G.sak, m0, M, 0, G.K, tid, va);
    stage_load<LB>(B, G.sbn, G.sbk, n0, G.N, 0, G.K, tid, vb);
    const int kq = (lane >> 4) * 8;
    for (int k0 = 0; k0 < G.K; k0 += 32) {
        stage_store<LA>(As, tid, va);
        stage_store<LB>(Bs, tid, vb);
        __syncthreads();
        if (k0 + 32 < G.K) {
            stage_load<LA>(A, G.sam, G.sak, m0, M, k0 + 32, G.K, tid, va);
            stage_load<LB>(B, G.sbn, G.sbk, n0, G.N, k0 + 32, G.K, tid, vb);
        }
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            a[i] = *(const bf16x8 *)&As[wm + 16 * i + (lane & 15)][kq];
            b[i] = *(const bf16x8 *)&Bs[wn + 16 * i + (lane & 15)][kq];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    if constexpr (VEC) {
        // the staging arrays are free after the loop's last barrier
        float(*Zs)[68] = reinterpret_cast<float(*)[68]>(&smem[0]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    Zs[wm + 16 * i + (lane >> 4) * 4 + e][wn + 16 * j + (lane & 15)] = acc[i][j][e];
        __syncthreads();
        const int rr = tid >> 2, c0 = (tid & 3) * 16;
        const int64_t gm = row0 + m0 + rr;
        float v[16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 t = *reinterpret_cast<const float4 *>(&Zs[rr][c0 + 4 * q]);
            v[4 * q] = t.x;
            v[4 * q + 1] = t.y;
            v[4 * q + 2] = t.z;
            v[4 * q + 3] = t.w;
        }
        if (G.epi == rti::EPI_DSILU) {
            const float *zp = G.Z + g * G.z_g + gm * G.ldz + n0 + c0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 z = *reinterpret_cast<const float4 *>(zp + 4 * q);
                v[4 * q] *= dsilu(z.x);
                v[4 * q + 1] *= dsilu(z.y);
                v[4 * q + 2] *= dsilu(z.z);
                v[4 * q + 3] *= dsilu(z.w);
            }
            __bf16 *cb = G.Cb + g * G.cb_g + gm * G.ldcb + n0 + c0;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                bf16x8 b;
#pragma unroll
                for (int e = 0; e < 8; ++e) b[e] = (__bf16)v[8 * q + e];
                *reinterpret_cast<bf16x8 *>(cb + 8 * q) = b;
            }
        }
        float *cf = G.Cf + g * G.cf_g + gm * G.ldcf + n0 + c0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            *reinterpret_cast<float4 *>(cf + 4 * q) = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
        return;
    }
    // epilogue
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm + 16 * i + (lane >> 4) * 4 + e;
                const int n = n0 + wn + 16 * j + (lane & 15);
                if (m >= M || n >= G.N) continue;
                const int64_t gm = row0 + m;
                float v = acc[i][j][e];
                switch (G.epi) {
                case rti::EPI_HIDDEN: {
                    const float z = v + G.bias[g * G.bias_g + n];
                    if (G.Cf) G.Cf[g * G.cf_g + gm * G.ldcf + n] = z;
                    G.Cb[g * G.cb_g + gm * G.ldcb + n] = (__bf16)silu(z);
                    break;
                }
                case rti::EPI_BIAS:
                    G.Cf[g * G.cf_g + gm * G.ldcf + n] = v + G.bias[g * G.bias_g + n];
                    break;
                case rti::EPI_DSILU: {
                    const float d = v * dsilu(G.Z[g * G.z_g + gm * G.ldz + n]);
                    G.Cf[g * G.cf_g + gm * G.ldcf + n] = d;
                    G.Cb[g * G.cb_g + gm * G.ldcb + n] = (__bf16)d;
                    break;
                }
                default:
                    G.Cf[g * G.cf_g + gm * G.ldcf + n] = v;
                    break;
                }
            }
}

// Weight-gradient product: both operands have unit stride along m (or n)
// and the long K (the batch) strided, C = sum_k A(m, k) B(k, n) with
// A(m, k) = A[k sak + m], B(k, n) = B[k sbk + n], EPI_NONE.  A 64x64 tile
// per block; the four waves split K in four contiguous quarters, each wave
// accumulating the whole tile for its quarter (4x4 16x16x32 MFMA tiles)
// with its own LDS staging, so the K loop has no block barrier.  A lane
// loads four k rows of eight consecutive m and writes each m's four k values
// as one 8-byte LDS store ([m][k] rows of 40).  The partial tiles are added
// in a fixed order, (w0 + w2) + (w1 + w3), through LDS.  Needs K % 128 == 0,
// M % 64 == 0, N % 64 == 0, 8 | the strides and 16-byte aligned bases.
__global__ __launch_bounds__(256) void k_gemm_wgrad(rti::GemmArgs G, int ntx, int nty, int ntz) {
    __shared__ __attribute__((aligned(16))) float smem[4 * 2 * 64 * 40 / 2];
    static_assert(sizeof(smem) >= 2 * 64 * 64 * sizeof(float), "reduction exceeds the LDS block");
    int tx, ty, g;
    if (!xcd_tile(ntx, nty, ntz, tx, ty, g)) return;
    const int m0 = ty * 64, n0 = tx * 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __bf16(*As)[40] = reinterpret_cast<__bf16(*)[40]>(&smem[0]) + wave * 128;  // this wave's [m][k]
    __bf16(*Bs)[40] = As + 64;                                                  // and [n][k]
    const __bf16 *__restrict__ A = G.A + g * G.a_g;
    const __bf16 *__restrict__ B = G.B + g * G.b_g;
    const int kq4 = G.K / 4;
    const int kb = wave * kq4;
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // lane: k rows kr .. kr + 3 of the 32-wide slice, m (or n) columns c0 .. c0 + 7
    const int kr = (lane >> 3) * 4, c0 = (lane & 7) * 8;
    const int kq = (lane >> 4) * 8;
    for (int k0 = kb; k0 < kb + kq4; k0 += 32) {
        bf16x8 va[4], vb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            va[t] = *(const bf16x8 *)(A + (int64_t)(k0 + kr + t) * G.sak + m0 + c0);
            vb[t] = *(const bf16x8 *)(B + (int64_t)(k0 + kr + t) * G.sbk + n0 + c0);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
            const bf16x4 a4 = {va[0][e], va[1][e], va[2][e], va[3][e]};
            const bf16x4 b4 = {vb[0][e], vb[1][e], vb[2][e], vb[3][e]};
            *(bf16x4 *)&As[c0 + e][kr] = a4;
            *(bf16x4 *)&Bs[c0 + e][kr] = b4;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        bf16x8 a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = *(const bf16x8 *)&As[16 * i + (lane & 15)][kq];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bf16x8 b = *(const bf16x8 *)&Bs[16 * j + (lane & 15)][kq];
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b, acc[i][j], 0, 0, 0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // fixed-order sum of the four partial tiles: (w0 + w2) + (w1 + w3)
    float(*R)[64][64] = reinterpret_cast<float(*)[64][64]>(&smem[0]);
    auto put = [&](int slot) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) R[slot][16 * i + (lane >> 4) * 4 + e][16 * j + (lane & 15)] = acc[i][j][e];
    };
    auto add = [&](int slot) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[i][j][e] += R[slot][16 * i + (lane >> 4) * 4 + e][16 * j + (lane & 15)];
    };
    __syncthreads();
    if (wave >= 2) put(wave - 2);
    __syncthreads();
    if (wave < 2) add(wave);
    __syncthreads();
    if (wave == 1) put(0);
    __syncthreads();
    if (wave != 0) return;
    add(0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + 16 * i + (lane >> 4) * 4 + e, n = n0 + 16 * j + (lane & 15);
                G.Cf[g * G.cf_g + (int64_t)m * G.ldcf + n] = acc[i][j][e];
            }
}

// First layer in FP32: thread o of a 256-thread block computes unit o of
// z1 = W1 x + b1 for up to 64 rows of network blockIdx.y; h1 = silu(z1) is
// stored split in two bf16 parts (hi, lo) for the next product, z1 (and x)
// for a backward pass.
__global__ __launch_bounds__(256) void k_l1_fwd(const float *__restrict__ params, const float *__restrict__ X, int B,
                                                float *__restrict__ Z, __bf16 *__restrict__ H, __bf16 *__restrict__ HL,
                                                float *__restrict__ Xkeep) {
    const int g = blockIdx.y, o = threadIdx.x;
    const int m0 = blockIdx.x * 64;
    if (m0 >= B) return;
    const float *__restrict__ W = params + g * rti::MLP_P + rti::OFF_W1 + o * 6;
    const float w0 = W[0], w1 = W[1], w2 = W[2], w3 = W[3], w4 = W[4], w5 = W[5];
    const float bias = params[g * rti::MLP_P + rti::OFF_B1 + o];
    const int m1 = min(B, m0 + 64);
    for (int m = m0; m < m1; ++m) {
        const int64_t r = (int64_t)g * B + m;
        const float *__restrict__ x = X + r * 6;
        float z = bias;
        z = fmaf(w0, x[0], z);
        z = fmaf(w1, x[1], z);
        z = fmaf(w2, x[2], z);
        z = fmaf(w3, x[3], z);
        z = fmaf(w4, x[4], z);
        z = fmaf(w5, x[5], z);
        if (Z) Z[r * rti::MLP_H + o] = z;
        const float h = silu(z);
        const __bf16 hh = (__bf16)h;
        H[r * rti::MLP_H + o] = hh;
        HL[r * rti::MLP_H + o] = (__bf16)(h - (float)hh);
        if (Xkeep && o < 6) Xkeep[r * 6 + o] = x[o];
    }
}

// Rows per partial of the FP32 layers' weight gradients: short serial
// chunks, many blocks.
constexpr int GRAD_ROWS = 32;

// First-layer gradients in FP32: dW1[o][i] = sum_m dz1[m][o] x[m][i] and
// db1[o] = sum_m dz1[m][o]; per block of GRAD_ROWS rows a sequential
// partial, then the partials summed in order.
__global__ __launch_bounds__(256) void k_l1_grad_part(const float *__restrict__ DZ, const float *__restrict__ X, int B,
                                                      float *__restrict__ part) {
    const int g = blockIdx.y, c = blockIdx.x, o = threadIdx.x;
    const int r0 = c * GRAD_ROWS, r1 = min(B, r0 + GRAD_ROWS);
    float a[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int m = r0; m < r1; ++m) {
        const int64_t r = (int64_t)g * B + m;
        const float d = DZ[r * rti::MLP_H + o];
        const float *__restrict__ x = X + r * 6;
#pragma unroll
        for (int i = 0; i < 6; ++i) a[i] = fmaf(d, x[i], a[i]);
        a[6] += d;
    }
    float *__restrict__ dst = part + (((int64_t)g * gridDim.x + c) * rti::MLP_H + o) * 7;
#pragma unroll
    for (int i = 0; i < 7; ++i) dst[i] = a[i];
}
__global__ __launch_bounds__(256) void k_l1_grad_final(const float *__restrict__ part, int nchunk,
                                                       float *__restrict__ grad) {
    const int g = blockIdx.x, o = threadIdx.x;
    float a[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < nchunk; ++c) {
        const float *__restrict__ src = part + (((int64_t)g * nchunk + c) * rti::MLP_H + o) * 7;
#pragma unroll
        for (int i = 0; i < 7; ++i) a[i] += src[i];
    }
    float *__restrict__ G = grad + (int64_t)g * rti::MLP_P;
#pragma unroll
    for (int i = 0; i < 6; ++i) G[rti::OFF_W1 + o * 6 + i] = a[i];
    G[rti::OFF_B1 + o] = a[6];
}

// Output layer in FP32: y[m][o] = b4[o] + sum_k W4[o][k] silu(z3[m][k]).
// One wave per row (the rows of a 64-row chunk of network blockIdx.y dealt
// to the block's four waves), lane l taking k = l + 64 q in order of q, then
// a butterfly sum over the lanes in a fixed pattern; W4 stays in registers.
__global__ __launch_bounds__(256) void k_l4_fwd(const float *__restrict__ params, const float *__restrict__ Z3, int B,
                                                float *__restrict__ Y) {
    const int g = blockIdx.y, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.x * 64;
    if (m0 >= B) return;
    const float *__restrict__ W = params + g * rti::MLP_P + rti::OFF_W4;
    float w[6][4];
#pragma unroll
    for (int o = 0; o < 6; ++o)
#pragma unroll
        for (int q = 0; q < 4; ++q) w[o][q] = W[o * rti::MLP_H + lane + 64 * q];
    const float *__restrict__ b4 = params + g * rti::MLP_P + rti::OFF_B4;
    const int m1 = min(B, m0 + 64);
    for (int m = m0 + wave; m < m1; m += 4) {
        const float *__restrict__ z = Z3 + ((int64_t)g * B + m) * rti::MLP_H;
        float h[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) h[q] = silu(z[lane + 64 * q]);
        float a[6];
#pragma unroll
        for (int o = 0; o < 6; ++o) {
            float t = w[o][0] * h[0];
#pragma unroll
            for (int q = 1; q < 4; ++q) t = fmaf(w[o][q], h[q], t);
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
            Y[((int64_t)g * B + m) * 6 + lane] = b4[lane] + v;
        }
    }
}

// Output-layer gradients in FP32: dW4[o][k] = sum_m dy[m][o] silu(z3[m][k]),
// db4[o] = sum_m dy[m][o]; per block of GRAD_ROWS rows a sequential partial
// (thread k: six dW4 partials, and db4[k] for k < 6), then the partials in
// order.
__global__ __launch_bounds__(256) void k_l4_grad_part(const float *__restrict__ DY, const float *__restrict__ Z3, int B,
                                                      float *__restrict__ part) {
    const int g = blockIdx.y, c = blockIdx.x, k = threadIdx.x;
    const int r0 = c * GRAD_ROWS, r1 = min(B, r0 + GRAD_ROWS);
    float a[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int m = r0; m < r1; ++m) {
        const int64_t r = (int64_t)g * B + m;
        const float h = silu(Z3[r * rti::MLP_H + k]);
        const float *__restrict__ d = DY + r * 6;
#pragma unroll
        for (int o = 0; o < 6; ++o) a[o] = fmaf(d[o], h, a[o]);
        if (k < 6) a[6] += d[k];
    }
    float *__restrict__ dst = part + (((int64_t)g * gridDim.x + c) * rti::MLP_H + k) * 7;
#pragma unroll
    for (int i = 0; i < 7; ++i) dst[i] = a[i];
}
__global__ __launch_bounds__(256) void k_l4_grad_final(const float *__restrict__ part, int nchunk,
                                                       float *__restrict__ grad) {
    const int g = blockIdx.x, k = threadIdx.x;
    float a[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < nchunk; ++c) {
        const float *__restrict__ src = part + (((int64_t)g * nchunk + c) * rti::MLP_H + k) * 7;
#pragma unroll
        for (int i = 0; i < 7; ++i) a[i] += src[i];
    }
    float *__restrict__ G = grad + (int64_t)g * rti::MLP_P;
#pragma unroll
    for (int o = 0; o < 6; ++o) G[rti::OFF_W4 + o * rti::MLP_H + k] = a[o];
    if (k < 6) G[rti::OFF_B4 + k] = a[6];
}

// Back-propagation through the output layer: dz3[m][k] =
// (sum_o dy[m][o] W4[o][k]) silu'(z3[m][k]), kept in FP32 and bf16.
__global__ __launch_bounds__(256) void k_l4_bwd(const float *__restrict__ params, const float *__restrict__ DY,
                                                const float *__restrict__ Z3, int B, float *__restrict__ DZ,
                                                __bf16 *__restrict__ DZB) {
    const int g = blockIdx.y, k = threadIdx.x;
    const int m0 = blockIdx.x * 64;
    if (m0 >= B) return;
    const float *__restrict__ W = params + g * rti::MLP_P + rti::OFF_W4;
    float w[6];
#pragma unroll
    for (int o = 0; o < 6; ++o) w[o] = W[o * rti::MLP_H + k];
    const int m1 = min(B, m0 + 64);
    for (int m = m0; m < m1; ++m) {
        const int64_t r = (int64_t)g * B + m;
        const float *__restrict__ d = DY + r * 6;
        float dh = 0.f;
#pragma unroll
        for (int o = 0; o < 6; ++o) dh = fmaf(d[o], w[o], dh);
        const float dz = dh * dsilu(Z3[r * rti::MLP_H + k]);
        DZ[r * rti::MLP_H + k] = dz;
        DZB[r * rti::MLP_H + k] = (__bf16)dz;
    }
}

// Forward product of a hidden layer in split bf16: for network blockIdx.z,
// z[m][n] = b[n] + sum_k h[m][k] W[n][k] over K = N = 256, with h given as
// its two bf16 parts (Hh, Hl, written by the previous layer) and W split
// from the FP32 master while staged; then Zout = z (FP32) and the parts of
// silu(z) for the next layer and the backward.  A 64x64 tile per block, 4
// waves of 2x2 16x16x32 tiles; LDS rows of 40 bf16 (80 bytes) so that every
// stage write and fragment read is one 16-byte access.
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(256) void k_gemm_x3(const __bf16 *__restrict__ Hh, const __bf16 *__restrict__ Hl,
                                                 const float *__restrict__ params, int64_t offW, int64_t offB, int B,
                                                 float *__restrict__ Zout, __bf16 *__restrict__ Oh,
                                                 __bf16 *__restrict__ Ol, int n_nets) {
    // one LDS block: the four staging arrays, reused for the output tile
    __shared__ __attribute__((aligned(16))) __bf16 stage[4][64][40];
    __bf16(&Ah)[64][40] = stage[0];
    __bf16(&Al)[64][40] = stage[1];
    __bf16(&Bh)[64][40] = stage[2];  // [n][k]
    __bf16(&Bl)[64][40] = stage[3];
    int tx, ty, g;
    if (!xcd_tile(rti::MLP_H / 64, (B + 63) / 64, n_nets, tx, ty, g)) return;
    const int m0 = ty * 64, n0 = tx * 64;
    if (m0 >= B) return;
    const int64_t K = rti::MLP_H;
    const __bf16 *__restrict__ Xh = Hh + (int64_t)g * B * K;
    const __bf16 *__restrict__ Xl = Hl + (int64_t)g * B * K;
    const float *__restrict__ W = params + (int64_t)g * rti::MLP_P + offW;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int r = tid >> 2, kc = (tid & 3) * 8;
    const int m = m0 + r, n = n0 + r;
    bf16x8v zero8;
#pragma unroll
    for (int e = 0; e < 8; ++e) zero8[e] = (__bf16)0.0f;
    for (int k0 = 0; k0 < K; k0 += 32) {
        // stage: thread t takes 8 consecutive k of row t/4 of each operand
        if (m < B) {
            *(bf16x8v *)&Ah[r][kc] = *(const bf16x8v *)(Xh + (int64_t)m * K + k0 + kc);
            *(bf16x8v *)&Al[r][kc] = *(const bf16x8v *)(Xl + (int64_t)m * K + k0 + kc);
        } else {
            *(bf16x8v *)&Ah[r][kc] = zero8;
            *(bf16x8v *)&Al[r][kc] = zero8;
        }
        {
            const float4 *src = reinterpret_cast<const float4 *>(W + (int64_t)n * K + k0 + kc);
            const float4 u0 = src[0], u1 = src[1];
            const float v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
            bf16x8v hi, lo;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const __bf16 t = (__bf16)v[e];
                hi[e] = t;
                lo[e] = (__bf16)(v[e] - (float)t);
            }
            *(bf16x8v *)&Bh[r][kc] = hi;
            *(bf16x8v *)&Bl[r][kc] = lo;
        }
        __syncthreads();
        const int kq = (lane >> 4) * 8;
        bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            ah[i] = *(const bf16x8 *)&Ah[wm + 16 * i + (lane & 15)][kq];
            al[i] = *(const bf16x8 *)&Al[wm + 16 * i + (lane & 15)][kq];
            bh[i] = *(const bf16x8 *)&Bh[wn + 16 * i + (lane & 15)][kq];
            bl[i] = *(const bf16x8 *)&Bl[wn + 16 * i + (lane & 15)][kq];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
        __syncthreads();
    }
    // epilogue through LDS (the staging buffers, free after the last
    // barrier): the tile of z = acc + bias, then every thread writes 16
    // consecutive values of one row as whole 16-byte stores of z and of the
    // two bf16 parts of silu(z)
    const float *__restrict__ bias = params + (int64_t)g * rti::MLP_P + offB;
    static_assert(sizeof(stage) >= 64 * 68 * sizeof(float), "output tile exceeds the staging block");
    float(*Zs)[68] = reinterpret_cast<float(*)[68]>(&stage[0][0][0]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int rr = wm + 16 * i + (lane >> 4) * 4 + e, cc = wn + 16 * j + (lane & 15);
                Zs[rr][cc] = acc[i][j][e] + bias[n0 + cc];
            }
    __syncthreads();
    {
        const int rr = tid >> 2, c0 = (tid & 3) * 16;
        const int mm = m0 + rr;
        if (mm < B) {
            const int64_t o = ((int64_t)g * B + mm) * K + n0 + c0;
            float v[16];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 t = *reinterpret_cast<const float4 *>(&Zs[rr][c0 + 4 * q]);
                v[4 * q] = t.x;
                v[4 * q + 1] = t.y;
                v[4 * q + 2] = t.z;
                v[4 * q + 3] = t.w;
                *reinterpret_cast<float4 *>(Zout + o + 4 * q) = t;
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                bf16x8v hi, lo;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float h = silu(v[8 * q + e]);
                    const __bf16 hh = (__bf16)h;
                    hi[e] = hh;
                    lo[e] = (__bf16)(h - (float)hh);
                }
                *reinterpret_cast<bf16x8v *>(Oh + o + 8 * q) = hi;
                *reinterpret_cast<bf16x8v *>(Ol + o + 8 * q) = lo;
            }
        }
    }
}

// out[g][n] = sum_m X[g][m][n], fixed order: per block of COLSUM_ROWS rows
// a sequential partial, then partials summed in order.
constexpr int COLSUM_ROWS = 64;
__global__ void k_colsum_part(const float *__restrict__ X, int64_t xg, int rows, int N, float *__restrict__ part) {
    const int g = blockIdx.z, n = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
    if (n >= N) return;
    const int r0 = c * COLSUM_ROWS, r1 = min(rows, r0 + COLSUM_ROWS);
    float s = 0.f;
    for (int r = r0; r < r1; ++r) s += X[g * xg + (int64_t)r * N + n];
    part[((int64_t)g * gridDim.y + c) * N + n] = s;
}
__global__ void k_colsum_final(const float *__restrict__ part, int nchunk, int N, float *__restrict__ out,
                               int64_t out_g) {
    const int g = blockIdx.y, n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int c = 0; c < nchunk; ++c) s += part[((int64_t)g * nchunk + c) * N + n];
    out[g * out_g + n] = s;
}

// AdamW with bias correction; refreshes the bf16 copy of the parameters.
__global__ void k_adamw(float *__restrict__ p, __bf16 *__restrict__ pb, float *__restrict__ m, float *__restrict__ v,
                        const float *__restrict__ gr, int64_t n, float lr, float b1, float b2, float eps, float wd,
                        float c1, float c2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float g = gr[i];
        float mi = b1 * m[i] + (1.f - b1) * g;
        float vi = b2 * v[i] + (1.f - b2) * g * g;
        m[i] = mi;
        v[i] = vi;
        float pi = p[i] - lr * ((mi * c1) / (sqrtf(vi * c2) + eps) + wd * p[i]);
        p[i] = pi;
        pb[i] = (__bf16)pi;
    }
}

// dy = 2 (y - t) / batch and per-block squared-error sums (fixed order).
__global__ __launch_bounds__(256) void k_mse_grad(const float *__restrict__ y, const float *__restrict__ t,
                                                  float *__restrict__ dy, int64_t n, float inv_batch,
                                                  float *__restrict__ part) {
    __shared__ float sh[256];
    float acc = 0.f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float d = y[i] - t[i];
        dy[i] = 2.f * d * inv_batch;
        acc += d * d;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_to_bf16(const float *__restrict__ x, __bf16 *__restrict__ y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (__bf16)x[i];
}

}  // namespace

namespace rti {

hipError_t launch_gemm(const GemmArgs &G, int groups, int max_rows, hipStream_t s) {
    const int ntx = (G.N + 63) / 64, nty = (max_rows + 63) / 64;
    dim3 grid(xcd_grid(ntx, nty, groups));
    // vector staging when every 8-element run it loads lies inside the
    // operand and starts on a 16-byte boundary
    auto al = [](const void *p, int64_t a, int64_t b) {
        return ((uintptr_t)p % 16 == 0) && a % 8 == 0 && b % 8 == 0;
    };
    const bool dims = !G.rows && G.M % 8 == 0 && G.N % 8 == 0 && G.K % 8 == 0;
    const bool a_mc = dims && G.sam == 1 && al(G.A, G.a_g, G.sak);
    const bool a_kc = dims && G.sak == 1 && al(G.A, G.a_g, G.sam);
    const bool b_nc = dims && G.sbn == 1 && al(G.B, G.b_g, G.sbk);
    const bool b_nc4 = dims && G.sbn == 1 && (uintptr_t)G.B % 4 == 0 && G.b_g % 2 == 0 && G.sbk % 8 == 0;
    // whole tiles and 16-byte aligned outputs: the LDS-staged epilogue
    auto al16 = [](const void *p, int64_t a, int64_t b) { return ((uintptr_t)p % 16 == 0) && a % 4 == 0 && b % 4 == 0; };
    const bool vec = dims && G.M % 64 == 0 && G.N % 64 == 0 &&
                     (G.epi == EPI_NONE || (G.epi == EPI_DSILU && al16(G.Z, G.z_g, G.ldz) &&
                                            (uintptr_t)G.Cb % 16 == 0 && G.cb_g % 8 == 0 && G.ldcb % 8 == 0)) &&
                     al16(G.Cf, G.cf_g, G.ldcf);
    if (a_mc && b_nc && G.epi == EPI_NONE && G.K % 128 == 0 && G.M % 64 == 0 && G.N % 64 == 0)
        hipLaunchKernelGGL(k_gemm_wgrad, grid, dim3(256), 0, s, G, ntx, nty, groups);
    else if (a_kc && b_nc4 && vec)
        hipLaunchKernelGGL((k_gemm<L_KC, L_MC4, true>), grid, dim3(256), 0, s, G, ntx, nty, groups);
    else if (a_kc && b_nc && vec)
        hipLaunchKernelGGL((k_gemm<L_KC, L_MC, true>), grid, dim3(256), 0, s, G, ntx, nty, groups);
    else if (a_mc && b_nc)
        hipLaunchKernelGGL((k_gemm<L_MC, L_MC>), grid, dim3(256), 0, s, G, ntx, nty, groups);
    else if (a_kc && b_nc)
        hipLaunchKernelGGL((k_gemm<L_KC, L_MC>), grid, dim3(256), 0, s, G, ntx, nty, groups);
    else if (a_kc && b_nc4)
        hipLaunchKernelGGL((k_gemm<L_KC, L_MC4>), grid, dim3(256), 0, s, G, ntx, nty, groups);
    else
        hipLaunchKernelGGL((k_gemm<L_GEN, L_GEN>), grid, dim3(256), 0, s, G, ntx, nty, groups);
    return hipGetLastError();
}

hipError_t launch_colsum(const float *X, int64_t xg, int rows, int N, int groups, float *part, float *out,
                         int64_t out_g, hipStream_t s) {
    // part holds groups x nchunk x N floats
    int nchunk = (rows + COLSUM_ROWS - 1) / COLSUM_ROWS;
    hipLaunchKernelGGL(k_colsum_part, dim3((N + 63) / 64, nchunk, groups), dim3(64), 0, s, X, xg, rows, N, part);
    hipLaunchKernelGGL(k_colsum_final, dim3((N + 63) / 64, groups), dim3(64), 0, s, (const float *)part, nchunk, N,
                       out, out_g);
    return hipGetLastError();
}

hipError_t launch_adamw(float *p, __bf16 *pb, float *m, float *v, const float *g, int64_t n, float lr, float b1,
                        float b2, float eps, float wd, int step, hipStream_t s) {
    float c1 = 1.0f / (1.0f - powf(b1, (float)step)), c2 = 1.0f / (1.0f - powf(b2, (float)step));
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_adamw, dim3(blocks), dim3(256), 0, s, p, pb, m, v, g, n, lr, b1, b2, eps, wd, c1, c2);
    return hipGetLastError();
}

hipError_t launch_mse_grad(const float *y, const float *t, float *dy, int64_t n, int batch, float *part, int nblk,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_mse_grad, dim3(nblk), dim3(256), 0, s, y, t, dy, n, 1.0f / (float)batch, part);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *x, __bf16 *y, int64_t n, hipStream_t s) {
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

}  // namespace rti

namespace rti {

size_t mlp_work_bytes(int n_nets, int batch) {
    size_t nb = (size_t)n_nets * batch;
    size_t nch = ((size_t)batch + GRAD_ROWS - 1) / GRAD_ROWS;
    return nb * MLP_IN * 4 + nb * MLP_OUT * 2 + nb * MLP_H * (3 * 4 + 6 * 2 + 2 * 4 + 2 * 2) +
           (size_t)n_nets * nch * MLP_H * 7 * 4 + 16 * 256;
}

void mlp_work_carve(void *base, int n_nets, int batch, MlpWork &w) {
    size_t nb = (size_t)n_nets * batch;
    size_t nch = ((size_t)batch + GRAD_ROWS - 1) / GRAD_ROWS;
    char *p = (char *)base;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += (bytes + 255) & ~(size_t)255;
        return (void *)r;
    };
    w.xf = (float *)take(nb * MLP_IN * 4);
    for (int i = 0; i < 3; ++i) w.z[i] = (float *)take(nb * MLP_H * 4);
    for (int i = 0; i < 3; ++i) w.h[i] = (__bf16 *)take(nb * MLP_H * 2);
    for (int i = 0; i < 3; ++i) w.hl[i] = (__bf16 *)take(nb * MLP_H * 2);
    w.dyb = (__bf16 *)take(nb * MLP_OUT * 2);
    for (int i = 0; i < 2; ++i) w.dzf[i] = (float *)take(nb * MLP_H * 4);
    for (int i = 0; i < 2; ++i) w.dzb[i] = (__bf16 *)take(nb * MLP_H * 2);
    // partials: nch x 7 x 256 per network for the FP32 layers, and
    // ceil(batch / COLSUM_ROWS) x 256 <= 7 nch x 256 for the column sums
    w.part = (float *)take((size_t)n_nets * nch * MLP_H * 7 * 4);
}

static GemmArgs gemm0() {
    GemmArgs G{};
    G.epi = EPI_NONE;
    return G;
}

// y = MLP(x) for n_nets networks of batch rows each.  keep: store the
// pre-activations for a backward pass.
hipError_t mlp_forward(int n, int B, const __bf16 *wb, const float *params, const float *x, float *y, const MlpWork &w,
                       bool keep, hipStream_t s) {
    // every layer's pre-activations go to z[l]: the next layer reads them
    (void)wb;
    (void)keep;
    hipLaunchKernelGGL(k_l1_fwd, dim3((B + 63) / 64, n), dim3(256), 0, s, params, x, B, w.z[0], w.h[0], w.hl[0],
                       w.xf);
    const dim3 grid(xcd_grid(MLP_H / 64, (B + 63) / 64, n));
    hipLaunchKernelGGL(k_gemm_x3, grid, dim3(256), 0, s, w.h[0], w.hl[0], params, OFF_W2, OFF_B2, B, w.z[1], w.h[1],
                       w.hl[1], n);
    hipLaunchKernelGGL(k_gemm_x3, grid, dim3(256), 0, s, w.h[1], w.hl[1], params, OFF_W3, OFF_B3, B, w.z[2], w.h[2],
                       w.hl[2], n);
    hipLaunchKernelGGL(k_l4_fwd, dim3((B + 63) / 64, n), dim3(256), 0, s, params, w.z[2], B, y);
    return hipGetLastError();
}

// grad = dL/dparams given dy = dL/dy, using the workspace of the last
// forward with keep = true.
hipError_t mlp_backward(int n, int B, const __bf16 *wb, const float *params, const float *dy, float *grad,
                        const MlpWork &w, hipStream_t s) {
    hipError_t e = hipSuccess;
    // weight gradient dW[o][i] = sum_b d[b][o] in[b][i]
    auto wgrad = [&](const __bf16 *d, int64_t dw, const __bf16 *in, int64_t iw, int64_t off) {
        GemmArgs G = gemm0();
        G.A = d;
        G.a_g = (int64_t)B * dw;
        G.sam = 1;
        G.sak = dw;
        G.B = in;
        G.b_g = (int64_t)B * iw;
        G.sbk = iw;
        G.sbn = 1;
        G.M = (int)dw;
        G.N = (int)iw;
        G.K = B;
        G.Cf = grad + off;
        G.cf_g = MLP_P;
        G.ldcf = iw;
        return launch_gemm(G, n, (int)dw, s);
    };
    // back-propagated signal dz = (d W) * silu'(z)
    auto bprop = [&](const __bf16 *d, int64_t dw, int64_t offW, const float *z, float *dzf, __bf16 *dzb) {
        GemmArgs G = gemm0();
        G.A = d;
        G.a_g = (int64_t)B * dw;
        G.sam = dw;
        G.sak = 1;
        G.B = wb + offW;
        G.b_g = MLP_P;
        G.sbk = MLP_H;
        G.sbn = 1;
        G.M = B;
        G.N = (int)MLP_H;
        G.K = (int)dw;
        G.epi = EPI_DSILU;
        G.Z = z;
        G.z_g = (int64_t)B * MLP_H;
        G.ldz = MLP_H;
        G.Cf = dzf;
        G.cf_g = (int64_t)B * MLP_H;
        G.ldcf = MLP_H;
        G.Cb = dzb;
        G.cb_g = (int64_t)B * MLP_H;
        G.ldcb = MLP_H;
        return launch_gemm(G, n, B, s);
    };
    // output layer (FP32): weight and bias gradients, then dz3 into buffer 0
    {
        const int nch4 = (B + GRAD_ROWS - 1) / GRAD_ROWS;
        hipLaunchKernelGGL(k_l4_grad_part, dim3(nch4, n), dim3(256), 0, s, dy, w.z[2], B, w.part);
        hipLaunchKernelGGL(k_l4_grad_final, dim3(n), dim3(256), 0, s, w.part, nch4, grad);
        hipLaunchKernelGGL(k_l4_bwd, dim3((B + 63) / 64, n), dim3(256), 0, s, params, dy, w.z[2], B, w.dzf[0],
                           w.dzb[0]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // layer 3: dz in buffer 0
    if ((e = wgrad(w.dzb[0], MLP_H, w.h[1], MLP_H, OFF_W3)) != hipSuccess) return e;
    if ((e = launch_colsum(w.dzf[0], (int64_t)B * MLP_H, B, (int)MLP_H, n, w.part, grad + OFF_B3, MLP_P, s)) !=
        hipSuccess)
        return e;
    if ((e = bprop(w.dzb[0], MLP_H, OFF_W3, w.z[1], w.dzf[1], w.dzb[1])) != hipSuccess) return e;
    // layer 2: dz in buffer 1
    if ((e = wgrad(w.dzb[1], MLP_H, w.h[0], MLP_H, OFF_W2)) != hipSuccess) return e;
    if ((e = launch_colsum(w.dzf[1], (int64_t)B * MLP_H, B, (int)MLP_H, n, w.part, grad + OFF_B2, MLP_P, s)) !=
        hipSuccess)
        return e;
    if ((e = bprop(w.dzb[1], MLP_H, OFF_W2, w.z[0], w.dzf[0], w.dzb[0])) != hipSuccess) return e;
    // layer 1 (FP32): dz in buffer 0, input x
    const int nch = (B + GRAD_ROWS - 1) / GRAD_ROWS;
    hipLaunchKernelGGL(k_l1_grad_part, dim3(nch, n), dim3(256), 0, s, w.dzf[0], w.xf, B, w.part);
    hipLaunchKernelGGL(k_l1_grad_final, dim3(n), dim3(256), 0, s, w.part, nch, grad);
    return hipGetLastError();
}

}  // namespace rti
