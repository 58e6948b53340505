// Relighting (Eq. 14 and, for an RGB transfer, Eq. 41 per channel): per
// splat and light environment the colour is the dot product of the splat's
// transfer vector with the light's SH coefficients,
//   colour[i][b][c] = sum_k T[i][c'][k] L[b][c][k],  c' = (C == 3 ? c : 0).
// With 16-bit transfers this is a batched GEMM on MFMA; the FP32 path uses
// VALU FMAs.  Both are bound by HBM bandwidth (colour writes dominate).
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "common.hpp"

namespace prtgs {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ pack

__global__ void pack_kernel(int64_t count, const float* __restrict__ src, void* __restrict__ dst, int dtype)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (dtype == PRTGS_BF16) {
        __hip_bfloat16* d = static_cast<__hip_bfloat16*>(dst);
        for (; i < count; i += stride) d[i] = __float2bfloat16(src[i]);
    } else {
        __half* d = static_cast<__half*>(dst);
        for (; i < count; i += stride) d[i] = __float2half(src[i]);
    }
}

// ------------------------------------------------------------------ FP32 path
// A block takes 64 splats: their transfer rows are staged in LDS and every
// thread owns up to MC output columns (b, c), keeping L[b][c][:] in registers.

constexpr int kRowsF32 = 64;
constexpr int kThreadsF32 = 256;

template <int K, int C, int MC, bool OUT16>
__global__ __launch_bounds__(kThreadsF32) void relight_f32_kernel(int n, const float* __restrict__ T, int B,
                                                                  const float* __restrict__ L, void* __restrict__ out)
{
    __shared__ float rows[kRowsF32 * C * K];
    const int cols = 3 * B;
    float lreg[MC][K];
    int chan[MC];
#pragma unroll
    for (int m = 0; m < MC; ++m) {
        int col = threadIdx.x + m * kThreadsF32;
        int cc = col < cols ? col : 0;
        chan[m] = (C == 3) ? (cc % 3) : 0;
#pragma unroll
        for (int k = 0; k < K; ++k) lreg[m][k] = col < cols ? L[(size_t)cc * K + k] : 0.0f;
    }
    for (int64_t base = (int64_t)blockIdx.x * kRowsF32; base < n; base += (int64_t)gridDim.x * kRowsF32) {
        const int nrows = (int)((n - base) < kRowsF32 ? (n - base) : kRowsF32);
        __syncthreads();
        for (int e = threadIdx.x; e < nrows * C * K; e += kThreadsF32) rows[e] = T[base * C * K + e];
        __syncthreads();
        for (int r = 0; r < nrows; ++r) {
#pragma unroll
            for (int m = 0; m < MC; ++m) {
                int col = threadIdx.x + m * kThreadsF32;
                if (col < cols) {
                    const float* tr = rows + (r * C + chan[m]) * K;
                    float acc = 0.0f;
#pragma unroll
                    for (int k = 0; k < K; ++k) acc = fmaf(tr[k], lreg[m][k], acc);
                    size_t o = (size_t)(base + r) * cols + col;
                    if (OUT16) static_cast<__half*>(out)[o] = __float2half(acc);
                    else static_cast<float*>(out)[o] = acc;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ MFMA path
// GEMM of 16-column tiles of outputs (b, c) against 16-splat row tiles with
// v_mfma_f32_16x16x32_{bf16,f16}, computed transposed: D = L' T'^T, so that
// lane l ends with D[4 (l / 16) + 0..3][l % 16] = colour[row l % 16][four
// consecutive columns] and writes them at once (8 bytes as 16-bit colours,
// 16 as FP32) into a wave-private LDS patch, from which each chunk of CT
// column tiles leaves in 16-byte stores of whole row pieces (each row of a
// chunk is contiguous in memory).  The 32-deep contraction of one MFMA is
// [L_hi ; L_lo] against [T_c' | T_c'] for channel c', where L_hi is the light
// rounded to 16 bits and L_lo the rounded remainder, so the light enters at
// ~FP32 precision; columns of other channels get zeros (C == 3 needs C such
// steps).  Lane l holds A[l % 16][8 (l / 16) + 0..7] (light, column l % 16)
// and B[8 (l / 16) + 0..7][l % 16] (transfer, row l % 16).
// Work item = one 16-row tile against a group of up to kGroupTiles column
// tiles (192 output columns: every light of a 64-light batch), so each
// transfer row is read once per group.  The block builds the light
// fragments of its group once, in LDS; each wave then walks row tiles on its
// own (no block barrier after the set-up), loading its transfer fragments
// once per tile and producing the group's columns in chunks.

// waves per block: 8 (the 3M x 64-light relight with 16-bit colours at 4
// waves took 0.32 ms, at 8 waves 0.29 ms)
template <bool OUT16>
constexpr int waves_mfma() { return 8; }
constexpr int kChunkTiles = 4;   // column tiles per chunk (64 output columns)
constexpr int kGroupTiles = 12;  // column tiles per group (3 chunks)

template <bool BF>
struct Frag;
template <>
struct Frag<true> {
    using vec = bf16x8;
    using elem = __bf16;
    static __device__ inline f32x4 mma(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
    static __device__ inline elem from_float(float x) { return (elem)x; }
};
template <>
struct Frag<false> {
    using vec = f16x8;
    using elem = _Float16;
    static __device__ inline f32x4 mma(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
    static __device__ inline elem from_float(float x) { return (elem)x; }
};

// IEEE binary16 bits of x, rounded to nearest even.
__device__ inline uint32_t half_bits(float x)
{
    const _Float16 h = (_Float16)x;
    return (uint32_t)__builtin_bit_cast(uint16_t, h);
}

template <int K, int C, bool BF, bool OUT16>
__global__ __launch_bounds__(waves_mfma<OUT16>() * kWave) void relight_mfma_kernel(int n, const void* __restrict__ Tv, int B,
                                                                          const float* __restrict__ L,
                                                                          void* __restrict__ out)
{
    using F = Frag<BF>;
    using vec = typename F::vec;
    using elem = typename F::elem;
    constexpr int kWavesMfma = waves_mfma<OUT16>();
    constexpr int kOutBytes = OUT16 ? 2 : 4;
    constexpr int CT = kChunkTiles;
    constexpr int kRowBytes = CT * 16 * kOutBytes;   // one row of a chunk: 128 or 256 B
    constexpr int kPatchStride = kRowBytes + 16;     // padded: the 16 rows fall in different banks
    __shared__ vec lsh[kGroupTiles][C][kWave];
    __shared__ __align__(16) unsigned char stage[kWavesMfma][16 * kPatchStride];
    const elem* T = static_cast<const elem*>(Tv);
    const int lane = threadIdx.x & (kWave - 1);
    const int wslot = threadIdx.x / kWave;
    const int g = lane / 16;   // k group of the lane's fragments; its 4 output columns 4g..4g+3
    const int li = lane % 16;  // column (light fragment) / row (transfer fragment, output) of the lane
    const int cols = 3 * B;
    const int group_col0 = blockIdx.y * kGroupTiles * 16;
    const int group_tiles = min(kGroupTiles, (cols - group_col0 + 15) / 16);

    // light fragments of the group's column tiles (wave w builds tiles w, w + waves, ...)
    for (int m = wslot; m < group_tiles; m += kWavesMfma) {
        const int col = group_col0 + m * 16 + li;
        const bool cvalid = col < cols;
        const int ch = cvalid ? col % 3 : 0;
#pragma unroll
        for (int st = 0; st < C; ++st) {
            vec v;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 8 * g + e;   // 0..31
                const int kk = k & 15;
                float x = 0.0f;
                if (cvalid && kk < K && (C == 1 || ch == st)) {
                    const float full = L[(size_t)col * K + kk];
                    const elem hi = F::from_float(full);
                    x = (k >= 16) ? (full - (float)hi) : full;
                }
                v[e] = F::from_float(x);
            }
            lsh[m][st][lane] = v;
        }
    }
    __syncthreads();

    unsigned char* my_stage = stage[wslot];
    const int ntiles_rows = (n + 15) / 16;
    const size_t row_stride = (size_t)cols * kOutBytes;
    for (int rt = blockIdx.x * kWavesMfma + wslot; rt < ntiles_rows; rt += gridDim.x * kWavesMfma) {
        const int64_t row = (int64_t)rt * 16 + li;
        const bool rvalid = row < n;
        vec tfrag[C];
#pragma unroll
        for (int st = 0; st < C; ++st) {
            if (K == 16 && rvalid) {
                tfrag[st] = *reinterpret_cast<const vec*>(T + ((size_t)row * C + st) * 16 + 8 * (g & 1));
            } else {
                vec v;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int kk = (8 * g + e) & 15;
                    v[e] = (rvalid && kk < K) ? T[((size_t)row * C + st) * K + kk] : F::from_float(0.0f);
                }
                tfrag[st] = v;
            }
        }
        const int nrows = (int)min((int64_t)16, (int64_t)n - (int64_t)rt * 16);
        for (int m0 = 0; m0 < group_tiles; m0 += CT) {
            const int chunk_col0 = group_col0 + m0 * 16;
            const int chunk_cols = min(CT * 16, cols - chunk_col0);
#pragma unroll
            for (int m = 0; m < CT; ++m) {
                if (m0 + m < group_tiles) {
                    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int st = 0; st < C; ++st) acc = F::mma(lsh[m0 + m][st][lane], tfrag[st], acc);
                    unsigned char* at = my_stage + li * kPatchStride + (m * 16 + 4 * g) * kOutBytes;
                    if (OUT16)
                        *reinterpret_cast<uint2*>(at) = make_uint2(half_bits(acc[0]) | (half_bits(acc[1]) << 16),
                                                                   half_bits(acc[2]) | (half_bits(acc[3]) << 16));
                    else
                        *reinterpret_cast<float4*>(at) = make_float4(acc[0], acc[1], acc[2], acc[3]);
                }
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            // 16 rows x kRowBytes, in 16-byte pieces; every row of the chunk is contiguous
            constexpr int kPiecesPerRow = kRowBytes / 16;
            unsigned char* obase = static_cast<unsigned char*>(out) + (size_t)rt * 16 * row_stride +
                                   (size_t)chunk_col0 * kOutBytes;
            const bool full_chunk = chunk_cols == CT * 16 && (row_stride % 16) == 0 &&
                                    (reinterpret_cast<uintptr_t>(out) % 16) == 0;
            if (full_chunk) {
#pragma unroll
                for (int pc = lane; pc < 16 * kPiecesPerRow; pc += kWave) {
                    const int r = pc / kPiecesPerRow, piece = pc % kPiecesPerRow;
                    if (r < nrows)
                        *reinterpret_cast<uint4*>(obase + r * row_stride + piece * 16) =
                            *reinterpret_cast<const uint4*>(my_stage + r * kPatchStride + piece * 16);
                }
            } else {
                for (int e = lane; e < 16 * chunk_cols; e += kWave) {
                    const int r = e / chunk_cols, c = e % chunk_cols;
                    if (r < nrows) {
                        if (OUT16)
                            reinterpret_cast<uint16_t*>(obase + r * row_stride)[c] =
                                reinterpret_cast<const uint16_t*>(my_stage + r * kPatchStride)[c];
                        else
                            reinterpret_cast<float*>(obase + r * row_stride)[c] =
                                reinterpret_cast<const float*>(my_stage + r * kPatchStride)[c];
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
    }
}

// ------------------------------------------------------------------ FP32 MFMA path
// FP32 transfers and colours on v_mfma_f32_16x16x4_f32, the 16-bit path's
// output scheme: D = L' T'^T per 16-row tile, lane l ending with
// D[4 (l / 16) + 0..3][l % 16], written to a wave-private LDS patch and
// stored as 16-byte pieces of whole rows.  Column tiles are per channel (16
// lights of one channel), so no MFMA multiplies zeros; a chunk is the three
// channels' tiles of kChunkLights32 lights, whose row piece (384 bytes) is
// three whole 128-byte lines.  Contraction: at step s (of K / 4) lane group g
// takes coefficient (K / 4) g + s, so a lane's transfer and light values for
// one channel are consecutive floats (one float4 at K = 16).  A block holds
// the light fragments of a group of 64 lights in LDS; its waves walk row
// tiles on their own.
constexpr int kLightsPerGroup32 = 64;
constexpr int kChunkLights32 = 32;

template <int K, int C>
__global__ __launch_bounds__(8 * kWave) void relight_mfma32_kernel(int n, const float* __restrict__ T, int B,
                                                                   const float* __restrict__ L,
                                                                   float* __restrict__ out)
{
    static_assert(K % 4 == 0, "K = 4 or 16");
    constexpr int kSteps = K / 4;
    constexpr int kWaves = 8;
    constexpr int kTiles = 3 * kLightsPerGroup32 / 16;   // 12 per-channel column tiles
    constexpr int kChunkCols = 3 * kChunkLights32;       // 96
    constexpr int kPatchStride = kChunkCols + 4;         // floats; padded rows
    typedef float fsteps __attribute__((ext_vector_type(kSteps)));
    __shared__ fsteps lf[kTiles][kWave];
    __shared__ __align__(16) float stage[kWaves][16 * kPatchStride];
    const int lane = threadIdx.x & (kWave - 1);
    const int wslot = threadIdx.x / kWave;
    const int g = lane / 16, li = lane % 16;
    const int cols = 3 * B;
    const int light0 = blockIdx.y * kLightsPerGroup32;
    const int group_lights = min(kLightsPerGroup32, B - light0);
    const int group_blocks = (group_lights + 15) / 16;   // 16-light blocks in the group

    // light fragments: tile m = 3 lb + c holds lights light0 + 16 lb + 0..15 of channel c
    for (int m = wslot; m < 3 * group_blocks; m += kWaves) {
        const int lb = m / 3, c = m % 3;
        const int b = light0 + 16 * lb + li;
        fsteps v;
#pragma unroll
        for (int st = 0; st < kSteps; ++st) v[st] = b < B ? L[((size_t)b * 3 + c) * K + kSteps * g + st] : 0.0f;
        lf[m][lane] = v;
    }
    __syncthreads();

    float* my_stage = stage[wslot];
    const int ntiles_rows = (n + 15) / 16;
    const bool vec_ok = (cols % 4) == 0 && (reinterpret_cast<uintptr_t>(out) % 16) == 0;
    for (int rt = blockIdx.x * kWaves + wslot; rt < ntiles_rows; rt += gridDim.x * kWaves) {
        const int64_t row = (int64_t)rt * 16 + li;
        const bool rvalid = row < n;
        fsteps tf[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (rvalid) {
                tf[c] = *reinterpret_cast<const fsteps*>(T + ((size_t)row * C + c) * K + kSteps * g);
            } else {
#pragma unroll
                for (int st = 0; st < kSteps; ++st) tf[c][st] = 0.0f;
            }
        }
        const int nrows = (int)min((int64_t)16, (int64_t)n - (int64_t)rt * 16);
        for (int lb0 = 0; lb0 < group_blocks; lb0 += kChunkLights32 / 16) {
#pragma unroll
            for (int j = 0; j < kChunkLights32 / 16; ++j) {
                if (lb0 + j < group_blocks) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
                        const fsteps a = lf[3 * (lb0 + j) + c][lane];
                        const fsteps bt = tf[C == 3 ? c : 0];
#pragma unroll
                        for (int st = 0; st < kSteps; ++st)
                            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[st], bt[st], acc, 0, 0, 0);
#pragma unroll
                        for (int i = 0; i < 4; ++i) my_stage[li * kPatchStride + 3 * (16 * j + 4 * g + i) + c] = acc[i];
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            const int first_light = light0 + 16 * lb0;
            const int chunk_cols = 3 * min(kChunkLights32, B - first_light);
            float* obase = out + (size_t)rt * 16 * cols + (size_t)3 * first_light;
            if (vec_ok && chunk_cols == kChunkCols) {
                // 16 rows x 24 pieces of 16 bytes
                for (int pc = lane; pc < 16 * (kChunkCols / 4); pc += kWave) {
                    const int r = pc / (kChunkCols / 4), piece = pc % (kChunkCols / 4);
                    if (r < nrows)
                        *reinterpret_cast<float4*>(obase + (size_t)r * cols + 4 * piece) =
                            *reinterpret_cast<const float4*>(my_stage + r * kPatchStride + 4 * piece);
                }
            } else {
                for (int e = lane; e < 16 * chunk_cols; e += kWave) {
                    const int r = e / chunk_cols, cc = e % chunk_cols;
                    if (r < nrows) obase[(size_t)r * cols + cc] = my_stage[r * kPatchStride + cc];
                }
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
    }
}

template <int K, int C>
hipError_t mfma32_launch(int n, const float* T, int B, const float* L, float* out, hipStream_t stream)
{
    const int groups = (B + kLightsPerGroup32 - 1) / kLightsPerGroup32;
    const int row_tiles = (n + 15) / 16;
    // about 8 waves per SIMD over 256 CUs in all, walking the row tiles
    int blocks = (256 * 4 * 8 / 8 + groups - 1) / groups;
    const int need = (row_tiles + 7) / 8;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((relight_mfma32_kernel<K, C>), dim3(blocks, groups), dim3(8 * kWave), 0, stream, n, T, B, L,
                       out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ backward

constexpr int kBwdRows = 1024;

// d_transfer[i][c'][k] = sum over (b, c -> c') of d_colour[i][b][c] L[b][c][k]
template <int K, int C>
__global__ void relight_dT_kernel(int n, int B, const float* __restrict__ L, const float* __restrict__ dC,
                                  float* __restrict__ dT)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * C * K) return;
    int k = (int)(idx % K);
    int cp = (int)((idx / K) % C);
    int64_t i = idx / ((int64_t)C * K);
    float acc = 0.0f;
    for (int b = 0; b < B; ++b) {
        if (C == 3) {
            acc = fmaf(dC[((size_t)i * B + b) * 3 + cp], L[((size_t)b * 3 + cp) * K + k], acc);
        } else {
            for (int c = 0; c < 3; ++c) acc = fmaf(dC[((size_t)i * B + b) * 3 + c], L[((size_t)b * 3 + c) * K + k], acc);
        }
    }
    dT[idx] = acc;
}

// partial[blk][b][c][k] = sum over the block's rows of d_colour[i][b][c] T[i][c'][k]
template <int K, int C>
__global__ void relight_dL_partial_kernel(int n, int B, const float* __restrict__ T, const float* __restrict__ dC,
                                          float* __restrict__ partial)
{
    const int outs = B * 3 * K;
    const int64_t r0 = (int64_t)blockIdx.x * kBwdRows;
    const int64_t r1 = r0 + kBwdRows < n ? r0 + kBwdRows : n;
    for (int o = threadIdx.x; o < outs; o += blockDim.x) {
        int k = o % K;
        int c = (o / K) % 3;
        int b = o / (3 * K);
        int cp = C == 3 ? c : 0;
        float sum = 0.0f, comp = 0.0f;
        for (int64_t i = r0; i < r1; ++i) {
            float x = dC[((size_t)i * B + b) * 3 + c] * T[((size_t)i * C + cp) * K + k];
            float y = x - comp;
            float t = sum + y;
            comp = (t - sum) - y;
            sum = t;
        }
        partial[(size_t)blockIdx.x * outs + o] = sum;
    }
}

__global__ void relight_dL_final_kernel(int nparts, int outs, const float* __restrict__ partial, float* __restrict__ dL)
{
    int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= outs) return;
    float sum = 0.0f, comp = 0.0f;
    for (int p = 0; p < nparts; ++p) {
        float y = partial[(size_t)p * outs + o] - comp;
        float t = sum + y;
        comp = (t - sum) - y;
        sum = t;
    }
    dL[o] = sum;
}

// ------------------------------------------------------------------ dispatch

template <int K, int C, int MC>
hipError_t f32_dispatch_out(int n, const float* T, int B, const float* L, void* out, bool out16, hipStream_t stream)
{
    int blocks = (int)((n + kRowsF32 - 1) / kRowsF32);
    if (blocks > 65536) blocks = 65536;
    if (out16)
        hipLaunchKernelGGL((relight_f32_kernel<K, C, MC, true>), dim3(blocks), dim3(kThreadsF32), 0, stream, n, T, B, L, out);
    else
        hipLaunchKernelGGL((relight_f32_kernel<K, C, MC, false>), dim3(blocks), dim3(kThreadsF32), 0, stream, n, T, B, L, out);
    return hipGetLastError();
}

template <int K, int C>
hipError_t f32_dispatch(int n, const float* T, int B, const float* L, void* out, bool out16, hipStream_t stream)
{
    int mc = (3 * B + kThreadsF32 - 1) / kThreadsF32;
    if (mc <= 1) return f32_dispatch_out<K, C, 1>(n, T, B, L, out, out16, stream);
    if (mc <= 2) return f32_dispatch_out<K, C, 2>(n, T, B, L, out, out16, stream);
    return f32_dispatch_out<K, C, 3>(n, T, B, L, out, out16, stream);
}

template <int K, int C, bool BF, bool OUT16>
hipError_t mfma_launch(int n, const void* T, int B, const float* L, void* out, hipStream_t stream)
{
    constexpr int kWavesMfma = waves_mfma<OUT16>();
    const int cols = 3 * B;
    const int groups = (cols + 16 * kGroupTiles - 1) / (16 * kGroupTiles);
    const int row_tiles = (n + 15) / 16;
    // about 8 waves per SIMD over 256 CUs in all, walking the row tiles
    int blocks = (256 * 4 * 8 / kWavesMfma + groups - 1) / groups;
    const int need = (row_tiles + kWavesMfma - 1) / kWavesMfma;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((relight_mfma_kernel<K, C, BF, OUT16>), dim3(blocks, groups), dim3(kWavesMfma * kWave), 0,
                       stream, n, T, B, L, out);
    return hipGetLastError();
}

template <int K, int C, bool BF>
hipError_t mfma_dispatch(int n, const void* T, int B, const float* L, void* out, bool out16, hipStream_t stream)
{
    if (out16) return mfma_launch<K, C, BF, true>(n, T, B, L, out, stream);
    return mfma_launch<K, C, BF, false>(n, T, B, L, out, stream);
}

template <int K, int C>
hipError_t relight_kc(int n, const void* T, prtgs_dtype tdt, int B, const float* L, void* out, prtgs_dtype odt,
                      hipStream_t stream)
{
    bool out16 = odt == PRTGS_F16;
    // FP32 on MFMA from one whole 16-light tile up (fewer lights would leave
    // most of each tile's products zero: the one-column kernel is better there)
    if constexpr (K % 4 == 0) {
        if (tdt == PRTGS_F32 && !out16 && B >= 16 && (reinterpret_cast<uintptr_t>(T) % 16) == 0)
            return mfma32_launch<K, C>(n, static_cast<const float*>(T), B, L, static_cast<float*>(out), stream);
    }
    if (tdt == PRTGS_F32) return f32_dispatch<K, C>(n, static_cast<const float*>(T), B, L, out, out16, stream);
    if (tdt == PRTGS_BF16) return mfma_dispatch<K, C, true>(n, T, B, L, out, out16, stream);
    return mfma_dispatch<K, C, false>(n, T, B, L, out, out16, stream);
}

template <int K>
hipError_t relight_k(int n, int C, const void* T, prtgs_dtype tdt, int B, const float* L, void* out, prtgs_dtype odt,
                     hipStream_t stream)
{
    if (C == 3) return relight_kc<K, 3>(n, T, tdt, B, L, out, odt, stream);
    return relight_kc<K, 1>(n, T, tdt, B, L, out, odt, stream);
}

template <int K, int C>
hipError_t relight_bwd_kc(int n, const float* T, int B, const float* L, const float* dC, float* dT, float* dL,
                          void* ws, hipStream_t stream)
{
    if (dT && n > 0) {
        int64_t total = (int64_t)n * C * K;
        int blocks = (int)((total + 255) / 256);
        hipLaunchKernelGGL((relight_dT_kernel<K, C>), dim3(blocks), dim3(256), 0, stream, n, B, L, dC, dT);
    }
    if (dL) {
        int outs = B * 3 * K;
        int nparts = (n + kBwdRows - 1) / kBwdRows;
        float* partial = reinterpret_cast<float*>(static_cast<char*>(ws) + kFlagBytes);
        if (nparts > 0)
            hipLaunchKernelGGL((relight_dL_partial_kernel<K, C>), dim3(nparts), dim3(256), 0, stream, n, B, T, dC, partial);
        hipLaunchKernelGGL(relight_dL_final_kernel, dim3((outs + 255) / 256), dim3(256), 0, stream, nparts, outs, partial, dL);
    }
    return hipGetLastError();
}

template <int K>
hipError_t relight_bwd_k(int n, int C, const float* T, int B, const float* L, const float* dC, float* dT, float* dL,
                         void* ws, hipStream_t stream)
{
    if (C == 3) return relight_bwd_kc<K, 3>(n, T, B, L, dC, dT, dL, ws, stream);
    return relight_bwd_kc<K, 1>(n, T, B, L, dC, dT, dL, ws, stream);
}

}  // namespace

hipError_t launch_pack(int64_t count, const float* src, void* dst, prtgs_dtype dtype, hipStream_t stream)
{
    int64_t blocks = (count + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, count, src, dst, (int)dtype);
    return hipGetLastError();
}

hipError_t launch_relight(int n, int K, int C, const void* T, prtgs_dtype tdt, int B, const float* L, void* out,
                          prtgs_dtype odt, hipStream_t stream)
{
    switch (K) {
        case 1: return relight_k<1>(n, C, T, tdt, B, L, out, odt, stream);
        case 4: return relight_k<4>(n, C, T, tdt, B, L, out, odt, stream);
        case 9: return relight_k<9>(n, C, T, tdt, B, L, out, odt, stream);
        case 16: return relight_k<16>(n, C, T, tdt, B, L, out, odt, stream);
        default: return hipErrorInvalidValue;
    }
}

size_t relight_backward_ws(int n, int K, int C, int B)
{
    (void)C;
    size_t nparts = (size_t)((n + kBwdRows - 1) / kBwdRows);
    return kFlagBytes + align256(sizeof(float) * nparts * (size_t)B * 3 * (size_t)K);
}

hipError_t launch_relight_backward(int n, int K, int C, const float* T, int B, const float* L, const float* dC,
                                   float* dT, float* dL, void* ws, hipStream_t stream)
{
    switch (K) {
        case 1: return relight_bwd_k<1>(n, C, T, B, L, dC, dT, dL, ws, stream);
        case 4: return relight_bwd_k<4>(n, C, T, B, L, dC, dT, dL, ws, stream);
        case 9: return relight_bwd_k<9>(n, C, T, B, L, dC, dT, dL, ws, stream);
        case 16: return relight_bwd_k<16>(n, C, T, B, L, dC, dT, dL, ws, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace prtgs
