// Shared device-side definitions of the PRTGS HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <stddef.h>
#include <stdint.h>

#include "prtgs.h"

namespace prtgs {

constexpr int kWave = 64;                 // CDNA wavefront width
constexpr float kBoxSigma = 3.0f;         // BVH boxes enclose the 3-sigma ellipsoid
constexpr size_t kFlagBytes = 256;        // flag word + padding at the head of a workspace
constexpr int kHitList = PRTGS_BOUNCE_HIT_LIST;   // bounce: hits listed per ray and round
constexpr int kBounceWavesPerSimd = 4;    // bounce (blend, two walks): resident waves per SIMD
constexpr int kFusedWavesPerSimd = 7;     // bounce (blend, one walk): resident waves per SIMD
constexpr int kIndexWavesPerSimd = 5;     // bounce (index matrix): resident waves per SIMD
constexpr int kBlendPartsMax = PRTGS_BLEND_PARTS_MAX;   // bounce (blend): direction parts with sums of their own
constexpr int kMaxRounds = PRTGS_BOUNCE_MAX_ROUNDS;     // bounce: traversal rounds per ray

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// What the blended bounce gathers for each hit: the hit splat's direct
// transfer (K floats) and then its albedo (3 floats), in leaf order, each
// splat padded to a power of two so that a record's gather touches one cache
// line (K = 16: 32 floats, 128 bytes).
__host__ __device__ constexpr int hit_stride(int K)
{
    int s = 4;
    while (s < K + 3) s *= 2;
    return s;
}

// Internal BVH node: the boxes of both children and their references.  A
// reference r >= 0 is an internal node, r < 0 the leaf ~r (a leaf rank).
// a = (L.lo.x, L.lo.y, L.lo.z, L.hi.x)  b = (L.hi.y, L.hi.z, R.lo.x, R.lo.y)
// c = (R.lo.z, R.hi.x, R.hi.y, R.hi.z)  d = (left ref, right ref, -, -)
struct __align__(16) Node {
    float4 a, b, c;
    int4 d;
};

// Ray-test record of one Gaussian, in leaf order: centre and opacity, then
// the rows of the whitening matrix W = diag(1/s) R^T (so that W^T W is the
// inverse covariance of Eq. 2); w0.w holds 1 / min(s) (rounding bounds).
struct __align__(16) Prim {
    float4 mo;   // mu.x, mu.y, mu.z, opacity
    float4 w0;   // W row 0, 1 / s_min
    float4 w1;   // W row 1, 0
    float4 w2;   // W row 2, 0
};

struct BvhHeader {
    int32_t n;
    int32_t max_depth;
    int32_t pad0, pad1;
    float lo[4];
    float hi[4];
};

// BVH buffer: header | internal nodes | Gaussian records | normals (float4,
// leaf order) | leaf-to-Gaussian permutation.
struct BvhLayout {
    size_t nodes, prims, normals, order, total;
};

inline BvhLayout bvh_layout(int n)
{
    BvhLayout L;
    size_t off = align256(sizeof(BvhHeader));
    L.nodes = off;
    off += align256(sizeof(Node) * (size_t)(n > 1 ? n - 1 : 1));
    L.prims = off;
    off += align256(sizeof(Prim) * (size_t)n);
    L.normals = off;
    off += align256(sizeof(float4) * (size_t)n);
    L.order = off;
    off += align256(sizeof(int32_t) * (size_t)n);
    L.total = off;
    return L;
}

// Cutoffs of the hit test, as used on the device.
struct HitParams {
    float cut;        // sigma_cut
    float cut2;       // sigma_cut^2
    float t_min;
    float T_eps;
    float alpha_min;
    float alpha_max;
};

// Load at a wave-uniform address through the constant address space, so the
// compiler issues a scalar (s_load) instead of a per-lane vector load.  Only
// for memory that no kernel writes while the loading kernel runs.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <class T>
__device__ inline T uniform_load(const T* p, size_t idx)
{
    static_assert(sizeof(T) % 4 == 0, "whole dwords only");
    T out;
    if constexpr (sizeof(T) % 16 == 0) {
        typedef const u32x4 __attribute__((address_space(4)))* cptr;
        const cptr src = (cptr)(p + idx);
        u32x4* dst = reinterpret_cast<u32x4*>(&out);
#pragma unroll
        for (size_t i = 0; i < sizeof(T) / 16; ++i) dst[i] = src[i];
    } else {
        typedef const uint32_t __attribute__((address_space(4)))* cptr;
        const cptr src = (cptr)(p + idx);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
        for (size_t i = 0; i < sizeof(T) / 4; ++i) dst[i] = src[i];
    }
    return out;
}

__device__ inline void raise_flag(unsigned* flags, unsigned bit)
{
    if (flags) atomicOr(flags, bit);
}

__device__ inline bool finite3(float a, float b, float c)
{
    return isfinite(a) && isfinite(b) && isfinite(c);
}

// Fill kernel used instead of hipMemsetAsync, so that callers may capture
// the library's work in a graph.
__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, size_t count);
hipError_t fill_u32(uint32_t* p, uint32_t v, size_t count, hipStream_t stream);

// ------------------------------------------------------------------------
// host-side entry points of the individual translation units
// ------------------------------------------------------------------------
hipError_t launch_direction_table(int S, uint64_t seed, int bands, double* d64, double* y64, float* d32,
                                  float* y32, hipStream_t stream);
hipError_t launch_direction_order(int S, int32_t* order, hipStream_t stream);
hipError_t launch_build_bvh(const prtgs_gaussians& g, void* bvh, void* ws, unsigned* flags, hipStream_t stream);
size_t build_workspace_bytes(int n);
hipError_t launch_leaf_order(const void* bvh, int n, int32_t* order, hipStream_t stream);

struct TransferArgs {
    const Node* nodes;
    const Prim* prims;
    const float4* normals;  // leaf order
    const int32_t* order;
    const float* dirs;      // [S][3]
    const float* Y;         // [S][K]
    const int32_t* dir_order;  // [S] directions in coherent (tile) order
    int S, K, n, first, count, channels;
    HitParams hp;
    float* transfer;        // [n][C][K]
    float* vis;             // [n][S] or null
    float* hit_table;       // [n][hit_stride(K)] leaf order (bounce scratch), or null
    const float* albedo;    // [n][3] original order (bounce)
    uint64_t* hitkey;       // bounce: per-lane hit lists of the persistent waves,
    float* hitalpha;        // [wave][64][kHitList] keys (t bits, leaf rank) and alphas
    float* partial;         // blend: [Q][n][3][K] each direction part's bounce sums
                            // (Q = blend_parts), added into transfer in part order
    int2* hitrec;           // blend: [wave][64][kHitList] (leaf rank, weight) of the
                            // hits blended in the current round, in blend order
    unsigned* queue;        // bounce: work counter (zeroed before the launch)
    float* rayw;            // [S][count] direction-order position: T c of each
                            // ray of the direct pass (0 below the horizon),
                            // summed against Y by the projection
    float* tcut;            // [count][S] direction-order position: depth of the
                            // farthest hit the direct pass used before the ray
                            // turned opaque (+inf if it never did), or null
    int32_t* index;         // index mode: [n][S] argmax hit (original index), or null
    float t_same;           // index mode: same-surface filter threshold
    int G;                  // sources per wave (group split); 1 = fan kernel
    int Q;                  // group split: waves per source group, each taking a
                            // contiguous share of the direction batches (part-major)
    int Q_req;              // the caller's direction parts (0 = the default)
    unsigned* flags;
    // blend in one walk per ray (transfer.hip, fused walk): each work item's
    // records (leaf rank, weight) in a chain of blocks of the arena
    uint64_t* rec;                 // arena of rec_words 8-byte words
    uint64_t rec_words;
    unsigned long long* rec_top;   // words taken so far (may pass rec_words)
    int64_t* item_head;            // [items] first block of each item, -1: none
    int32_t* item_deferred;        // [items] 1: its records did not fit, the two-walk pass redoes it
};
// A record block: word 0 the next block of the item (~0: none), words 1-16
// the 64 lanes' record counts (16 bits each), then the records, lane by lane.
constexpr int kRecHeaderWords = 17;
hipError_t launch_transfer_direct(const TransferArgs& a, hipStream_t stream, unsigned long long* stats = nullptr);
hipError_t launch_transfer_bounce(const TransferArgs& a, hipStream_t stream);
// the blended bounce in one walk per ray: visibility, projection and bounce (needs the arena)
hipError_t launch_transfer_fused(const TransferArgs& a, hipStream_t stream);
// the index matrix in one walk per ray (its visibility with it), then, if project, the direct transfer
hipError_t launch_index_fused(const TransferArgs& a, hipStream_t stream, bool project);
// the one walk with its work tallied into stats[8] (visibility and records not kept)
hipError_t launch_fused_stats(const TransferArgs& a, hipStream_t stream, unsigned long long* stats);
hipError_t launch_transfer_index(const TransferArgs& a, hipStream_t stream);
// the blended bounce's walk with its work tallied into stats[8] (no transfer written)
hipError_t launch_bounce_stats(const TransferArgs& a, hipStream_t stream, unsigned long long* stats);
hipError_t launch_self_transfer(int n, int S, int K, const float* dirs, const float* normals, const float* albedo,
                                const int32_t* index, const float* t_prev, int c_prev, float* t_out, unsigned* flags,
                                hipStream_t stream);
hipError_t launch_add(float* acc, const float* x, size_t count, hipStream_t stream);
// Direction parts of the direct pass and its adjoint: the S directions of a source group are
// split into Q contiguous runs of batches, one wave each, and the waves take
// them part-major (every group's first part, then every group's second ...).
// The thousands of waves resident together then trace nearly the same
// directions from different sources: they walk the tree in the same order,
// so its hot nodes stay in L2, and every XCD (blocks go to the 8 XCDs in
// turn) gets every part, also where many directions fall below the surfaces'
// horizon.  Measured at 100k x 256 (8 sources per wave): Q = 1, 4, 8, 32
// give 31.8, 23.4, 21.1, 19.4 ms; with 16 sources per wave Q = 16, 32, 64
// give 18.1, 16.9, 16.3 ms; at 1M x 512 Q = 1, 8, 32, 128: 1021, 935, 934,
// 938 ms.  One batch per wave, at most 64 parts.  `requested` (1 .. 64, 0 =
// this default) is the caller's choice, capped at the number of batches.
inline int direction_parts(int G, int S, int requested)
{
    const int batches = (S + kWave / G - 1) / (kWave / G);
    int Q = requested > 0 ? requested : 64;
    return std::max(std::min(Q, batches), 1);
}

// Direction parts of the blended bounce: each keeps sums of its own (a
// [Q][n][3][K] buffer added in part order at the end), so the count is capped
// by kBlendPartsMax.
inline int blend_parts(int G, int S, int requested)
{
    return std::min(direction_parts(G, S, requested), kBlendPartsMax);
}

// Persistent waves of the bounce launches for n sources (any group size): as
// many as the 1024 SIMDs hold at the kernel's occupancy; the hit-list scratch
// holds this many waves.
enum WalkKind { kWalkBlend, kWalkFused, kWalkIndex };
__host__ __device__ inline int bounce_waves(int n, int kind)
{
    const int per = kind == kWalkIndex ? kIndexWavesPerSimd : kind == kWalkFused ? kFusedWavesPerSimd
                                                                                   : kBounceWavesPerSimd;
    const int cap = 1024 * per;
    return n < cap ? n : cap;
}

struct BackwardArgs {
    TransferArgs fwd;
    const float* d_transfer;  // [n][1][K]
    const float* vis_in;      // [n][S] forward visibilities (original order), or null
    float* g_W;               // [n][9] scratch: dLoss/dW, leaf order
    float* g_mu;              // [n][3] scratch, leaf order
    float* g_o;               // [n]    scratch, leaf order
    float* g_n;               // [n][3] scratch, leaf order
    const float* quats;       // original order inputs
    const float* log_scales;
    prtgs_grads out;
};
hipError_t launch_transfer_backward(const BackwardArgs& a, hipStream_t stream);

// Gaussian splatting (splat.hip).
struct SplatCamera {
    float view[12];        // world to camera, rows of [R | t]
    float fx, fy, cx, cy;
    int width, height;
    float near_z;
    float background[3];
    float lim[4];          // x/z and y/z bounds (1.3 x the frustum) for the projection Jacobian
};
struct SplatBuffers {
    float4* uv;                // screen centre, cut on q, unused
    float4* conic_o;
    float* depth;
    int4* rect;
    uint32_t* count;
    uint64_t* offset;
    unsigned long long* total;
    uint2* ranges;
    uint64_t *keys, *keys_alt;
    uint32_t *vals, *vals_alt;
    void* scan_temp;
    size_t scan_temp_bytes;
    void* sort_temp;
    size_t sort_temp_bytes;
    int64_t max_instances;
    unsigned* flags;
};
size_t splat_sort_temp_bytes(int64_t max_instances);
size_t splat_scan_temp_bytes(int n);
hipError_t launch_splat_front(int n, const SplatCamera& cam, const float* means, const float* quats,
                              const float* log_scales, const float* opacity, const SplatBuffers& b, hipStream_t stream);
hipError_t launch_splat_back(int n, const SplatCamera& cam, int64_t instances, const float* colours, int64_t stride,
                             const SplatBuffers& b, float* image, float* final_T, hipStream_t stream);

hipError_t launch_glossy(int n, int S, int K, const float* dirs, const float* Y, const float* normals,
                         const float* albedo, const float* roughness, const float* metallic, const float* vis,
                         float* out, unsigned* flags, hipStream_t stream);
hipError_t launch_glossy_view(int n, int K, const float* M, const float* means, const float eye[3], float* z,
                              hipStream_t stream);

hipError_t launch_pack(int64_t count, const float* src, void* dst, prtgs_dtype dtype, hipStream_t stream);
hipError_t launch_relight(int n, int K, int C, const void* T, prtgs_dtype tdt, int B, const float* L,
                          void* out, prtgs_dtype odt, hipStream_t stream);
hipError_t launch_relight_backward(int n, int K, int C, const float* T, int B, const float* L,
                                   const float* dC, float* dT, float* dL, void* ws, hipStream_t stream);
size_t relight_backward_ws(int n, int K, int C, int B);

}  // namespace prtgs
