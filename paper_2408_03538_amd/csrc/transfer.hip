// Transfer precompute: visibility along S directions from every splat centre
// through the other Gaussians (Sec. 4.4), projected with max(0, n.w) onto
// real SH (Eq. 7, 9, 29), and the one-bounce self-transfer (Eq. 20-22,
// 30-33) with the hits of each ray blended front to back.
//
// Work split ("group"): a wave takes G Morton-adjacent sources and D = 64/G
// directions at a time, consecutive in the coherent direction order (8 x 8
// stratum tiles, Morton order inside, so aligned runs stay in one octant and
// a compact patch of the sphere); lane l traces source l / D along direction
// l % D.  Neighbouring origins share the Gaussians around them, nearby
// directions share the far field.  Each lane accumulates the SH projection
// of its own rays (compensated sums); the D lanes of a source are added at
// the end.  Small scenes use the "fan" split instead (one source per wave,
// its hemisphere directions compacted over the lanes) to fill the GPU.
#include "trace.hpp"

namespace prtgs {

namespace {

constexpr int kBlock = 256;
constexpr float kFourPi = 12.566370614359172f;
constexpr float kInvPi = 0.31830988618379067f;
constexpr int kBounceBuffer = 16;   // nearest hits kept per ray and round

__device__ inline void kahan_add(float& sum, float& comp, float x)
{
    float y = x - comp;
    float t = sum + y;
    comp = (t - sum) - y;
    sum = t;
}

// Sum of v over each aligned run of D lanes (D a power of two).
__device__ inline float segment_sum(float v, int D)
{
    for (int off = D / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Mean direction of the traced lanes (uniform after the reduction) and
// whether they all lie in one octant.
struct BatchDir {
    float mean[3];
    int oct;
    bool uniform_oct;
};

__device__ inline BatchDir batch_dir(const RayDir& d, bool traced)
{
    BatchDir b;
    b.mean[0] = traced ? d.wx : 0.0f;
    b.mean[1] = traced ? d.wy : 0.0f;
    b.mean[2] = traced ? d.wz : 0.0f;
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) b.mean[q] += __shfl_xor(b.mean[q], off, kWave);
    const uint64_t m = __ballot(traced);
    const int first = __builtin_ctzll(m);
    const int oct = octant(d);
    b.oct = __builtin_amdgcn_readlane(oct, first);
    b.uniform_oct = __ballot(traced && oct != b.oct) == 0ull;
    return b;
}

// Traversal with the octant fast path when the batch allows it.
template <bool kCount, class LeafFn>
__device__ inline void traverse_batch(const TransferArgs& a, const RayDir& d, const BatchDir& bd, float ox, float oy,
                                      float oz, bool& live, float& tlo, float& thi, LeafFn& leaf, RayCounts* cnt)
{
    if (bd.uniform_oct)
        packet_traverse<kCount, true>(a.nodes, a.n, d, ox, oy, oz, live, tlo, thi, a.flags, leaf, cnt, bd.mean, bd.oct);
    else
        packet_traverse<kCount, false>(a.nodes, a.n, d, ox, oy, oz, live, tlo, thi, a.flags, leaf, cnt, bd.mean, 0);
}

// ---------------------------------------------------------------------------
// direct transfer, group split
// stats (kCount): [0] traced rays, [1] child-box tests, [2] Gaussian tests
// (single-ray work, summed over rays), [3] wave node visits, [4] wave
// Gaussian-record visits (summed over waves and batches).
// ---------------------------------------------------------------------------
template <int K, bool kCount>
__global__ __launch_bounds__(kBlock) void direct_kernel(TransferArgs a, unsigned long long* stats)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int G = a.G;
    const int D = kWave / G;
    const int gwave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int local = gwave * G + lane / D;
    const bool valid = local < a.count;
    const int rank = a.first + (valid ? local : 0);
    const float4 mo = a.prims[rank].mo;
    const float ox = mo.x, oy = mo.y, oz = mo.z;
    const float4 nrm = a.normals[rank];
    const int orig = valid ? a.order[rank] : 0;
    const HitParams hp = a.hp;
    float acc[K], cmp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        acc[k] = 0.0f;
        cmp[k] = 0.0f;
    }
    RayCounts cnt;
    uint32_t traced_rays = 0;
    for (int b0 = 0; b0 < a.S; b0 += D) {
        const int pos = b0 + (lane % D);
        const bool inrange = pos < a.S;
        const int s = inrange ? a.dir_order[pos] : 0;
        const RayDir d = make_dir(a.dirs[3 * s], a.dirs[3 * s + 1], a.dirs[3 * s + 2]);
        const float c = nrm.x * d.wx + nrm.y * d.wy + nrm.z * d.wz;
        const bool traced = valid && inrange && c > 0.0f;
        if (!kCount && valid && inrange && !traced && a.vis) a.vis[(size_t)orig * a.S + s] = -1.0f;
        if (__ballot(traced) == 0ull) continue;
        if (kCount && traced) ++traced_rays;
        const BatchDir bd = batch_dir(d, traced);
        bool live = traced;
        float T = 1.0f;
        float tlo = hp.t_min, thi = INFINITY;
        auto leaf = [&](int r, bool box_hit) {
            const Prim p = uniform_load(a.prims, r);
            const PreHit q = gaussian_pre(p, ox, oy, oz, d, hp);
            const bool cand = q.maybe & box_hit & live & (r != rank);
            if (__ballot(cand) == 0ull) return;
            HitResult h;
            const bool hit = gaussian_exact(p, q, ox, oy, oz, d, hp, h) & cand;
            T = hit ? T * (1.0f - h.alpha) : T;
            const bool opaque = T < hp.T_eps;
            live = live & !opaque;
            T = opaque ? 0.0f : T;
        };
        traverse_batch<kCount>(a, d, bd, ox, oy, oz, live, tlo, thi, leaf, &cnt);
        if (!kCount && traced) {
            const float f = T * c;
#pragma unroll
            for (int k = 0; k < K; ++k) kahan_add(acc[k], cmp[k], f * a.Y[(size_t)s * K + k]);
            if (a.vis) a.vis[(size_t)orig * a.S + s] = T;
        }
    }
    if (kCount) {
        atomicAdd(&stats[0], (unsigned long long)traced_rays);
        atomicAdd(&stats[1], (unsigned long long)cnt.box_tests);
        atomicAdd(&stats[2], (unsigned long long)cnt.prim_tests);
        if (lane == 0) {
            atomicAdd(&stats[3], (unsigned long long)cnt.wave_nodes);
            atomicAdd(&stats[4], (unsigned long long)cnt.wave_leaves);
        }
        return;
    }
    const float scale = kFourPi / (float)a.S;
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = segment_sum(acc[k] - cmp[k], D) * scale;
    if (valid && (lane % D) == 0) {
        for (int ch = 0; ch < a.channels; ++ch) {
            float* out = a.transfer + ((size_t)orig * a.channels + ch) * K;
#pragma unroll
            for (int k = 0; k < K; ++k) out[k] = acc[k];
        }
        if (a.tdir_sorted) {
#pragma unroll
            for (int k = 0; k < K; ++k) a.tdir_sorted[(size_t)rank * K + k] = acc[k];
            const int j = orig;
            a.albedo_sorted[rank] = make_float4(a.albedo[3 * (size_t)j], a.albedo[3 * (size_t)j + 1],
                                                a.albedo[3 * (size_t)j + 2], 0.0f);
        }
    }
}

// ---------------------------------------------------------------------------
// direct transfer, fan split (small scenes): one wave per source; the
// directions above its horizon are compacted (coherent order) into a
// per-wave list in LDS and traced 64 at a time.
// ---------------------------------------------------------------------------
constexpr int kFanMaxDirs = 1024;   // per-wave direction list capacity (LDS)

template <int K>
__global__ __launch_bounds__(kBlock) void direct_fan_kernel(TransferArgs a)
{
    __shared__ int16_t list[kBlock / kWave][kFanMaxDirs];
    const int lane = threadIdx.x & (kWave - 1);
    const int wslot = threadIdx.x / kWave;
    const int local = (blockIdx.x * kBlock + threadIdx.x) / kWave;   // source of this wave
    if (local >= a.count) return;                                     // whole wave leaves together
    const int rank = a.first + local;
    const float4 mo = uniform_load(a.prims, rank).mo;
    const float ox = mo.x, oy = mo.y, oz = mo.z;
    const float4 nrm = uniform_load(a.normals, rank);
    const int orig = uniform_load(a.order, rank);
    const HitParams hp = a.hp;
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    float acc[K], cmp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        acc[k] = 0.0f;
        cmp[k] = 0.0f;
    }
    for (int seg = 0; seg < a.S; seg += kFanMaxDirs) {
        const int seg_n = min(kFanMaxDirs, a.S - seg);
        int count = 0;
        for (int c0 = 0; c0 < seg_n; c0 += kWave) {
            const int pos = c0 + lane;
            const int s = pos < seg_n ? a.dir_order[seg + pos] : 0;
            const float c =
                pos < seg_n ? nrm.x * a.dirs[3 * s] + nrm.y * a.dirs[3 * s + 1] + nrm.z * a.dirs[3 * s + 2] : 0.0f;
            const uint64_t m = __ballot(c > 0.0f);
            if (c > 0.0f) list[wslot][count + __popcll(m & lt_mask)] = (int16_t)pos;
            else if (pos < seg_n && a.vis) a.vis[(size_t)orig * a.S + s] = -1.0f;
            count += __popcll(m);
        }
        __builtin_amdgcn_wave_barrier();
        for (int b0 = 0; b0 < count; b0 += kWave) {
            const int idx = b0 + lane;
            const bool traced = idx < count;
            const int s = a.dir_order[seg + list[wslot][traced ? idx : 0]];
            const RayDir d = make_dir(a.dirs[3 * s], a.dirs[3 * s + 1], a.dirs[3 * s + 2]);
            const float c = nrm.x * d.wx + nrm.y * d.wy + nrm.z * d.wz;
            const BatchDir bd = batch_dir(d, traced);
            bool live = traced;
            float T = 1.0f;
            float tlo = hp.t_min, thi = INFINITY;
            auto leaf = [&](int r, bool box_hit) {
                const Prim p = uniform_load(a.prims, r);
                const PreHit q = gaussian_pre(p, ox, oy, oz, d, hp);
                const bool cand = q.maybe & box_hit & live & (r != rank);
                if (__ballot(cand) == 0ull) return;
                HitResult h;
                const bool hit = gaussian_exact(p, q, ox, oy, oz, d, hp, h) & cand;
                T = hit ? T * (1.0f - h.alpha) : T;
                const bool opaque = T < hp.T_eps;
                live = live & !opaque;
                T = opaque ? 0.0f : T;
            };
            traverse_batch<false>(a, d, bd, ox, oy, oz, live, tlo, thi, leaf, (RayCounts*)nullptr);
            if (traced) {
                const float f = T * c;
#pragma unroll
                for (int k = 0; k < K; ++k) kahan_add(acc[k], cmp[k], f * a.Y[(size_t)s * K + k]);
                if (a.vis) a.vis[(size_t)orig * a.S + s] = T;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    const float scale = kFourPi / (float)a.S;
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = segment_sum(acc[k] - cmp[k], kWave) * scale;
    if (lane == 0) {
        for (int ch = 0; ch < a.channels; ++ch) {
            float* out = a.transfer + ((size_t)orig * a.channels + ch) * K;
#pragma unroll
            for (int k = 0; k < K; ++k) out[k] = acc[k];
        }
        if (a.tdir_sorted) {
#pragma unroll
            for (int k = 0; k < K; ++k) a.tdir_sorted[(size_t)rank * K + k] = acc[k];
            a.albedo_sorted[rank] = make_float4(a.albedo[3 * (size_t)orig], a.albedo[3 * (size_t)orig + 1],
                                                a.albedo[3 * (size_t)orig + 2], 0.0f);
        }
    }
}

// ---------------------------------------------------------------------------
// one bounce, group split
// ---------------------------------------------------------------------------

// Strict order of hits along a ray: by t*, then by leaf rank.
__device__ inline bool key_less(float ta, int ja, float tb, int jb) { return ta < tb || (ta == tb && ja < jb); }

// The hits of each ray are needed front to back (weight alpha_j T_j, T_j the
// transmittance in front of hit j), up to the one that takes the
// transmittance below T_eps.  A ray keeps the KB nearest hits beyond the
// last processed one, sorted in registers (boxes beyond the KB-th nearest so
// far are culled), blends them in order after the traversal, and repeats
// from its last hit while the buffer came back full and transparent.
template <int K, int KB>
__global__ __launch_bounds__(kBlock) void bounce_kernel(TransferArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int G = a.G;
    const int D = kWave / G;
    const int gwave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int local = gwave * G + lane / D;
    const bool valid = local < a.count;
    const int rank = a.first + (valid ? local : 0);
    const float4 mo = a.prims[rank].mo;
    const float ox = mo.x, oy = mo.y, oz = mo.z;
    const float4 nrm = a.normals[rank];
    const int orig = valid ? a.order[rank] : 0;
    const HitParams hp = a.hp;

    float acc[3][K];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[ch][k] = 0.0f;

    for (int b0 = 0; b0 < a.S; b0 += D) {
        const int pos = b0 + (lane % D);
        const bool inrange = pos < a.S;
        const int s = inrange ? a.dir_order[pos] : 0;
        const RayDir d = make_dir(a.dirs[3 * s], a.dirs[3 * s + 1], a.dirs[3 * s + 2]);
        const float c = nrm.x * d.wx + nrm.y * d.wy + nrm.z * d.wz;
        bool pending = valid && inrange && c > 0.0f;
        if (__ballot(pending) == 0ull) continue;
        const BatchDir bd = batch_dir(d, pending);
        const float wc = c * kInvPi;
        float T = 1.0f;
        float t_last = -INFINITY;
        int j_last = -1;
        // Each full round consumes KB hits of at most n - 1, hence the cap.
        int rounds = a.n / KB + 2;
        while (__ballot(pending) != 0ull) {
            if (--rounds < 0) {
                raise_flag(a.flags, PRTGS_FLAG_BAD_TREE);
                break;
            }
            float bt[KB], ba[KB];
            int bj[KB];
#pragma unroll
            for (int q = 0; q < KB; ++q) {
                bt[q] = INFINITY;
                bj[q] = 0x7fffffff;
                ba[q] = 0.0f;
            }
            bool live = pending;
            float tlo = fmaxf(hp.t_min, t_last), thi = INFINITY;
            auto leaf = [&](int r, bool box_hit) {
                const Prim p = uniform_load(a.prims, r);
                const PreHit q = gaussian_pre(p, ox, oy, oz, d, hp);
                const bool cand = q.maybe & box_hit & live & (r != rank);
                if (__ballot(cand) == 0ull) return;
                HitResult h;
                const bool hit = gaussian_exact(p, q, ox, oy, oz, d, hp, h) & cand;
                if (hit && key_less(t_last, j_last, h.t, r) && key_less(h.t, r, bt[KB - 1], bj[KB - 1])) {
                    float ct = h.t, ca = h.alpha;
                    int cj = r;
#pragma unroll
                    for (int q2 = 0; q2 < KB; ++q2) {
                        const bool lt = key_less(ct, cj, bt[q2], bj[q2]);
                        const float tt = bt[q2], ta = ba[q2];
                        const int tj = bj[q2];
                        bt[q2] = lt ? ct : tt;
                        bj[q2] = lt ? cj : tj;
                        ba[q2] = lt ? ca : ta;
                        ct = lt ? tt : ct;
                        cj = lt ? tj : cj;
                        ca = lt ? ta : ca;
                    }
                    thi = bt[KB - 1];   // beyond the KB-th nearest nothing is needed this round
                }
            };
            traverse_batch<false>(a, d, bd, ox, oy, oz, live, tlo, thi, leaf, (RayCounts*)nullptr);
            if (pending) {
                int used = 0;
#pragma unroll
                for (int q = 0; q < KB; ++q) {
                    if (bt[q] < INFINITY && pending) {
                        const int r = bj[q];
                        const float w = ba[q] * T * wc;
                        const float4 rho = a.albedo_sorted[r];
                        float tv[K];
                        if constexpr (K % 4 == 0) {
                            const float4* td = reinterpret_cast<const float4*>(a.tdir_sorted + (size_t)r * K);
#pragma unroll
                            for (int k4 = 0; k4 < K / 4; ++k4) {
                                const float4 v = td[k4];
                                tv[4 * k4] = v.x;
                                tv[4 * k4 + 1] = v.y;
                                tv[4 * k4 + 2] = v.z;
                                tv[4 * k4 + 3] = v.w;
                            }
                        } else {
#pragma unroll
                            for (int k = 0; k < K; ++k) tv[k] = a.tdir_sorted[(size_t)r * K + k];
                        }
                        const float r0 = rho.x * w, r1 = rho.y * w, r2 = rho.z * w;
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            acc[0][k] = fmaf(r0, tv[k], acc[0][k]);
                            acc[1][k] = fmaf(r1, tv[k], acc[1][k]);
                            acc[2][k] = fmaf(r2, tv[k], acc[2][k]);
                        }
                        T *= 1.0f - ba[q];
                        t_last = bt[q];
                        j_last = r;
                        ++used;
                        if (T < hp.T_eps) pending = false;
                    }
                }
                // more hits may lie beyond a full, still transparent buffer
                if (used < KB) pending = false;
            }
        }
    }
    const float scale = kFourPi / (float)a.S;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[ch][k] = segment_sum(acc[ch][k], D) * scale;
    if (valid && (lane % D) == 0) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float* out = a.transfer + ((size_t)orig * 3 + ch) * K;
#pragma unroll
            for (int k = 0; k < K; ++k) out[k] += acc[ch][k];
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int group_blocks(int count, int G)
{
    int waves = (count + G - 1) / G;
    return (waves + kBlock / kWave - 1) / (kBlock / kWave);
}

template <int K>
hipError_t launch_direct_k(const TransferArgs& a, unsigned long long* stats, hipStream_t stream)
{
    if (stats) {
        hipLaunchKernelGGL((direct_kernel<K, true>), dim3(group_blocks(a.count, a.G)), dim3(kBlock), 0, stream, a,
                           stats);
    } else if (a.G == 1) {
        hipLaunchKernelGGL(direct_fan_kernel<K>, dim3(group_blocks(a.count, 1)), dim3(kBlock), 0, stream, a);
    } else {
        hipLaunchKernelGGL((direct_kernel<K, false>), dim3(group_blocks(a.count, a.G)), dim3(kBlock), 0, stream, a,
                           stats);
    }
    return hipGetLastError();
}

template <int K>
hipError_t launch_bounce_k(const TransferArgs& a, hipStream_t stream)
{
    hipLaunchKernelGGL((bounce_kernel<K, kBounceBuffer>), dim3(group_blocks(a.count, a.G)), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_transfer_direct(const TransferArgs& a, hipStream_t stream, unsigned long long* stats)
{
    if (a.count <= 0) return hipSuccess;
    switch (a.K) {
        case 1: return launch_direct_k<1>(a, stats, stream);
        case 4: return launch_direct_k<4>(a, stats, stream);
        case 9: return launch_direct_k<9>(a, stats, stream);
        case 16: return launch_direct_k<16>(a, stats, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_transfer_bounce(const TransferArgs& a, hipStream_t stream)
{
    if (a.count <= 0) return hipSuccess;
    switch (a.K) {
        case 1: return launch_bounce_k<1>(a, stream);
        case 4: return launch_bounce_k<4>(a, stream);
        case 9: return launch_bounce_k<9>(a, stream);
        case 16: return launch_bounce_k<16>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace prtgs
