// Transfer precompute: visibility along S directions from every splat centre
// through the other Gaussians (Sec. 4.4), projected with max(0, n.w) onto
// real SH (Eq. 7, 9, 29), and the one-bounce self-transfer (Eq. 20-22,
// 30-33) with the hits of each ray blended front to back.
//
// Work split ("group"): a wave takes G Morton-adjacent sources and D = 64/G
// directions at a time, consecutive in the coherent direction order (8 x 8
// stratum tiles, Morton order inside, so aligned runs stay in one octant and
// a compact patch of the sphere); lane l traces source l / D along direction
// l % D.  The direction batches of a group are shared among Q waves, issued
// part-major, so that the waves in flight trace the same directions.
// Neighbouring origins share the Gaussians around them, nearby directions
// share the far field.  Each ray's weight T max(n . w, 0) is
// stored, and a second kernel projects every source's S weights onto SH
// with compensated FP32 sums, in direction order, so the transfer does not
// depend on the split.
// Small scenes use the "fan" split instead (one source per wave, its
// hemisphere directions compacted over the lanes) to fill the GPU.
#include "trace.hpp"

namespace prtgs {

namespace {

constexpr int kBlock = 256;
constexpr float kFourPi = 12.566370614359172f;
constexpr float kInvPi = 0.31830988618379067f;

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

// Traversal with the octant fast path when the batch allows it; kStep as in
// packet_traverse (kChooseFirst: the direct pass, kLoadFirst: the bounce walks).
template <bool kCount, int kStep = kChooseFirst, class LeafFn>
__device__ inline void traverse_batch(const TransferArgs& a, const RayDir& d, const BatchDir& bd, float ox, float oy,
                                      float oz, bool& live, float& tlo, float& thi, LeafFn& leaf, RayCounts* cnt)
{
    if (bd.uniform_oct)
        packet_traverse<kCount, true, kStep>(a.nodes, a.n, d, ox, oy, oz, live, tlo, thi, a.flags, leaf, cnt, bd.mean,
                                             bd.oct);
    else
        packet_traverse<kCount, false, kStep>(a.nodes, a.n, d, ox, oy, oz, live, tlo, thi, a.flags, leaf, cnt,
                                              bd.mean, 0);
}

// ---------------------------------------------------------------------------
// direct transfer, group split
// Each ray's T max(n . w, 0) goes to rayw and project_kernel forms the SH
// sums: with no sums held across the traversal the kernel fits 64 VGPRs, 8
// waves per SIMD, which hides more of the latency of its dependent record
// loads than the 5 waves that the register-held sums allowed.
// stats (kCount): [0] traced rays, [1] child-box tests, [2] Gaussian tests
// (single-ray work, summed over rays), [3] wave node visits, [4] wave
// Gaussian-record visits (summed over waves and batches).
// ---------------------------------------------------------------------------
template <bool kCount>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void direct_kernel(TransferArgs a,
                                                                                                unsigned long long* stats)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int G = a.G;
    const int D = kWave / G;
    const int gwave = (int)(((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave);
    // part-major: wave w takes direction part w / groups of source group
    // w % groups (spare waves of the last block get part >= Q: no work)
    const int groups = (a.count + G - 1) / G;
    const int part = gwave / groups;
    const int local = (gwave % groups) * G + lane / D;
    const bool valid = local < a.count && part < a.Q;
    const int rank = a.first + (valid ? local : 0);
    const float4 mo = a.prims[rank].mo;
    const float ox = mo.x, oy = mo.y, oz = mo.z;
    const float4 nrm = a.normals[rank];
    const int orig = valid ? a.order[rank] : 0;
    const HitParams hp = a.hp;
    RayCounts cnt;
    uint32_t traced_rays = 0;
    const int nb = (a.S + D - 1) / D;
    for (int bi = part * nb / a.Q; bi < (part + 1) * nb / a.Q; ++bi) {
        const int b0 = bi * D;
        const int pos = b0 + (lane % D);
        const bool inrange = pos < a.S;
        const int s = inrange ? a.dir_order[pos] : 0;
        const RayDir d = make_dir(a.dirs[3 * s], a.dirs[3 * s + 1], a.dirs[3 * s + 2]);
        const float c = nrm.x * d.wx + nrm.y * d.wy + nrm.z * d.wz;
        const bool traced = valid && inrange && c > 0.0f;
        if (!kCount && valid && inrange && !traced) {
            a.rayw[(size_t)pos * a.count + local] = 0.0f;
            if (a.vis) a.vis[(size_t)orig * a.S + s] = -1.0f;
            if (a.tcut) a.tcut[(size_t)local * a.S + pos] = 0.0f;
        }
        if (__ballot(traced) == 0ull) continue;
        if (kCount && traced) ++traced_rays;
        const BatchDir bd = batch_dir(d, traced);
        bool live = traced;
        float T = 1.0f, tfar = 0.0f;
        float tlo = hp.t_min, thi = INFINITY;
        auto leaf = [&](int r, bool box_hit) {
            const Prim p = uniform_load(a.prims, r);
            const PreHit q = gaussian_pre(p, ox, oy, oz, d, hp);
            const bool cand = q.maybe & box_hit & live & (r != rank);
            if (__ballot(cand) == 0ull) return;
            HitResult h;
            const bool hit = gaussian_exact(p, q, ox, oy, oz, d, hp, h) & cand;
            T = hit ? T * (1.0f - h.alpha) : T;
            tfar = hit ? fmaxf(tfar, h.t) : tfar;
            const bool opaque = T < hp.T_eps;
            live = live & !opaque;
            T = opaque ? 0.0f : T;
        };
        traverse_batch<kCount>(a, d, bd, ox, oy, oz, live, tlo, thi, leaf, &cnt);
        if (!kCount && traced) {
            a.rayw[(size_t)pos * a.count + local] = T * c;
            if (a.vis) a.vis[(size_t)orig * a.S + s] = T;
            if (a.tcut) a.tcut[(size_t)local * a.S + pos] = T == 0.0f ? tfar : INFINITY;
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
    }
}

// The SH projection of the direct pass (Eq. 29 over the S directions):
// one thread per source sums rayw[pos] Y(w_s) over the direction-order
// positions (loads of 8 positions in flight; the direction's Y row is uniform
// across the wave and comes through the scalar unit), then writes the
// transfer (copied to every channel) and, for a bounce, the leaf-order copies.
// The sums are compensated FP32 dot products (Ogita, Rump and Oishi's Dot2):
// each product's rounding error comes from an FMA and each addition's from
// Neumaier's branch-free TwoSum variant, both carried in a second float, so
// the result is as if summed in about twice the precision and then rounded.
// The order is fixed (direction order), so the transfer is the same for
// every work split.
__device__ inline void dot2_add(float w, float y, float& sum, float& comp)
{
#pragma clang fp contract(off)   // p and t must be the rounded product and sum
    const float p = w * y;
    const float pe = fmaf(w, y, -p);          // w y - p exactly
    const float t = sum + p;
    const float se = fabsf(sum) >= fabsf(p) ? (sum - t) + p : (p - t) + sum;   // sum + p - t exactly
    sum = t;
    comp += pe + se;
}

template <int K>
__global__ __launch_bounds__(kBlock) void project_kernel(TransferArgs a)
{
    const int local = blockIdx.x * kBlock + threadIdx.x;
    if (local >= a.count) return;
    const int rank = a.first + local;
    float acc[K], cmp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        acc[k] = 0.0f;
        cmp[k] = 0.0f;
    }
    constexpr int kAhead = 8;
    int pos = 0;
    for (; pos + kAhead <= a.S; pos += kAhead) {
        float w[kAhead];
#pragma unroll
        for (int u = 0; u < kAhead; ++u) w[u] = a.rayw[(size_t)(pos + u) * a.count + local];
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
            const float* y = a.Y + (size_t)a.dir_order[pos + u] * K;
#pragma unroll
            for (int k = 0; k < K; ++k) dot2_add(w[u], y[k], acc[k], cmp[k]);
        }
    }
    for (; pos < a.S; ++pos) {
        const float w = a.rayw[(size_t)pos * a.count + local];
        const float* y = a.Y + (size_t)a.dir_order[pos] * K;
#pragma unroll
        for (int k = 0; k < K; ++k) dot2_add(w, y[k], acc[k], cmp[k]);
    }
    const float scale = kFourPi / (float)a.S;
    float t[K];
#pragma unroll
    for (int k = 0; k < K; ++k) t[k] = (acc[k] + cmp[k]) * scale;
    const int orig = a.order[rank];
    for (int ch = 0; a.transfer && ch < a.channels; ++ch) {
        float* out = a.transfer + ((size_t)orig * a.channels + ch) * K;
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] = t[k];
    }
    if (a.hit_table) {
        constexpr int W = hit_stride(K);
        float* row = a.hit_table + (size_t)rank * W;
#pragma unroll
        for (int k = 0; k < K; ++k) row[k] = t[k];
#pragma unroll
        for (int c = 0; c < 3; ++c) row[K + c] = a.albedo[3 * (size_t)orig + c];
        if constexpr (K % 4 == 0) row[K + 3] = 0.0f;   // the albedo's float4 is read whole
    }
}

// ---------------------------------------------------------------------------
// direct transfer, fan split (small scenes): one wave per source; the
// directions above its horizon are compacted (coherent order) into a
// per-wave list in LDS and traced 64 at a time.  Rays go to rayw like those
// of the group split, so both give the same transfer.
// ---------------------------------------------------------------------------
constexpr int kFanMaxDirs = 1024;   // per-wave direction list capacity (LDS)

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
            else if (pos < seg_n) {
                a.rayw[(size_t)(seg + pos) * a.count + local] = 0.0f;
                if (a.vis) a.vis[(size_t)orig * a.S + s] = -1.0f;
                if (a.tcut) a.tcut[(size_t)local * a.S + seg + pos] = 0.0f;
            }
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
            float T = 1.0f, tfar = 0.0f;
            float tlo = hp.t_min, thi = INFINITY;
            auto leaf = [&](int r, bool box_hit) {
                const Prim p = uniform_load(a.prims, r);
                const PreHit q = gaussian_pre(p, ox, oy, oz, d, hp);
                const bool cand = q.maybe & box_hit & live & (r != rank);
                if (__ballot(cand) == 0ull) return;
                HitResult h;
                const bool hit = gaussian_exact(p, q, ox, oy, oz, d, hp, h) & cand;
                T = hit ? T * (1.0f - h.alpha) : T;
                tfar = hit ? fmaxf(tfar, h.t) : tfar;
                const bool opaque = T < hp.T_eps;
                live = live & !opaque;
                T = opaque ? 0.0f : T;
            };
            traverse_batch<false>(a, d, bd, ox, oy, oz, live, tlo, thi, leaf, (RayCounts*)nullptr);
            if (traced) {
                a.rayw[(size_t)(seg + list[wslot][idx]) * a.count + local] = T * c;
                if (a.vis) a.vis[(size_t)orig * a.S + s] = T;
                if (a.tcut) a.tcut[(size_t)local * a.S + seg + list[wslot][idx]] = T == 0.0f ? tfar : INFINITY;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------------------
// one bounce, group split
// ---------------------------------------------------------------------------

// Strict order of hits along a ray, by t* then by leaf rank, as one 64-bit
// key: t* >= 0, so its bit pattern orders like the value (+ 0 turns -0 into
// +0).  kNoHit (t = inf) sorts after every hit.
__device__ inline uint64_t hit_key(float t, int j)
{
    return ((uint64_t)__float_as_uint(t + 0.0f) << 32) | (uint32_t)j;
}
constexpr uint64_t kNoHit = 0x7f800000ffffffffull;
__device__ inline float key_t(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ inline int key_j(uint64_t k) { return (int)(uint32_t)k; }

// The hits of each ray are needed front to back (weight alpha_j T_j, T_j the
// transmittance in front of hit j), up to the one that takes the
// transmittance below T_eps.  The traversal appends every hit beyond the last
// blended one and no farther than the depth the direct pass needed to a list
// of the lane's own in device memory, unsorted (the traversal meets them in
// no useful order), contiguous per lane so that its appends fill whole cache
// lines (interleaving the lanes' entries instead left lines part-written
// when evicted: 3.6x the appended bytes were written back, and the million-
// splat bounce took 2.65 s against 2.41 s).  Afterwards the lane blends the
// list nearest first, kBlend hits at a time: one pass over the list (each
// lane reading its own entries in order) keeps the kBlend nearest unblended
// keys in a sorted register buffer
// (merge_chunk folds in kScan entries at a time), and
// each blended hit's weight goes to a per-lane record list; the records are
// summed into the transfer once the round's selection is over, so that the
// 3K sums are not live during the traversal or the scans.  A
// list that fills up is compacted around the mean depth of its hits: those
// beyond it are dropped and every later hit beyond it is refused (k_over), so
// the list stays complete in front of k_over; the lane blends it and, if
// still transparent, traverses again from its last hit.  The launch is
// persistent: a fixed set of waves takes groups of sources from a counter,
// so the lists are sized by the waves, not the scene.
constexpr int kSelBlend = 16;   // hits selected per pass over the list: the blend in two walks,
constexpr int kSelFused = 8;    // the blend in one walk (its fewer registers let it run 7 waves per SIMD),
constexpr int kSelIndex = 8;    // and the index walk
constexpr int kCheck = 8;   // depth checkpoints per ray and round

// Compare-exchange of two (key, alpha) pairs: the smaller key ends in a.
__device__ inline void cas_pair(uint64_t& ka, float& aa, uint64_t& kb, float& ab)
{
    const bool sw = kb < ka;
    const uint64_t tk = ka;
    const float ta = aa;
    ka = sw ? kb : ka;
    aa = sw ? ab : aa;
    kb = sw ? tk : kb;
    ab = sw ? ta : ab;
}

// Folds a chunk of N keys (ineligible ones set to kNoHit) into the sorted
// buffer of the B smallest: a sorting network orders the chunk (Batcher's
// odd-even merge sort), the buffer followed by the chunk reversed is
// bitonic, so one half-cleaner step leaves the B smallest of both in the
// buffer, and the bitonic merge network sorts them.  At B = 8, N = 8 that is
// 34 VALU per entry against 56 for an insertion into the buffer, which one
// lane or another needs at almost every entry.
template <int N, int B>
__device__ inline void merge_chunk(uint64_t (&kk)[N], float (&aa)[N], uint64_t (&bk)[B], float (&ba)[B])
{
    static_assert((B == 8 || B == 16) && (N == 4 || N == 8), "networks for 4 or 8 entries into 8 or 16");
    auto c = [&](int i, int j) { cas_pair(kk[i], aa[i], kk[j], aa[j]); };
    if constexpr (N == 4) {
        c(0, 1); c(2, 3); c(0, 2); c(1, 3); c(1, 2);
    } else {
        c(0, 1); c(2, 3); c(4, 5); c(6, 7);
        c(0, 2); c(1, 3); c(4, 6); c(5, 7);
        c(1, 2); c(5, 6);
        c(0, 4); c(1, 5); c(2, 6); c(3, 7);
        c(2, 4); c(3, 5);
        c(1, 2); c(3, 4); c(5, 6);
    }
#pragma unroll
    for (int q = B - N; q < B; ++q) {
        const bool lt = kk[B - 1 - q] < bk[q];
        bk[q] = lt ? kk[B - 1 - q] : bk[q];
        ba[q] = lt ? aa[B - 1 - q] : ba[q];
    }
    // bitonic merge of the B-entry buffer: half-cleaners at distance B/2, ..., 1
#pragma unroll
    for (int dist = B / 2; dist >= 1; dist >>= 1)
#pragma unroll
        for (int i = 0; i < B; ++i)
            if ((i & dist) == 0) cas_pair(bk[i], ba[i], bk[i + dist], ba[i + dist]);
}

// A hit splat's direct transfer and albedo from the leaf-order hit table
// (one row of hit_stride(K) floats: float4 loads where K is a multiple of 4).
template <int K>
__device__ inline void load_hit(const float* table, int r, float (&tv)[K], float4& rho)
{
    constexpr int W = hit_stride(K);
    const float* row = table + (size_t)r * W;
    if constexpr (K % 4 == 0) {
        const float4* v4 = reinterpret_cast<const float4*>(row);
#pragma unroll
        for (int k4 = 0; k4 < K / 4; ++k4) {
            const float4 v = v4[k4];
            tv[4 * k4] = v.x;
            tv[4 * k4 + 1] = v.y;
            tv[4 * k4 + 2] = v.z;
            tv[4 * k4 + 3] = v.w;
        }
        rho = v4[K / 4];
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) tv[k] = row[k];
        rho = make_float4(row[K], row[K + 1], row[K + 2], 0.0f);
    }
}

// Sums a lane's blended-hit records (leaf rank, weight), in blend order, into
// its source's 3 K bounce sums of direction part `part` (Eq. 20-22, 30-33:
// rho_j,c w t_dir[j] per record), the D lanes of a source summed first.  One
// wave owns a (part, source) pair, so the read-modify-write needs no atomics.
template <int K>
__device__ inline void sum_records(const TransferArgs& a, const int2* rec, int cnt, int D, bool valid, int part,
                                   int orig, float scale)
{
    const int lane = threadIdx.x & (kWave - 1);
    float acc[3][K];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[ch][k] = 0.0f;
    for (int q = 0; q < cnt; ++q) {
        const int2 e = rec[q];
        const int r = e.x;
        const float w = __int_as_float(e.y);
        float4 rho;
        float tv[K];
        load_hit<K>(a.hit_table, r, tv, rho);
        const float r0 = rho.x * w, r1 = rho.y * w, r2 = rho.z * w;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            acc[0][k] = fmaf(r0, tv[k], acc[0][k]);
            acc[1][k] = fmaf(r1, tv[k], acc[1][k]);
            acc[2][k] = fmaf(r2, tv[k], acc[2][k]);
        }
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float* out = a.partial + (((size_t)part * a.n + orig) * 3 + ch) * K;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float v = segment_sum(acc[ch][k], D) * scale;
            if (valid && (lane % D) == 0) out[k] += v;
        }
    }
}

// sum_records with the loads of U records (record, albedo, direct transfer)
// issued together before their FMAs, which run in the same order: the same
// sums, for the pass that reads every record back from the arena.
template <int K, int U>
__device__ inline void sum_records_batched(const TransferArgs& a, const int2* rec, int cnt, int D, bool valid,
                                           int part, int orig, float scale)
{
    const int lane = threadIdx.x & (kWave - 1);
    float acc[3][K];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[ch][k] = 0.0f;
    for (int q0 = 0; q0 < cnt; q0 += U) {
        int2 e[U];
        float4 rho[U];
        float tv[U][K];
#pragma unroll
        for (int u = 0; u < U; ++u) e[u] = q0 + u < cnt ? rec[q0 + u] : make_int2(0, 0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = e[u].x;
            load_hit<K>(a.hit_table, r, tv[u], rho[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (q0 + u < cnt) {
                const float w = __int_as_float(e[u].y);
                const float r0 = rho[u].x * w, r1 = rho[u].y * w, r2 = rho[u].z * w;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    acc[0][k] = fmaf(r0, tv[u][k], acc[0][k]);
                    acc[1][k] = fmaf(r1, tv[u][k], acc[1][k]);
                    acc[2][k] = fmaf(r2, tv[u][k], acc[2][k]);
                }
            }
        }
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float* out = a.partial + (((size_t)part * a.n + orig) * 3 + ch) * K;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float v = segment_sum(acc[ch][k], D) * scale;
            if (valid && (lane % D) == 0) out[k] += v;
        }
    }
}

// Exclusive prefix sum of v over the lanes of the wave.
__device__ inline int lane_prefix(int v)
{
    const int lane = threadIdx.x & (kWave - 1);
    int incl = v;
    for (int off = 1; off < kWave; off <<= 1) {
        const int up = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += up;
    }
    return incl - v;
}

// One-walk blend: the round's records (each lane's cnt of them) go to a new
// block at the end of the item's chain, to be summed once every direct
// transfer exists (accumulate_kernel).  An item whose block does not fit in
// the arena is marked deferred: its later rounds write nothing, the
// accumulation skips it and the two-walk pass redoes it.
__device__ inline void emit_records(const TransferArgs& a, const int2* lrec, int cnt, int item, int64_t& prev_block,
                                    bool& item_def)
{
    const int lane = threadIdx.x & (kWave - 1);
    int tot = cnt;
    for (int off = kWave / 2; off >= 1; off >>= 1) tot += __shfl_xor(tot, off, kWave);
    if (tot == 0 || item_def) return;   // uniform
    const unsigned long long need = (unsigned long long)kRecHeaderWords + (unsigned long long)tot;
    unsigned long long at = 0;
    if (lane == 0) at = atomicAdd(a.rec_top, need);
    at = ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(at >> 32)) << 32) |
         (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)at);
    if (at + need > a.rec_words) {
        item_def = true;
        if (lane == 0) {
            a.item_deferred[item] = 1;
            raise_flag(a.flags, PRTGS_FLAG_RECORDS_DEFERRED);
        }
        return;
    }
    uint64_t* blk = a.rec + at;
    if (lane == 0) {
        blk[0] = ~0ull;   // the end of the chain until a next block links in
        if (prev_block < 0) a.item_head[item] = (int64_t)at;
        else a.rec[prev_block] = at;
    }
    reinterpret_cast<uint16_t*>(blk + 1)[lane] = (uint16_t)cnt;
    int2* dst = reinterpret_cast<int2*>(blk + kRecHeaderWords) + lane_prefix(cnt);
    for (int q = 0; q < cnt; ++q) dst[q] = lrec[q];
    prev_block = (int64_t)at;
}

// kIndex: the paper's own bounce instead of the blend -- the same walk, but
// each ray records the hit of largest alpha_j T_j max(-w . n_j, 0) among the
// hits with T_j <= t_same (the nearer one on equal weights) in the index
// matrix (-1: none, or not traced), and nothing is accumulated.  kScan list
// entries are loaded together in the selection.
// kCount (blend only): the walk also tallies its work into stats (see
// launch_bounce_stats); the results are the same.
// kFused (blend only): one walk per ray for both passes.  No cut comes from a
// direct pass: until the running product of the hits found falls below
// T_eps (in traversal order, as the direct pass multiplies them) the walk
// lists every hit; from then on the farthest of those hits is the cut, the
// checkpoints split [t_lo, cut] (the last one holding that product, the
// others T, a bound that the hits found later tighten), and the walk goes on
// as the two-walk blend does.  At the end of its rounds the ray's blend gives
// its visibility (the product over all its hits, 0 once below T_eps), written
// where the direct pass writes it, with the deepest cut found; the blended
// hits' records go to the arena (emit_records) instead of being summed.
template <int K, bool kIndex, int kScan, bool kCount = false, bool kFused = false>
__device__ __forceinline__ void bounce_walk(const TransferArgs& a, unsigned long long* stats = nullptr)
{
    constexpr int M = kHitList;
    constexpr int kBlend = kIndex ? kSelIndex : kFused ? kSelFused : kSelBlend;
    constexpr int kKind = kIndex ? kWalkIndex : kFused ? kWalkFused : kWalkBlend;
    const int lane = threadIdx.x & (kWave - 1);
    const int G = a.G;
    const int D = kWave / G;
    const int wslot = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    // the grid is whole blocks: a wave past the lists' capacity has none and
    // leaves before it takes work (no block-wide barrier follows)
    if (wslot >= bounce_waves(a.n, kKind)) return;
    // (two-walk pass after a one-walk blend) nothing to redo unless the walk deferred an item
    if (!kFused && a.item_deferred &&
        !(__atomic_load_n(a.flags, __ATOMIC_RELAXED) & PRTGS_FLAG_RECORDS_DEFERRED))
        return;
    // each lane's list is contiguous (entry q at [q]): a lane's appends fill whole cache lines
    uint64_t* const lkey = a.hitkey + (size_t)wslot * M * kWave + (size_t)lane * M;
    float* const lalpha = a.hitalpha + (size_t)wslot * M * kWave + (size_t)lane * M;
    int2* const lrec = kIndex ? nullptr : a.hitrec + (size_t)wslot * M * kWave + (size_t)lane * M;
    const int groups = (a.count + G - 1) / G;
    const HitParams hp = a.hp;
    RayCounts rc;   // (kCount) single-ray traversal work, hits blended and listed, rounds
    uint32_t n_traced = 0, n_blended = 0, n_listed = 0, n_rounds = 0;

    for (;;) {
        // items are (direction part, source group), taken part-major as in the
        // direct pass, so the waves in flight trace nearly the same directions
        int item = 0;
        if (lane == 0) item = (int)atomicAdd(a.queue, 1u);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= groups * a.Q) break;   // uniform: every wave leaves once the counter passes the last item
        // (two-walk pass after a one-walk blend) only the items whose records did not fit
        if (!kFused && a.item_deferred && a.item_deferred[item] == 0) continue;
        const int part = item / groups, grp = item % groups;
        int64_t prev_block = -1;   // (kFused) the item's last record block
        bool item_def = false;     // (kFused) the item's records did not fit

        const int local = grp * G + lane / D;
        const bool valid = local < a.count;
        const int rank = a.first + (valid ? local : 0);
        const float4 mo = a.prims[rank].mo;
        const float ox = mo.x, oy = mo.y, oz = mo.z;
        const float4 nrm = a.normals[rank];
        const int orig = valid ? a.order[rank] : 0;
        const float scale = kFourPi / (float)a.S;

        const int nb = (a.S + D - 1) / D;
        for (int bi = part * nb / a.Q; bi < (part + 1) * nb / a.Q; ++bi) {
            const int b0 = bi * D;
            const int pos = b0 + (lane % D);
            const bool inrange = pos < a.S;
            const int s = inrange ? a.dir_order[pos] : 0;
            const RayDir d = make_dir(a.dirs[3 * s], a.dirs[3 * s + 1], a.dirs[3 * s + 2]);
            const float c = nrm.x * d.wx + nrm.y * d.wy + nrm.z * d.wz;
            bool pending = valid && inrange && c > 0.0f;
            if (kIndex && valid && inrange && !pending) a.index[(size_t)orig * a.S + s] = -1;
            if (kFused && !kCount && valid && inrange && !pending) {   // below the horizon, as the direct pass writes it
                a.rayw[(size_t)pos * a.count + local] = 0.0f;
                if (a.vis) a.vis[(size_t)orig * a.S + s] = -1.0f;
                a.tcut[(size_t)local * a.S + pos] = 0.0f;
            }
            if (__ballot(pending) == 0ull) continue;
            const bool traced = pending;
            if (kCount && traced) ++n_traced;
            BatchDir bd = batch_dir(d, pending);
#pragma unroll
            for (int k = 0; k < 3; ++k)   // uniform: kept in scalar registers through the walk
                bd.mean[k] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(bd.mean[k])));
            const float wc = c * kInvPi;
            // No hit beyond tc can carry weight: the direct pass saw the
            // transmittance fall below T_eps using hits no farther than tc.
            // (kFused: no cut yet; tck is the deepest the walk has found.)
            const float tc = kFused ? INFINITY : (pending ? a.tcut[(size_t)local * a.S + pos] : 0.0f);
            float tck = tc;
            float T = 1.0f;
            float bestW = 0.0f;   // (kIndex) largest weight so far and its leaf rank
            int bestr = -1;
            bool started = false;
            uint64_t k_last = 0;   // key of the last blended hit (once started)
            int rounds = 0;
            while (__ballot(pending) != 0ull) {
                // A traversal that ran out of its budget flagged the tree: stop.
                // Every round blends at least one listed hit (compact keeps the
                // nearest), so a ray ends within as many rounds as it has hits;
                // the cap bounds the work of a pathological scene.
                // (No early exit for the lanes that stop: the record emission
                // needs every lane of the wave active; a stopped lane traces,
                // lists and blends nothing.)
                if (pending && (__atomic_load_n(a.flags, __ATOMIC_RELAXED) & PRTGS_FLAG_BAD_TREE)) pending = false;
                if (pending && ++rounds > kMaxRounds) {
                    raise_flag(a.flags, PRTGS_FLAG_ROUND_CAP);
                    pending = false;
                }
                if (kCount && pending) ++n_rounds;
                int cnt = 0;
                float sum_t = 0.0f;         // of the listed hits (compaction pivot)
                uint64_t k_over = kNoHit;   // hits from here on wait for the next round
                bool live = pending;
                float tlo = started ? fmaxf(hp.t_min, key_t(k_last)) : hp.t_min, thi = tck;
                float Tr = T, tfar = 0.0f;   // (kFused, no cut yet) product and depth of the hits found
                // Checkpoints tlo + (b + 1) tstep split [tlo, tc]: P[b] is T times
                // the (1 - alpha) of the hits found so far in front of checkpoint
                // b.  The hits in front of it are a subset of all of them, so
                // once P[b] < T_eps the walk ends there and nothing beyond the
                // checkpoint is needed.
                float tstep = tck < INFINITY ? (tck - tlo) * (1.0f / (float)kCheck) : 0.0f;
                float P[kCheck];
#pragma unroll
                for (int b = 0; b < kCheck; ++b) P[b] = T;
                // Full list: keep the hits in front of their mean depth.  At
                // least one goes (if rounding keeps them all, the farthest) and
                // at least one stays (the nearest, also when every listed depth
                // is the same and the mean rounds to it or below), so the round
                // blends a hit and the next one starts beyond it.
                auto compact = [&]() {
                    uint64_t kmin = kNoHit;   // every listed key is below k_over
                    for (int q = 0; q < cnt; ++q) {
                        const uint64_t k = lkey[q];
                        kmin = k < kmin ? k : kmin;
                    }
                    uint64_t pivot = hit_key(sum_t / (float)cnt, 0);
                    pivot = pivot > kmin ? pivot : kmin + 1;
                    if (pivot < k_over) k_over = pivot;
                    int kept = 0;
                    float kept_sum = 0.0f;
                    uint64_t kmax = 0;
                    int imax = 0;
                    for (int q = 0; q < cnt; ++q) {
                        const uint64_t k = lkey[q];
                        const float al = lalpha[q];
                        if (k < k_over) {
                            lkey[kept] = k;
                            lalpha[kept] = al;
                            if (k > kmax) {
                                kmax = k;
                                imax = kept;
                            }
                            kept_sum += key_t(k);
                            ++kept;
                        }
                    }
                    if (kept == cnt) {   // drop the farthest: move the last entry into its slot
                        k_over = kmax;
                        kept_sum -= key_t(kmax);
                        --kept;
                        lkey[imax] = lkey[kept];
                        lalpha[imax] = lalpha[kept];
                    }
                    cnt = kept;
                    sum_t = kept_sum;
                    thi = fminf(thi, key_t(k_over));
                };
                auto leaf = [&](int r, bool box_hit) {
                    const Prim p = uniform_load(a.prims, r);
                    const PreHit q = gaussian_pre(p, ox, oy, oz, d, hp);
                    // no r != rank test: the ray starts at the source's own mean, so its own
                    // Gaussian peaks at t* = 0 exactly (a zero offset in both stages) and fails
                    // t* > t_min >= 0; without the test the lane's rank need not stay in a
                    // register through the walk (it was spilled and reloaded at every leaf)
                    const bool cand = q.maybe & box_hit & live;
                    if (__ballot(cand) == 0ull) return;
                    HitResult h;
                    const bool hit = gaussian_exact(p, q, ox, oy, oz, d, hp, h) & cand;
                    const uint64_t key = hit_key(h.t, r);
                    const bool ins = hit & (h.t <= thi) & (!started | (key > k_last)) & (key < k_over);
                    if (ins) {
                        if (tstep > 0.0f) {
                            float cut = INFINITY;
#pragma unroll
                            for (int b = 0; b < kCheck; ++b) {
                                const float tb = tlo + tstep * (float)(b + 1);
                                P[b] = h.t <= tb ? P[b] * (1.0f - h.alpha) : P[b];
                                cut = P[b] < hp.T_eps ? fminf(cut, tb) : cut;
                            }
                            thi = fminf(thi, cut);
                            if (kFused) tck = fminf(tck, cut);
                        } else if (kFused) {
                            Tr *= 1.0f - h.alpha;
                            tfar = fmaxf(tfar, h.t);
                            if (Tr < hp.T_eps) {
                                // every hit found so far lies in front of tfar: the cut
                                tck = tfar;
                                thi = fminf(thi, tfar);
                                tstep = (tck - tlo) * (1.0f / (float)kCheck);
#pragma unroll
                                for (int b = 0; b < kCheck - 1; ++b) P[b] = T;
                                P[kCheck - 1] = Tr;
                            }
                        }
                        if (cnt == M) compact();
                        if (key < k_over) {
                            lkey[cnt] = key;
                            lalpha[cnt] = h.alpha;
                            sum_t += h.t;
                            ++cnt;
                        }
                    }
                };
                traverse_batch<kCount, kLoadFirst>(a, d, bd, ox, oy, oz, live, tlo, thi, leaf,
                                             kCount ? &rc : (RayCounts*)nullptr);
                if (kCount && pending) n_listed += cnt;

                int maxcnt = pending ? cnt : 0;
                for (int off = 32; off >= 1; off >>= 1) maxcnt = max(maxcnt, __shfl_xor(maxcnt, off, kWave));
                bool done = false;
                bool more = pending && cnt > 0;   // listed hits left to blend
                int nrec = 0;                     // hits blended this round (at most cnt)
                while (__ballot(more) != 0ull) {
                    uint64_t bk[kBlend];
                    float ba[kBlend];
#pragma unroll
                    for (int q = 0; q < kBlend; ++q) {
                        bk[q] = kNoHit;
                        ba[q] = 0.0f;
                    }
                    for (int q0 = 0; q0 < maxcnt; q0 += kScan) {
                        // kScan keys' loads in flight together; the buffer carries
                        // each key's list position (bits in a float), and only the
                        // selected entries' alphas are read, after the pass
                        uint64_t kk[kScan];
                        float aa[kScan];
#pragma unroll
                        for (int u = 0; u < kScan; ++u) {
                            const int q = q0 + u;
                            const bool inl = more && q < cnt;
                            kk[u] = inl ? lkey[q] : kNoHit;
                            aa[u] = __int_as_float(q);
                        }
                        bool anysel = false;
#pragma unroll
                        for (int u = 0; u < kScan; ++u) {
                            const uint64_t k = kk[u];
                            const bool sel = (k != kNoHit) & (!started | (k > k_last)) & (k < k_over) &
                                             (k < bk[kBlend - 1]);
                            kk[u] = sel ? k : kNoHit;
                            anysel |= sel;
                        }
                        if (__ballot(anysel) != 0ull) merge_chunk<kScan, kBlend>(kk, aa, bk, ba);
                    }
                    // the selected entries' alphas (their loads in flight together)
#pragma unroll
                    for (int q = 0; q < kBlend; ++q)
                        ba[q] = (more && bk[q] != kNoHit) ? lalpha[__float_as_int(ba[q])] : 0.0f;
                    int got = 0;
#pragma unroll
                    for (int q = 0; q < kBlend; ++q) {
                        // one hit's loads at a time: hoisting all of them would
                        // hold kBlend (K + 4) registers at once
                        asm volatile("" ::: "memory");
                        if (kIndex && more && !done && bk[q] != kNoHit) {
                            const int r = key_j(bk[q]);
                            if (T <= a.t_same) {
                                const float4 nj = a.normals[r];
                                const float f = -(d.wx * nj.x + d.wy * nj.y + d.wz * nj.z);
                                const float W = ba[q] * T * fmaxf(f, 0.0f);
                                if (W > bestW) {
                                    bestW = W;
                                    bestr = r;
                                }
                            }
                            T *= 1.0f - ba[q];
                            k_last = bk[q];
                            started = true;
                            ++got;
                            // no later hit can outweigh the best one: its W_j <= T_j <= T
                            // (each FP32 product by a factor <= 1 stays <= T); the one walk
                            // goes on for the ray's visibility
                            if (T < hp.T_eps || (!kFused && T <= bestW)) done = true;
                        } else if (!kIndex && more && !done && bk[q] != kNoHit) {
                            // the hit's weight, summed into the transfer after the selection
                            lrec[nrec] = make_int2(key_j(bk[q]), __float_as_int(ba[q] * T * wc));
                            ++nrec;
                            T *= 1.0f - ba[q];
                            k_last = bk[q];
                            started = true;
                            ++got;
                            if (T < hp.T_eps) done = true;
                        }
                    }
                    // a buffer that came back short held the last listed hits
                    if (done || got < kBlend) more = false;
                }
                if (kCount) n_blended += nrec;
                // a list that overflowed and is still transparent: traverse on
                if (done || k_over == kNoHit) pending = false;
                // Sum the round's blended hits in blend order and add them to
                // the source's transfer (the D lanes of a source summed
                // first).  The sums live only here, not across the selection
                // or the traversal, which keeps both free of spills.
                if constexpr (kFused && !kIndex) {
                    if constexpr (!kCount) emit_records(a, lrec, nrec, item, prev_block, item_def);
                } else if constexpr (!kIndex) {
                    sum_records<K>(a, lrec, nrec, D, valid, part, orig, scale);
                }
            }
            if (kFused && traced) {
                // the ray's visibility (Eq. 4's product over every hit, 0 once below
                // T_eps), as the direct pass writes it, and the deepest cut found
                const float V = T < hp.T_eps ? 0.0f : T;
                if constexpr (!kCount) {
                    a.rayw[(size_t)pos * a.count + local] = V * c;
                    if (a.vis) a.vis[(size_t)orig * a.S + s] = V;
                    a.tcut[(size_t)local * a.S + pos] = tck;
                }
            }
            if (kIndex && traced) a.index[(size_t)orig * a.S + s] = bestr >= 0 ? a.order[bestr] : -1;
        }
    }
    if constexpr (kCount) {
        atomicAdd(&stats[0], (unsigned long long)n_traced);
        atomicAdd(&stats[1], (unsigned long long)rc.box_tests);
        atomicAdd(&stats[2], (unsigned long long)rc.prim_tests);
        if (lane == 0) {
            atomicAdd(&stats[3], (unsigned long long)rc.wave_nodes);
            atomicAdd(&stats[4], (unsigned long long)rc.wave_leaves);
        }
        atomicAdd(&stats[5], (unsigned long long)n_blended);
        atomicAdd(&stats[6], (unsigned long long)n_listed);
        atomicAdd(&stats[7], (unsigned long long)n_rounds);
    }
}

// The walks hold different registers at their peak (the two-walk blend its
// 3K sums, the one-walk blend and the index mode none), so each gets the
// occupancy, buffer and scan width that measured fastest: the two-walk blend
// 4 waves per SIMD, a 16-hit buffer and 4 entries per step (fewer passes over
// the lists than with 8 hits: the million-splat transfer call 3.34 -> 3.29
// s); the one-walk blend 7 waves and 8 hits (its time is the latency of its
// dependent loads, so resident waves pay more than fewer passes over the lists
// or spill traffic: 5 / 6 / 7 / 8 waves 2214 / 2101-2123 / 2093 / 2447 ms at
// 1M x 512, with 22 / 62 / 68 / 113 VGPRs spilled); the index walk 5 waves, 8
// hits; 4 entries per step for all.
template <int K>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kBounceWavesPerSimd))) void bounce_kernel(
    TransferArgs a)
{
    bounce_walk<K, false, 4>(a);
}
template <int K>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kIndexWavesPerSimd))) void index_kernel(
    TransferArgs a)
{
    bounce_walk<K, true, 4>(a);
}
// the blend's walk with its work tallied (prtgs_traversal_stats)
template <int K>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kBounceWavesPerSimd))) void bounce_count_kernel(
    TransferArgs a, unsigned long long* stats)
{
    bounce_walk<K, false, 4, true>(a, stats);
}
// the index matrix in one walk per ray (visibility and index, no records)
template <int K>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kIndexWavesPerSimd))) void fused_index_kernel(
    TransferArgs a)
{
    bounce_walk<K, true, 4, false, true>(a);
}
// the blend in one walk per ray, and the same with its work tallied
template <int K>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kFusedWavesPerSimd))) void fused_kernel(
    TransferArgs a)
{
    bounce_walk<K, false, 4, false, true>(a);
}
template <int K>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kFusedWavesPerSimd))) void fused_count_kernel(
    TransferArgs a, unsigned long long* stats)
{
    bounce_walk<K, false, 4, true, true>(a, stats);
}

// The one-walk blend's records summed once every direct transfer exists: one
// wave per work item, its blocks in the order the walk wrote them, each
// lane's records in blend order (sum_records, the arithmetic of the two-walk
// blend).  Deferred items are left to the two-walk pass.
constexpr int kAccBatch = 4;   // records whose loads the record sums issue together

template <int K>
__global__ __launch_bounds__(kBlock) void accumulate_kernel(TransferArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int G = a.G, D = kWave / G;
    const int groups = (a.count + G - 1) / G;
    const int items = groups * a.Q;
    const float scale = kFourPi / (float)a.S;
    for (int item = (int)((blockIdx.x * kBlock + threadIdx.x) / kWave); item < items;
         item += (int)(gridDim.x * (kBlock / kWave))) {
        if (a.item_deferred[item]) continue;
        int64_t at = a.item_head[item];
        const int part = item / groups, grp = item % groups;
        const int local = grp * G + lane / D;
        const bool valid = local < a.count;
        const int orig = valid ? a.order[a.first + local] : 0;
        while (at >= 0) {
            const uint64_t* blk = a.rec + at;
            const int cnt = reinterpret_cast<const uint16_t*>(blk + 1)[lane];
            const int2* rec = reinterpret_cast<const int2*>(blk + kRecHeaderWords) + lane_prefix(cnt);
            sum_records_batched<K, kAccBatch>(a, rec, cnt, D, valid, part, orig, scale);
            const uint64_t nx = blk[0];
            at = nx == ~0ull ? -1 : (int64_t)nx;
        }
    }
}

// ---------------------------------------------------------------------------
// the paper's recursive self-transfer: one gather step over the index matrix
// (one wave per source, lanes over directions, then a wave reduction)
// ---------------------------------------------------------------------------
template <int K, int CP>
__global__ __launch_bounds__(kBlock) void self_transfer_kernel(int n, int S, const float* __restrict__ dirs,
                                                               const float* __restrict__ normals,
                                                               const float* __restrict__ albedo,
                                                               const int32_t* __restrict__ index,
                                                               const float* __restrict__ t_prev,
                                                               float* __restrict__ t_out, unsigned* flags)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int i = (blockIdx.x * kBlock + threadIdx.x) / kWave;   // source of this wave
    if (i >= n) return;                                           // whole wave leaves together
    const float nx = normals[3 * (size_t)i], ny = normals[3 * (size_t)i + 1], nz = normals[3 * (size_t)i + 2];
    float acc[3][K];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[ch][k] = 0.0f;
    for (int s0 = 0; s0 < S; s0 += kWave) {
        const int s = s0 + lane;
        if (s >= S) continue;
        const int j = index[(size_t)i * S + s];
        if (j < -1 || j >= n) {
            if (flags) raise_flag(flags, PRTGS_FLAG_BAD_INDEX);
            continue;
        }
        const float c = nx * dirs[3 * s] + ny * dirs[3 * s + 1] + nz * dirs[3 * s + 2];
        if (j < 0 || !(c > 0.0f)) continue;
        const float w = c * kInvPi;
        const float r[3] = {albedo[3 * (size_t)j] * w, albedo[3 * (size_t)j + 1] * w, albedo[3 * (size_t)j + 2] * w};
        const float* tp = t_prev + (size_t)j * CP * K;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch)
#pragma unroll
            for (int k = 0; k < K; ++k) acc[ch][k] = fmaf(r[ch], tp[(CP == 3 ? ch : 0) * K + k], acc[ch][k]);
    }
    const float scale = kFourPi / (float)S;
    float mine = 0.0f;   // lane l < 3K ends up with element l
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float v = segment_sum(acc[ch][k], kWave);
            mine = lane == ch * K + k ? v : mine;
        }
    if (lane < 3 * K) t_out[(size_t)i * 3 * K + lane] = mine * scale;
}

// transfer += the parts' bounce sums, added in part order
__global__ void add_parts_kernel(float* __restrict__ acc, const float* __restrict__ parts, size_t count, int Q)
{
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x) {
        float v = acc[e];
        for (int q = 0; q < Q; ++q) v += parts[(size_t)q * count + e];
        acc[e] = v;
    }
}

__global__ void add_kernel(float* __restrict__ acc, const float* __restrict__ x, size_t count)
{
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
        acc[e] += x[e];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int group_blocks(int count, int G, int Q = 1)
{
    const int64_t waves = (int64_t)((count + G - 1) / G) * Q;
    return (int)((waves + kBlock / kWave - 1) / (kBlock / kWave));
}

template <int K>
hipError_t launch_direct_k(const TransferArgs& a, unsigned long long* stats, hipStream_t stream)
{
    TransferArgs b = a;
    b.Q = a.G == 1 ? 1 : direction_parts(a.G, a.S, a.Q_req);
    if (stats) {
        hipLaunchKernelGGL((direct_kernel<true>), dim3(group_blocks(a.count, a.G, b.Q)), dim3(kBlock), 0, stream, b,
                           stats);
        return hipGetLastError();
    }
    if (a.G == 1)
        hipLaunchKernelGGL(direct_fan_kernel, dim3(group_blocks(a.count, 1)), dim3(kBlock), 0, stream, b);
    else
        hipLaunchKernelGGL((direct_kernel<false>), dim3(group_blocks(a.count, a.G, b.Q)), dim3(kBlock), 0, stream, b,
                           stats);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(project_kernel<K>, dim3((a.count + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

template <int K, bool kIndex>
hipError_t launch_bounce_k(const TransferArgs& a, hipStream_t stream, unsigned long long* stats = nullptr)
{
    hipError_t e = fill_u32(a.queue, 0u, 1, stream);
    if (e != hipSuccess) return e;
    TransferArgs b = a;
    b.Q = kIndex ? direction_parts(a.G, a.S, a.Q_req) : blend_parts(a.G, a.S, a.Q_req);
    if constexpr (!kIndex) {
        e = fill_u32(reinterpret_cast<uint32_t*>(b.partial), 0u, (size_t)b.Q * a.n * 3 * a.K, stream);
        if (e != hipSuccess) return e;
    }
    const int64_t items = (int64_t)((a.count + a.G - 1) / a.G) * b.Q;
    const int cap = bounce_waves(a.n, kIndex ? kWalkIndex : kWalkBlend);   // the hit lists hold this many
    const int waves = items < cap ? (int)items : cap;
    const dim3 grid((waves + kBlock / kWave - 1) / (kBlock / kWave));
    if constexpr (kIndex) {
        hipLaunchKernelGGL(index_kernel<K>, grid, dim3(kBlock), 0, stream, b);
    } else if (stats) {
        hipLaunchKernelGGL(bounce_count_kernel<K>, grid, dim3(kBlock), 0, stream, b, stats);
    } else {
        hipLaunchKernelGGL(bounce_kernel<K>, grid, dim3(kBlock), 0, stream, b);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        const size_t count = (size_t)a.n * 3 * a.K;
        hipLaunchKernelGGL(add_parts_kernel, dim3((unsigned)std::min<size_t>((count + 255) / 256, 65536)), dim3(256), 0,
                           stream, a.transfer, b.partial, count, b.Q);
    }
    return hipGetLastError();
}

// The blend in one walk per ray: the walk (visibility, cut depths, records),
// the projection (the direct transfers the records need), the records' sums,
// the two-walk pass over the items whose records did not fit (a launch whose
// waves skip every other item), and the parts added in order.
template <int K>
hipError_t launch_fused_k(const TransferArgs& a, hipStream_t stream, unsigned long long* stats)
{
    TransferArgs b = a;
    b.Q = blend_parts(a.G, a.S, a.Q_req);
    const int64_t items = (int64_t)((a.count + a.G - 1) / a.G) * b.Q;
    hipError_t e = fill_u32(a.queue, 0u, 1, stream);
    if (e == hipSuccess) e = fill_u32(reinterpret_cast<uint32_t*>(a.rec_top), 0u, 2, stream);
    if (e == hipSuccess) e = fill_u32(reinterpret_cast<uint32_t*>(a.item_head), 0xffffffffu, 2 * (size_t)items, stream);
    if (e == hipSuccess) e = fill_u32(reinterpret_cast<uint32_t*>(a.item_deferred), 0u, (size_t)items, stream);
    if (e == hipSuccess && !stats)
        e = fill_u32(reinterpret_cast<uint32_t*>(b.partial), 0u, (size_t)b.Q * a.n * 3 * a.K, stream);
    if (e != hipSuccess) return e;
    const int cap = bounce_waves(a.n, kWalkFused);
    const int waves = items < cap ? (int)items : cap;
    const dim3 grid((waves + kBlock / kWave - 1) / (kBlock / kWave));
    if (stats) {
        hipLaunchKernelGGL(fused_count_kernel<K>, grid, dim3(kBlock), 0, stream, b, stats);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(fused_kernel<K>, grid, dim3(kBlock), 0, stream, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(project_kernel<K>, dim3((a.count + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t acc_blocks = std::min<int64_t>((items + kBlock / kWave - 1) / (kBlock / kWave), 65536);
    hipLaunchKernelGGL(accumulate_kernel<K>, dim3((unsigned)acc_blocks), dim3(kBlock), 0, stream, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = fill_u32(a.queue, 0u, 1, stream)) != hipSuccess) return e;
    const int bcap = bounce_waves(a.n, kWalkBlend);
    const int bwaves = items < bcap ? (int)items : bcap;
    hipLaunchKernelGGL(bounce_kernel<K>, dim3((bwaves + kBlock / kWave - 1) / (kBlock / kWave)), dim3(kBlock), 0,
                       stream, b);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const size_t count = (size_t)a.n * 3 * a.K;
    hipLaunchKernelGGL(add_parts_kernel, dim3((unsigned)std::min<size_t>((count + 255) / 256, 65536)), dim3(256), 0,
                       stream, a.transfer, b.partial, count, b.Q);
    return hipGetLastError();
}

// The index matrix in one walk per ray (the visibility with it), then, for a
// transfer, the projection.
template <int K>
hipError_t launch_index_fused_k(const TransferArgs& a, hipStream_t stream, bool project)
{
    hipError_t e = fill_u32(a.queue, 0u, 1, stream);
    if (e != hipSuccess) return e;
    TransferArgs b = a;
    b.Q = direction_parts(a.G, a.S, a.Q_req);
    const int64_t items = (int64_t)((a.count + a.G - 1) / a.G) * b.Q;
    const int cap = bounce_waves(a.n, kWalkIndex);
    const int waves = items < cap ? (int)items : cap;
    hipLaunchKernelGGL(fused_index_kernel<K>, dim3((waves + kBlock / kWave - 1) / (kBlock / kWave)), dim3(kBlock), 0,
                       stream, b);
    if ((e = hipGetLastError()) != hipSuccess || !project) return e;
    hipLaunchKernelGGL(project_kernel<K>, dim3((a.count + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_index_fused(const TransferArgs& a, hipStream_t stream, bool project)
{
    if (a.count <= 0) return hipSuccess;
    switch (a.K) {
        case 1: return launch_index_fused_k<1>(a, stream, project);
        case 4: return launch_index_fused_k<4>(a, stream, project);
        case 9: return launch_index_fused_k<9>(a, stream, project);
        case 16: return launch_index_fused_k<16>(a, stream, project);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_transfer_fused(const TransferArgs& a, hipStream_t stream)
{
    if (a.count <= 0) return hipSuccess;
    switch (a.K) {
        case 1: return launch_fused_k<1>(a, stream, nullptr);
        case 4: return launch_fused_k<4>(a, stream, nullptr);
        case 9: return launch_fused_k<9>(a, stream, nullptr);
        case 16: return launch_fused_k<16>(a, stream, nullptr);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fused_stats(const TransferArgs& a, hipStream_t stream, unsigned long long* stats)
{
    if (a.count <= 0) return hipSuccess;
    switch (a.K) {
        case 1: return launch_fused_k<1>(a, stream, stats);
        case 4: return launch_fused_k<4>(a, stream, stats);
        case 9: return launch_fused_k<9>(a, stream, stats);
        case 16: return launch_fused_k<16>(a, stream, stats);
        default: return hipErrorInvalidValue;
    }
}

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
        case 1: return launch_bounce_k<1, false>(a, stream);
        case 4: return launch_bounce_k<4, false>(a, stream);
        case 9: return launch_bounce_k<9, false>(a, stream);
        case 16: return launch_bounce_k<16, false>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bounce_stats(const TransferArgs& a, hipStream_t stream, unsigned long long* stats)
{
    if (a.count <= 0) return hipSuccess;
    switch (a.K) {
        case 1: return launch_bounce_k<1, false>(a, stream, stats);
        case 4: return launch_bounce_k<4, false>(a, stream, stats);
        case 9: return launch_bounce_k<9, false>(a, stream, stats);
        case 16: return launch_bounce_k<16, false>(a, stream, stats);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_transfer_index(const TransferArgs& a, hipStream_t stream)
{
    if (a.count <= 0) return hipSuccess;
    switch (a.K) {
        case 1: return launch_bounce_k<1, true>(a, stream);
        case 4: return launch_bounce_k<4, true>(a, stream);
        case 9: return launch_bounce_k<9, true>(a, stream);
        case 16: return launch_bounce_k<16, true>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

template <int K>
hipError_t launch_self_k(int n, int S, const float* dirs, const float* normals, const float* albedo,
                         const int32_t* index, const float* t_prev, int c_prev, float* t_out, unsigned* flags,
                         hipStream_t stream)
{
    const int blocks = (int)(((int64_t)n * kWave + kBlock - 1) / kBlock);
    if (c_prev == 3)
        hipLaunchKernelGGL((self_transfer_kernel<K, 3>), dim3(blocks), dim3(kBlock), 0, stream, n, S, dirs, normals,
                           albedo, index, t_prev, t_out, flags);
    else
        hipLaunchKernelGGL((self_transfer_kernel<K, 1>), dim3(blocks), dim3(kBlock), 0, stream, n, S, dirs, normals,
                           albedo, index, t_prev, t_out, flags);
    return hipGetLastError();
}

hipError_t launch_self_transfer(int n, int S, int K, const float* dirs, const float* normals, const float* albedo,
                                const int32_t* index, const float* t_prev, int c_prev, float* t_out, unsigned* flags,
                                hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    switch (K) {
        case 1: return launch_self_k<1>(n, S, dirs, normals, albedo, index, t_prev, c_prev, t_out, flags, stream);
        case 4: return launch_self_k<4>(n, S, dirs, normals, albedo, index, t_prev, c_prev, t_out, flags, stream);
        case 9: return launch_self_k<9>(n, S, dirs, normals, albedo, index, t_prev, c_prev, t_out, flags, stream);
        case 16: return launch_self_k<16>(n, S, dirs, normals, albedo, index, t_prev, c_prev, t_out, flags, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_add(float* acc, const float* x, size_t count, hipStream_t stream)
{
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(add_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, acc, x, count);
    return hipGetLastError();
}

}  // namespace prtgs
