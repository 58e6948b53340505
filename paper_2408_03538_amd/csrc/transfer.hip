// Transfer precompute: visibility along S directions from every splat centre
// through the other Gaussians (Sec. 4.4), projected with max(0, n.w) onto
// real SH (Eq. 7, 9, 29), and the one-bounce self-transfer (Eq. 20-22,
// 30-33) with the hits of each ray blended front to back.
//
// Work split: lane = source splat (64 Morton-adjacent sources per wave),
// loop over directions inside the lane, one packet traversal per direction
// (trace.hpp).  Each lane owns its source's SH accumulators, so the
// projection needs no cross-lane reduction; it is a compensated (Kahan) sum
// over directions.
#include "trace.hpp"

namespace prtgs {

namespace {

constexpr int kBlock = 256;
constexpr float kFourPi = 12.566370614359172f;

__device__ inline void kahan_add(float& sum, float& comp, float x)
{
    float y = x - comp;
    float t = sum + y;
    comp = (t - sum) - y;
    sum = t;
}

// stats (kCount): [0] traced rays, [1] child-box tests, [2] Gaussian tests
// (single-ray work, summed over rays), [3] wave node visits, [4] wave
// Gaussian-record visits (summed over waves and directions).
template <int K, bool kCount>
__global__ __launch_bounds__(kBlock) void direct_kernel(TransferArgs a, unsigned long long* stats)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int local = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = local < a.count;
    const int rank = a.first + (valid ? local : 0);
    const Prim src = a.prims[rank];
    const float ox = src.mo.x, oy = src.mo.y, oz = src.mo.z;
    const float nx = src.w0.w, ny = src.w1.w, nz = src.w2.w;
    const int orig = valid ? a.order[rank] : 0;
    (void)lane;

    float acc[K], cmp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        acc[k] = 0.0f;
        cmp[k] = 0.0f;
    }
    const HitParams hp = a.hp;
    RayCounts cnt;
    uint32_t traced_rays = 0;
    for (int s = 0; s < a.S; ++s) {
        const RayDir d = make_dir(uniform_load(a.dirs, 3 * s), uniform_load(a.dirs, 3 * s + 1),
                                 uniform_load(a.dirs, 3 * s + 2));
        const float c = nx * d.wx + ny * d.wy + nz * d.wz;
        const bool traced = valid && c > 0.0f;
        float V = -1.0f;
        if (kCount && traced) ++traced_rays;
        if (__ballot(traced) != 0ull) {
            bool live = traced;
            float T = 1.0f;
            float tlo = hp.t_min, thi = INFINITY;
            packet_traverse<kCount>(a.nodes, a.n, d, ox, oy, oz, live, tlo, thi, a.flags, [&](int r) {
                const Prim p = uniform_load(a.prims, r);
                HitResult h;
                if (live && r != rank && gaussian_hit(p, ox, oy, oz, d, hp, h)) {
                    T *= 1.0f - h.alpha;
                    if (T < hp.T_eps) {
                        live = false;
                        T = 0.0f;
                    }
                }
            }, &cnt);
            if (traced) {
                V = T;
                const float f = V * c;
#pragma unroll
                for (int k = 0; k < K; ++k) kahan_add(acc[k], cmp[k], f * uniform_load(a.Y, s * K + k));
            }
        }
        if (!kCount && a.vis && valid) a.vis[(size_t)orig * a.S + s] = V;
    }
    if (kCount) {
        atomicAdd(&stats[0], (unsigned long long)traced_rays);
        atomicAdd(&stats[1], (unsigned long long)cnt.box_tests);
        atomicAdd(&stats[2], (unsigned long long)cnt.prim_tests);
        if ((threadIdx.x & (kWave - 1)) == 0) {
            atomicAdd(&stats[3], (unsigned long long)cnt.wave_nodes);
            atomicAdd(&stats[4], (unsigned long long)cnt.wave_leaves);
        }
        return;
    }
    if (!valid) return;
    const float scale = kFourPi / (float)a.S;
    for (int ch = 0; ch < a.channels; ++ch) {
        float* out = a.transfer + ((size_t)orig * a.channels + ch) * K;
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] = acc[k] * scale;
    }
    if (a.tdir_sorted) {
#pragma unroll
        for (int k = 0; k < K; ++k) a.tdir_sorted[(size_t)rank * K + k] = acc[k] * scale;
    }
}

// Strict order of hits along a ray: by t*, then by leaf rank.
__device__ inline bool key_less(float ta, int ja, float tb, int jb) { return ta < tb || (ta == tb && ja < jb); }

template <int K, int KB>
__global__ __launch_bounds__(kBlock) void bounce_kernel(TransferArgs a)
{
    const int local = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = local < a.count;
    const int rank = a.first + (valid ? local : 0);
    const Prim src = a.prims[rank];
    const float ox = src.mo.x, oy = src.mo.y, oz = src.mo.z;
    const float nx = src.w0.w, ny = src.w1.w, nz = src.w2.w;
    const int orig = valid ? a.order[rank] : 0;
    const HitParams hp = a.hp;
    constexpr float kInvPi = 0.31830988618379067f;

    float acc[3][K];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[ch][k] = 0.0f;

    for (int s = 0; s < a.S; ++s) {
        const RayDir d = make_dir(uniform_load(a.dirs, 3 * s), uniform_load(a.dirs, 3 * s + 1),
                                 uniform_load(a.dirs, 3 * s + 2));
        const float c = nx * d.wx + ny * d.wy + nz * d.wz;
        bool pending = valid && c > 0.0f;
        float T = 1.0f;
        float t_last = -INFINITY;
        int j_last = -1;
        // Rounds: gather the KB nearest hits beyond the last processed one,
        // then blend them in order; repeat while the buffer came back full.
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
            int m = 0;
            bool live = pending;
            float tlo = fmaxf(hp.t_min, t_last), thi = INFINITY;
            packet_traverse(a.nodes, a.n, d, ox, oy, oz, live, tlo, thi, a.flags, [&](int r) {
                const Prim p = uniform_load(a.prims, r);
                HitResult h;
                if (live && r != rank && gaussian_hit(p, ox, oy, oz, d, hp, h) && key_less(t_last, j_last, h.t, r) &&
                    key_less(h.t, r, bt[KB - 1], bj[KB - 1])) {
                    float ct = h.t, ca = h.alpha;
                    int cj = r;
#pragma unroll
                    for (int q = 0; q < KB; ++q) {
                        if (key_less(ct, cj, bt[q], bj[q])) {
                            float tt = bt[q]; bt[q] = ct; ct = tt;
                            int tj = bj[q]; bj[q] = cj; cj = tj;
                            float ta = ba[q]; ba[q] = ca; ca = ta;
                        }
                    }
                    m = m < KB ? m + 1 : KB;
                    if (m == KB) thi = bt[KB - 1];
                }
            });
            if (pending) {
#pragma unroll
                for (int q = 0; q < KB; ++q) {
                    if (q < m && pending) {
                        const int r = bj[q];
                        const float w = ba[q] * T;
                        const int jo = a.order[r];
                        const float wc = w * c * kInvPi;
                        const float rho[3] = {a.albedo[3 * (size_t)jo] * wc, a.albedo[3 * (size_t)jo + 1] * wc,
                                              a.albedo[3 * (size_t)jo + 2] * wc};
                        const float* td = a.tdir_sorted + (size_t)r * K;
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            const float v = td[k];
                            acc[0][k] = fmaf(rho[0], v, acc[0][k]);
                            acc[1][k] = fmaf(rho[1], v, acc[1][k]);
                            acc[2][k] = fmaf(rho[2], v, acc[2][k]);
                        }
                        T *= 1.0f - ba[q];
                        t_last = bt[q];
                        j_last = r;
                        if (T < hp.T_eps) pending = false;
                    }
                }
                if (m < KB) pending = false;
            }
        }
    }
    if (!valid) return;
    const float scale = kFourPi / (float)a.S;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float* out = a.transfer + ((size_t)orig * 3 + ch) * K;
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] += acc[ch][k] * scale;
    }
}

template <int K>
hipError_t launch_direct_k(const TransferArgs& a, unsigned long long* stats, hipStream_t stream)
{
    int blocks = (a.count + kBlock - 1) / kBlock;
    if (stats)
        hipLaunchKernelGGL((direct_kernel<K, true>), dim3(blocks), dim3(kBlock), 0, stream, a, stats);
    else
        hipLaunchKernelGGL((direct_kernel<K, false>), dim3(blocks), dim3(kBlock), 0, stream, a, stats);
    return hipGetLastError();
}

template <int K>
hipError_t launch_bounce_k(const TransferArgs& a, hipStream_t stream)
{
    int blocks = (a.count + kBlock - 1) / kBlock;
    hipLaunchKernelGGL((bounce_kernel<K, 8>), dim3(blocks), dim3(kBlock), 0, stream, a);
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
