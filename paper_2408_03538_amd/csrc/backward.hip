// Adjoint of the direct transfer (Eq. 7, 9, 29 with alpha at the peak of
// each Gaussian along the ray): dLoss/d(mean, quaternion, log-scale,
// opacity, normal) from dLoss/dt_dir.
//
// For a traced ray of source i in direction w, with V = prod(1 - alpha_j)
// over its hits and g = (4 pi / S) sum_k dt_i[k] Y_k(w):
//   dLoss/dV = g c,  dLoss/dc = g V  (c = n_i . w, so dn_i += g V w),
//   dLoss/dalpha_j = -g c V / (1 - alpha_j),
//   alpha_j = o_j exp(-d_j^2 / 2):  d o_j = dalpha E_j,  d(d_j^2) = -dalpha alpha_j / 2,
//   d_j^2 = |p|^2 with p = W_j (x* - mu_j), x* = mu_i + t* w; t* minimises d^2
//   along the ray, so d(d^2) = 2 p . (dW (x* - mu_j) + W (dmu_i - dmu_j)).
// Rays whose transmittance fell below T_eps have V held at 0 and carry no
// gradient; a clamped alpha (alpha_max) has none either.  Each ray is
// traced twice: once for V, once to scatter the per-hit terms.  Lanes of a
// wave visit Gaussians together (packet traversal), so the per-Gaussian
// terms are summed across the wave first and added with one set of atomics.
#include "trace.hpp"

namespace prtgs {

namespace {

constexpr int kBlock = 256;
constexpr float kFourPi = 12.566370614359172f;

__device__ inline float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ inline float segment_sum(float v, int D)
{
    for (int off = D / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

struct BatchDir {
    float mean[3];
    int oct;
    bool uniform_oct;
};

// Mean direction of the traced lanes and whether they share an octant.
__device__ inline BatchDir batch_dir(const RayDir& d, bool traced)
{
    BatchDir b;
    b.mean[0] = traced ? d.wx : 0.0f;
    b.mean[1] = traced ? d.wy : 0.0f;
    b.mean[2] = traced ? d.wz : 0.0f;
#pragma unroll
    for (int q = 0; q < 3; ++q) b.mean[q] = wave_sum(b.mean[q]);
    const int first = __builtin_ctzll(__ballot(traced));
    const int oct = octant(d);
    b.oct = __builtin_amdgcn_readlane(oct, first);
    b.uniform_oct = __ballot(traced && oct != b.oct) == 0ull;
    return b;
}

template <class LeafFn>
__device__ inline void traverse_batch(const TransferArgs& a, const RayDir& d, const BatchDir& bd, float ox, float oy,
                                      float oz, bool& live, float& tlo, float& thi, LeafFn& leaf)
{
    if (bd.uniform_oct)
        packet_traverse<false, true, kLeavesFirst>(a.nodes, a.n, d, ox, oy, oz, live, tlo, thi, a.flags, leaf,
                                                   nullptr, bd.mean, bd.oct);
    else
        packet_traverse<false, false, kLeavesFirst>(a.nodes, a.n, d, ox, oy, oz, live, tlo, thi, a.flags, leaf,
                                                    nullptr, bd.mean, 0);
}

template <int K>
__global__ __launch_bounds__(kBlock) void transfer_backward_kernel(BackwardArgs ba)
{
    const TransferArgs& a = ba.fwd;
    const int lane = threadIdx.x & (kWave - 1);
    const int G = a.G;
    const int D = kWave / G;
    // direction parts taken part-major, as in the forward pass (spare waves
    // of the last block get part >= Q: no work)
    const int gwave = (int)(((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave);
    const int groups = (a.count + G - 1) / G;
    const int part = gwave / groups;
    const int local = (gwave % groups) * G + lane / D;
    const bool valid = local < a.count && part < a.Q;
    const int rank = valid ? local : 0;
    const float4 mo = a.prims[rank].mo;
    const float ox = mo.x, oy = mo.y, oz = mo.z;
    const float4 nrm = a.normals[rank];
    const int orig = a.order[rank];
    const HitParams hp = a.hp;

    float dt[K];
#pragma unroll
    for (int k = 0; k < K; ++k) dt[k] = valid ? ba.d_transfer[(size_t)orig * K + k] : 0.0f;
    float gmi[3] = {0.0f, 0.0f, 0.0f};   // dLoss/dmu_i through the ray origin
    float gni[3] = {0.0f, 0.0f, 0.0f};   // dLoss/dn_i
    const float wq = kFourPi / (float)a.S;

    const int nb = (a.S + D - 1) / D;
    for (int bi = part * nb / a.Q; bi < (part + 1) * nb / a.Q; ++bi) {
        const int b0 = bi * D;
        const int pos = b0 + (lane % D);
        const bool inrange = pos < a.S;
        const int s = inrange ? a.dir_order[pos] : 0;
        const RayDir d = make_dir(a.dirs[3 * s], a.dirs[3 * s + 1], a.dirs[3 * s + 2]);
        const float c = nrm.x * d.wx + nrm.y * d.wy + nrm.z * d.wz;
        const bool traced = valid && inrange && c > 0.0f;
        if (__ballot(traced) == 0ull) continue;
        float g = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) g = fmaf(dt[k], a.Y[(size_t)s * K + k], g);
        g *= wq;
        const BatchDir bd = batch_dir(d, traced);
        bool live = traced;
        float T = 1.0f;
        float tlo = hp.t_min, thi = INFINITY;
        if (ba.vis_in) {
            // the forward's visibility of this ray (negative: not traced there)
            T = traced ? fmaxf(ba.vis_in[(size_t)orig * a.S + s], 0.0f) : 0.0f;
        } else {
            // pass 1: transmittance
            auto leaf1 = [&](int r, bool box_hit) {
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
            traverse_batch(a, d, bd, ox, oy, oz, live, tlo, thi, leaf1);
        }
        const bool carries = traced && T > 0.0f;
        if (carries) {
            gni[0] += g * T * d.wx;
            gni[1] += g * T * d.wy;
            gni[2] += g * T * d.wz;
        }
        if (__ballot(carries && g != 0.0f) == 0ull) continue;
        // pass 2: per-hit adjoint (the same hits: these lanes ran pass 1 to the end)
        const float gV = g * c * T;   // dLoss/dV times V
        live = carries && g != 0.0f;
        tlo = hp.t_min;
        thi = INFINITY;
        auto leaf2 = [&](int r, bool box_hit) {
            const Prim p = uniform_load(a.prims, r);
            const PreHit q = gaussian_pre(p, ox, oy, oz, d, hp);
            const bool cand = q.maybe & box_hit & live & (r != rank);
            if (__ballot(cand) == 0ull) return;
            HitResult h;
            const bool hit = gaussian_exact(p, q, ox, oy, oz, d, hp, h) & cand;
            const bool contrib = hit & (p.mo.w * h.E < hp.alpha_max);   // a clamped alpha has no gradient
            float go = 0.0f, gw[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, gm[3] = {0, 0, 0};
            if (contrib) {
                const float alpha = h.alpha;
                const float dal = -gV / (1.0f - alpha);
                go = dal * h.E;
                const float dd2 = -0.5f * dal * alpha;
                const float q0 = 2.0f * dd2 * h.p0, q1 = 2.0f * dd2 * h.p1, q2 = 2.0f * dd2 * h.p2;
                // d(d^2)/dW = 2 p (x* - mu_j)^T
                gw[0] = q0 * h.x0; gw[1] = q0 * h.x1; gw[2] = q0 * h.x2;
                gw[3] = q1 * h.x0; gw[4] = q1 * h.x1; gw[5] = q1 * h.x2;
                gw[6] = q2 * h.x0; gw[7] = q2 * h.x1; gw[8] = q2 * h.x2;
                // d(d^2)/dmu_i = -d(d^2)/dmu_j = 2 W^T p
                const float u0 = p.w0.x * q0 + p.w1.x * q1 + p.w2.x * q2;
                const float u1 = p.w0.y * q0 + p.w1.y * q1 + p.w2.y * q2;
                const float u2 = p.w0.z * q0 + p.w1.z * q1 + p.w2.z * q2;
                gm[0] = -u0; gm[1] = -u1; gm[2] = -u2;
                gmi[0] += u0; gmi[1] += u1; gmi[2] += u2;
            }
            const uint64_t who = __ballot(contrib);
            if (who == 0ull) return;
            if (__popcll(who) == 1) {
                if (contrib) {
                    atomicAdd(&ba.g_o[r], go);
                    for (int k = 0; k < 9; ++k) atomicAdd(&ba.g_W[9 * (size_t)r + k], gw[k]);
                    for (int k = 0; k < 3; ++k) atomicAdd(&ba.g_mu[3 * (size_t)r + k], gm[k]);
                }
                return;
            }
            go = wave_sum(go);
#pragma unroll
            for (int k = 0; k < 9; ++k) gw[k] = wave_sum(gw[k]);
#pragma unroll
            for (int k = 0; k < 3; ++k) gm[k] = wave_sum(gm[k]);
            if (lane == 0) {
                atomicAdd(&ba.g_o[r], go);
                for (int k = 0; k < 9; ++k) atomicAdd(&ba.g_W[9 * (size_t)r + k], gw[k]);
                for (int k = 0; k < 3; ++k) atomicAdd(&ba.g_mu[3 * (size_t)r + k], gm[k]);
            }
        };
        traverse_batch(a, d, bd, ox, oy, oz, live, tlo, thi, leaf2);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        gmi[q] = segment_sum(gmi[q], D);
        gni[q] = segment_sum(gni[q], D);
    }
    if (!valid || (lane % D) != 0) return;
    for (int q = 0; q < 3; ++q) {
        atomicAdd(&ba.g_mu[3 * (size_t)rank + q], gmi[q]);
        atomicAdd(&ba.g_n[3 * (size_t)rank + q], gni[q]);   // the source's other parts add theirs
    }
}

// Per Gaussian: chain dW into d(log s) and d(quaternion) and add every
// gradient into the caller's buffers (original order).  W = diag(1/s) R^T,
// so dlog s_a = -sum_b dW_ab W_ab and dR_ba = dW_ab / s_a; R(q/|q|) is
// differentiated by hand and the normalisation projected out.
__global__ void backward_finalize_kernel(BackwardArgs ba)
{
    const TransferArgs& a = ba.fwd;
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n) return;
    const int j = a.order[r];
    const prtgs_grads& out = ba.out;
    if (out.d_opacity) out.d_opacity[j] += ba.g_o[r];
    if (out.d_means)
        for (int q = 0; q < 3; ++q) out.d_means[3 * (size_t)j + q] += ba.g_mu[3 * (size_t)r + q];
    if (out.d_normals)
        for (int q = 0; q < 3; ++q) out.d_normals[3 * (size_t)j + q] += ba.g_n[3 * (size_t)r + q];
    if (!out.d_log_scales && !out.d_quats) return;
    float gW[3][3];
    for (int q = 0; q < 9; ++q) gW[q / 3][q % 3] = ba.g_W[9 * (size_t)r + q];
    const Prim p = uniform_load(a.prims, r);
    const float W[3][3] = {{p.w0.x, p.w0.y, p.w0.z}, {p.w1.x, p.w1.y, p.w1.z}, {p.w2.x, p.w2.y, p.w2.z}};
    if (out.d_log_scales)
        for (int aa = 0; aa < 3; ++aa)
            out.d_log_scales[3 * (size_t)j + aa] -= gW[aa][0] * W[aa][0] + gW[aa][1] * W[aa][1] + gW[aa][2] * W[aa][2];
    if (!out.d_quats) return;
    float is[3];
    for (int aa = 0; aa < 3; ++aa) is[aa] = expf(-ba.log_scales[3 * (size_t)j + aa]);
    float dR[3][3];   // dR[b][a] = gW[a][b] / s_a
    for (int aa = 0; aa < 3; ++aa)
        for (int b = 0; b < 3; ++b) dR[b][aa] = gW[aa][b] * is[aa];
    float qw = ba.quats[4 * (size_t)j], qx = ba.quats[4 * (size_t)j + 1], qy = ba.quats[4 * (size_t)j + 2],
          qz = ba.quats[4 * (size_t)j + 3];
    const float qn = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    if (!(qn > 0.0f)) return;
    const float w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
    float gw_ = 2.0f * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
    float gx = 2.0f * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2.0f * x * dR[1][1] - w * dR[1][2] + z * dR[2][0] +
                       w * dR[2][1] - 2.0f * x * dR[2][2]);
    float gy = 2.0f * (-2.0f * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] - w * dR[2][0] +
                       z * dR[2][1] - 2.0f * y * dR[2][2]);
    float gz = 2.0f * (-2.0f * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] - 2.0f * z * dR[1][1] +
                       y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
    const float dotq = gw_ * w + gx * x + gy * y + gz * z;
    out.d_quats[4 * (size_t)j + 0] += (gw_ - w * dotq) / qn;
    out.d_quats[4 * (size_t)j + 1] += (gx - x * dotq) / qn;
    out.d_quats[4 * (size_t)j + 2] += (gy - y * dotq) / qn;
    out.d_quats[4 * (size_t)j + 3] += (gz - z * dotq) / qn;
}

template <int K>
hipError_t launch_bwd_k(const BackwardArgs& a, hipStream_t stream)
{
    BackwardArgs b = a;
    b.fwd.Q = direction_parts(a.fwd.G, a.fwd.S, a.fwd.Q_req);
    const int64_t waves = (int64_t)((a.fwd.count + a.fwd.G - 1) / a.fwd.G) * b.fwd.Q;
    const int blocks = (int)((waves + kBlock / kWave - 1) / (kBlock / kWave));
    hipLaunchKernelGGL(transfer_backward_kernel<K>, dim3(blocks), dim3(kBlock), 0, stream, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(backward_finalize_kernel, dim3((a.fwd.n + 255) / 256), dim3(256), 0, stream, b);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_transfer_backward(const BackwardArgs& a, hipStream_t stream)
{
    switch (a.fwd.K) {
        case 1: return launch_bwd_k<1>(a, stream);
        case 4: return launch_bwd_k<4>(a, stream);
        case 9: return launch_bwd_k<9>(a, stream);
        case 16: return launch_bwd_k<16>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace prtgs
