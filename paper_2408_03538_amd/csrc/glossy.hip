// Glossy transfer matrices (Sec. 4.5, Eq. 36-41) with the BRDF of Sec. 4.2,
// and the per-frame view step that turns a matrix into a transfer vector.
//
// Per splat, over the S stratified directions (input index s, output p, both
// in the upper hemisphere of the normal):
//   t'_c[a][b] = wq^2 sum_s sum_p Y_a(s) T_c(s, p) Y_b(p),   wq = 4 pi / S
//   T_c(s, p)  = V_s c_s ((1 - m) rho_c / pi) + V_s G1(c_s) D(s, p) F_c(s, p) / (4 (c_p (1 - k) + k))
// (the Smith term of the output side divided by its c_p by hand; G1(x) =
// x / (x (1 - k) + k), D = GGX with alpha = r^2, k = (r + 1)^2 / 8).  With
// F_c = F0_c (1 - w) + w, w = (1 - wo.h)^5, the specular part splits into two
// channel-free matrices, t'_c = F0_c A + B + ((1 - m) rho_c / pi) t h^T, with
// t_a = wq sum_s Y_a V_s c_s and h_b = wq sum_p Y_b(p).
//
// One wave per splat.  The hemisphere's directions are listed in LDS; A and B
// are built 16 output directions at a time by v_mfma_f32_16x16x4_f32, each
// lane evaluating the BRDF for the (s, p) pair its B-operand slot holds, so
// the VALU does only the BRDF and the matrix cores the contraction over s;
// the 16 x 16 block U[a][p] then goes through LDS once for the contraction
// over p (a second MFMA chain).
#include "common.hpp"
#include "sh.hpp"

namespace prtgs {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kGlossyWaves = 4;   // waves per block, fewer when their LDS would pass 64 KB
constexpr int kPB = 2;            // 16-direction output blocks per pass over the input directions
constexpr int kPad = 16 * kPB;    // the hemisphere list is padded to a multiple of this
constexpr float kPi = 3.14159265358979323846f;

// A wave's LDS: the hemisphere list for up to S + kPad entries (direction w
// and c = n . w; n x w and V G1(c), or V G1(c) alone in the lean layout,
// which recomputes n x w per use; table row), the two U blocks in transit,
// and t, h.  The lean layout (24 instead of 36 bytes per entry) lets more
// waves share a CU where the list is long: at S = 512, 4 waves per block
// instead of 2 (1M x 512: 149 -> 124 ms); at S = 256 the stored n x w is 3%
// faster.
struct GlossyLds {
    float4* dir;
    float4* crs;   // n x w and V G1 (full layout)
    float* vg;     // V G1 (lean layout)
    int* idx;
    float (*u)[16][17];
    float (*red)[16];
};

__host__ __device__ inline size_t glossy_lds_bytes_per_wave(int S, bool lean)
{
    const size_t e = (size_t)S + kPad;
    return e * (lean ? 24 : 36) + 2 * 16 * 17 * 4 + 2 * 16 * 4;
}

// The lean layout where the full one would hold fewer than kGlossyWaves
// waves per block within 64 KB.
__host__ __device__ inline bool glossy_lean(int S)
{
    return kGlossyWaves * glossy_lds_bytes_per_wave(S, false) > 65536;
}

template <bool kLean>
__device__ inline GlossyLds glossy_lds(char* base, int S)
{
    const size_t e = (size_t)S + kPad;
    const size_t we = kLean ? 4 : 16;   // bytes of the second per-entry array
    GlossyLds L;
    L.dir = reinterpret_cast<float4*>(base);
    L.crs = reinterpret_cast<float4*>(base + e * 16);
    L.vg = reinterpret_cast<float*>(base + e * 16);
    L.idx = reinterpret_cast<int*>(base + e * (16 + we));
    L.u = reinterpret_cast<float(*)[16][17]>(base + e * (20 + we));
    L.red = reinterpret_cast<float(*)[16]>(base + e * (20 + we) + 2 * 16 * 17 * 4);
    return L;
}

__device__ inline float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int K, bool kLean>
__global__ __launch_bounds__(64 * kGlossyWaves) void glossy_kernel(int n, int S, const float* __restrict__ dirs,
                                                                   const float* __restrict__ Y,
                                                                   const float* __restrict__ normals,
                                                                   const float* __restrict__ albedo,
                                                                   const float* __restrict__ roughness,
                                                                   const float* __restrict__ metallic,
                                                                   const float* __restrict__ vis,
                                                                   float* __restrict__ out, unsigned* flags)
{
    extern __shared__ __align__(16) char glossy_smem[];
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int i = blockIdx.x * ((int)blockDim.x >> 6) + wave;
    if (i >= n) return;                  // whole waves only: each wave has its own LDS, no block barrier
    const GlossyLds L = glossy_lds<kLean>(glossy_smem + (size_t)wave * glossy_lds_bytes_per_wave(S, kLean), S);

    float nx = normals[3 * (size_t)i], ny = normals[3 * (size_t)i + 1], nz = normals[3 * (size_t)i + 2];
    const float r = roughness[i], m = metallic[i];
    const float rho[3] = {albedo[3 * (size_t)i], albedo[3 * (size_t)i + 1], albedo[3 * (size_t)i + 2]};
    const float nn = nx * nx + ny * ny + nz * nz;
    float* o = out + (size_t)i * 3 * K * K;
    if (!(nn > 0.0f && isfinite(nn) && r > 0.0f && r <= 1.0f && m >= 0.0f && m <= 1.0f)) {
        if (lane == 0) raise_flag(flags, PRTGS_FLAG_NONFINITE);
        for (int e = lane; e < 3 * K * K; e += 64) o[e] = 0.0f;
        return;
    }
    const float inv_n = rsqrtf(nn);
    nx *= inv_n;
    ny *= inv_n;
    nz *= inv_n;
    const float a2 = r * r * r * r;
    const float a2_pi = a2 / kPi;
    const float k = (r + 1.0f) * (r + 1.0f) * 0.125f, omk = 1.0f - k;
    const float wq = 4.0f * kPi / (float)S;

    // hemisphere list; t_a and h_b on the way
    const float* vrow = vis + (size_t)i * S;
    int H = 0;
    float t_part[K], h_part[K];
#pragma unroll
    for (int a = 0; a < K; ++a) t_part[a] = h_part[a] = 0.0f;
    for (int base = 0; base < S; base += 64) {
        const int s = base + lane;
        float wx = 0.0f, wy = 0.0f, wz = 0.0f, c = 0.0f;
        if (s < S) {
            wx = dirs[3 * s];
            wy = dirs[3 * s + 1];
            wz = dirs[3 * s + 2];
            c = nx * wx + ny * wy + nz * wz;
        }
        const bool up = s < S && c > 0.0f;
        const uint64_t ball = __ballot(up);
        if (up) {
            const int pos = H + __popcll(ball & ((1ull << lane) - 1ull));
            const float V = fmaxf(vrow[s], 0.0f);
            L.dir[pos] = make_float4(wx, wy, wz, c);
            if constexpr (kLean)
                L.vg[pos] = V * c / (c * omk + k);
            else
                L.crs[pos] = make_float4(ny * wz - nz * wy, nz * wx - nx * wz, nx * wy - ny * wx, V * c / (c * omk + k));
            L.idx[pos] = s;
#pragma unroll
            for (int a = 0; a < K; ++a) {
                const float y = Y[(size_t)s * K + a];
                t_part[a] = fmaf(y, V * c, t_part[a]);
                h_part[a] += y;
            }
        }
        H += __popcll(ball);
    }
    // pad to a whole number of kPad-entry blocks with finite, weightless entries
    const int Hp = (H + kPad - 1) & ~(kPad - 1);
    if (H + lane < Hp) {
        L.dir[H + lane] = make_float4(nx, ny, nz, 1.0f);
        if constexpr (kLean)
            L.vg[H + lane] = 0.0f;
        else
            L.crs[H + lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        L.idx[H + lane] = 0;
    }
#pragma unroll
    for (int a = 0; a < K; ++a) {
        const float tv = wave_sum(t_part[a]), hv = wave_sum(h_part[a]);
        if (lane == 0) {
            L.red[0][a] = wq * tv;
            L.red[1][a] = wq * hv;
        }
    }
    // the list is read across lanes from here on
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");

    const int col = lane & 15, quad = lane >> 4;
    f32x4 mA = {0.0f, 0.0f, 0.0f, 0.0f}, mB = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int p0 = 0; p0 < Hp; p0 += kPad) {
        // this lane's output directions (B-operand column) in the pass's blocks
        float4 wp[kPB], cp[kPB];
        float qp[kPB];
        f32x4 uA[kPB], uB[kPB];
#pragma unroll
        for (int b = 0; b < kPB; ++b) {
            const int pj = p0 + 16 * b + col;
            wp[b] = L.dir[pj];
            if constexpr (kLean)
                cp[b] = make_float4(ny * wp[b].z - nz * wp[b].y, nz * wp[b].x - nx * wp[b].z, nx * wp[b].y - ny * wp[b].x,
                                    0.0f);
            else
                cp[b] = L.crs[pj];
            qp[b] = pj < H ? 0.25f / (wp[b].w * omk + k) : 0.0f;
            uA[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            uB[b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        }
        for (int s0 = 0; s0 < Hp; s0 += 4) {
            const int js = s0 + quad;                     // this lane's input direction (B-operand row)
            const float4 ws = L.dir[js];
            const float4 cs = kLean ? make_float4(ny * ws.z - nz * ws.y, nz * ws.x - nx * ws.z, nx * ws.y - ny * ws.x,
                                                  L.vg[js])
                                    : L.crs[js];
            const int row = L.idx[js];
            // A operand: Y_a(s) with a = col
            const float ya = col < K ? Y[(size_t)row * K + col] : 0.0f;
#pragma unroll
            for (int b = 0; b < kPB; ++b) {
                // BRDF for (s, p) with the unnormalised half vector v = ws + wp:
                // D = alpha^2 / (pi x^2), x |v|^2 = |n x v|^2 + (n . v)^2 alpha^2
                // (no cancellation as n . h -> 1), and wo . h = |v| / 2
                const float hx = ws.x + wp[b].x, hy = ws.y + wp[b].y, hz = ws.z + wp[b].z;
                const float hl2 = fmaxf(hx * hx + hy * hy + hz * hz, 1e-30f);
                const float qx = cs.x + cp[b].x, qy = cs.y + cp[b].y, qz = cs.z + cp[b].z;
                const float nv = ws.w + wp[b].w;
                const float xh = fmaf(nv * nv, a2, qx * qx + qy * qy + qz * qz);
                const float voh = fminf(0.5f * hl2 * __builtin_amdgcn_rsqf(hl2), 1.0f);
                const float e = cs.w * a2_pi * (hl2 * hl2) * __builtin_amdgcn_rcpf(xh * xh);
                const float t1 = 1.0f - voh, t2 = t1 * t1;
                const float eB = e * (t2 * t2 * t1);
                const float eA = e - eB;
                uA[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ya, eA, uA[b], 0, 0, 0);
                uB[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(ya, eB, uB[b], 0, 0, 0);
            }
        }
#pragma unroll
        for (int b = 0; b < kPB; ++b) {
            // U[a][p] (a = 4 quad + j, p = col): scale by the output side's q_p and
            // pass through LDS as the A operand of the contraction over p
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                L.u[0][4 * quad + j][col] = uA[b][j] * qp[b];
                L.u[1][4 * quad + j][col] = uB[b][j] * qp[b];
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int pl = 4 * kk + quad;             // local output direction of this k slot
                const int rowp = L.idx[p0 + 16 * b + pl];
                const float yb = col < K ? Y[(size_t)rowp * K + col] : 0.0f;
                mA = __builtin_amdgcn_mfma_f32_16x16x4f32(L.u[0][col][pl], yb, mA, 0, 0, 0);
                mB = __builtin_amdgcn_mfma_f32_16x16x4f32(L.u[1][col][pl], yb, mB, 0, 0, 0);
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
    }
    // t'_c[a][b] = wq^2 (F0_c A + B) + (1 - m) rho_c / pi t_a h_b, lane holds a = 4 quad + j, b = col
    const float w2 = wq * wq;
    if (col < K) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int a = 4 * quad + j;
            if (a < K) {
                const float th = L.red[0][a] * L.red[1][col];
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const float F0 = 0.04f * (1.0f - m) + m * rho[ch];
                    o[((size_t)ch * K + a) * K + col] = w2 * fmaf(F0, mA[j], mB[j]) + (1.0f - m) * rho[ch] / kPi * th;
                }
            }
        }
    }
}

// z[i][c][a] = sum_b t'[i][c][a][b] Y_b(w_i), w_i = (eye - mu_i) / |eye - mu_i|;
// one wave per splat, lanes over (c, a).
template <int K>
__global__ void glossy_view_kernel(int n, const float* __restrict__ M, const float* __restrict__ means, float ex,
                                   float ey, float ez, float* __restrict__ z)
{
    const int i = blockIdx.x * 4 + ((int)threadIdx.x >> 6), lane = (int)threadIdx.x & 63;
    if (i >= n) return;
    const double dx = (double)ex - means[3 * (size_t)i], dy = (double)ey - means[3 * (size_t)i + 1],
                 dz = (double)ez - means[3 * (size_t)i + 2];
    const double len = sqrt(dx * dx + dy * dy + dz * dz);
    double yb[kMaxBands * kMaxBands];
    const int bands = K == 16 ? 4 : 3;
    if (len > 0.0) {
        real_sh(bands, dx / len, dy / len, dz / len, yb);
    } else {
        for (int b = 0; b < K; ++b) yb[b] = 0.0;
    }
    if (lane < 3 * K) {
        const float* row = M + ((size_t)i * 3 * K + lane) * K;
        float acc = 0.0f;
#pragma unroll
        for (int b = 0; b < K; ++b) acc = fmaf(row[b], (float)yb[b], acc);
        z[((size_t)i * 3) * K + lane] = acc;
    }
}

}  // namespace

hipError_t launch_glossy(int n, int S, int K, const float* dirs, const float* Y, const float* normals,
                         const float* albedo, const float* roughness, const float* metallic, const float* vis,
                         float* out, unsigned* flags, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const bool lean = glossy_lean(S);
    const size_t per_wave = glossy_lds_bytes_per_wave(S, lean);
    int waves = kGlossyWaves;
    while (waves > 1 && (size_t)waves * per_wave > 65536) --waves;
    const dim3 grid((n + waves - 1) / waves), block(64 * waves);
    const size_t lds = (size_t)waves * per_wave;
#define PRTGS_GLOSSY_LAUNCH(KK, LL)                                                                                  \
    hipLaunchKernelGGL((glossy_kernel<KK, LL>), grid, block, lds, stream, n, S, dirs, Y, normals, albedo, roughness, \
                       metallic, vis, out, flags)
    if (K == 16 && lean)
        PRTGS_GLOSSY_LAUNCH(16, true);
    else if (K == 16)
        PRTGS_GLOSSY_LAUNCH(16, false);
    else if (lean)
        PRTGS_GLOSSY_LAUNCH(9, true);
    else
        PRTGS_GLOSSY_LAUNCH(9, false);
#undef PRTGS_GLOSSY_LAUNCH
    return hipGetLastError();
}

hipError_t launch_glossy_view(int n, int K, const float* M, const float* means, const float eye[3], float* z,
                              hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const dim3 grid((n + 3) / 4), block(256);
    if (K == 16)
        hipLaunchKernelGGL(glossy_view_kernel<16>, grid, block, 0, stream, n, M, means, eye[0], eye[1], eye[2], z);
    else
        hipLaunchKernelGGL(glossy_view_kernel<9>, grid, block, 0, stream, n, M, means, eye[0], eye[1], eye[2], z);
    return hipGetLastError();
}

}  // namespace prtgs
