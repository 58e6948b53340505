// Gaussian splatting of per-splat colours (the 3DGS rasterizer the paper
// renders with, Sec. 3.1: Sigma = R S S^T R^T, the 2D footprint
// Sigma' = J W Sigma W^T J^T, front-to-back alpha blending of Eq. 4).
//
// Per frame: project every Gaussian (footprint, screen centre, the radius
// beyond which its alpha is below 1/255), bin it into the 16 x 16-pixel
// tiles its footprint square touches, sort the (tile, depth) keys, find each
// tile's range, and blend each tile's Gaussians front to back in one block
// per tile with batches staged in LDS.
#include <cstring>

#include "common.hpp"
#include "sort.hpp"

namespace prtgs {

namespace {

constexpr int kTile = 16;
constexpr int kTilePixels = kTile * kTile;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTStop = 1e-4f;
constexpr float kDilate = 0.3f;   // low-pass added to the 2D covariance (pixels^2)
constexpr int kSub = 8;           // a wave's share of a tile: an 8 x 8-pixel quarter
constexpr int kUnroll = 8;        // Gaussians evaluated together in the blend loop

// Smallest value of q(x, y) = A dx^2 + 2 B dx dy + C dy^2 (dx = x - u, dy = y - v)
// over the rectangle [x0, x1] x [y0, y1]: 0 with the centre inside, else the
// least of the four edges' minima (q is convex, each edge is a clamped 1-D
// quadratic).  A, C > 0 (a positive definite conic).
__device__ inline float rect_min_q(float u, float v, float A, float B, float C, float x0, float y0, float x1,
                                   float y1)
{
    if (u >= x0 && u <= x1 && v >= y0 && v <= y1) return 0.0f;
    const float ex0 = x0 - u, ex1 = x1 - u, ey0 = y0 - v, ey1 = y1 - v;
    auto along_y = [&](float dx) {   // edge x = u + dx, y free in [y0, y1]
        const float dy = fminf(fmaxf(-B * dx / C, ey0), ey1);
        return A * dx * dx + 2.0f * B * dx * dy + C * dy * dy;
    };
    auto along_x = [&](float dy) {   // edge y = v + dy
        const float dx = fminf(fmaxf(-B * dy / A, ex0), ex1);
        return A * dx * dx + 2.0f * B * dx * dy + C * dy * dy;
    };
    return fminf(fminf(along_y(ex0), along_y(ex1)), fminf(along_x(ey0), along_x(ey1)));
}

// Does the ellipse q <= cut reach a pixel centre of the given pixel block
// (clipped to the image)?
__device__ inline bool block_touched(float4 uvc, float4 co, int px0, int py0, int size, int width, int height)
{
    const float x0 = (float)px0 + 0.5f, y0 = (float)py0 + 0.5f;
    const float x1 = (float)(min(px0 + size, width) - 1) + 0.5f, y1 = (float)(min(py0 + size, height) - 1) + 0.5f;
    return rect_min_q(uvc.x, uvc.y, co.x, co.y, co.z, x0, y0, x1, y1) <= uvc.z;
}

__global__ void splat_preprocess_kernel(int n, SplatCamera cam, const float* __restrict__ means,
                                        const float* __restrict__ quats, const float* __restrict__ log_scales,
                                        const float* __restrict__ opacity, float4* __restrict__ uv,
                                        float4* __restrict__ conic_o, float* __restrict__ depth,
                                        int4* __restrict__ rect, uint32_t* __restrict__ count, unsigned* flags)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    count[i] = 0;
    const float mx = means[3 * (size_t)i], my = means[3 * (size_t)i + 1], mz = means[3 * (size_t)i + 2];
    const float o = opacity[i];
    float qw = quats[4 * (size_t)i], qx = quats[4 * (size_t)i + 1], qy = quats[4 * (size_t)i + 2],
          qz = quats[4 * (size_t)i + 3];
    const float s0 = expf(log_scales[3 * (size_t)i]), s1 = expf(log_scales[3 * (size_t)i + 1]),
                s2 = expf(log_scales[3 * (size_t)i + 2]);
    const float qn2 = qw * qw + qx * qx + qy * qy + qz * qz;
    if (!(finite3(mx, my, mz) && isfinite(o) && finite3(s0, s1, s2) && qn2 > 0.0f && isfinite(qn2))) {
        raise_flag(flags, PRTGS_FLAG_NONFINITE);
        return;
    }
    // camera space
    const float* V = cam.view;
    const float x = V[0] * mx + V[1] * my + V[2] * mz + V[3];
    const float y = V[4] * mx + V[5] * my + V[6] * mz + V[7];
    const float z = V[8] * mx + V[9] * my + V[10] * mz + V[11];
    if (!(z >= cam.near_z)) return;
    const float dmax2 = 2.0f * logf(255.0f * o);   // alpha >= 1/255 inside x^T conic x <= dmax2
    if (!(dmax2 > 0.0f)) return;
    // Sigma = R S S^T R^T, R from the normalised quaternion
    const float inv = rsqrtf(qn2);
    qw *= inv;
    qx *= inv;
    qy *= inv;
    qz *= inv;
    const float R[3][3] = {{1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
                           {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
                           {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
    const float s[3] = {s0 * s0, s1 * s1, s2 * s2};
    // M = W R (camera rotation times Gaussian rotation); Sigma_c = M diag(s^2) M^T
    float M[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) M[r][c] = V[4 * r] * R[0][c] + V[4 * r + 1] * R[1][c] + V[4 * r + 2] * R[2][c];
    // the Jacobian of the projection at the centre, its x/z, y/z held inside 1.3 x the frustum
    const float tx = fminf(fmaxf(x / z, cam.lim[0]), cam.lim[1]) * z;
    const float ty = fminf(fmaxf(y / z, cam.lim[2]), cam.lim[3]) * z;
    const float iz = 1.0f / z;
    const float J00 = cam.fx * iz, J02 = -cam.fx * tx * iz * iz;
    const float J11 = cam.fy * iz, J12 = -cam.fy * ty * iz * iz;
    // T = J M (2 x 3); Sigma' = T diag(s^2) T^T
    float T0[3], T1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T0[c] = J00 * M[0][c] + J02 * M[2][c];
        T1[c] = J11 * M[1][c] + J12 * M[2][c];
    }
    const float a = T0[0] * T0[0] * s[0] + T0[1] * T0[1] * s[1] + T0[2] * T0[2] * s[2] + kDilate;
    const float b = T0[0] * T1[0] * s[0] + T0[1] * T1[1] * s[1] + T0[2] * T1[2] * s[2];
    const float c = T1[0] * T1[0] * s[0] + T1[1] * T1[1] * s[1] + T1[2] * T1[2] * s[2] + kDilate;
    const float det = a * c - b * b;
    if (!(det > 0.0f)) return;
    const float idet = 1.0f / det;
    // the cut q <= dmax2 with a margin over float32 rounding of q (relative
    // error a few eps times the footprint's condition number)
    const float mid = 0.5f * (a + c);
    const float root = sqrtf(fmaxf(mid * mid - det, 0.0f));
    const float kappa = (mid + root) * (mid + root) / det;
    const float cut = dmax2 * (1.0f + 1e-3f + 64.0f * 5.96e-8f * kappa);
    const float u = cam.fx * x * iz + cam.cx, v = cam.fy * y * iz + cam.cy;
    // the ellipse's bounding box: half-widths sqrt(Sigma'_xx cut), sqrt(Sigma'_yy cut)
    const float rx = sqrtf(a * cut) + 1e-3f, ry = sqrtf(c * cut) + 1e-3f;
    const int ntx = (cam.width + kTile - 1) / kTile, nty = (cam.height + kTile - 1) / kTile;
    const float fx0 = floorf((u - rx - 0.5f) / kTile), fx1 = floorf((u + rx - 0.5f) / kTile);
    const float fy0 = floorf((v - ry - 0.5f) / kTile), fy1 = floorf((v + ry - 0.5f) / kTile);
    // off screen (or not finite): nothing to draw; clamp in float before converting
    if (!(fx1 >= 0.0f && fx0 <= (float)(ntx - 1) && fy1 >= 0.0f && fy0 <= (float)(nty - 1))) return;
    const int x0 = (int)fmaxf(fx0, 0.0f), x1 = (int)fminf(fx1, (float)(ntx - 1));
    const int y0 = (int)fmaxf(fy0, 0.0f), y1 = (int)fminf(fy1, (float)(nty - 1));
    const float4 uvc = make_float4(u, v, cut, 0.0f);
    const float4 co = make_float4(c * idet, -b * idet, a * idet, o);
    // the tiles of the box that the ellipse reaches
    uint32_t k = 0;
    for (int ty = y0; ty <= y1; ++ty)
        for (int tx = x0; tx <= x1; ++tx)
            k += block_touched(uvc, co, tx * kTile, ty * kTile, kTile, cam.width, cam.height) ? 1u : 0u;
    if (k == 0) return;
    uv[i] = uvc;
    conic_o[i] = co;
    depth[i] = z;
    rect[i] = make_int4(x0, y0, x1, y1);
    count[i] = k;
}

__global__ void splat_total_kernel(int n, const uint64_t* __restrict__ offset, const uint32_t* __restrict__ count,
                                   unsigned long long* __restrict__ total)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *total = offset[n - 1] + count[n - 1];
}

// One (tile, depth) key per tile the Gaussian reaches, in the order the count
// was taken; should the test ever come out differently here, the slots left
// over get a tile number past the last, which sorts to the end and is ignored.
__global__ void splat_duplicate_kernel(int n, SplatCamera cam, int ntx, int ntiles,
                                       const uint64_t* __restrict__ offset, const uint32_t* __restrict__ count,
                                       const int4* __restrict__ rect, const float4* __restrict__ uv,
                                       const float4* __restrict__ conic_o, const float* __restrict__ depth,
                                       uint64_t* __restrict__ keys, uint32_t* __restrict__ vals, int64_t max_instances)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t cnt = count[i];
    if (cnt == 0) return;
    const int4 rc = rect[i];
    const uint64_t e0 = offset[i];
    if ((int64_t)(e0 + cnt) > max_instances) return;   // the host reports the shortfall
    const float4 uvc = uv[i], co = conic_o[i];
    // depth > 0, so its bit pattern orders like the value
    const uint64_t d = __float_as_uint(depth[i]);
    uint32_t k = 0;
    for (int ty = rc.y; ty <= rc.w && k < cnt; ++ty)
        for (int tx = rc.x; tx <= rc.z && k < cnt; ++tx)
            if (block_touched(uvc, co, tx * kTile, ty * kTile, kTile, cam.width, cam.height)) {
                keys[e0 + k] = ((uint64_t)(ty * ntx + tx) << 32) | d;
                vals[e0 + k] = (uint32_t)i;
                ++k;
            }
    for (; k < cnt; ++k) {
        keys[e0 + k] = ((uint64_t)ntiles << 32) | d;
        vals[e0 + k] = (uint32_t)i;
    }
}

__global__ void splat_ranges_kernel(int64_t total, uint32_t ntiles, const uint64_t* __restrict__ keys,
                                    uint2* __restrict__ ranges)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const uint32_t tile = (uint32_t)(keys[e] >> 32);
    if (tile >= ntiles) return;
    if (e == 0 || (uint32_t)(keys[e - 1] >> 32) != tile) ranges[tile].x = (uint32_t)e;
    if (e == total - 1 || (uint32_t)(keys[e + 1] >> 32) != tile) ranges[tile].y = (uint32_t)(e + 1);
}

// One block per 16 x 16 tile, one wave per 8 x 8 quarter.  The tile's
// Gaussians come in batches of 256 staged in LDS; while staging, each thread
// marks which quarters its Gaussian reaches, and a wave passes over the
// Gaussians that miss its quarter without touching its pixels.
__global__ __launch_bounds__(kTilePixels) void splat_render_kernel(SplatCamera cam, int ntx,
                                                                   const uint2* __restrict__ ranges,
                                                                   const uint32_t* __restrict__ vals,
                                                                   const float4* __restrict__ uv,
                                                                   const float4* __restrict__ conic_o,
                                                                   const float* __restrict__ colours,
                                                                   int64_t stride, float* __restrict__ image,
                                                                   float* __restrict__ final_T)
{
    __shared__ float2 s_uv[kTilePixels];
    __shared__ float4 s_co[kTilePixels];
    __shared__ float4 s_col[kTilePixels];   // rgb + the quarter mask in .w
    const int tile = blockIdx.x;
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int tx0 = (tile % ntx) * kTile, ty0 = (tile / ntx) * kTile;
    const int px = tx0 + (wave & 1) * kSub + (lane & 7);
    const int py = ty0 + (wave >> 1) * kSub + (lane >> 3);
    const bool inside = px < cam.width && py < cam.height;
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const uint2 rg = ranges[tile];
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    bool done = !inside;
    for (uint32_t base = rg.x; base < rg.y; base += kTilePixels) {
        if (__syncthreads_count(done ? 1 : 0) == kTilePixels) break;
        const uint32_t e = base + threadIdx.x;
        if (e < rg.y) {
            const uint32_t g = vals[e];
            const float4 uvc = uv[g], co = conic_o[g];
            const float* cg = colours + (size_t)g * stride;
            unsigned mask = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (block_touched(uvc, co, tx0 + (q & 1) * kSub, ty0 + (q >> 1) * kSub, kSub, cam.width, cam.height))
                    mask |= 1u << q;
            s_uv[threadIdx.x] = make_float2(uvc.x, uvc.y);
            s_co[threadIdx.x] = co;
            s_col[threadIdx.x] = make_float4(cg[0], cg[1], cg[2], __uint_as_float(mask));
        }
        __syncthreads();
        const int nb = (int)min((uint32_t)kTilePixels, rg.y - base);
        // kUnroll Gaussians at a time: their alphas are independent, so they are
        // evaluated together, then blended one after another in list order
        for (int j0 = 0; j0 < nb; j0 += kUnroll) {
            unsigned hit4 = 0;
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
                if (j0 + u < nb) hit4 |= ((__float_as_uint(s_col[j0 + u].w) >> wave) & 1u) << u;
            if (hit4 == 0) continue;                      // uniform across the wave
            if (__all(done)) break;
            float al[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int j = min(j0 + u, nb - 1);
                const float2 c = s_uv[j];
                const float4 co = s_co[j];
                const float dx = c.x - fx, dy = c.y - fy;
                const float power = -0.5f * (co.x * dx * dx + co.z * dy * dy) - co.y * dx * dy;
                const float alpha = fminf(kAlphaMax, co.w * __expf(power));
                al[u] = ((hit4 >> u) & 1u) && power <= 0.0f && alpha >= kAlphaMin ? alpha : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                if (done || al[u] == 0.0f) continue;
                const float Tn = T * (1.0f - al[u]);
                if (Tn < kTStop) {
                    done = true;
                    continue;
                }
                const float4 col = s_col[j0 + u];
                const float w = al[u] * T;
                C0 = fmaf(col.x, w, C0);
                C1 = fmaf(col.y, w, C1);
                C2 = fmaf(col.z, w, C2);
                T = Tn;
            }
        }
        __syncthreads();
    }
    if (!inside) return;
    const size_t p = (size_t)py * cam.width + px;
    image[3 * p] = C0 + T * cam.background[0];
    image[3 * p + 1] = C1 + T * cam.background[1];
    image[3 * p + 2] = C2 + T * cam.background[2];
    if (final_T) final_T[p] = T;
}

}  // namespace

size_t splat_sort_temp_bytes(int64_t max_instances) { return sortk::sort_scratch_bytes(max_instances); }

size_t splat_scan_temp_bytes(int n) { return sortk::scan_scratch_bytes(n); }

hipError_t launch_splat_front(int n, const SplatCamera& cam, const float* means, const float* quats,
                              const float* log_scales, const float* opacity, const SplatBuffers& b,
                              hipStream_t stream)
{
    const int blocks = (n + 255) / 256;
    hipLaunchKernelGGL(splat_preprocess_kernel, dim3(blocks), dim3(256), 0, stream, n, cam, means, quats, log_scales,
                       opacity, b.uv, b.conic_o, b.depth, b.rect, b.count, b.flags);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = sortk::exclusive_scan<uint32_t, uint64_t>(b.count, b.offset, n, b.scan_temp, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(splat_total_kernel, dim3(1), dim3(64), 0, stream, n, b.offset, b.count, b.total);
    return hipGetLastError();
}

hipError_t launch_splat_back(int n, const SplatCamera& cam, int64_t instances, const float* colours, int64_t stride,
                             const SplatBuffers& b, float* image, float* final_T, hipStream_t stream)
{
    const int ntx = (cam.width + kTile - 1) / kTile, nty = (cam.height + kTile - 1) / kTile;
    const int ntiles = ntx * nty;
    hipError_t e = fill_u32(reinterpret_cast<uint32_t*>(b.ranges), 0u, 2 * (size_t)ntiles, stream);
    if (e != hipSuccess) return e;
    const uint64_t* sorted_keys = b.keys;   // where the sort leaves the pairs
    const uint32_t* sorted_vals = b.vals;
    if (instances > 0) {
        hipLaunchKernelGGL(splat_duplicate_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, n, cam, ntx, ntiles,
                           b.offset, b.count, b.rect, b.uv, b.conic_o, b.depth, b.keys, b.vals, b.max_instances);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        // enough key bits for every tile number and the past-the-end one
        unsigned tile_bits = 1;
        while ((1u << tile_bits) <= (unsigned)ntiles) ++tile_bits;
        bool in_alt = false;
        e = sortk::radix_sort_pairs<uint64_t, uint32_t>(b.keys, b.vals, b.keys_alt, b.vals_alt, instances, 0,
                                                        32 + (int)tile_bits, b.sort_temp, stream, &in_alt);
        if (e != hipSuccess) return e;
        if (in_alt) {
            sorted_keys = b.keys_alt;
            sorted_vals = b.vals_alt;
        }
        hipLaunchKernelGGL(splat_ranges_kernel, dim3((unsigned)((instances + 255) / 256)), dim3(256), 0, stream,
                           instances, (uint32_t)ntiles, sorted_keys, b.ranges);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(splat_render_kernel, dim3(ntiles), dim3(kTilePixels), 0, stream, cam, ntx, b.ranges,
                       sorted_vals, b.uv, b.conic_o, colours, stride, image, final_T);
    return hipGetLastError();
}

}  // namespace prtgs
