// Linear BVH over the Gaussians' 3-sigma boxes (the Gaussian ray tracer of
// Sec. 4.4 is built on a BVH): scene bounds -> 30-bit Morton codes of the
// centres -> stable LSD radix sort (sort.hpp) -> per-leaf ray-test records (Eq. 1-2) ->
// Karras hierarchy -> bottom-up refit of the child boxes.
#include "common.hpp"
#include "sort.hpp"

namespace prtgs {

namespace {

constexpr int kReduceBlock = 256;

struct BuildWs {
    size_t keys0, vals0, keys1, vals1, hist, leafbox, ibox, parent_int, parent_leaf, counters, partial, total;
};

BuildWs build_ws_layout(int n)
{
    BuildWs w;
    size_t nr = (size_t)((n + kReduceBlock - 1) / kReduceBlock);
    size_t off = kFlagBytes;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    w.keys0 = take(4 * (size_t)n);
    w.vals0 = take(4 * (size_t)n);
    w.keys1 = take(4 * (size_t)n);
    w.vals1 = take(4 * (size_t)n);
    w.hist = take(sortk::sort_scratch_bytes(n));
    w.leafbox = take(24 * (size_t)n);
    w.ibox = take(24 * (size_t)(n > 1 ? n - 1 : 1));
    w.parent_int = take(4 * (size_t)(n > 1 ? n - 1 : 1));
    w.parent_leaf = take(4 * (size_t)n);
    w.counters = take(4 * (size_t)(n > 1 ? n - 1 : 1));
    w.partial = take(32 * nr);
    w.total = off;
    return w;
}

// ---------------------------------------------------------------- bounds

__global__ void bounds_partial_kernel(const float* __restrict__ means, int n, float* __restrict__ partial)
{
    __shared__ float s[6][kReduceBlock];
    int i = blockIdx.x * kReduceBlock + threadIdx.x;
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    if (i < n) {
        for (int a = 0; a < 3; ++a) {
            float m = means[3 * (size_t)i + a];
            if (isfinite(m)) {
                v[a] = m;
                v[3 + a] = m;
            }
        }
    }
    for (int a = 0; a < 6; ++a) s[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int st = kReduceBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            for (int a = 0; a < 3; ++a) {
                s[a][threadIdx.x] = fminf(s[a][threadIdx.x], s[a][threadIdx.x + st]);
                s[3 + a][threadIdx.x] = fmaxf(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + st]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[8 * (size_t)blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void bounds_final_kernel(const float* __restrict__ partial, int nparts, BvhHeader* hdr, int n)
{
    __shared__ float s[6][kReduceBlock];
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int p = threadIdx.x; p < nparts; p += kReduceBlock) {
        for (int a = 0; a < 3; ++a) {
            v[a] = fminf(v[a], partial[8 * (size_t)p + a]);
            v[3 + a] = fmaxf(v[3 + a], partial[8 * (size_t)p + 3 + a]);
        }
    }
    for (int a = 0; a < 6; ++a) s[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int st = kReduceBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            for (int a = 0; a < 3; ++a) {
                s[a][threadIdx.x] = fminf(s[a][threadIdx.x], s[a][threadIdx.x + st]);
                s[3 + a][threadIdx.x] = fmaxf(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + st]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        hdr->n = n;
        hdr->max_depth = 0;
        for (int a = 0; a < 3; ++a) {
            float lo = s[a][0], hi = s[3 + a][0];
            if (!(lo <= hi)) {   // no finite centre at all
                lo = 0.0f;
                hi = 1.0f;
            }
            hdr->lo[a] = lo;
            hdr->hi[a] = hi;
        }
        hdr->lo[3] = 0.0f;
        hdr->hi[3] = 0.0f;
    }
}

// ---------------------------------------------------------------- Morton

__device__ inline uint32_t spread10(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void morton_kernel(const float* __restrict__ means, int n, const BvhHeader* __restrict__ hdr,
                              uint32_t* __restrict__ keys, int32_t* __restrict__ vals)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
        float lo = hdr->lo[a], hi = hdr->hi[a];
        float ext = hi - lo;
        float u = ext > 0.0f ? (means[3 * (size_t)i + a] - lo) / ext : 0.5f;
        if (!(u >= 0.0f)) u = 0.0f;   // also catches NaN
        if (u > 1.0f) u = 1.0f;
        q[a] = (uint32_t)fminf(u * 1024.0f, 1023.0f);
    }
    keys[i] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    vals[i] = i;
}

// ---------------------------------------------------------------- leaves
// One record per leaf rank r (Gaussian j = order[r]): q -> R, s = exp(log s),
// W = diag(1/s) R^T, and the box mu +- sigma_box sqrt(diag(Sigma)), Sigma =
// R diag(s^2) R^T (Eq. 2), padded for rounding.

__global__ void leaf_kernel(const prtgs_gaussians g, const int32_t* __restrict__ order, Prim* __restrict__ prims,
                            float4* __restrict__ normals, float* __restrict__ leafbox, int32_t* __restrict__ order_out,
                            unsigned* flags)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= g.n) return;
    int j = order[r];
    order_out[r] = j;
    float mx = g.means[3 * (size_t)j], my = g.means[3 * (size_t)j + 1], mz = g.means[3 * (size_t)j + 2];
    float qw = g.quats[4 * (size_t)j], qx = g.quats[4 * (size_t)j + 1], qy = g.quats[4 * (size_t)j + 2],
          qz = g.quats[4 * (size_t)j + 3];
    float l0 = g.log_scales[3 * (size_t)j], l1 = g.log_scales[3 * (size_t)j + 1], l2 = g.log_scales[3 * (size_t)j + 2];
    float op = g.opacity[j];
    float nx = g.normals[3 * (size_t)j], ny = g.normals[3 * (size_t)j + 1], nz = g.normals[3 * (size_t)j + 2];
    float qn2 = qw * qw + qx * qx + qy * qy + qz * qz;
    bool ok = finite3(mx, my, mz) && finite3(qw, qx, qy) && isfinite(qz) && finite3(l0, l1, l2) && isfinite(op) &&
              finite3(nx, ny, nz) && qn2 > 0.0f;
    if (!ok) {
        raise_flag(flags, PRTGS_FLAG_NONFINITE);
        // neutral record: a transparent point far from everything
        qw = 1.0f; qx = qy = qz = 0.0f; qn2 = 1.0f;
        l0 = l1 = l2 = -20.0f;
        op = 0.0f;
        if (!finite3(mx, my, mz)) mx = my = mz = 0.0f;
        if (!finite3(nx, ny, nz)) { nx = ny = 0.0f; nz = 1.0f; }
    }
    float inv = rsqrtf(qn2);
    qw *= inv; qx *= inv; qy *= inv; qz *= inv;
    float R[3][3] = {
        {1.0f - 2.0f * (qy * qy + qz * qz), 2.0f * (qx * qy - qw * qz), 2.0f * (qx * qz + qw * qy)},
        {2.0f * (qx * qy + qw * qz), 1.0f - 2.0f * (qx * qx + qz * qz), 2.0f * (qy * qz - qw * qx)},
        {2.0f * (qx * qz - qw * qy), 2.0f * (qy * qz + qw * qx), 1.0f - 2.0f * (qx * qx + qy * qy)}};
    float s[3] = {expf(l0), expf(l1), expf(l2)};
    float is[3] = {expf(-l0), expf(-l1), expf(-l2)};
    Prim p;
    p.mo = make_float4(mx, my, mz, op);
    p.w0 = make_float4(R[0][0] * is[0], R[1][0] * is[0], R[2][0] * is[0], fmaxf(is[0], fmaxf(is[1], is[2])));
    p.w1 = make_float4(R[0][1] * is[1], R[1][1] * is[1], R[2][1] * is[1], 0.0f);
    p.w2 = make_float4(R[0][2] * is[2], R[1][2] * is[2], R[2][2] * is[2], 0.0f);
    prims[r] = p;
    normals[r] = make_float4(nx, ny, nz, 0.0f);
    float m[3] = {mx, my, mz};
    float mag = fmaxf(fabsf(mx), fmaxf(fabsf(my), fabsf(mz)));
    for (int a = 0; a < 3; ++a) {
        float var = R[a][0] * R[a][0] * s[0] * s[0] + R[a][1] * R[a][1] * s[1] * s[1] + R[a][2] * R[a][2] * s[2] * s[2];
        float h = kBoxSigma * sqrtf(var) * (1.0f + 1e-5f) + 4e-7f * (1.0f + mag);
        leafbox[6 * (size_t)r + a] = m[a] - h;
        leafbox[6 * (size_t)r + 3 + a] = m[a] + h;
    }
}

// ---------------------------------------------------------------- Karras
// Hierarchy of Karras (HPG 2012) over the sorted codes; equal codes are told
// apart by their leaf rank, so every internal node i covers a key range
// whose common prefix is longer than its parent's.

__device__ inline int prefix_len(const uint32_t* __restrict__ codes, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    uint32_t a = codes[i], b = codes[j];
    if (a != b) return __clz(a ^ b);
    return 32 + __clz((uint32_t)i ^ (uint32_t)j);
}

__global__ void karras_kernel(const uint32_t* __restrict__ codes, int n, Node* __restrict__ nodes,
                              int32_t* __restrict__ parent_int, int32_t* __restrict__ parent_leaf)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int d = (prefix_len(codes, n, i, i + 1) - prefix_len(codes, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = prefix_len(codes, n, i, i - d);
    int lmax = 2;
    while (prefix_len(codes, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(codes, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = prefix_len(codes, n, i, j);
    int s = 0;
    int t = l;
    do {
        t = (t + 1) >> 1;
        if (prefix_len(codes, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int gamma = i + s * d + min(d, 0);
    int lo = min(i, j), hi = max(i, j);
    int left = (lo == gamma) ? ~gamma : gamma;
    int right = (hi == gamma + 1) ? ~(gamma + 1) : gamma + 1;
    nodes[i].d = make_int4(left, right, 0, 0);
    if (left < 0) parent_leaf[~left] = i; else parent_int[left] = i;
    if (right < 0) parent_leaf[~right] = i; else parent_int[right] = i;
    if (i == 0) parent_int[0] = -1;
}

// ---------------------------------------------------------------- refit
// One thread per leaf climbs towards the root; the second thread to reach a
// node (atomic counter) writes the node's child boxes and continues.

__device__ inline void load_box(const float* p, float* b)
{
    for (int a = 0; a < 6; ++a) b[a] = __hip_atomic_load(p + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void refit_kernel(int n, Node* __restrict__ nodes, const int32_t* __restrict__ parent_int,
                             const int32_t* __restrict__ parent_leaf, const float* __restrict__ leafbox,
                             float* __restrict__ ibox, uint32_t* __restrict__ counters, BvhHeader* hdr)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int depth = 1;
    for (int p = parent_leaf[r]; p >= 0; p = parent_int[p]) ++depth;
    atomicMax(&hdr->max_depth, depth);
    int p = parent_leaf[r];
    while (p >= 0) {
        uint32_t prev = __hip_atomic_fetch_add(&counters[p], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == 0) return;
        int4 refs = nodes[p].d;
        float bl[6], br[6];
        if (refs.x < 0) load_box(leafbox + 6 * (size_t)(~refs.x), bl); else load_box(ibox + 6 * (size_t)refs.x, bl);
        if (refs.y < 0) load_box(leafbox + 6 * (size_t)(~refs.y), br); else load_box(ibox + 6 * (size_t)refs.y, br);
        Node nd;
        nd.a = make_float4(bl[0], bl[1], bl[2], bl[3]);
        nd.b = make_float4(bl[4], bl[5], br[0], br[1]);
        nd.c = make_float4(br[2], br[3], br[4], br[5]);
        nd.d = refs;
        nodes[p] = nd;
        float* ob = ibox + 6 * (size_t)p;
        for (int a = 0; a < 3; ++a) {
            __hip_atomic_store(ob + a, fminf(bl[a], br[a]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(ob + 3 + a, fmaxf(bl[3 + a], br[3 + a]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        p = parent_int[p];
    }
}

}  // namespace

size_t build_workspace_bytes(int n) { return build_ws_layout(n).total; }

hipError_t launch_build_bvh(const prtgs_gaussians& g, void* bvh, void* ws, unsigned* flags, hipStream_t stream)
{
    const int n = g.n;
    BvhLayout L = bvh_layout(n);
    BuildWs W = build_ws_layout(n);
    char* b = static_cast<char*>(bvh);
    char* w = static_cast<char*>(ws);
    BvhHeader* hdr = reinterpret_cast<BvhHeader*>(b);
    Node* nodes = reinterpret_cast<Node*>(b + L.nodes);
    Prim* prims = reinterpret_cast<Prim*>(b + L.prims);
    float4* normals = reinterpret_cast<float4*>(b + L.normals);
    int32_t* order_out = reinterpret_cast<int32_t*>(b + L.order);
    uint32_t* keys[2] = {reinterpret_cast<uint32_t*>(w + W.keys0), reinterpret_cast<uint32_t*>(w + W.keys1)};
    int32_t* vals[2] = {reinterpret_cast<int32_t*>(w + W.vals0), reinterpret_cast<int32_t*>(w + W.vals1)};
    void* hist = w + W.hist;   // sort scratch
    float* leafbox = reinterpret_cast<float*>(w + W.leafbox);
    float* ibox = reinterpret_cast<float*>(w + W.ibox);
    int32_t* parent_int = reinterpret_cast<int32_t*>(w + W.parent_int);
    int32_t* parent_leaf = reinterpret_cast<int32_t*>(w + W.parent_leaf);
    uint32_t* counters = reinterpret_cast<uint32_t*>(w + W.counters);
    float* partial = reinterpret_cast<float*>(w + W.partial);

    hipError_t e;
    int nr = (n + kReduceBlock - 1) / kReduceBlock;
    hipLaunchKernelGGL(bounds_partial_kernel, dim3(nr), dim3(kReduceBlock), 0, stream, g.means, n, partial);
    hipLaunchKernelGGL(bounds_final_kernel, dim3(1), dim3(kReduceBlock), 0, stream, partial, nr, hdr, n);
    int blocks = (n + 255) / 256;
    hipLaunchKernelGGL(morton_kernel, dim3(blocks), dim3(256), 0, stream, g.means, n, hdr, keys[0], vals[0]);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    bool in_alt = false;
    if ((e = sortk::radix_sort_pairs<uint32_t, int32_t>(keys[0], vals[0], keys[1], vals[1], n, 0, 32, hist, stream,
                                                        &in_alt)) != hipSuccess)
        return e;
    const int cur = in_alt ? 1 : 0;

    hipLaunchKernelGGL(leaf_kernel, dim3(blocks), dim3(256), 0, stream, g, vals[cur], prims, normals, leafbox,
                       order_out, flags);
    if (n > 1) {
        if ((e = fill_u32(counters, 0u, (size_t)(n - 1), stream)) != hipSuccess) return e;
        int iblocks = (n - 1 + 255) / 256;
        hipLaunchKernelGGL(karras_kernel, dim3(iblocks), dim3(256), 0, stream, keys[cur], n, nodes, parent_int,
                           parent_leaf);
        hipLaunchKernelGGL(refit_kernel, dim3(blocks), dim3(256), 0, stream, n, nodes, parent_int, parent_leaf,
                           leafbox, ibox, counters, hdr);
    }
    return hipGetLastError();
}

hipError_t launch_leaf_order(const void* bvh, int n, int32_t* order, hipStream_t stream)
{
    BvhLayout L = bvh_layout(n);
    return hipMemcpyAsync(order, static_cast<const char*>(bvh) + L.order, sizeof(int32_t) * (size_t)n,
                          hipMemcpyDeviceToDevice, stream);
}

}  // namespace prtgs
