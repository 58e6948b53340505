// Direction / SH-basis table: S stratified equal-area directions and the
// real orthonormal spherical harmonics at them (SH projection, Eq. 8-11),
// generated in FP64 on the device.
#include "common.hpp"
#include "sh.hpp"

namespace prtgs {

namespace {

// SplitMix64 (Steele, Lea & Flood 2014): output `idx` of the stream seeded
// with `seed` is the finaliser applied to seed + (idx + 1) * golden gamma.
__device__ inline uint64_t mix64(uint64_t seed, uint64_t idx)
{
    uint64_t z = seed + (idx + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline double unit53(uint64_t seed, uint64_t idx)
{
    return (double)(mix64(seed, idx) >> 11) * 0x1.0p-53;
}

__global__ void direction_table_kernel(int S, int nu, int nv, uint64_t seed, int bands, double* d64, double* y64,
                                       float* d32, float* y32)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    int a = s / nv, b = s - a * nv;
    double xi = unit53(seed, 2ull * (uint64_t)s);
    double eta = unit53(seed, 2ull * (uint64_t)s + 1ull);
    double z = 1.0 - 2.0 * ((double)a + xi) / (double)nu;
    double phi = 2.0 * 3.14159265358979323846 * ((double)b + eta) / (double)nv;
    double r = sqrt(fmax(0.0, 1.0 - z * z));
    double sp, cp;
    sincos(phi, &sp, &cp);
    float fx = (float)(r * cp), fy = (float)(r * sp), fz = (float)z;
    if (d32) {
        d32[3 * s + 0] = fx;
        d32[3 * s + 1] = fy;
        d32[3 * s + 2] = fz;
    }
    if (d64) {
        d64[3 * s + 0] = (double)fx;
        d64[3 * s + 1] = (double)fy;
        d64[3 * s + 2] = (double)fz;
    }
    // the basis is evaluated at the FP32 direction, renormalised in FP64
    double ux = fx, uy = fy, uz = fz;
    double len = sqrt(ux * ux + uy * uy + uz * uz);
    ux /= len;
    uy /= len;
    uz /= len;
    double Y[kMaxBands * kMaxBands];
    real_sh(bands, ux, uy, uz, Y);
    int K = bands * bands;
    for (int k = 0; k < K; ++k) {
        if (y64) y64[(size_t)s * K + k] = Y[k];
        if (y32) y32[(size_t)s * K + k] = (float)Y[k];
    }
}

// Rank of stratum s in a coherent order: strata are grouped into tiles of
// (up to) 8 z-bands x 8 phi-sectors, tiles in row-major order, row-major
// inside a tile, so that 64 consecutive directions cover a compact patch.
__device__ inline int tile_key(int s, int nu, int nv)
{
    int a = s / nv, b = s - a * nv;
    int ta = nu < 8 ? nu : 8;
    int tb = 64 / ta;
    if (tb > nv) tb = nv;
    int ntb = (nv + tb - 1) / tb;
    int ia = a % ta, ib = b % tb;
    int within = ia * tb + ib;
    if (ta == 8 && tb == 8) {   // full tiles in Morton order: aligned runs of 2^k are compact
        within = 0;
        for (int bit = 0; bit < 3; ++bit) within |= (((ib >> bit) & 1) << (2 * bit)) | (((ia >> bit) & 1) << (2 * bit + 1));
    }
    return ((a / ta) * ntb + (b / tb)) * (ta * tb) + within;
}

__global__ void direction_order_kernel(int S, int nu, int nv, int32_t* order)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    if (S > 8192) {   // the quadratic ranking below is for table sizes in use; keep large tables in place
        order[s] = s;
        return;
    }
    int key = tile_key(s, nu, nv);
    int rank = 0;   // keys are distinct: the rank is the count of smaller keys
    for (int u = 0; u < S; ++u) rank += tile_key(u, nu, nv) < key;
    order[rank] = s;
}

}  // namespace

void stratified_grid(int S, int* nu, int* nv)
{
    int r = 1;
    while ((r + 1) * (r + 1) <= S) ++r;
    int u = 1;
    for (int d = 1; d <= r; ++d)
        if (S % d == 0) u = d;
    *nu = u;
    *nv = S / u;
}

hipError_t launch_direction_table(int S, uint64_t seed, int bands, double* d64, double* y64, float* d32,
                                  float* y32, hipStream_t stream)
{
    int nu, nv;
    stratified_grid(S, &nu, &nv);
    int threads = 64;
    int blocks = (S + threads - 1) / threads;
    hipLaunchKernelGGL(direction_table_kernel, dim3(blocks), dim3(threads), 0, stream, S, nu, nv, seed, bands, d64,
                       y64, d32, y32);
    return hipGetLastError();
}

hipError_t launch_direction_order(int S, int32_t* order, hipStream_t stream)
{
    int nu, nv;
    stratified_grid(S, &nu, &nv);
    hipLaunchKernelGGL(direction_order_kernel, dim3((S + 63) / 64), dim3(64), 0, stream, S, nu, nv, order);
    return hipGetLastError();
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, size_t count)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = v;
}

hipError_t fill_u32(uint32_t* p, uint32_t v, size_t count, hipStream_t stream)
{
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, v, count);
    return hipGetLastError();
}

}  // namespace prtgs
