// Device-wide exclusive scan and stable LSD radix sort of (key, value)
// pairs, shared by the BVH build (Morton codes) and the splat rasterizer
// (tile and depth keys).
//
// Scan: three launches -- per-tile sums, one block scanning the tile sums,
// then each tile scanned in LDS and offset by its tile's base.
// Sort: per 8-bit digit, tile histograms in digit-major order, one exclusive
// scan over them (giving each tile's output base per digit), then a stable
// scatter in which the lanes of one wave find equal digits by bitwise
// ballots.
#pragma once

#include "common.hpp"

namespace prtgs {
namespace sortk {
namespace {   // each translation unit keeps its own copies of the kernels

constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;   // consecutive items per thread
constexpr int kScanTile = kScanBlock * kScanItems;
constexpr int kScanSumsBlock = 1024;

inline int64_t sort_tiles(int64_t n) { return (n + kSortTile - 1) / kSortTile; }
inline int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

// Scratch of a scan over n items: one 64-bit sum per scan tile.
inline size_t scan_scratch_bytes(int64_t n) { return align256(8 * (size_t)(scan_tiles(n) + 1)); }

// Scratch of a sort of n pairs: the digit histograms, then the scratch of
// their scan.
inline size_t sort_hist_bytes(int64_t n) { return align256(4 * 256 * (size_t)sort_tiles(n)); }
inline size_t sort_scratch_bytes(int64_t n) { return sort_hist_bytes(n) + scan_scratch_bytes(256 * sort_tiles(n)); }

// ---------------------------------------------------------------- scan

template <class In>
__global__ __launch_bounds__(kScanBlock) void scan_reduce_kernel(const In* __restrict__ in, int64_t n,
                                                                 uint64_t* __restrict__ tile_sums)
{
    __shared__ uint64_t ws[kScanBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint64_t s = 0;
    for (int it = 0; it < kScanItems; ++it) {
        const int64_t i = base + (int64_t)it * kScanBlock + threadIdx.x;
        if (i < n) s += (uint64_t)in[i];
    }
    for (int off = kWave / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) ws[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < kScanBlock / kWave; ++w) t += ws[w];
        tile_sums[blockIdx.x] = t;
    }
}

// Exclusive scan of the tile sums in place, by one block: each thread takes
// a contiguous run, the run totals are scanned in LDS.
__global__ __launch_bounds__(kScanSumsBlock) void scan_tile_sums_kernel(uint64_t* __restrict__ sums, int64_t count)
{
    __shared__ uint64_t part[kScanSumsBlock];
    const int64_t per = (count + kScanSumsBlock - 1) / kScanSumsBlock;
    const int64_t beg = (int64_t)threadIdx.x * per;
    const int64_t end = beg + per < count ? beg + per : count;
    uint64_t local = 0;
    for (int64_t i = beg; i < end; ++i) local += sums[i];
    part[threadIdx.x] = local;
    __syncthreads();
    for (int off = 1; off < kScanSumsBlock; off <<= 1) {
        const uint64_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0ull;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint64_t run = part[threadIdx.x] - local;
    for (int64_t i = beg; i < end; ++i) {
        const uint64_t v = sums[i];
        sums[i] = run;
        run += v;
    }
}

// Each tile: thread t scans its kScanItems consecutive items, the thread
// totals are scanned across the block (waves by shuffles, then the wave
// totals), and the tile's base is added.  in == out is allowed.
template <class In, class Out>
__global__ __launch_bounds__(kScanBlock) void scan_apply_kernel(const In* in, Out* out, int64_t n,
                                                                const uint64_t* __restrict__ tile_base)
{
    __shared__ uint64_t ws[kScanBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t first = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint64_t v[kScanItems];
    uint64_t total = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = first + k < n ? (uint64_t)in[first + k] : 0ull;
        total += v[k];
    }
    uint64_t incl = total;   // inclusive scan of the thread totals within the wave
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t up = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += up;
    }
    if (lane == kWave - 1) ws[wave] = incl;
    __syncthreads();
    uint64_t run = tile_base[blockIdx.x] + incl - total;
    for (int w = 0; w < wave; ++w) run += ws[w];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (first + k < n) out[first + k] = (Out)run;
        run += v[k];
    }
}

// out[i] = sum of in[0..i) (64-bit running sums, stored as Out).
template <class In, class Out>
hipError_t exclusive_scan(const In* in, Out* out, int64_t n, void* scratch, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    uint64_t* sums = static_cast<uint64_t*>(scratch);
    const int64_t tiles = scan_tiles(n);
    hipLaunchKernelGGL((scan_reduce_kernel<In>), dim3((unsigned)tiles), dim3(kScanBlock), 0, stream, in, n, sums);
    hipLaunchKernelGGL(scan_tile_sums_kernel, dim3(1), dim3(kScanSumsBlock), 0, stream, sums, tiles);
    hipLaunchKernelGGL((scan_apply_kernel<In, Out>), dim3((unsigned)tiles), dim3(kScanBlock), 0, stream, in, out, n,
                       sums);
    return hipGetLastError();
}

// ---------------------------------------------------------------- radix sort

template <class Key>
__global__ __launch_bounds__(kSortBlock) void radix_hist_kernel(const Key* __restrict__ keys, int64_t n, int shift,
                                                                uint32_t* __restrict__ hist, int64_t ntiles)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
        const int64_t i = base + (int64_t)it * kSortBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

template <class Key, class Val>
__global__ __launch_bounds__(kSortBlock) void radix_scatter_kernel(const Key* __restrict__ kin,
                                                                   const Val* __restrict__ vin, Key* __restrict__ kout,
                                                                   Val* __restrict__ vout, int64_t n, int shift,
                                                                   const uint32_t* __restrict__ offsets, int64_t ntiles)
{
    constexpr int kWaves = kSortBlock / kWave;
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kWaves][256];
    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    const int lane = tid % kWave;
    run[tid] = offsets[(size_t)tid * ntiles + blockIdx.x];
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
        for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const int64_t i = base + (int64_t)it * kSortBlock + tid;
        const bool valid = i < n;
        const Key key = valid ? kin[i] : (Key)0;
        const Val val = valid ? vin[i] : (Val)0;
        const uint32_t dig = (uint32_t)(key >> shift) & 255u;
        uint64_t same = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t ones = __ballot(valid && ((dig >> bit) & 1u));
            same &= ((dig >> bit) & 1u) ? ones : ~ones;
        }
        const uint32_t rank = (uint32_t)__popcll(same & lt_mask);
        if (valid && rank == 0) wcnt[wave][dig] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[dig] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][dig];
            if ((int64_t)pos < n) {
                kout[pos] = key;
                vout[pos] = val;
            }
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kWaves; ++w) add += wcnt[w][tid];
        run[tid] += add;
        __syncthreads();
    }
}

// Sorts n pairs (k0, v0) by key bits [begin_bit, end_bit), one 8-bit digit
// per pass, ping-ponging with (k1, v1); *in_alt tells whether the sorted
// pairs ended in (k1, v1).  n must stay below 2^31 (32-bit positions).
// scratch: sort_scratch_bytes(n).
template <class Key, class Val>
hipError_t radix_sort_pairs(Key* k0, Val* v0, Key* k1, Val* v1, int64_t n, int begin_bit, int end_bit,
                            void* scratch, hipStream_t stream, bool* in_alt)
{
    *in_alt = false;
    if (n <= 1 || begin_bit >= end_bit) return hipSuccess;
    if (n >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    const int64_t ntiles = sort_tiles(n);
    uint32_t* hist = static_cast<uint32_t*>(scratch);
    void* scan_scratch = static_cast<char*>(scratch) + sort_hist_bytes(n);
    Key* keys[2] = {k0, k1};
    Val* vals[2] = {v0, v1};
    int cur = 0;
    for (int shift = begin_bit; shift < end_bit; shift += 8) {
        hipLaunchKernelGGL((radix_hist_kernel<Key>), dim3((unsigned)ntiles), dim3(kSortBlock), 0, stream, keys[cur], n,
                           shift, hist, ntiles);
        hipError_t e = exclusive_scan<uint32_t, uint32_t>(hist, hist, 256 * ntiles, scan_scratch, stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((radix_scatter_kernel<Key, Val>), dim3((unsigned)ntiles), dim3(kSortBlock), 0, stream,
                           keys[cur], vals[cur], keys[cur ^ 1], vals[cur ^ 1], n, shift, hist, ntiles);
        cur ^= 1;
    }
    *in_alt = cur == 1;
    return hipGetLastError();
}

}  // namespace
}  // namespace sortk
}  // namespace prtgs
