// k_scan.hip -- exclusive prefix sum of a uint32 array (reduce-then-scan).
// A first kernel writes every tile's sum.  Up to kScanDirect tiles, each
// workgroup of the second kernel adds up the sums of the tiles before its own
// (at most a few loads per thread) and scans its tile from there; above that
// (the total work of those sums grows with the square of the tile count), one
// workgroup scans the tile sums in between.
//
// Used for every offset computation of the path: ordered outlier positions
// (per-segment counts), Huffman word offsets (per-chunk word counts), RLE run
// positions and, in decompression, chunk word offsets and run starts.  Batches
// scan one concatenated array; a field's offsets are differences of two
// prefix values, which stay exact in modulo-2^32 arithmetic as long as the
// field's own total is below 2^32.
#include "ebc_dev.h"
#include "ebc_launch.h"

namespace ebc {

constexpr int kScanItems = 16;
constexpr uint32_t kScanTile = kBlock * kScanItems;
constexpr uint32_t kScanDirect = 1024;  // default: tiles up to which the tile sums are not scanned first

// exclusive scan of one value per thread over the block; *total = block sum
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* total)
{
    __shared__ uint32_t s_w[kWavesPerBlock];
    const int w = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan_u32(v);
    if (lane_id() == kWave - 1) s_w[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kWavesPerBlock; ++k) {
        off += k < w ? s_w[k] : 0u;
        tot += s_w[k];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__device__ __forceinline__ void load_items(const uint32_t* a, uint32_t n, uint32_t base,
                                           uint32_t v[kScanItems])
{
    const uint32_t i0 = base + threadIdx.x * kScanItems;
    if (i0 + kScanItems <= n) {
#pragma unroll
        for (int k = 0; k < kScanItems; k += 4) {
            uint4 t = *(const uint4*)(a + i0 + k);
            v[k] = t.x, v[k + 1] = t.y, v[k + 2] = t.z, v[k + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = i0 + k < n ? a[i0 + k] : 0u;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* __restrict__ a, uint32_t n,
                                                        uint32_t* __restrict__ sums)
{
    uint32_t v[kScanItems];
    load_items(a, n, blockIdx.x * kScanTile, v);
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += v[k];
    s = wave_sum_u32(s);
    __shared__ uint32_t s_w[kWavesPerBlock];
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kWavesPerBlock; ++k) t += s_w[k];
        sums[blockIdx.x] = t;
    }
}

// single block: exclusive scan of the block sums, total in sums[nb]
__global__ __launch_bounds__(kBlock) void k_scan_top(uint32_t* __restrict__ sums, uint32_t nb)
{
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += kScanTile) {
        uint32_t v[kScanItems];
        load_items(sums, nb, base, v);
        uint32_t loc = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) loc += v[k];
        uint32_t tot;
        uint32_t off = block_excl_scan(loc, &tot) + carry;
        const uint32_t i0 = base + threadIdx.x * kScanItems;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (i0 + k < nb) sums[i0 + k] = off;
            off += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

// total of an empty array
__global__ void k_scan_empty(uint32_t* __restrict__ a) { a[0] = 0; }

// sum of one value per thread over the block
__device__ __forceinline__ uint32_t block_sum(uint32_t v)
{
    __shared__ uint32_t s_r[kWavesPerBlock];
    v = wave_sum_u32(v);
    if (lane_id() == 0) s_r[threadIdx.x / kWave] = v;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int k = 0; k < kWavesPerBlock; ++k) t += s_r[k];
    return t;
}

// SCANNED: sums[] already holds the exclusive prefix of the tile sums
template <bool SCANNED>
__global__ __launch_bounds__(kBlock) void k_scan_down(uint32_t* __restrict__ a, uint32_t n,
                                                      const uint32_t* __restrict__ sums,
                                                      uint32_t nb)
{
    uint32_t pre = 0;
    if (SCANNED) {
        pre = sums[blockIdx.x];
    } else {
        for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kBlock) pre += sums[b];
        pre = block_sum(pre);
    }
    uint32_t v[kScanItems];
    const uint32_t base = blockIdx.x * kScanTile;
    load_items(a, n, base, v);
    uint32_t loc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) loc += v[k];
    uint32_t tot;
    uint32_t off = block_excl_scan(loc, &tot) + pre;
    const uint32_t i0 = base + threadIdx.x * kScanItems;
    if (i0 + kScanItems <= n) {
#pragma unroll
        for (int k = 0; k < kScanItems; k += 4) {
            uint4 t;
            t.x = off, off += v[k];
            t.y = off, off += v[k + 1];
            t.z = off, off += v[k + 2];
            t.w = off, off += v[k + 3];
            *(uint4*)(a + i0 + k) = t;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (i0 + k < n) a[i0 + k] = off;
            off += v[k];
        }
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) a[n] = pre + tot;
}

uint32_t scan_tmp_words(uint32_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_scan(uint32_t* a, uint32_t n, uint32_t* tmp, hipStream_t s, uint32_t direct_max)
{
    if (direct_max == 0) direct_max = kScanDirect;
    if (n == 0) {
        hipLaunchKernelGGL(k_scan_empty, dim3(1), dim3(1), 0, s, a);
        return hipGetLastError();
    }
    const uint32_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s, a, n, tmp);
    if (nb <= direct_max) {
        hipLaunchKernelGGL(k_scan_down<false>, dim3(nb), dim3(kBlock), 0, s, a, n, tmp, nb);
    } else {
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, tmp, nb);
        hipLaunchKernelGGL(k_scan_down<true>, dim3(nb), dim3(kBlock), 0, s, a, n, tmp, nb);
    }
    return hipGetLastError();
}

}  // namespace ebc
