// k_estimate.hip -- compressibility estimates of Sec. III-B on the device.
//
// From the histogram (Sec. III-B.1): entropy H = -sum p_i log2 p_i, the
// probability p1 of the most likely symbol, and the bounds of the Huffman
// redundancy R = <b> - H: R+ = p1 + 0.086, and R- = 1 - H(p1, 1 - p1) when
// p1 > 0.4 (0 otherwise; a single symbol costs one bit), so that
// H + R- <= <b> <= H + R+ holds before any codebook is built.  The workflow
// they predict: run-length coding when H + R+ <= 1.09, Huffman when
// H + R- > 1.09, undecided otherwise.
//
// Smoothness (Sec. III-B.2): a sampled binary madogram of the quant-codes.
// Sample k draws SplitMix64(seed, k) (the generator of Steele, Lea and Flood
// used as a counter-based one: the output after k + 1 steps from the seed);
// its high half picks a position a in [0, n), its low half a distance d in
// [1, dmax], both by multiply-shift; a pair past the field's end is skipped.
// Per distance the kernel counts the pairs and those whose codes differ, in
// exact integers.
#include "ebc_dev.h"
#include "ebc_launch.h"

namespace ebc {

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// One workgroup per field: the histogram estimates.
__global__ __launch_bounds__(kBlock) void k_estimate_hist(const FieldDesc* __restrict__ F,
                                                          EstDev* __restrict__ est)
{
    const FieldDesc& fd = F[blockIdx.x];
    const auto* dy = kconst(fd.dyn);
    EstDev* e = est + blockIdx.x;
    if (dy->status != ST_OK || dy->codec == ARC_CONST) return;
    const double n = (double)fd.n;
    double h = 0.0;
    uint32_t mx = 0;
    for (uint32_t s = threadIdx.x; s < fd.n_bins; s += kBlock) {
        const uint32_t c = fd.hist[s];
        if (c) {
            const double p = (double)c / n;
            h -= p * log2(p);
            mx = max(mx, c);
        }
    }
    __shared__ double s_h[kBlock];
    __shared__ uint32_t s_m[kBlock];
    s_h[threadIdx.x] = h;
    s_m[threadIdx.x] = mx;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double H = 0.0;
    for (int k = 0; k < kBlock; ++k) {
        H += s_h[k];
        mx = max(mx, s_m[k]);
    }
    const double p1 = (double)mx / n;
    double lo = 0.0;
    if (p1 >= 1.0) lo = 1.0;
    else if (p1 > 0.4) lo = 1.0 - (-p1 * log2(p1) - (1.0 - p1) * log2(1.0 - p1));
    const double hi = p1 + 0.086;
    e->entropy = H;
    e->p1 = p1;
    e->r_lo = lo;
    e->r_hi = hi;
    e->hist_max = mx;
    e->predict = H + hi <= 1.09 ? 1 : (H + lo > 1.09 ? 0 : 2);
}

// Sampled binary madogram: grid-stride over the samples, per-distance
// counters privatised in LDS and added to the field's record at the end.
__global__ __launch_bounds__(kBlock) void k_madogram(const FieldDesc* __restrict__ F,
                                                     EstDev* __restrict__ est, uint64_t samples,
                                                     uint64_t seed)
{
    const FieldDesc& fd = F[blockIdx.y];
    const auto* dy = kconst(fd.dyn);
    EstDev* e = est + blockIdx.y;
    if (dy->status != ST_OK || dy->codec == ARC_CONST) return;
    __shared__ uint32_t s_sum[kMadoDist + 1], s_cnt[kMadoDist + 1];
    for (uint32_t d = threadIdx.x; d <= kMadoDist; d += kBlock) s_sum[d] = s_cnt[d] = 0;
    __syncthreads();
    const uint64_t n = fd.n;
    const EBC_G uint16_t* __restrict__ q = fd.q;
    for (uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x; k < samples;
         k += (uint64_t)gridDim.x * kBlock) {
        const uint64_t r = splitmix64(seed, k);
        const uint64_t a = ((r >> 32) * n) >> 32;
        const uint32_t d = 1 + (uint32_t)(((r & 0xFFFFFFFFull) * kMadoDist) >> 32);
        if (a + d >= n) continue;
        atomicAdd(&s_cnt[d], 1u);
        if (q[a] != q[a + d]) atomicAdd(&s_sum[d], 1u);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d <= kMadoDist; d += kBlock) {
        if (s_cnt[d]) atomicAdd((unsigned long long*)&e->mado_cnt[d], (unsigned long long)s_cnt[d]);
        if (s_sum[d]) atomicAdd((unsigned long long*)&e->mado_sum[d], (unsigned long long)s_sum[d]);
    }
}

__global__ void k_estimate_clear(EstDev* __restrict__ est, int nf)
{
    uint64_t* p = (uint64_t*)est;
    const uint64_t words = (uint64_t)nf * (sizeof(EstDev) / 8);
    for (uint64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x) p[i] = 0;
}

hipError_t launch_estimate(const FieldDesc* F, int nf, EstDev* est, uint64_t samples, uint64_t seed,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_estimate_clear, dim3(4), dim3(kBlock), 0, s, est, nf);
    hipLaunchKernelGGL(k_estimate_hist, dim3(nf), dim3(kBlock), 0, s, F, est);
    if (samples) {
        const uint64_t want = (samples + kBlock * 64 - 1) / (kBlock * 64);  // ~64 samples per thread
        const uint32_t g = want < 1 ? 1u : want > 1024 ? 1024u : (uint32_t)want;
        hipLaunchKernelGGL(k_madogram, dim3(g, nf), dim3(kBlock), 0, s, F, est, samples, seed);
    }
    return hipGetLastError();
}

}  // namespace ebc
