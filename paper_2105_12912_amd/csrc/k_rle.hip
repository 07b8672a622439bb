// k_rle.hip -- run-length encoding of the quant-codes and its inverse.
//
// Sec. III-B: a run of equal symbols is stored as a (value, count) tuple; the
// run lengths are metadata.  Runs are maximal and taken over the whole code
// array in row-major order.  Encoding marks run starts (a code differing from
// its predecessor), counts them per tile, scans the counts, and compacts
// (value, start) pairs in order; lengths are differences of successive
// starts.  Decoding scans the stored lengths into starts and expands each
// output tile from the runs that overlap it.
#include "ebc_dev.h"
#include "ebc_launch.h"

namespace ebc {

constexpr int kRleItems = kRleTile / kBlock;  // 16 codes per thread

// load 16 codes owned by this thread and the flags "starts a run"
__device__ __forceinline__ uint32_t run_flags(const FieldDesc& fd, uint64_t lo, uint16_t c[kRleItems])
{
    __shared__ uint16_t s_last[kBlock];
    const uint64_t i0 = lo + (uint64_t)threadIdx.x * kRleItems;
    const uint64_t n = fd.n;
    const EBC_G uint16_t* __restrict__ q = fd.q;
    if (i0 + kRleItems <= n) {
        const uint4 a = *(const EBC_G uint4*)(q + i0);
        const uint4 b = *(const EBC_G uint4*)(q + i0 + 8);
        const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int k = 0; k < 8; ++k) c[2 * k] = w[k] & 0xFFFF, c[2 * k + 1] = w[k] >> 16;
    } else {
#pragma unroll
        for (int k = 0; k < kRleItems; ++k) c[k] = i0 + k < n ? q[i0 + k] : 0;
    }
    s_last[threadIdx.x] = c[kRleItems - 1];
    __syncthreads();
    uint32_t prev;
    bool have_prev;
    if (threadIdx.x > 0) {
        prev = s_last[threadIdx.x - 1];
        have_prev = true;
    } else {
        have_prev = lo > 0;
        prev = have_prev ? q[lo - 1] : 0u;
    }
    uint32_t flags = 0;
#pragma unroll
    for (int k = 0; k < kRleItems; ++k) {
        if (i0 + k < n && (!have_prev || c[k] != prev)) flags |= 1u << k;
        prev = c[k];
        have_prev = true;
    }
    __syncthreads();
    return flags;
}

__device__ __forceinline__ uint32_t block_excl_scan_rle(uint32_t v, uint32_t* total)
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

// Both encode passes are persistent (grid stride over the tiles).
// Grid-stride step past field fd's RLE tiles (those of a field that is not
// run-length coded): the first tile index of this workgroup's stride at or
// beyond the field's end, so such a field costs one iteration per workgroup.
__device__ __forceinline__ uint32_t skip_field(const FieldDesc& fd, uint32_t t)
{
    const uint32_t end = fd.rt_base + fd.n_rt;
    return t + ((end - t + gridDim.x - 1) / gridDim.x) * gridDim.x;
}

__global__ __launch_bounds__(kBlock) void k_rle_count(const FieldDesc* __restrict__ F, int nf,
                                                      uint32_t* __restrict__ rcnt, uint32_t units)
{
    for (uint32_t t = blockIdx.x; t < units;) {
        const int f = find_field<&FieldDesc::rt_base>(F, nf, t);
        const FieldDesc& fd = F[f];
        const auto* dy = kconst(fd.dyn);
        if (dy->status != ST_OK || !rle_codec(dy->codec)) {
            t = skip_field(fd, t);
            continue;
        }
        uint16_t c[kRleItems];
        const uint32_t flags = run_flags(fd, (uint64_t)(t - fd.rt_base) * kRleTile, c);
        uint32_t tot;
        block_excl_scan_rle(__popc(flags), &tot);
        if (threadIdx.x == 0) rcnt[t] = tot;
        t += gridDim.x;
    }
}

// what: kRleValArc writes the run values into the archive (RLE codec),
// kRleValSym into the run-value stream of the Huffman pass (RLE+VLE codec),
// kRleStart the run starts (both codecs; they overwrite the outlier delta
// scratch, so only after the outlier list is written).
constexpr int kRleValArc = 1, kRleValSym = 2, kRleStart = 4;

__global__ __launch_bounds__(kBlock) void k_rle_write(const FieldDesc* __restrict__ F, int nf,
                                                      const uint32_t* __restrict__ roff, uint32_t units,
                                                      int what)
{
    for (uint32_t t = blockIdx.x; t < units; t += gridDim.x) {
        const int f = find_field<&FieldDesc::rt_base>(F, nf, t);
        const FieldDesc& fd = F[f];
        const auto* dy = kconst(fd.dyn);
        const int32_t codec = dy->codec;
        const bool val_arc = (what & kRleValArc) && codec == ARC_RLE;
        const bool val_sym = (what & kRleValSym) && codec == ARC_RLE_VLE;
        const bool starts = (what & kRleStart) && rle_codec(codec);
        if (dy->status != ST_OK || !(val_arc || val_sym || starts)) {
            t = skip_field(fd, t) - gridDim.x;  // the loop step adds it back
            continue;
        }
        const uint64_t lo = (uint64_t)(t - fd.rt_base) * kRleTile;
        // the tile's output offset is loaded before its codes, so its latency
        // overlaps theirs
        const uint32_t base = roff[t] - roff[fd.rt_base];
        uint16_t c[kRleItems];
        const uint32_t flags = run_flags(fd, lo, c);
        uint32_t tot;
        uint32_t pos = block_excl_scan_rle(__popc(flags), &tot) + base;
        EBC_G uint16_t* val = val_arc ? (EBC_G uint16_t*)(fd.arc + kHdr) : fd.vsym;
        const uint64_t i0 = lo + (uint64_t)threadIdx.x * kRleItems;
#pragma unroll
        for (int k = 0; k < kRleItems; ++k) {
            if (flags & (1u << k)) {
                if (val_arc || val_sym) val[pos] = c[k];
                if (starts) fd.rstart[pos] = (uint32_t)(i0 + k);
                ++pos;
            }
        }
    }
}

// RLE+VLE compress: the run count of each field (from the scanned tile
// counts) and its run-value histogram cleared; one workgroup per field.
__global__ __launch_bounds__(kBlock) void k_rle_total(const FieldDesc* __restrict__ F,
                                                      const uint32_t* __restrict__ roff)
{
    const FieldDesc& fd = F[blockIdx.x];
    EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || dy->codec != ARC_RLE_VLE) return;
    for (uint32_t b = threadIdx.x; b < fd.n_bins; b += kBlock) fd.vhist[b] = 0;
    if (threadIdx.x == 0) dy->n_runs = roff[fd.rt_base + fd.n_rt] - roff[fd.rt_base];
}

// RLE+VLE compress: histogram of the run values, kRleTile values per
// workgroup, privatised in LDS (the codes' histogram of Sec. II-A step 5,
// taken over the value stream).
__global__ __launch_bounds__(kBlock) void k_rle_vhist(const FieldDesc* __restrict__ F, int nf,
                                                      uint32_t units)
{
    extern __shared__ uint32_t sh[];
    for (uint32_t t = blockIdx.x; t < units; t += gridDim.x) {
        const int f = find_field<&FieldDesc::rt_base>(F, nf, t);
        const FieldDesc& fd = F[f];
        const auto* dy = kconst(fd.dyn);
        const uint64_t R = dy->n_runs;
        const uint64_t lo = (uint64_t)(t - fd.rt_base) * kRleTile;
        if (dy->status != ST_OK || dy->codec != ARC_RLE_VLE || lo >= R) {
            t = skip_field(fd, t) - gridDim.x;
            continue;
        }
        // wide bins: LDS slots as in construction (code 0, then a window
        // around the centre), other values counted in HBM directly
        const uint32_t nb = fd.n_bins, ns = hist_slots(nb), wlo = hist_win_lo(nb);
        const bool wide = nb > kMaxBins;
        for (uint32_t b = threadIdx.x; b < ns; b += kBlock) sh[b] = 0;
        __syncthreads();
        const uint64_t hi = min(lo + (uint64_t)kRleTile, R);
        for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
            const uint32_t v = fd.vsym[i];
            if (!wide) {
                atomicAdd(&sh[v], 1u);
            } else {
                const uint32_t dj = v - wlo;  // codes below the window wrap to large values
                if (v == 0) atomicAdd(&sh[0], 1u);
                else if (dj < kHistWin - 1) atomicAdd(&sh[dj + 1], 1u);
                else atomicAdd(&fd.vhist[v], 1u);
            }
        }
        __syncthreads();
        for (uint32_t b = threadIdx.x; b < ns; b += kBlock)
            if (sh[b]) atomicAdd(&fd.vhist[wide && b ? wlo + b - 1 : b], sh[b]);
        __syncthreads();
    }
}

// lengths = differences of successive starts; grid-stride over the runs
__global__ __launch_bounds__(kBlock) void k_rle_len(const FieldDesc* __restrict__ F)
{
    const FieldDesc& fd = F[blockIdx.y];
    const auto* dy = kconst(fd.dyn);
    if (dy->status != ST_OK || !rle_codec(dy->codec)) return;
    const uint64_t R = dy->n_runs;
    EBC_G uint32_t* len = (EBC_G uint32_t*)(fd.arc + dy->off_rlen);
    for (uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x; k < R;
         k += (uint64_t)gridDim.x * kBlock) {
        const uint64_t end = k + 1 < R ? fd.rstart[k + 1] : fd.n;
        len[k] = (uint32_t)(end - fd.rstart[k]);
    }
}

// ------------------------------------------------------------- decoding
// Run lengths from the archive into the batch-wide array.  A run must be
// non-empty and no longer than the field; the scan that follows works modulo
// 2^32, so the cover check below also needs the starts to increase.
__global__ __launch_bounds__(kBlock) void k_rle_prep(const FieldDesc* __restrict__ F, int nf,
                                                     uint32_t* __restrict__ starts)
{
    const uint32_t t = blockIdx.x;
    const int f = find_field<&FieldDesc::rl_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    const uint32_t k = (t - fd.rl_base) * kBlock + threadIdx.x;
    if (!rle_codec(fd.codec_hdr) || k >= fd.n_runs_hdr) return;
    const uint32_t L = ((const EBC_G uint32_t*)(fd.arc + fd.off_rlen))[k];
    if (L == 0 || (uint64_t)L > fd.n) atomicMin(&fd.dyn->status, ST_ERR_ARCHIVE);
    starts[fd.rle_base + k] = L;
}

// After the scan: the runs must cover the field exactly.  With every length
// in [1, n], the relative starts (mod 2^32) increase strictly exactly when no
// prefix sum wrapped, and then the last one is the true total, which must
// equal n.  One thread per run (the run-length prep grid).
__global__ __launch_bounds__(kBlock) void k_rle_check(const FieldDesc* __restrict__ F, int nf,
                                                      const uint32_t* __restrict__ starts)
{
    const uint32_t t = blockIdx.x;
    const int f = find_field<&FieldDesc::rl_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    const uint32_t k = (t - fd.rl_base) * kBlock + threadIdx.x;
    if (!rle_codec(fd.codec_hdr) || k >= fd.n_runs_hdr) return;
    const uint32_t* S = starts + fd.rle_base;
    const uint32_t s0 = S[0];
    const uint32_t a = S[k] - s0, b = S[k + 1] - s0;
    bool bad = b <= a;
    if (k + 1 == fd.n_runs_hdr && (uint64_t)b != fd.n) bad = true;
    if (bad) atomicMin(&fd.dyn->status, ST_ERR_ARCHIVE);
}

// After the check: for every output tile, the run that holds its first
// element (the largest r with start[r] <= tile start) and the number of runs
// it overlaps, one thread per tile, so that every tile's searches are in
// flight at once rather than one thread per workgroup searching while the
// others wait.  tmap[2t] = first run, tmap[2t + 1] = run count.
__global__ __launch_bounds__(kBlock) void k_rle_tilemap(const FieldDesc* __restrict__ F, int nf,
                                                        uint32_t units, const uint32_t* __restrict__ starts,
                                                        uint32_t* __restrict__ tmap)
{
    const uint32_t t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= units) return;
    const int f = find_field<&FieldDesc::rt_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    if (fd.dyn->status != ST_OK || !rle_codec(fd.codec_hdr)) return;
    const uint32_t* S = starts + fd.rle_base;
    const uint32_t s0 = S[0];
    const uint64_t lo = (uint64_t)(t - fd.rt_base) * kRleTile;
    const uint64_t hi = min(lo + (uint64_t)kRleTile, fd.n);
    uint32_t a = 0, b = fd.n_runs_hdr - 1;
    while (a < b) {
        const uint32_t m = (a + b + 1) >> 1;
        if ((uint64_t)(S[m] - s0) <= lo) a = m;
        else b = m - 1;
    }
    uint32_t c = a, d = fd.n_runs_hdr - 1;  // the run holding the tile's last element
    while (c < d) {
        const uint32_t m = (c + d + 1) >> 1;
        if ((uint64_t)(S[m] - s0) <= hi - 1) c = m;
        else d = m - 1;
    }
    tmap[2 * t] = a;
    tmap[2 * t + 1] = c - a + 1;
}

// runs of one tile staged in LDS by the expansion (a tile with more runs
// searches them in HBM)
constexpr uint32_t kRleStage = 1024;

// The kRleItems codes from element i0 on: the run holding i0 by binary search
// over the tile's nr run starts (relative to the field), then a forward walk.
template <class START, class VAL>
__device__ __forceinline__ void expand_codes(uint64_t i0, uint32_t nr, uint16_t c[kRleItems], START start,
                                             VAL value)
{
    uint32_t a = 0, b = nr - 1;
    while (a < b) {
        const uint32_t m = (a + b + 1) >> 1;
        if ((uint64_t)start(m) <= i0) a = m;
        else b = m - 1;
    }
#pragma unroll
    for (int k = 0; k < kRleItems; ++k) {
        const uint64_t i = i0 + k;
        while (a + 1 < nr && (uint64_t)start(a + 1) <= i) ++a;
        c[k] = value(a);
    }
}

__global__ __launch_bounds__(kBlock) void k_rle_expand(const FieldDesc* __restrict__ F, int nf,
                                                       const uint32_t* __restrict__ starts,
                                                       const uint32_t* __restrict__ tmap)
{
    __shared__ uint32_t s_start[kRleStage];
    __shared__ uint16_t s_val[kRleStage];
    const uint32_t t = blockIdx.x;
    const int f = find_field<&FieldDesc::rt_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || !rle_codec(fd.codec_hdr)) return;
    const uint32_t* S = starts + fd.rle_base;
    const uint32_t s0 = S[0];
    const uint64_t lo = (uint64_t)(t - fd.rt_base) * kRleTile;
    const uint64_t hi = min(lo + (uint64_t)kRleTile, fd.n);
    const uint32_t rlo = tmap[2 * t], nr = tmap[2 * t + 1];  // nr <= kRleTile: runs are non-empty
    const EBC_G uint16_t* val = fd.rval;
    const bool staged = nr <= kRleStage;  // uniform over the workgroup
    if (staged) {
        for (uint32_t i = threadIdx.x; i < nr; i += kBlock) {
            s_start[i] = S[rlo + i] - s0;
            s_val[i] = val[rlo + i];
        }
    }
    __syncthreads();
    const uint64_t i0 = lo + (uint64_t)threadIdx.x * kRleItems;
    if (i0 >= hi) return;
    uint16_t c[kRleItems];
    if (staged)
        expand_codes(i0, nr, c, [&](uint32_t k) { return s_start[k]; }, [&](uint32_t k) { return s_val[k]; });
    else
        expand_codes(i0, nr, c, [&](uint32_t k) { return S[rlo + k] - s0; },
                     [&](uint32_t k) { return (uint16_t)val[rlo + k]; });
    EBC_G uint16_t* __restrict__ q = fd.q;
    if (i0 + kRleItems <= hi) {
        uint4 x, y;
        x.x = c[0] | ((uint32_t)c[1] << 16), x.y = c[2] | ((uint32_t)c[3] << 16);
        x.z = c[4] | ((uint32_t)c[5] << 16), x.w = c[6] | ((uint32_t)c[7] << 16);
        y.x = c[8] | ((uint32_t)c[9] << 16), y.y = c[10] | ((uint32_t)c[11] << 16);
        y.z = c[12] | ((uint32_t)c[13] << 16), y.w = c[14] | ((uint32_t)c[15] << 16);
        *(EBC_G uint4*)(q + i0) = x;
        *(EBC_G uint4*)(q + i0 + 8) = y;
    } else {
        for (int k = 0; k < kRleItems; ++k)
            if (i0 + k < hi) q[i0 + k] = c[k];
    }
}

// The two encode passes stream the codes with a grid the device holds whole
// (8 workgroups of 256 per CU): with half that many workgroups in flight the
// count and write stages on a 1.2e8-value field took 75 and 101 us instead
// of 63 and 81.
constexpr uint32_t kRleBlocks = 2048;

hipError_t launch_rle_count(const FieldDesc* F, int nf, uint32_t units, uint32_t* rcnt, hipStream_t s)
{
    if (!units) return hipSuccess;
    const uint32_t g = units < kRleBlocks ? units : kRleBlocks;
    hipLaunchKernelGGL(k_rle_count, dim3(g), dim3(kBlock), 0, s, F, nf, rcnt, units);
    return hipGetLastError();
}

hipError_t launch_rle_write(const FieldDesc* F, int nf, uint32_t units, const uint32_t* roff, int what,
                            hipStream_t s)
{
    if (!units) return hipSuccess;
    const uint32_t g = units < kRleBlocks ? units : kRleBlocks;
    hipLaunchKernelGGL(k_rle_write, dim3(g), dim3(kBlock), 0, s, F, nf, roff, units, what);
    return hipGetLastError();
}

hipError_t launch_rle_vle_prep(const FieldDesc* F, int nf, uint32_t units, const uint32_t* roff,
                               uint32_t n_bins, hipStream_t s)
{
    hipLaunchKernelGGL(k_rle_total, dim3(nf), dim3(kBlock), 0, s, F, roff);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !units) return e;
    e = launch_rle_write(F, nf, units, roff, kRleValSym, s);
    if (e != hipSuccess) return e;
    const uint32_t g = units < kPersistentBlocks ? units : kPersistentBlocks;
    hipLaunchKernelGGL(k_rle_vhist, dim3(g), dim3(kBlock), (size_t)hist_slots(n_bins) * 4, s, F, nf, units);
    return hipGetLastError();
}

hipError_t launch_rle_len(const FieldDesc* F, int nf, uint32_t max_units, hipStream_t s)
{
    const uint32_t g = max(1u, min(max_units, 2048u));
    hipLaunchKernelGGL(k_rle_len, dim3(g, nf), dim3(kBlock), 0, s, F);
    return hipGetLastError();
}

hipError_t launch_rle_decode(const FieldDesc* F, int nf, uint32_t rl_units, uint32_t rt_units,
                             uint32_t* starts, uint32_t* tmap, uint32_t* tmp, uint32_t n_starts,
                             uint32_t scan_direct, hipStream_t s)
{
    if (!rl_units) return hipSuccess;
    hipLaunchKernelGGL(k_rle_prep, dim3(rl_units), dim3(kBlock), 0, s, F, nf, starts);
    hipError_t e = launch_scan(starts, n_starts, tmp, s, scan_direct);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rle_check, dim3(rl_units), dim3(kBlock), 0, s, F, nf, starts);
    if (rt_units) {
        hipLaunchKernelGGL(k_rle_tilemap, dim3((rt_units + kBlock - 1) / kBlock), dim3(kBlock), 0, s, F, nf,
                           rt_units, starts, tmap);
        hipLaunchKernelGGL(k_rle_expand, dim3(rt_units), dim3(kBlock), 0, s, F, nf, starts, tmap);
    }
    return hipGetLastError();
}

}  // namespace ebc
