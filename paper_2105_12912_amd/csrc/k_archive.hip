// k_archive.hip -- archive layout, header and padding, descriptor upload.
//
// Archive format v2 (little-endian, 128-byte header, every section starts on
// a 16-byte boundary, padding is zero):
//   Huffman: u8 len[n_bins] | u16 sbits[n_sub] | u32 words[n_words]
//            (sbits: bit count of every sub-chunk of hs = min(hc, 256)
//            symbols; chunks of hc symbols start on a word, their sub-chunks
//            follow each other without padding)
//   RLE:     u16 val[n_runs] | u32 len[n_runs]
//   RLE+VLE: u8 len[n_bins] | u16 sbits | u32 words (the run values as a
//            Huffman stream of their own) | u32 rlen[n_runs]
//   all:     u32 outlier_index[n_out] | i32 outlier_delta[n_out]
// The paper leaves the container unspecified; the header records everything
// a decoder needs (dims, chunking, codec, step, section counts).
#include "ebc_dev.h"
#include "ebc_launch.h"

namespace ebc {

// Section offsets and total size from the scanned counts; checks capacity.
__global__ void k_layout(const FieldDesc* __restrict__ F, int nf, const uint32_t* __restrict__ soff,
                         const uint32_t* __restrict__ woff, const uint32_t* __restrict__ roff)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const FieldDesc& fd = F[f];
    EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK) return;
    if (dy->codec == ARC_CONST) {
        dy->total = kHdr;
        if (kHdr > fd.arc_cap) dy->status = ST_ERR_OUT_TOO_SMALL;
        return;
    }
    const uint64_t no = soff[fd.seg_base + fd.n_seg] - soff[fd.seg_base];
    dy->n_out = no;
    uint64_t off_o;
    if (dy->codec == ARC_HUFFMAN) {
        const uint64_t nw = woff[fd.hch_base + fd.n_hch] - woff[fd.hch_base];
        dy->n_words = nw;
        dy->n_runs = 0;
        dy->off_sbits = align16(kHdr + fd.n_bins);
        dy->off_words = align16(dy->off_sbits + 2ull * fd.n_sub);
        off_o = align16(dy->off_words + 4ull * nw);
    } else if (dy->codec == ARC_RLE_VLE) {
        // the Huffman stream of the R run values, then the run lengths
        const uint64_t R = roff[fd.rt_base + fd.n_rt] - roff[fd.rt_base];
        const uint64_t nch = (R + fd.hc - 1) / fd.hc, nsub = (R + fd.hs - 1) / fd.hs;
        const uint64_t nw = woff[fd.hch_base + nch] - woff[fd.hch_base];
        dy->n_runs = R;
        dy->n_words = nw;
        dy->off_sbits = align16(kHdr + fd.n_bins);
        dy->off_words = align16(dy->off_sbits + 2ull * nsub);
        dy->off_rlen = align16(dy->off_words + 4ull * nw);
        off_o = align16(dy->off_rlen + 4ull * R);
    } else {
        const uint64_t R = roff[fd.rt_base + fd.n_rt] - roff[fd.rt_base];
        dy->n_runs = R;
        dy->n_words = 0;
        dy->off_rlen = align16(kHdr + 2ull * R);
        off_o = align16(dy->off_rlen + 4ull * R);
    }
    dy->off_oidx = off_o;
    dy->off_oval = align16(off_o + 4ull * no);
    dy->total = align16(dy->off_oval + 4ull * no);
    if (dy->total > fd.arc_cap) dy->status = ST_ERR_OUT_TOO_SMALL;
}

__device__ __forceinline__ void zero_gap(EBC_G uint8_t* a, uint64_t from, uint64_t to, int lane)
{
    for (uint64_t i = from + lane; i < to; i += kWave) a[i] = 0;
}

// One wavefront per field: header bytes, Huffman length section, and the
// zero padding between sections.
__global__ void k_header(const FieldDesc* __restrict__ F, int nf)
{
    const int f = blockIdx.x;
    const FieldDesc& fd = F[f];
    const auto* dy = kconst(fd.dyn);
    if (dy->status != ST_OK) return;
    EBC_G uint8_t* a = fd.arc;
    const int l = threadIdx.x;
    __shared__ uint32_t h[32];
    if (l < 32) h[l] = 0;
    __syncthreads();
    if (l == 0) {
        h[0] = 0x31434245u;  // "EBC1"
        h[1] = 2u;           // version 2, flags 0
        h[2] = (uint32_t)fd.rank | ((uint32_t)dy->codec << 8) | ((uint32_t)fd.eb_mode << 16) |
               ((uint32_t)fd.dtype << 24);
        h[3] = fd.n_bins;
        const uint64_t dims[3] = {fd.nx, fd.ny, fd.nz};
        for (int k = 0; k < 3; ++k) {
            h[4 + 2 * k] = (uint32_t)dims[k];
            h[5 + 2 * k] = (uint32_t)(dims[k] >> 32);
        }
        const uint32_t ch[3] = {fd.rank == 1 ? 256u : fd.rank == 2 ? 16u : 8u,
                                fd.rank == 1 ? 1u : fd.rank == 2 ? 16u : 8u,
                                fd.rank == 3 ? 8u : 1u};
        h[10] = ch[0], h[11] = ch[1], h[12] = ch[2];
        h[13] = fd.hc;
        const double dd[3] = {fd.eb, dy->eb_abs, dy->ebx2};
        for (int k = 0; k < 3; ++k) {
            const uint64_t b = (uint64_t)__double_as_longlong(dd[k]);
            h[14 + 2 * k] = (uint32_t)b;
            h[15 + 2 * k] = (uint32_t)(b >> 32);
        }
        // constant value as f64 (exact for an fp32 field)
        const uint64_t cb = dy->codec == ARC_CONST ? (uint64_t)__double_as_longlong((double)dy->mn) : 0ull;
        h[20] = (uint32_t)cb;
        h[21] = (uint32_t)(cb >> 32);
        const uint64_t na = dy->codec == ARC_HUFFMAN ? (uint64_t)fd.n_hch : dy->n_runs;  // RLE, RLE+VLE: runs
        const uint64_t v[4] = {dy->codec == ARC_CONST ? 0ull : dy->n_out,
                               dy->codec == ARC_CONST ? 0ull : na, dy->n_words, dy->total};
        for (int k = 0; k < 4; ++k) {
            h[22 + 2 * k] = (uint32_t)v[k];
            h[23 + 2 * k] = (uint32_t)(v[k] >> 32);
        }
        h[30] = huff_codec(dy->codec) ? fd.hs : 0u;
        h[31] = 0;
    }
    __syncthreads();
    if (l < 32) ((EBC_G uint32_t*)a)[l] = h[l];
    if (dy->codec == ARC_CONST) return;
    const uint64_t no = dy->n_out;
    if (huff_codec(dy->codec)) {
        const bool vle = dy->codec == ARC_RLE_VLE;
        const uint64_t nsub = vle ? (dy->n_runs + fd.hs - 1) / fd.hs : fd.n_sub;
#pragma unroll 8
        for (uint32_t s = l; s < fd.n_bins; s += kWave) a[kHdr + s] = fd.len[s];
        zero_gap(a, kHdr + fd.n_bins, dy->off_sbits, l);
        zero_gap(a, dy->off_sbits + 2ull * nsub, dy->off_words, l);
        const uint64_t words_end = dy->off_words + 4ull * dy->n_words;
        if (vle) {
            zero_gap(a, words_end, dy->off_rlen, l);
            zero_gap(a, dy->off_rlen + 4ull * dy->n_runs, dy->off_oidx, l);
        } else {
            zero_gap(a, words_end, dy->off_oidx, l);
        }
    } else {
        zero_gap(a, kHdr + 2ull * dy->n_runs, dy->off_rlen, l);
        zero_gap(a, dy->off_rlen + 4ull * dy->n_runs, dy->off_oidx, l);
    }
    zero_gap(a, dy->off_oidx + 4ull * no, dy->off_oval, l);
    zero_gap(a, dy->off_oval + 4ull * no, dy->total, l);
}

// Async result record: archive size (0 on error) and status.
__global__ void k_result(const FieldDesc* __restrict__ F, uint64_t* __restrict__ res)
{
    const EBC_G FieldDyn* dy = F[0].dyn;
    res[0] = dy->status == ST_OK ? dy->total : 0ull;
    ((int32_t*)(res + 1))[0] = dy->status;
    ((int32_t*)(res + 1))[1] = dy->codec;
}

__global__ void k_status(const FieldDesc* __restrict__ F, int32_t* __restrict__ st)
{
    *st = F[0].dyn->status;
}

// Batch result records in the caller's order: {archive bytes (0 on error),
// status, codec} = 16 bytes per field.
__global__ void k_batch_results(const FieldDesc* __restrict__ F, int nf, uint64_t* __restrict__ res)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nf) return;
    const FieldDesc& fd = F[k];
    const EBC_G FieldDyn* dy = fd.dyn;
    uint64_t* r = res + 2ull * fd.slot;
    r[0] = dy->status == ST_OK ? dy->total : 0ull;
    r[1] = (uint64_t)(uint32_t)dy->status | ((uint64_t)(uint32_t)dy->codec << 32);
}

__global__ void k_batch_status(const FieldDesc* __restrict__ F, int nf, int32_t* __restrict__ st)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nf) return;
    st[F[k].slot] = F[k].dyn->status;
}

// Upload up to kDescPerLaunch descriptors passed by value.
__global__ void k_put_desc(DescBlob blob, FieldDesc* __restrict__ dst)
{
    const int k = threadIdx.x;
    if (k < blob.count) dst[blob.first + k] = blob.d[k];
}

hipError_t launch_layout(const FieldDesc* F, int nf, const uint32_t* soff, const uint32_t* woff,
                         const uint32_t* roff, hipStream_t s)
{
    hipLaunchKernelGGL(k_layout, dim3((nf + 63) / 64), dim3(64), 0, s, F, nf, soff, woff, roff);
    return hipGetLastError();
}

hipError_t launch_header(const FieldDesc* F, int nf, hipStream_t s)
{
    hipLaunchKernelGGL(k_header, dim3(nf), dim3(kWave), 0, s, F, nf);
    return hipGetLastError();
}

hipError_t launch_result(const FieldDesc* F, uint64_t* res, hipStream_t s)
{
    hipLaunchKernelGGL(k_result, dim3(1), dim3(1), 0, s, F, res);
    return hipGetLastError();
}

hipError_t launch_status(const FieldDesc* F, int32_t* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_status, dim3(1), dim3(1), 0, s, F, st);
    return hipGetLastError();
}

hipError_t launch_batch_results(const FieldDesc* F, int nf, uint64_t* res, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_results, dim3((nf + 63) / 64), dim3(64), 0, s, F, nf, res);
    return hipGetLastError();
}

hipError_t launch_batch_status(const FieldDesc* F, int nf, int32_t* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_status, dim3((nf + 63) / 64), dim3(64), 0, s, F, nf, st);
    return hipGetLastError();
}

hipError_t upload_descs(const FieldDesc* host, int nf, FieldDesc* dev, hipStream_t s)
{
    for (int first = 0; first < nf; first += kDescPerLaunch) {
        DescBlob b;
        b.first = first;
        b.count = min(kDescPerLaunch, nf - first);
        for (int k = 0; k < b.count; ++k) b.d[k] = host[first + k];
        hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(kDescPerLaunch), 0, s, b, dev);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace ebc
