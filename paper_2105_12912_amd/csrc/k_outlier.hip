// k_outlier.hip -- ordered outlier list: compaction at compression, scatter
// at decompression.
//
// Sec. IV-B.1 (modified quantisation): an out-of-range delta keeps its code
// slot as the placeholder 0 and is stored exactly in a separate list; before
// reconstruction the list is fused back (Algorithm 1, decompression half).
// The list is ordered by linear index.  Compression already counted the
// outliers of every row segment (the x-extent of one construct wave-tile);
// after a scan of those counts, each segment with outliers is compacted by
// one wavefront with ballot ranks.  Decompression scatters the list into a
// dense delta scratch, validates it against the codes and, for 3D fields,
// queues the chunks that hold outliers for the reconstruction fix-up.
#include "ebc_dev.h"
#include "ebc_launch.h"

namespace ebc {

constexpr uint32_t kSegPerBlock = kBlock;  // one segment per thread

uint32_t outlier_write_units(uint32_t n_seg) { return (n_seg + kSegPerBlock - 1) / kSegPerBlock; }

// element range [a, b) of segment s
__device__ __forceinline__ void seg_range(const FieldDesc& fd, uint32_t s, uint64_t& a, uint64_t& b)
{
    if (fd.rank == 1) {
        a = (uint64_t)s * 256;
        b = min(a + 256, fd.n);
    } else {
        const uint32_t xs = fd.xs;
        const uint64_t row = s / fd.nxb;
        const uint32_t xb = s % fd.nxb;
        a = row * fd.nx + (uint64_t)xb * xs;
        b = row * fd.nx + min((uint64_t)(xb + 1) * xs, (uint64_t)fd.nx);
    }
}

// One thread per row segment (at most 256 elements).  A thread whose
// segment holds outliers scans its codes for the placeholder 0 and writes
// the outliers in index order from the segment's scanned offset; all such
// threads of a wave scan concurrently.
__global__ __launch_bounds__(kBlock) void k_outlier_write(const FieldDesc* __restrict__ F, int nf,
                                                          const uint32_t* __restrict__ soff)
{
    const uint32_t t = blockIdx.x;
    const int f = find_field<&FieldDesc::ow_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    const auto* dy = kconst(fd.dyn);
    if (dy->status != ST_OK || dy->codec == ARC_CONST || dy->n_out == 0) return;
    const uint32_t sg = (t - fd.ow_base) * kSegPerBlock + threadIdx.x;
    if (sg >= fd.n_seg) return;
    const uint32_t* off = soff + fd.seg_base;
    const uint32_t o0 = off[sg], o1 = off[sg + 1];
    if (o0 == o1) return;
    EBC_G uint32_t* oidx = (EBC_G uint32_t*)(fd.arc + dy->off_oidx);
    EBC_G int32_t* oval = (EBC_G int32_t*)(fd.arc + dy->off_oval);
    uint32_t pos = o0 - off[0];
    const uint32_t end = o1 - off[0];
    uint64_t a, b;
    seg_range(fd, sg, a, b);
    const EBC_G uint16_t* q = fd.q;
    uint64_t i = a;
    // 8 codes at a time where aligned
    for (; i < b && (i & 7); ++i)
        if (q[i] == 0 && pos < end) oidx[pos] = (uint32_t)i, oval[pos] = fd.dsc[i], ++pos;
    // 32 codes at a time with their deltas loaded alongside (the deltas of
    // non-outliers are never used), so a block costs one memory round trip
    // however many outliers it holds
    for (; i + 32 <= b && pos < end; i += 32) {
        uint4 cv[4], dv[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) cv[k] = *(const EBC_G uint4*)(q + i + 8 * k);
#pragma unroll
        for (int k = 0; k < 8; ++k) dv[k] = *(const EBC_G uint4*)(fd.dsc + i + 4 * k);
#pragma unroll
        for (int e = 0; e < 32; ++e) {
            const uint4& c4 = cv[e / 8];
            const uint32_t cw = (e / 2) % 4 == 0 ? c4.x : (e / 2) % 4 == 1 ? c4.y : (e / 2) % 4 == 2 ? c4.z : c4.w;
            const uint4& d4 = dv[e / 4];
            const uint32_t dw = e % 4 == 0 ? d4.x : e % 4 == 1 ? d4.y : e % 4 == 2 ? d4.z : d4.w;
            if (((cw >> (16 * (e & 1))) & 0xFFFFu) == 0 && pos < end) {
                oidx[pos] = (uint32_t)(i + e);
                oval[pos] = (int32_t)dw;
                ++pos;
            }
        }
    }
    for (; i + 8 <= b && pos < end; i += 8) {
        const uint4 v = *(const EBC_G uint4*)(q + i);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (((w[k / 2] >> (16 * (k & 1))) & 0xFFFFu) == 0 && pos < end) {
                oidx[pos] = (uint32_t)(i + k);
                oval[pos] = fd.dsc[i + k];
                ++pos;
            }
        }
    }
    for (; i < b && pos < end; ++i)
        if (q[i] == 0) oidx[pos] = (uint32_t)i, oval[pos] = fd.dsc[i], ++pos;
}

// ------------------------------------------------------------- decoding
// one thread per listed outlier: index in range, strictly ascending, code 0
__global__ __launch_bounds__(kBlock) void k_outlier_scatter(const FieldDesc* __restrict__ F, int nf)
{
    const uint32_t t = blockIdx.x;
    const int f = find_field<&FieldDesc::sc_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || fd.codec_hdr == ARC_CONST) return;
    const uint64_t k = (uint64_t)(t - fd.sc_base) * kBlock + threadIdx.x;
    if (k >= fd.n_out_hdr) return;
    const EBC_G uint32_t* oidx = (const EBC_G uint32_t*)(fd.arc + fd.off_oidx);
    const EBC_G int32_t* oval = (const EBC_G int32_t*)(fd.arc + fd.off_oval);
    const uint32_t i = oidx[k];
    bool bad = i >= fd.n || (k > 0 && oidx[k - 1] >= i);
    if (!bad) bad = fd.q[i] != 0;
    if (bad) {
        atomicMin(&dy->status, ST_ERR_ARCHIVE);
        return;
    }
    fd.dsc[i] = oval[k];
    if (fd.rank == 3) {
        // queue this outlier's 8x8x8 chunk for the reconstruction fix-up,
        // once: the first outlier to set the chunk's flag appends it (the
        // flags were cleared by the reconstruction, which ran before)
        const uint32_t nx = fd.nx, ny = fd.ny;
        const uint32_t x = i % nx, yz = i / nx;
        const uint32_t y = yz % ny, z = yz / ny;
        const uint32_t wb = ((z >> 3) * (fd.nyb * kWavesPerBlock) + (y >> 3)) * fd.nxb + (x >> 8);
        const uint32_t bit = 1u << ((x & 255) >> 3);
        if ((atomicOr(&fd.oflag[wb], bit) & bit) == 0) fd.fixl[atomicAdd(&dy->fix_count, 1u)] = i;
    }
}

hipError_t launch_outlier_write(const FieldDesc* F, int nf, uint32_t units, const uint32_t* soff,
                                hipStream_t s)
{
    if (!units) return hipSuccess;
    hipLaunchKernelGGL(k_outlier_write, dim3(units), dim3(kBlock), 0, s, F, nf, soff);
    return hipGetLastError();
}

hipError_t launch_outlier_scatter(const FieldDesc* F, int nf, uint32_t units, hipStream_t s)
{
    if (!units) return hipSuccess;
    hipLaunchKernelGGL(k_outlier_scatter, dim3(units), dim3(kBlock), 0, s, F, nf);
    return hipGetLastError();
}

}  // namespace ebc
