// k_recon.hip -- Lorenzo reconstruction as an N-D partial sum, with the
// outlier fuse and dequantisation folded in.
//
// Sec. IV-B.2: with q' = q - r (outliers substituted, Sec. IV-B.1), the
// reconstructed integers are the inclusive N-D prefix sum of q' within each
// chunk, and the N-D sum splits into one-axis passes (x, then y, then z;
// Algorithm 1, decompression half).  Output = d * (2 eb) rounded once to fp32.
//
// Mapping (same tiles and lane layout as construction): a lane owns four
// consecutive x.  The x pass is a within-lane prefix plus the totals of the
// quads to its left in the chunk row (one DPP row shift in 3D, two lane
// shuffles in 2D, a full-wave scan for the 256-long 1D chunk).  The y pass is
// a scan across the lanes of a chunk column with DPP row shifts (8 lanes in
// 3D, the 16 lanes of a DPP row in 2D); the z pass is a running sum in
// registers as the wave walks the chunk's planes.  Integer sums wrap modulo
// 2^32 exactly as the CPU recurrence truncated to int32 does.
#include "ebc_dev.h"
#include "ebc_launch.h"

namespace ebc {

template <bool VEC>
__device__ __forceinline__ void load_codes(const EBC_G uint16_t* __restrict__ q, uint64_t i, int nvalid,
                                           uint32_t c[4])
{
    if (VEC) {
        if (nvalid == 4) {
            const u32x2 t = ld_nt_u2(q + i);
            c[0] = t.x & 0xFFFF, c[1] = t.x >> 16, c[2] = t.y & 0xFFFF, c[3] = t.y >> 16;
        } else {
            c[0] = c[1] = c[2] = c[3] = 1;  // never used; non-zero so no outlier lookup
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) c[k] = k < nvalid ? q[i + k] : 1u;
    }
}

template <bool VEC>
__device__ __forceinline__ void store_quad(EBC_G float* __restrict__ o, uint64_t i, int nvalid,
                                           const float v[4])
{
    if (VEC) {
        if (nvalid == 4) st_nt_f4(o + i, f32x4{v[0], v[1], v[2], v[3]});
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nvalid) o[i + k] = v[k];
    }
}

// q' for a quad: code - r, or the exact outlier delta where the code is 0
__device__ __forceinline__ void fuse4(const uint32_t c[4], int nvalid, int32_t r,
                                      const EBC_G int32_t* __restrict__ dsc, uint64_t i, uint32_t qp[4],
                                      uint32_t& zeros)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (c[k] == 0 && k < nvalid) {
            qp[k] = (uint32_t)dsc[i + k];
            ++zeros;
        } else {
            qp[k] = c[k] - (uint32_t)r;
        }
    }
}

__device__ __forceinline__ void dequant4(const uint32_t s[4], double ebx2, float v[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (float)((double)(int32_t)s[k] * ebx2);
}

template <int RANK, bool VEC>
__global__ __launch_bounds__(kBlock) void k_reconstruct(const FieldDesc* __restrict__ F, int nf)
{
    const uint32_t t = blockIdx.x;
    const int f = find_field<&FieldDesc::wg_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    const EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || dy->codec == ARC_CONST) return;
    const int l = lane_id();
    const uint32_t w = threadIdx.x / kWave;
    const uint32_t tl = t - fd.wg_base;
    const int32_t r = (int32_t)(fd.n_bins / 2);
    const double ebx2 = dy->ebx2;
    const EBC_G uint16_t* __restrict__ q = fd.q;
    const EBC_G int32_t* __restrict__ dsc = fd.dsc;
    EBC_G float* __restrict__ out = fd.outf;
    uint32_t zeros = 0;

    if (RANK == 1) {
        const uint32_t wt = tl * kWavesPerBlock + w;
        if (wt < fd.n_wave_tiles) {
            const uint64_t n = fd.n;
            uint32_t c[4][4];
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                const uint64_t i0 = (uint64_t)wt * 1024 + ch * 256 + 4 * l;
                const int nv = i0 >= n ? 0 : (int)min<uint64_t>(4, n - i0);
                if (VEC && nv == 4) load_codes<true>(q, i0, 4, c[ch]);
                else load_codes<false>(q, i0, nv, c[ch]);
            }
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                const uint64_t i0 = (uint64_t)wt * 1024 + ch * 256 + 4 * l;
                const int nv = i0 >= n ? 0 : (int)min<uint64_t>(4, n - i0);
                uint32_t s[4];
                fuse4(c[ch], nv, r, dsc, i0, s, zeros);
                s[1] += s[0], s[2] += s[1], s[3] += s[2];
                // exclusive prefix of the lane totals over the 256-long chunk
                const uint32_t excl = wave_incl_scan_u32(s[3]) - s[3];
#pragma unroll
                for (int k = 0; k < 4; ++k) s[k] += excl;
                float v[4];
                dequant4(s, ebx2, v);
                if (VEC && nv == 4) store_quad<true>(out, i0, 4, v);
                else store_quad<false>(out, i0, nv, v);
            }
        }
    } else {
        const uint32_t wx = fd.wx, wy = kWavesPerBlock / wx;
        const uint32_t wxi = w % wx, wyi = w / wx;
        const uint32_t nxb = fd.nxb, nyb = fd.nyb;
        const uint32_t xb = tl % nxb, yb = (tl / nxb) % nyb, zb = tl / (nxb * nyb);
        const uint32_t nx = fd.nx, ny = fd.ny, nz = fd.nz;
        if (RANK == 3) {
            // lane = 8 * xq + y, one z-plane of an 8x8x8 chunk pair per step
            const uint32_t y = l & 7, xq = l >> 3;
            const uint32_t x0 = xb * fd.xs + wxi * 32 + 4 * xq;
            const uint32_t yy = yb * 8 * wy + wyi * 8 + y;
            const uint32_t z0 = zb * 8;
            const int nv_x = x0 >= nx ? 0 : (int)min<uint32_t>(4, nx - x0);
            uint32_t zprev[4] = {0, 0, 0, 0};
            // the whole 8-plane column of codes in flight at once
            uint32_t c[8][4];
#pragma unroll
            for (int iz = 0; iz < 8; ++iz) {
                const bool ok = yy < ny && z0 + iz < nz;
                load_codes<VEC>(q, ((uint64_t)(z0 + iz) * ny + yy) * nx + x0, ok ? nv_x : 0, c[iz]);
            }
#pragma unroll
            for (int iz = 0; iz < 8; ++iz) {
                const uint32_t z = z0 + iz;
                const int nv = (yy < ny && z < nz) ? nv_x : 0;
                const uint64_t i0 = ((uint64_t)z * ny + yy) * nx + x0;
                uint32_t s[4];
                fuse4(c[iz], nv, r, dsc, i0, s, zeros);
                // x pass: within the quad, then the quad to the left in the chunk
                s[1] += s[0], s[2] += s[1], s[3] += s[2];
                uint32_t left = dpp_shr_u<8>(s[3]);
                if ((xq & 1) == 0) left = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) s[k] += left;
                // y pass: inclusive scan over the 8 lanes of the chunk column
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    uint32_t a = dpp_shr_u<1>(s[k]);
                    s[k] += y >= 1 ? a : 0u;
                    a = dpp_shr_u<2>(s[k]);
                    s[k] += y >= 2 ? a : 0u;
                    a = dpp_shr_u<4>(s[k]);
                    s[k] += y >= 4 ? a : 0u;
                    // z pass: running sum over the planes of the chunk
                    s[k] += zprev[k];
                    zprev[k] = s[k];
                }
                float v[4];
                dequant4(s, ebx2, v);
                store_quad<VEC>(out, i0, nv, v);
            }
        } else {
            // lane = 16 * xq + y, four 16x16 chunks along x per wave
            const uint32_t y = l & 15, xq = l >> 4;
            const uint32_t yy = yb * 16 * wy + wyi * 16 + y;
            const bool yok = yy < ny;
            // the four chunks of the wave in flight at once
            uint32_t c[4][4];
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                const uint32_t x0 = xb * fd.xs + wxi * 64 + 16 * ch + 4 * xq;
                const int nv = (!yok || x0 >= nx) ? 0 : (int)min<uint32_t>(4, nx - x0);
                load_codes<VEC>(q, (uint64_t)yy * nx + x0, nv, c[ch]);
            }
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                const uint32_t x0 = xb * fd.xs + wxi * 64 + 16 * ch + 4 * xq;
                const int nv = (!yok || x0 >= nx) ? 0 : (int)min<uint32_t>(4, nx - x0);
                const uint64_t i0 = (uint64_t)yy * nx + x0;
                uint32_t s[4];
                fuse4(c[ch], nv, r, dsc, i0, s, zeros);
                // x pass: within the quad, then over the 4 quads of the chunk row
                s[1] += s[0], s[2] += s[1], s[3] += s[2];
                const uint32_t tot = s[3];
                uint32_t inc = tot;
                uint32_t a = (uint32_t)__shfl_up((int)inc, 16);
                inc += xq >= 1 ? a : 0u;
                a = (uint32_t)__shfl_up((int)inc, 32);
                inc += xq >= 2 ? a : 0u;
                const uint32_t left = inc - tot;
                // y pass: the 16 rows of a chunk are the 16 lanes of a DPP row
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    s[k] += left;
                    s[k] += dpp_shr_u<1>(s[k]);
                    s[k] += dpp_shr_u<2>(s[k]);
                    s[k] += dpp_shr_u<4>(s[k]);
                    s[k] += dpp_shr_u<8>(s[k]);
                }
                float v[4];
                dequant4(s, ebx2, v);
                store_quad<VEC>(out, i0, nv, v);
            }
        }
    }
    // zero codes seen by this workgroup (checked against the outlier count)
    const uint32_t zs = wave_sum_u32(zeros);
    __shared__ uint32_t s_z[kWavesPerBlock];
    if (l == 0) s_z[w] = zs;
    __syncthreads();
    if (threadIdx.x == 0) fd.zpart[tl] = s_z[0] + s_z[1] + s_z[2] + s_z[3];
}

// decompression epilogue: the code-0 count must equal the outlier count
__global__ __launch_bounds__(kBlock) void k_recon_check(const FieldDesc* __restrict__ F)
{
    const FieldDesc& fd = F[blockIdx.x];
    EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || fd.codec_hdr == ARC_CONST) return;
    uint64_t z = 0;
    for (uint32_t i = threadIdx.x; i < fd.wg_tiles; i += kBlock) z += fd.zpart[i];
    z = wave_sum_u64(z);
    __shared__ uint64_t s_z[kWavesPerBlock];
    if (lane_id() == 0) s_z[threadIdx.x / kWave] = z;
    __syncthreads();
    if (threadIdx.x == 0) {
        z = s_z[0] + s_z[1] + s_z[2] + s_z[3];
        dy->zero_count = z;
        if (z != fd.n_out_hdr) dy->status = ST_ERR_ARCHIVE;
    }
}

// decompression prologue: per-field device scalars from the header values
__global__ void k_dinit(const FieldDesc* __restrict__ F, int nf)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const FieldDesc& fd = F[f];
    FieldDyn d = {};
    d.status = ST_OK;
    d.codec = fd.codec_hdr;
    d.ebx2 = fd.ebx2_hdr;
    d.n_out = fd.n_out_hdr;
    *fd.dyn = d;
}

// constant field (range zero): every element is the stored value
__global__ __launch_bounds__(kBlock) void k_fill_const(const FieldDesc* __restrict__ F, int nf)
{
    const uint32_t u = blockIdx.x;
    const int f = find_field<&FieldDesc::range_base>(F, nf, u);
    const FieldDesc& fd = F[f];
    if (fd.codec_hdr != ARC_CONST || fd.dyn->status != ST_OK) return;
    const uint64_t lo = (uint64_t)(u - fd.range_base) * kRangeUnit;
    const uint64_t hi = min(lo + (uint64_t)kRangeUnit, fd.n);
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock) fd.outf[i] = fd.cval;
}

hipError_t launch_reconstruct(const FieldDesc* F, int nf, int rank, bool vec, uint32_t wg_tiles,
                              hipStream_t s)
{
    if (wg_tiles == 0) return hipSuccess;
    const dim3 g(wg_tiles), b(kBlock);
    if (rank == 1) {
        if (vec) hipLaunchKernelGGL((k_reconstruct<1, true>), g, b, 0, s, F, nf);
        else hipLaunchKernelGGL((k_reconstruct<1, false>), g, b, 0, s, F, nf);
    } else if (rank == 2) {
        if (vec) hipLaunchKernelGGL((k_reconstruct<2, true>), g, b, 0, s, F, nf);
        else hipLaunchKernelGGL((k_reconstruct<2, false>), g, b, 0, s, F, nf);
    } else {
        if (vec) hipLaunchKernelGGL((k_reconstruct<3, true>), g, b, 0, s, F, nf);
        else hipLaunchKernelGGL((k_reconstruct<3, false>), g, b, 0, s, F, nf);
    }
    return hipGetLastError();
}

hipError_t launch_recon_check(const FieldDesc* F, int nf, hipStream_t s)
{
    hipLaunchKernelGGL(k_recon_check, dim3(nf), dim3(kBlock), 0, s, F);
    return hipGetLastError();
}

hipError_t launch_dinit(const FieldDesc* F, int nf, hipStream_t s)
{
    hipLaunchKernelGGL(k_dinit, dim3((nf + 63) / 64), dim3(64), 0, s, F, nf);
    return hipGetLastError();
}

hipError_t launch_fill_const(const FieldDesc* F, int nf, uint32_t units, hipStream_t s)
{
    if (!units) return hipSuccess;
    hipLaunchKernelGGL(k_fill_const, dim3(units), dim3(kBlock), 0, s, F, nf);
    return hipGetLastError();
}

}  // namespace ebc
