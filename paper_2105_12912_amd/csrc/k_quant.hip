// k_quant.hip -- value range, quantisation step, dual-quantisation Lorenzo
// construction with fused histogram and outlier bookkeeping.
//
// Method: dual-quantisation (Sec. IV-A.1 "prequant"/"postquant", Algorithm 1
// compression half) with the first-order Lorenzo predictor (Sec. IV-B.2
// formulas) inside independent chunks (Sec. II-A step 1; 256 / 16x16 /
// 8x8x8), and the modified quantisation of Sec. IV-B.1 (code 0 marks an
// outlier whose delta is kept exactly).  The histogram of Sec. II-A step 5 is
// privatised per workgroup in LDS.
//
// Lorenzo difference as separable backward differences: with zero outside the
// chunk, d - p = Dz Dy Dx d, where Dx v(x) = v(x) - v(x-1) (v(-1) = 0 at a
// chunk start), and likewise for y and z.  A lane owns four consecutive x and
// walks y (and z) sequentially, so Dy and Dz are register-only; Dx needs one
// value from the lane on its left (DPP row shift).
#include "ebc_dev.h"
#include "ebc_launch.h"

namespace ebc {

// ---------------------------------------------------------------- value range
__global__ __launch_bounds__(kBlock) void k_range(const FieldDesc* __restrict__ F, int nf)
{
    const uint32_t u = blockIdx.x;
    const int f = find_field<&FieldDesc::range_base>(F, nf, u);
    const FieldDesc& fd = F[f];
    const uint64_t lo = (uint64_t)(u - fd.range_base) * kRangeUnit;
    const uint64_t hi = min(lo + (uint64_t)kRangeUnit, fd.n);
    const EBC_G float* __restrict__ in = fd.in;
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0u, bad = 0u;
    const bool aligned = ((uintptr_t)in & 15u) == 0;
    for (uint64_t i = lo + 4u * threadIdx.x; i < hi; i += 4u * kBlock) {
        float v[4];
        if (aligned && i + 3 < hi) {
            const f32x4 t = ld_nt_f4(in + i);
            v[0] = t.x, v[1] = t.y, v[2] = t.z, v[3] = t.w;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                bad |= !isfinite(v[k]);
                uint32_t key = float_key(v[k]);
                kmin = min(kmin, key);
                kmax = max(kmax, key);
            }
        } else {
            for (int k = 0; k < 4; ++k) {
                if (i + k < hi) {
                    float s = in[i + k];
                    bad |= !isfinite(s);
                    uint32_t key = float_key(s);
                    kmin = min(kmin, key);
                    kmax = max(kmax, key);
                }
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, o));
        kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, o));
        bad |= (uint32_t)__shfl_xor((int)bad, o);
    }
    __shared__ uint32_t s_red[3][kWavesPerBlock];
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) s_red[0][w] = kmin, s_red[1][w] = kmax, s_red[2][w] = bad;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kWavesPerBlock; ++k) {
            kmin = min(kmin, s_red[0][k]);
            kmax = max(kmax, s_red[1][k]);
            bad |= s_red[2][k];
        }
        EBC_G uint32_t* rp = fd.rpart + 3ull * (u - fd.range_base);
        rp[0] = kmin, rp[1] = kmax, rp[2] = bad;
    }
}

// ilogb of a positive finite double, exact for subnormals too.
__device__ __forceinline__ int ilogb_pos(double x)
{
    uint64_t b = (uint64_t)__double_as_longlong(x) & 0x7FFFFFFFFFFFFFFFull;
    int ex = (int)(b >> 52);
    if (ex == 0) {
        uint64_t m = b & ((1ull << 52) - 1);
        return (63 - __clzll((long long)m)) - 1074;
    }
    return ex - 1023;
}

// ------------------------------------------------------ quantisation step
// One workgroup per field: reduce the range partials, then derive
//   eb_abs = eb (ABS) or eb * (max - min) (REL, Sec. II-B.1 table caption),
//   eps = 2^max(ilogb(M) - ilogb(eb_abs) - 21, -22), rejected when > 2^-4,
//   ebx2 = (eb_abs * (1 - eps)) * 2, inv = 1 / ebx2,
// so that |x - xhat| <= eb survives the final fp32 rounding.  A REL field
// whose range is zero is stored as a constant.  Also zeroes the histogram.
__global__ __launch_bounds__(kBlock) void k_params(const FieldDesc* __restrict__ F)
{
    const FieldDesc& fd = F[blockIdx.x];
    EBC_G FieldDyn* dy = fd.dyn;
    for (uint32_t b = threadIdx.x; b < fd.n_bins; b += kBlock) fd.hist[b] = 0;
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0u, bad = 0u;
    for (uint32_t u = threadIdx.x; u < fd.range_units; u += kBlock) {
        const EBC_G uint32_t* rp = fd.rpart + 3ull * u;
        kmin = min(kmin, rp[0]);
        kmax = max(kmax, rp[1]);
        bad |= rp[2];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, o));
        kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, o));
        bad |= (uint32_t)__shfl_xor((int)bad, o);
    }
    __shared__ uint32_t s_red[3][kWavesPerBlock];
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) s_red[0][w] = kmin, s_red[1][w] = kmax, s_red[2][w] = bad;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int k = 1; k < kWavesPerBlock; ++k) {
        kmin = min(kmin, s_red[0][k]);
        kmax = max(kmax, s_red[1][k]);
        bad |= s_red[2][k];
    }
    FieldDyn d = {};
    d.status = ST_OK;
    d.codec = ARC_HUFFMAN;
    if (bad) {
        d.status = ST_ERR_NONFINITE;
        *dy = d;
        return;
    }
    const float mn = key_float(kmin), mx = key_float(kmax);
    d.mn = mn, d.mx = mx;
    const double range = (double)mx - (double)mn;
    const double M = fmax(fabs((double)mn), fabs((double)mx));
    if (fd.eb_mode == MODE_REL && range == 0.0) {
        d.codec = ARC_CONST;
        *dy = d;
        return;
    }
    const double eb_abs = fd.eb_mode == MODE_REL ? fd.eb * range : fd.eb;
    d.eb_abs = eb_abs;
    if (!(eb_abs > 0.0) || !isfinite(eb_abs)) {
        d.status = ST_ERR_EB_TOO_SMALL;
    } else if (eb_abs > 0x1p1000) {
        d.status = ST_ERR_EB;
    } else {
        int e = -22;
        if (M != 0.0) e = max(ilogb_pos(M) - ilogb_pos(eb_abs) - 21, -22);
        if (e > -4) {
            d.status = ST_ERR_EB_TOO_SMALL;
        } else {
            const double eps = __longlong_as_double((long long)((uint64_t)(1023 + e) << 52));
            const double shrunk = eb_abs * (1.0 - eps);
            d.ebx2 = shrunk * 2.0;
            d.inv = 1.0 / d.ebx2;
        }
    }
    *dy = d;
}

// ------------------------------------------------------ Lorenzo construct
template <bool VEC>
__device__ __forceinline__ void load_quad(const EBC_G float* __restrict__ p, uint64_t i, int nvalid,
                                          float v[4])
{
    if (VEC) {
        if (nvalid == 4) {
            const f32x4 t = ld_nt_f4(p + i);
            v[0] = t.x, v[1] = t.y, v[2] = t.z, v[3] = t.w;
        } else {
            v[0] = v[1] = v[2] = v[3] = 0.f;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = k < nvalid ? p[i + k] : 0.f;
    }
}

template <bool VEC>
__device__ __forceinline__ void store_codes(EBC_G uint16_t* __restrict__ q, uint64_t i, int nvalid,
                                            const uint32_t c[4])
{
    if (VEC) {
        if (nvalid == 4) {
            uint2 t;
            t.x = c[0] | (c[1] << 16);
            t.y = c[2] | (c[3] << 16);
            *(EBC_G uint2*)(q + i) = t;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nvalid) q[i + k] = (uint16_t)c[k];
    }
}

struct QuantCtx {
    double inv;
    int32_t r;
    uint32_t center;  // private count of the centre bin r (the dominant code)
};

// prequant one quad: d = rint(x * inv) in fp64 (Sec. IV-A.1)
__device__ __forceinline__ void prequant4(const float v[4], double inv, int32_t d[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) d[k] = (int32_t)__builtin_rint((double)v[k] * inv);
}

// postquant one quad of deltas: code, outlier scratch, histogram.
// Returns a 4-bit mask of outliers among the valid elements.
__device__ __forceinline__ uint32_t postquant4(const int32_t dl[4], int nvalid, QuantCtx& qc,
                                               uint32_t c[4], EBC_G int32_t* __restrict__ dsc,
                                               uint64_t i, uint32_t* sh_hist)
{
    uint32_t om = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool in = dl[k] > -qc.r && dl[k] < qc.r;
        c[k] = in ? (uint32_t)(dl[k] + qc.r) : 0u;
        if (k < nvalid) {
            if (!in) {
                om |= 1u << k;
                dsc[i + k] = dl[k];
            }
            if (c[k] == (uint32_t)qc.r) qc.center++;
            else atomicAdd(&sh_hist[c[k]], 1u);
        }
    }
    return om;
}

// Outliers of one row segment, summed over the LX lanes of this lane's group.
__device__ __forceinline__ uint32_t group_count(uint32_t om, int lx, int g)
{
    const uint64_t any = ballot(om != 0);
    if (any == 0) return 0;
    uint32_t cnt = 0;
    const uint64_t gmask = lx == 64 ? ~0ull : (((1ull << lx) - 1) << (g * lx));
#pragma unroll
    for (int k = 0; k < 4; ++k) cnt += __popcll(ballot((om >> k) & 1u) & gmask);
    return cnt;
}

template <int RANK, bool VEC>
__global__ __launch_bounds__(kBlock) void k_construct(const FieldDesc* __restrict__ F, int nf,
                                                      uint32_t* __restrict__ seg_cnt)
{
    extern __shared__ uint32_t sh_hist[];
    const uint32_t t = blockIdx.x;
    const int f = find_field<&FieldDesc::wg_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    const EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || dy->codec == ARC_CONST) return;
    const uint32_t nb = fd.n_bins;
    for (uint32_t b = threadIdx.x; b < nb; b += kBlock) sh_hist[b] = 0;
    __syncthreads();

    QuantCtx qc;
    qc.inv = dy->inv;
    qc.r = (int32_t)(nb / 2);
    qc.center = 0;
    const int l = lane_id();
    const uint32_t wt = (t - fd.wg_base) * kWavesPerBlock + threadIdx.x / kWave;
    const EBC_G float* __restrict__ in = fd.in;
    EBC_G uint16_t* __restrict__ qo = fd.q;
    EBC_G int32_t* __restrict__ dsc = fd.dsc;
    uint32_t* __restrict__ segs = seg_cnt + fd.seg_base;

    if (wt < fd.n_wave_tiles) {
        if (RANK == 1) {
            // wave-tile: 4 chunks of 256; lane owns x = c*256 + 4*l + k
            const uint64_t n = fd.n;
            float v[4][4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint64_t i0 = (uint64_t)wt * 1024 + c * 256 + 4 * l;
                const int nv = i0 >= n ? 0 : (int)min<uint64_t>(4, n - i0);
                if (VEC && nv == 4) load_quad<true>(in, i0, 4, v[c]);
                else load_quad<false>(in, i0, nv, v[c]);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint64_t i0 = (uint64_t)wt * 1024 + c * 256 + 4 * l;
                const int nv = i0 >= n ? 0 : (int)min<uint64_t>(4, n - i0);
                int32_t d[4], dl[4];
                prequant4(v[c], qc.inv, d);
                int left = __shfl_up(d[3], 1);
                if (l == 0) left = 0;
                dl[0] = d[0] - left, dl[1] = d[1] - d[0], dl[2] = d[2] - d[1], dl[3] = d[3] - d[2];
                uint32_t code[4];
                const uint32_t om = postquant4(dl, nv, qc, code, dsc, i0, sh_hist);
                if (VEC && nv == 4) store_codes<true>(qo, i0, 4, code);
                else store_codes<false>(qo, i0, nv, code);
                const uint32_t cnt = group_count(om, 64, 0);
                const uint64_t seg = (uint64_t)wt * 4 + c;
                if (l == 0 && seg < fd.n_seg) segs[seg] = cnt;
            }
        } else {
            const int lx = (int)fd.lx;
            const int xl = l % lx, g = l / lx;
            const uint32_t nxb = fd.nxb, nyb = fd.nyb;
            const uint32_t xb = wt % nxb;
            const uint32_t yb = (wt / nxb) % nyb;
            const uint32_t zb = wt / (nxb * nyb);
            const uint32_t nx = fd.nx, ny = fd.ny, nz = fd.nz;
            const uint32_t x0 = xb * 4u * lx + 4u * xl;
            const int nv_x = x0 >= nx ? 0 : (int)min<uint32_t>(4, nx - x0);
            // chunk-row of x: 16 elements (4 lanes) in 2D, 8 elements (2 lanes) in 3D
            const bool x_first = RANK == 2 ? (xl % 4) == 0 : (xl % 2) == 0;
            constexpr int CY = RANK == 2 ? 16 : 8;
            constexpr int CZ = RANK == 2 ? 1 : 8;
            const uint32_t y0 = yb * (uint32_t)(CY * (kWave / lx)) + (uint32_t)(CY * g);
            const uint32_t z0 = zb * CZ;
            int32_t fprev[CY][4];
#pragma unroll
            for (int j = 0; j < CY; ++j)
#pragma unroll
                for (int k = 0; k < 4; ++k) fprev[j][k] = 0;
            for (int iz = 0; iz < CZ; ++iz) {
                const uint32_t z = z0 + iz;
                float v[CY][4];
#pragma unroll
                for (int j = 0; j < CY; ++j) {
                    const uint32_t y = y0 + j;
                    const bool rowok = y < ny && z < nz;
                    const uint64_t i0 = ((uint64_t)z * ny + y) * nx + x0;
                    load_quad<VEC>(in, i0, rowok ? nv_x : 0, v[j]);
                }
                int32_t eprev[4] = {0, 0, 0, 0};
#pragma unroll
                for (int j = 0; j < CY; ++j) {
                    const uint32_t y = y0 + j;
                    const bool rowok = y < ny && z < nz;
                    const int nv = rowok ? nv_x : 0;
                    const uint64_t i0 = ((uint64_t)z * ny + y) * nx + x0;
                    int32_t d[4], e[4], dl[4];
                    prequant4(v[j], qc.inv, d);
                    int left = dpp_shr1(d[3]);
                    if (x_first) left = 0;
                    e[0] = d[0] - left, e[1] = d[1] - d[0], e[2] = d[2] - d[1], e[3] = d[3] - d[2];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int32_t fy = e[k] - eprev[k];  // Dy Dx d
                        eprev[k] = e[k];
                        if (RANK == 3) {
                            dl[k] = fy - fprev[j][k];  // Dz Dy Dx d
                            fprev[j][k] = fy;
                        } else {
                            dl[k] = fy;
                        }
                    }
                    uint32_t code[4];
                    const uint32_t om = postquant4(dl, nv, qc, code, dsc, i0, sh_hist);
                    store_codes<VEC>(qo, i0, nv, code);
                    const uint32_t cnt = group_count(om, lx, g);
                    if (xl == 0 && rowok) segs[((uint64_t)z * ny + y) * nxb + xb] = cnt;
                }
            }
        }
    }
    // centre-bin counts: wave reduction, then one LDS add per wave
    const uint32_t cs = wave_sum_u32(qc.center);
    if (l == 0 && cs) atomicAdd(&sh_hist[qc.r], cs);
    __syncthreads();
    EBC_G uint32_t* hp = fd.hpart + (uint64_t)(t - fd.wg_base) * nb;
    for (uint32_t b = threadIdx.x; b < nb; b += kBlock) hp[b] = sh_hist[b];
}

// ------------------------------------------------------ histogram reduce
// grid (ceil(n_bins / 256), kHistSplit, nf): split the partial rows of a
// field over kHistSplit workgroups, then add into the field histogram.
constexpr int kHistSplit = 64;
__global__ __launch_bounds__(kBlock) void k_hist_reduce(const FieldDesc* __restrict__ F)
{
    const FieldDesc& fd = F[blockIdx.z];
    if (fd.dyn->status != ST_OK || fd.dyn->codec == ARC_CONST) return;
    const uint32_t b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= fd.n_bins) return;
    const uint32_t nb = fd.n_bins;
    uint32_t s = 0;
    for (uint32_t r = blockIdx.y; r < fd.wg_tiles; r += kHistSplit) s += fd.hpart[(uint64_t)r * nb + b];
    if (s) atomicAdd(&fd.hist[b], s);
}

// ------------------------------------------------------------- launchers
hipError_t launch_range(const FieldDesc* F, int nf, uint32_t units, hipStream_t s)
{
    if (units == 0) return hipSuccess;
    hipLaunchKernelGGL(k_range, dim3(units), dim3(kBlock), 0, s, F, nf);
    return hipGetLastError();
}

hipError_t launch_params(const FieldDesc* F, int nf, hipStream_t s)
{
    hipLaunchKernelGGL(k_params, dim3(nf), dim3(kBlock), 0, s, F);
    return hipGetLastError();
}

hipError_t launch_construct(const FieldDesc* F, int nf, int rank, bool vec, uint32_t wg_tiles,
                            uint32_t n_bins, uint32_t* seg_cnt, hipStream_t s)
{
    if (wg_tiles == 0) return hipSuccess;
    const size_t sh = (size_t)n_bins * sizeof(uint32_t);
    const dim3 g(wg_tiles), b(kBlock);
    if (rank == 1) {
        if (vec) hipLaunchKernelGGL((k_construct<1, true>), g, b, sh, s, F, nf, seg_cnt);
        else hipLaunchKernelGGL((k_construct<1, false>), g, b, sh, s, F, nf, seg_cnt);
    } else if (rank == 2) {
        if (vec) hipLaunchKernelGGL((k_construct<2, true>), g, b, sh, s, F, nf, seg_cnt);
        else hipLaunchKernelGGL((k_construct<2, false>), g, b, sh, s, F, nf, seg_cnt);
    } else {
        if (vec) hipLaunchKernelGGL((k_construct<3, true>), g, b, sh, s, F, nf, seg_cnt);
        else hipLaunchKernelGGL((k_construct<3, false>), g, b, sh, s, F, nf, seg_cnt);
    }
    return hipGetLastError();
}

hipError_t launch_hist_reduce(const FieldDesc* F, int nf, uint32_t n_bins, hipStream_t s)
{
    dim3 g((n_bins + kBlock - 1) / kBlock, kHistSplit, nf);
    hipLaunchKernelGGL(k_hist_reduce, g, dim3(kBlock), 0, s, F);
    return hipGetLastError();
}

}  // namespace ebc
