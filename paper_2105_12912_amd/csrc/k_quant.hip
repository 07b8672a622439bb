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
// chunk start), and likewise for y and z.  A lane owns four consecutive x.
// 2D: lane = 16 xq + y, so the 16 rows of a 16x16 chunk are the 16 lanes of a
// DPP row (Dy is one row shift) and Dx takes the left quad from lane - 16;
// a wave walks four chunks along x.  3D: lane = 8 xq + y covers 32 x by 8 y,
// Dy is a row shift by 1, Dx by 8, and the wave walks the 8 z-planes of its
// chunks keeping Dy Dx of the previous plane in registers for Dz.  1D: a wave
// covers four 256-long chunks.  Every load and store is a 16-byte quad per
// lane; each quad is read and written once.
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

// Value range of an fp64 field: the same ordered-key min / max, with 64-bit
// keys; the partials take the unit's three 64-bit words (min, max, bad).
__device__ __forceinline__ uint64_t double_key(double f)
{
    const uint64_t b = (uint64_t)__double_as_longlong(f);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double key_double(uint64_t k)
{
    const uint64_t b = (k & 0x8000000000000000ull) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    return __longlong_as_double((long long)b);
}

__global__ __launch_bounds__(kBlock) void k_range64(const FieldDesc* __restrict__ F, int nf)
{
    const uint32_t u = blockIdx.x;
    const int f = find_field<&FieldDesc::range_base>(F, nf, u);
    const FieldDesc& fd = F[f];
    const uint64_t lo = (uint64_t)(u - fd.range_base) * kRangeUnit;
    const uint64_t hi = min(lo + (uint64_t)kRangeUnit, fd.n);
    const EBC_G double* __restrict__ in = fd.in64;
    uint64_t kmin = ~0ull, kmax = 0ull;
    uint32_t bad = 0u;
    for (uint64_t i = lo + 2u * threadIdx.x; i < hi; i += 2u * kBlock) {
        for (int k = 0; k < 2; ++k) {
            if (i + k < hi) {
                const double v = in[i + k];
                bad |= !isfinite(v);
                const uint64_t key = double_key(v);
                kmin = min(kmin, key);
                kmax = max(kmax, key);
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        kmin = min(kmin, (uint64_t)__shfl_xor((long long)kmin, o));
        kmax = max(kmax, (uint64_t)__shfl_xor((long long)kmax, o));
        bad |= (uint32_t)__shfl_xor((int)bad, o);
    }
    __shared__ uint64_t s_red[3][kWavesPerBlock];
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) s_red[0][w] = kmin, s_red[1][w] = kmax, s_red[2][w] = bad;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kWavesPerBlock; ++k) {
            kmin = min(kmin, s_red[0][k]);
            kmax = max(kmax, s_red[1][k]);
            bad |= (uint32_t)s_red[2][k];
        }
        EBC_G uint64_t* rp = (EBC_G uint64_t*)fd.rpart + 3ull * (u - fd.range_base);
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
    const bool f64 = fd.dtype == 1;
    // keys widened to 64 bits (fp32 keys sit in the low word)
    uint64_t kmin = ~0ull, kmax = 0ull;
    uint32_t bad = 0u;
    // several partials in flight per wait
    if (f64) {
#pragma unroll 8
        for (uint32_t u = threadIdx.x; u < fd.range_units; u += kBlock) {
            const EBC_G uint64_t* rp = (const EBC_G uint64_t*)fd.rpart + 3ull * u;
            kmin = min(kmin, rp[0]);
            kmax = max(kmax, rp[1]);
            bad |= (uint32_t)rp[2];
        }
    } else {
#pragma unroll 8
        for (uint32_t u = threadIdx.x; u < fd.range_units; u += kBlock) {
            const EBC_G uint32_t* rp = fd.rpart + 3ull * u;
            kmin = min(kmin, (uint64_t)rp[0]);
            kmax = max(kmax, (uint64_t)rp[1]);
            bad |= rp[2];
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        kmin = min(kmin, (uint64_t)__shfl_xor((long long)kmin, o));
        kmax = max(kmax, (uint64_t)__shfl_xor((long long)kmax, o));
        bad |= (uint32_t)__shfl_xor((int)bad, o);
    }
    __shared__ uint64_t s_red[3][kWavesPerBlock];
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) s_red[0][w] = kmin, s_red[1][w] = kmax, s_red[2][w] = bad;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int k = 1; k < kWavesPerBlock; ++k) {
        kmin = min(kmin, s_red[0][k]);
        kmax = max(kmax, s_red[1][k]);
        bad |= (uint32_t)s_red[2][k];
    }
    FieldDyn d = {};
    d.status = ST_OK;
    d.codec = ARC_HUFFMAN;
    if (bad) {
        d.status = ST_ERR_NONFINITE;
        *dy = d;
        return;
    }
    const double mn = f64 ? key_double(kmin) : (double)key_float((uint32_t)kmin);
    const double mx = f64 ? key_double(kmax) : (double)key_float((uint32_t)kmax);
    d.mn = mn, d.mx = mx;
    const double range = mx - mn;  // exact for fp32 ends, rounded once for fp64 ends
    const double M = fmax(fabs(mn), fabs(mx));
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
        // fp32 output: eps = 2^max(k - 21, -22), rejected above 2^-4;
        // fp64 output: eps = 2^max(k - 48, -49), k > 27 rejected (the codes
        // would leave the int32 range of the Lorenzo arithmetic);
        // k = ilogb(M) - ilogb(eb_abs)
        int e = f64 ? -49 : -22;
        bool too_small = false;
        if (M != 0.0) {
            const int k = ilogb_pos(M) - ilogb_pos(eb_abs);
            if (f64) {
                too_small = k > 27;
                e = max(k - 48, -49);
            } else {
                e = max(k - 21, -22);
                too_small = e > -4;
            }
        }
        if (too_small) {
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
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef f64x2 f64x2_a8 __attribute__((aligned(8)));

// fp64 quads: two 16-byte loads (VEC: 16-byte aligned rows)
template <bool VEC>
__device__ __forceinline__ void load_quad(const EBC_G double* __restrict__ p, uint64_t i, int nvalid,
                                          double v[4])
{
    if (nvalid == 4) {
        f64x2 a, b;
        if (VEC) {
            a = __builtin_nontemporal_load((const EBC_G f64x2*)(p + i));
            b = __builtin_nontemporal_load((const EBC_G f64x2*)(p + i + 2));
        } else {
            a = *(const EBC_G f64x2_a8*)(p + i);
            b = *(const EBC_G f64x2_a8*)(p + i + 2);
        }
        v[0] = a.x, v[1] = a.y, v[2] = b.x, v[3] = b.y;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = k < nvalid ? p[i + k] : 0.0;
    }
}

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
    } else if (nvalid == 4) {
        const f32x4 t = *(const EBC_G f32x4_a4*)(p + i);
        v[0] = t.x, v[1] = t.y, v[2] = t.z, v[3] = t.w;
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
    } else if (nvalid == 4 && (i & 1) == 0) {
        // four codes at an even index: one dword-aligned 8-byte store
        const u32x2 t = {c[0] | (c[1] << 16), c[2] | (c[3] << 16)};
        *(EBC_G u32x2_a4*)(q + i) = t;
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
    uint32_t lo;      // wide bins: first code of the LDS window (slot 1)
    EBC_G uint32_t* ghist;  // wide bins: the field histogram, for codes outside the window
};

// prequant one quad: d = rint(x * inv) in fp64 (Sec. IV-A.1)
template <class T>
__device__ __forceinline__ void prequant4(const T v[4], double inv, int32_t d[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) d[k] = (int32_t)__builtin_rint((double)v[k] * inv);
}

template <class T> __device__ __forceinline__ const EBC_G T* field_in(const FieldDesc& fd);
template <> __device__ __forceinline__ const EBC_G float* field_in<float>(const FieldDesc& fd) { return fd.in; }
template <> __device__ __forceinline__ const EBC_G double* field_in<double>(const FieldDesc& fd) { return fd.in64; }

// postquant one quad of deltas: code, outlier scratch, histogram.
// Returns a 4-bit mask of outliers among the valid elements.
// WIDE (n_bins > kMaxBins): LDS slot 0 counts code 0, slots 1 .. kHistWin-1
// the codes lo .. lo + kHistWin - 2 around the centre; any other code is
// counted straight into the field histogram in HBM (rare for a predictable
// field, whose deltas cluster around zero).
template <bool WIDE>
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
            if (c[k] == (uint32_t)qc.r) {
                qc.center++;
            } else if (!WIDE) {
                atomicAdd(&sh_hist[c[k]], 1u);
            } else {
                // slot 1 + (c - lo) for lo <= c < lo + kHistWin - 1 (unsigned
                // difference: codes below lo wrap to large values)
                const uint32_t dj = c[k] - qc.lo;
                if (c[k] == 0) atomicAdd(&sh_hist[0], 1u);
                else if (dj < kHistWin - 1) atomicAdd(&sh_hist[dj + 1], 1u);
                else atomicAdd(&qc.ghist[c[k]], 1u);
            }
        }
    }
    return om;
}

// Outliers of one row among the lanes of that row: `rowmask` selects the
// lanes holding the row, `om` holds this lane's 4-bit outlier mask.
__device__ __forceinline__ uint32_t row_count(uint32_t om, uint64_t rowmask)
{
    const uint64_t any = ballot(om != 0);
    if (any == 0) return 0;
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) cnt += __popcll(ballot((om >> k) & 1u) & rowmask);
    return cnt;
}

// One workgroup tile: quantise, record outliers, count codes into the LDS
// histogram and outlier counts per row segment into `s_cnt` (2D/3D).
template <int RANK, bool VEC, class T, bool WIDE>
__device__ __forceinline__ void construct_tile(const FieldDesc& fd, uint32_t tl, QuantCtx& qc,
                                               uint32_t* sh_hist, uint32_t* s_cnt,
                                               uint32_t* __restrict__ segs)
{
    const int l = lane_id();
    const int w = threadIdx.x / kWave;
    const EBC_G T* __restrict__ in = field_in<T>(fd);
    EBC_G uint16_t* __restrict__ qo = fd.q;
    EBC_G int32_t* __restrict__ dsc = fd.dsc;
    if (RANK == 1) {
        // wave tile: 4 chunks of 256; lane owns x = c*256 + 4*l + k
        const uint32_t wt = tl * kWavesPerBlock + w;
        if (wt < fd.n_wave_tiles) {
            const uint64_t n = fd.n;
            T v[4][4];
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
                const uint32_t om = postquant4<WIDE>(dl, nv, qc, code, dsc, i0, sh_hist);
                if (VEC && nv == 4) store_codes<true>(qo, i0, 4, code);
                else store_codes<false>(qo, i0, nv, code);
                const uint32_t cnt = row_count(om, ~0ull);
                const uint64_t seg = (uint64_t)wt * 4 + c;
                if (l == 0 && seg < fd.n_seg) segs[seg] = cnt;
            }
        }
    } else {
        // workgroup tile: wx waves along x by wy along y
        const uint32_t wx = fd.wx, wy = kWavesPerBlock / wx;
        const uint32_t wxi = w % wx, wyi = w / wx;
        const uint32_t nxb = fd.nxb, nyb = fd.nyb;
        const uint32_t xb = tl % nxb, yb = (tl / nxb) % nyb, zb = tl / (nxb * nyb);
        const uint32_t nx = fd.nx, ny = fd.ny, nz = fd.nz;
        if (RANK == 3) {
            // lane = 8 * xq + y: y-neighbour at lane - 1, x-neighbour at lane - 8
            const uint32_t y = l & 7, xq = l >> 3;
            const uint32_t x0 = xb * fd.xs + wxi * 32 + 4 * xq;
            const uint32_t yy = yb * 8 * wy + wyi * 8 + y;
            const uint32_t z0 = zb * 8;
            const int nv_x = x0 >= nx ? 0 : (int)min<uint32_t>(4, nx - x0);
            const uint64_t rowmask = 0x0101010101010101ull << y;
            int32_t fprev[4] = {0, 0, 0, 0};
            // planes in flight kAhead ahead of the one being processed (the
            // loop is unrolled, so only those planes occupy registers)
            constexpr int kAhead = 1;
            T v[8][4];
#pragma unroll
            for (int iz = 0; iz < kAhead; ++iz) {
                const bool ok = yy < ny && z0 + iz < nz;
                load_quad<VEC>(in, ((uint64_t)(z0 + iz) * ny + yy) * nx + x0, ok ? nv_x : 0, v[iz]);
            }
#pragma unroll
            for (int iz = 0; iz < 8; ++iz) {
                if (iz + kAhead < 8) {
                    const bool ok = yy < ny && z0 + iz + kAhead < nz;
                    load_quad<VEC>(in, ((uint64_t)(z0 + iz + kAhead) * ny + yy) * nx + x0, ok ? nv_x : 0,
                                   v[iz + kAhead]);
                }
                const uint32_t z = z0 + iz;
                const bool rowok = yy < ny && z < nz;
                const int nv = rowok ? nv_x : 0;
                const uint64_t i0 = ((uint64_t)z * ny + yy) * nx + x0;
                int32_t d[4], e[4], dl[4];
                prequant4(v[iz], qc.inv, d);
                int left = dpp_shr<8>(d[3]);
                if ((xq & 1) == 0) left = 0;  // x chunk boundary
                e[0] = d[0] - left, e[1] = d[1] - d[0], e[2] = d[2] - d[1], e[3] = d[3] - d[2];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    int up = dpp_keep(dpp_shr<1>(e[k]));
                    if (y == 0) up = 0;  // y chunk boundary
                    const int32_t fy = e[k] - up;   // Dy Dx d
                    dl[k] = fy - fprev[k];          // Dz Dy Dx d
                    fprev[k] = fy;
                }
                uint32_t code[4];
                const uint32_t om = postquant4<WIDE>(dl, nv, qc, code, dsc, i0, sh_hist);
                store_codes<VEC>(qo, i0, nv, code);
                const uint32_t cnt = row_count(om, rowmask);
                if (xq == 0 && cnt) atomicAdd(&s_cnt[wyi * 64 + iz * 8 + y], cnt);
            }
        } else {
            // lane = 16 * xq + y: y-neighbour at lane - 1 (same DPP row),
            // x-neighbour at lane - 16; four 16x16 chunks along x per wave
            const uint32_t y = l & 15, xq = l >> 4;
            const uint32_t yy = yb * 16 * wy + wyi * 16 + y;
            const uint64_t rowmask = 0x0001000100010001ull << y;
            const bool yok = yy < ny;
            uint32_t rowcnt = 0;
            // the four chunks of the wave in flight at once
            T v[4][4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint32_t x0 = xb * fd.xs + wxi * 64 + 16 * c + 4 * xq;
                const int nv = (!yok || x0 >= nx) ? 0 : (int)min<uint32_t>(4, nx - x0);
                load_quad<VEC>(in, (uint64_t)yy * nx + x0, nv, v[c]);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint32_t x0 = xb * fd.xs + wxi * 64 + 16 * c + 4 * xq;
                const int nv = (!yok || x0 >= nx) ? 0 : (int)min<uint32_t>(4, nx - x0);
                const uint64_t i0 = (uint64_t)yy * nx + x0;
                int32_t d[4], dl[4];
                prequant4(v[c], qc.inv, d);
                int left = __shfl_up(d[3], 16);
                if (xq == 0) left = 0;  // x chunk boundary
                int32_t e[4] = {d[0] - left, d[1] - d[0], d[2] - d[1], d[3] - d[2]};
#pragma unroll
                for (int k = 0; k < 4; ++k) dl[k] = e[k] - dpp_keep(dpp_shr<1>(e[k]));  // y = 0 reads 0
                uint32_t code[4];
                const uint32_t om = postquant4<WIDE>(dl, nv, qc, code, dsc, i0, sh_hist);
                store_codes<VEC>(qo, i0, nv, code);
                rowcnt += row_count(om, rowmask);
            }
            if (xq == 0 && rowcnt) atomicAdd(&s_cnt[wyi * 16 + y], rowcnt);
        }
    }
}

// Flush the LDS histogram of field `fd` into its partial row for this
// workgroup and clear it.  Row (b - wg_base) mod G is unique per workgroup b
// of the grid G among those that visit the field.
template <bool WIDE>
__device__ __forceinline__ void flush_hist(const FieldDesc& fd, QuantCtx& qc, uint32_t* sh_hist)
{
    const uint32_t cs = wave_sum_u32(qc.center);
    qc.center = 0;
    if (lane_id() == 0 && cs) atomicAdd(&sh_hist[WIDE ? (uint32_t)qc.r - qc.lo + 1u : (uint32_t)qc.r], cs);
    __syncthreads();
    const uint32_t G = gridDim.x, nb = hist_slots(fd.n_bins);
    const uint32_t row = (blockIdx.x + G - fd.wg_base % G) % G;
    EBC_G uint32_t* hp = fd.hpart + (uint64_t)row * nb;
    for (uint32_t b = threadIdx.x; b < nb; b += kBlock) {
        hp[b] = sh_hist[b];
        sh_hist[b] = 0;
    }
    __syncthreads();
}

// Persistent over the workgroup tiles of one (rank, layout) group: the grid
// strides over the tiles, so each workgroup visits every field in one run of
// consecutive tiles and flushes one partial histogram per field it visits.
template <int RANK, bool VEC, class T, bool WIDE>
__global__ __launch_bounds__(kBlock) void k_construct(const FieldDesc* __restrict__ F, int nf,
                                                      uint32_t n_tiles, uint32_t* __restrict__ seg_cnt)
{
    extern __shared__ uint32_t sh_hist[];
    __shared__ uint32_t s_cnt[2][kWavesPerBlock * 64];  // outliers per row, double-buffered
    const uint32_t nb = F[0].n_bins;
    for (uint32_t b = threadIdx.x; b < hist_slots(nb); b += kBlock) sh_hist[b] = 0;
    s_cnt[0][threadIdx.x] = 0;
    s_cnt[1][threadIdx.x] = 0;
    __syncthreads();
    QuantCtx qc;
    qc.center = 0;
    int cur = -1, par = 0;
    uint32_t cur_lo = 0, cur_hi = 0;  // tile range of field `cur`
    for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        // a workgroup stays in one field for a run of tiles: search the
        // descriptors only when it leaves the current field's range
        const int f = t >= cur_lo && t < cur_hi ? cur : find_field<&FieldDesc::wg_base>(F, nf, t);
        const FieldDesc& fd = F[f];
        const auto* dy = kconst(fd.dyn);  // scalar loads: no wait on the previous tile's stores
        if (dy->status != ST_OK || dy->codec == ARC_CONST) continue;  // uniform over the workgroup
        if (f != cur) {
            if (cur >= 0) flush_hist<WIDE>(F[cur], qc, sh_hist);
            cur = f;
            cur_lo = fd.wg_base;
            cur_hi = fd.wg_base + fd.wg_tiles;
            qc.inv = dy->inv;
            qc.r = (int32_t)(nb / 2);
            qc.lo = hist_win_lo(nb);
            qc.ghist = fd.hist;
        }
        const uint32_t tl = t - fd.wg_base;
        uint32_t* cnt = s_cnt[par];
        construct_tile<RANK, VEC, T, WIDE>(fd, tl, qc, sh_hist, cnt, seg_cnt + fd.seg_base);
        if (RANK >= 2) {
            __syncthreads();
            // one outlier count per row segment of this tile; the buffer is
            // cleared for the tile after next
            const uint32_t wx = fd.wx, wy = kWavesPerBlock / wx;
            const uint32_t nxb = fd.nxb, nyb = fd.nyb;
            const uint32_t xb = tl % nxb, yb = (tl / nxb) % nyb, zb = tl / (nxb * nyb);
            const uint32_t rows = RANK == 3 ? 64 : 16;  // rows per wave-row of the tile
            uint32_t* segs = seg_cnt + fd.seg_base;
            const uint32_t r = threadIdx.x;
            if (r < wy * rows) {
                const uint32_t wyi = r / rows, rr = r % rows;
                uint32_t z, yy;
                if (RANK == 3) z = zb * 8 + rr / 8, yy = yb * 8 * wy + wyi * 8 + rr % 8;
                else z = 0, yy = yb * 16 * wy + wyi * 16 + rr;
                if (z < fd.nz && yy < fd.ny) segs[((uint64_t)z * fd.ny + yy) * nxb + xb] = cnt[r];
            }
            cnt[r] = 0;
            par ^= 1;
        }
    }
    if (cur >= 0) flush_hist<WIDE>(F[cur], qc, sh_hist);
}

// ------------------------------------------------------ histogram reduce
// grid (ceil(slots / 256), kHistSplit, nf): split the partial rows of a
// field over kHistSplit workgroups, then add into the field histogram (for
// wide bins, slot j holds code 0 or code lo + j - 1; the codes outside the
// window were already counted there by construction).
constexpr int kHistSplit = 64;
__global__ __launch_bounds__(kBlock) void k_hist_reduce(const FieldDesc* __restrict__ F)
{
    const FieldDesc& fd = F[blockIdx.z];
    const auto* dy = kconst(fd.dyn);
    if (dy->status != ST_OK || dy->codec == ARC_CONST) return;
    const uint32_t b = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t nb = hist_slots(fd.n_bins);
    if (b >= nb) return;
    uint32_t s = 0;
#pragma unroll 8
    for (uint32_t r = blockIdx.y; r < fd.hrows; r += kHistSplit) s += fd.hpart[(uint64_t)r * nb + b];
    const uint32_t code = fd.n_bins > kMaxBins && b != 0 ? hist_win_lo(fd.n_bins) + b - 1 : b;
    if (s) atomicAdd(&fd.hist[code], s);
}

// ------------------------------------------------------------- launchers
hipError_t launch_range(const FieldDesc* F, int nf, uint32_t units, bool f64, hipStream_t s)
{
    if (units == 0) return hipSuccess;
    if (f64) hipLaunchKernelGGL(k_range64, dim3(units), dim3(kBlock), 0, s, F, nf);
    else hipLaunchKernelGGL(k_range, dim3(units), dim3(kBlock), 0, s, F, nf);
    return hipGetLastError();
}

hipError_t launch_params(const FieldDesc* F, int nf, hipStream_t s)
{
    hipLaunchKernelGGL(k_params, dim3(nf), dim3(kBlock), 0, s, F);
    return hipGetLastError();
}

template <class T, bool W>
static hipError_t occupancy(int rank, bool vec, size_t sh, int* per)
{
    if (rank == 1)
        return vec ? hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_construct<1, true, T, W>, kBlock, sh)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_construct<1, false, T, W>, kBlock, sh);
    if (rank == 2)
        return vec ? hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_construct<2, true, T, W>, kBlock, sh)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_construct<2, false, T, W>, kBlock, sh);
    return vec ? hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_construct<3, true, T, W>, kBlock, sh)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(per, k_construct<3, false, T, W>, kBlock, sh);
}

// Workgroups of one construction variant that the device holds at once (the
// default persistent grid); 0 if the query fails.
uint32_t construct_resident_blocks(int rank, bool vec, uint32_t n_bins, bool f64)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const size_t sh = (size_t)hist_slots(n_bins) * sizeof(uint32_t);
    const bool w = n_bins > kMaxBins;
    const hipError_t e = f64 ? (w ? occupancy<double, true>(rank, vec, sh, &per)
                                  : occupancy<double, false>(rank, vec, sh, &per))
                             : (w ? occupancy<float, true>(rank, vec, sh, &per)
                                  : occupancy<float, false>(rank, vec, sh, &per));
    if (e != hipSuccess || per <= 0 || cus <= 0) return 0;
    return (uint32_t)(per * cus);
}

template <class T, bool W>
static void construct_launch(const FieldDesc* F, int nf, int rank, bool vec, uint32_t wg_tiles,
                             dim3 g, size_t sh, uint32_t* seg_cnt, hipStream_t s)
{
    const dim3 b(kBlock);
    if (rank == 1) {
        if (vec) hipLaunchKernelGGL((k_construct<1, true, T, W>), g, b, sh, s, F, nf, wg_tiles, seg_cnt);
        else hipLaunchKernelGGL((k_construct<1, false, T, W>), g, b, sh, s, F, nf, wg_tiles, seg_cnt);
    } else if (rank == 2) {
        if (vec) hipLaunchKernelGGL((k_construct<2, true, T, W>), g, b, sh, s, F, nf, wg_tiles, seg_cnt);
        else hipLaunchKernelGGL((k_construct<2, false, T, W>), g, b, sh, s, F, nf, wg_tiles, seg_cnt);
    } else {
        if (vec) hipLaunchKernelGGL((k_construct<3, true, T, W>), g, b, sh, s, F, nf, wg_tiles, seg_cnt);
        else hipLaunchKernelGGL((k_construct<3, false, T, W>), g, b, sh, s, F, nf, wg_tiles, seg_cnt);
    }
}

hipError_t launch_construct(const FieldDesc* F, int nf, int rank, bool vec, bool f64, uint32_t wg_tiles,
                            uint32_t blocks, uint32_t n_bins, uint32_t* seg_cnt, hipStream_t s)
{
    if (wg_tiles == 0) return hipSuccess;
    const size_t sh = (size_t)hist_slots(n_bins) * sizeof(uint32_t);
    const dim3 g(blocks);
    if (n_bins > kMaxBins) {
        if (f64) construct_launch<double, true>(F, nf, rank, vec, wg_tiles, g, sh, seg_cnt, s);
        else construct_launch<float, true>(F, nf, rank, vec, wg_tiles, g, sh, seg_cnt, s);
    } else {
        if (f64) construct_launch<double, false>(F, nf, rank, vec, wg_tiles, g, sh, seg_cnt, s);
        else construct_launch<float, false>(F, nf, rank, vec, wg_tiles, g, sh, seg_cnt, s);
    }
    return hipGetLastError();
}

hipError_t launch_hist_reduce(const FieldDesc* F, int nf, uint32_t n_bins, hipStream_t s)
{
    dim3 g((hist_slots(n_bins) + kBlock - 1) / kBlock, kHistSplit, nf);
    hipLaunchKernelGGL(k_hist_reduce, g, dim3(kBlock), 0, s, F);
    return hipGetLastError();
}

}  // namespace ebc
