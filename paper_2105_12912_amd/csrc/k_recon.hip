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

// Four codes kept packed (two per 32-bit word) so that a whole tile's loads
// fit in few registers; codes of absent elements read as 1 (never the
// outlier placeholder).
template <bool VEC>
__device__ __forceinline__ u32x2 load_packed(const EBC_G uint16_t* __restrict__ q, uint64_t i, int nvalid)
{
    if (VEC && nvalid == 4) return ld_nt_u2(q + i);
    if (nvalid == 4 && (i & 1) == 0) return *(const EBC_G u32x2_a4*)(q + i);  // dword-aligned
    uint32_t c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = k < nvalid ? q[i + k] : 1u;
    u32x2 t;
    t.x = c[0] | (c[1] << 16);
    t.y = c[2] | (c[3] << 16);
    return t;
}

__device__ __forceinline__ void unpack4(u32x2 t, uint32_t c[4])
{
    c[0] = t.x & 0xFFFF, c[1] = t.x >> 16, c[2] = t.y & 0xFFFF, c[3] = t.y >> 16;
}

template <bool VEC>
__device__ __forceinline__ void store_quad(EBC_G float* __restrict__ o, uint64_t i, int nvalid,
                                           const float v[4])
{
    if (VEC && nvalid == 4) {
        st_nt_f4(o + i, f32x4{v[0], v[1], v[2], v[3]});
    } else if (nvalid == 4) {
        *(EBC_G f32x4_a4*)(o + i) = f32x4{v[0], v[1], v[2], v[3]};  // dword-aligned
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
            // consume the loaded value inside the (rare) branch, so that the
            // wait for it stays here and the common path never waits on the
            // loads and stores in flight
            asm volatile("" ::"v"(qp[k]));
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

// fp64 archives: the product rounded once, in binary64
__device__ __forceinline__ void dequant4(const uint32_t s[4], double ebx2, double v[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (double)(int32_t)s[k] * ebx2;
}

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef f64x2 f64x2_a8 __attribute__((aligned(8)));

// an fp64 quad: two 16-byte stores (non-temporal on 16-byte aligned rows)
template <bool VEC>
__device__ __forceinline__ void store_quad(EBC_G double* __restrict__ o, uint64_t i, int nvalid,
                                           const double v[4])
{
    if (nvalid == 4) {
        if (VEC) {
            __builtin_nontemporal_store(f64x2{v[0], v[1]}, (EBC_G f64x2*)(o + i));
            __builtin_nontemporal_store(f64x2{v[2], v[3]}, (EBC_G f64x2*)(o + i + 2));
        } else {
            *(EBC_G f64x2_a8*)(o + i) = f64x2{v[0], v[1]};
            *(EBC_G f64x2_a8*)(o + i + 2) = f64x2{v[2], v[3]};
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k < nvalid) o[i + k] = v[k];
    }
}

// output element type of a field: fp32, or fp64 for fp64 archives
template <class OT> __device__ __forceinline__ EBC_G OT* field_out(const FieldDesc& fd);
template <> __device__ __forceinline__ EBC_G float* field_out<float>(const FieldDesc& fd) { return fd.outf; }
template <> __device__ __forceinline__ EBC_G double* field_out<double>(const FieldDesc& fd) { return fd.outd; }

// This lane's quads of one workgroup tile: four 256-long chunks' quads (1D),
// four chunks along x (2D) or the eight z-planes of the chunk column (3D).
template <int RANK>
struct RTile {
    static constexpr int NQ = RANK == 3 ? 8 : 4;
    u32x2 raw[NQ];
};

// lane geometry of a tile: first element of quad k and its valid count
template <int RANK>
__device__ __forceinline__ void rquad(const FieldDesc& fd, uint32_t tl, int k, uint64_t& i0, int& nv)
{
    const int l = lane_id();
    const uint32_t w = threadIdx.x / kWave;
    if (RANK == 1) {
        const uint32_t wt = tl * kWavesPerBlock + w;
        i0 = (uint64_t)wt * 1024 + k * 256 + 4 * l;
        nv = (wt >= fd.n_wave_tiles || i0 >= fd.n) ? 0 : (int)min<uint64_t>(4, fd.n - i0);
        if (nv == 0) i0 = 0;
        return;
    }
    const uint32_t wx = fd.wx, wy = kWavesPerBlock / wx;
    const uint32_t wxi = w % wx, wyi = w / wx;
    const uint32_t nxb = fd.nxb, nyb = fd.nyb;
    const uint32_t xb = tl % nxb, yb = (tl / nxb) % nyb, zb = tl / (nxb * nyb);
    const uint32_t nx = fd.nx, ny = fd.ny, nz = fd.nz;
    uint32_t x0, yy, z;
    if (RANK == 3) {
        const uint32_t y = l & 7, xq = l >> 3;
        x0 = xb * fd.xs + wxi * 32 + 4 * xq;
        yy = yb * 8 * wy + wyi * 8 + y;
        z = zb * 8 + k;
    } else {
        const uint32_t y = l & 15, xq = l >> 4;
        x0 = xb * fd.xs + wxi * 64 + 16 * k + 4 * xq;
        yy = yb * 16 * wy + wyi * 16 + y;
        z = 0;
    }
    const bool ok = x0 < nx && yy < ny && z < nz;
    nv = ok ? (int)min<uint32_t>(4, nx - x0) : 0;
    i0 = ok ? ((uint64_t)z * ny + yy) * nx + x0 : 0;
}

// With 16-byte rows (VEC) every quad is loaded with one unconditional vector
// load (an absent quad reads the start of the code array; the tail quad of a
// 1D field may read up to 6 bytes past the codes, into the outlier scratch
// that follows them), so the number of memory operations per tile is fixed
// and the compiler never has to wait for stores before a load's use.
template <int RANK, bool VEC>
__device__ __forceinline__ void rtile_load(const FieldDesc& fd, uint32_t tl, RTile<RANK>& T)
{
#pragma unroll
    for (int k = 0; k < RTile<RANK>::NQ; ++k) {
        uint64_t i0;
        int nv;
        rquad<RANK>(fd, tl, k, i0, nv);
        if (VEC) T.raw[k] = ld_nt_u2(fd.q + (nv > 0 ? i0 : 0));
        else T.raw[k] = load_packed<false>(fd.q, i0, nv);
    }
}

template <int RANK, bool VEC, class OT>
__device__ __forceinline__ void rtile_process(const FieldDesc& fd, uint32_t tl, const RTile<RANK>& T,
                                              double ebx2, uint32_t& zeros)
{
    const int l = lane_id();
    const int32_t r = (int32_t)(fd.n_bins / 2);
    const EBC_G int32_t* __restrict__ dsc = fd.dsc;
    EBC_G OT* __restrict__ out = field_out<OT>(fd);
    uint32_t zprev[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < RTile<RANK>::NQ; ++k) {
        uint64_t i0;
        int nv;
        rquad<RANK>(fd, tl, k, i0, nv);
        uint32_t c[4], s[4];
        unpack4(T.raw[k], c);
        if (VEC) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (j >= nv) c[j] = 1u;  // absent: never the outlier placeholder
        }
        fuse4(c, nv, r, dsc, i0, s, zeros);
        s[1] += s[0], s[2] += s[1], s[3] += s[2];  // x pass within the quad
        if (RANK == 1) {
            // exclusive prefix of the lane totals over the 256-long chunk
            const uint32_t excl = wave_incl_scan_u32(s[3]) - s[3];
#pragma unroll
            for (int j = 0; j < 4; ++j) s[j] += excl;
        } else if (RANK == 3) {
            const uint32_t y = l & 7, xq = l >> 3;
            uint32_t left = dpp_shr_u<8>(s[3]);  // the quad to the left in the chunk
            if ((xq & 1) == 0) left = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                s[j] += left;
                // y pass: inclusive scan over the 8 lanes of the chunk column
                uint32_t a = dpp_shr_u<1>(s[j]);
                s[j] += y >= 1 ? a : 0u;
                a = dpp_shr_u<2>(s[j]);
                s[j] += y >= 2 ? a : 0u;
                a = dpp_shr_u<4>(s[j]);
                s[j] += y >= 4 ? a : 0u;
                // z pass: running sum over the planes of the chunk
                s[j] += zprev[j];
                zprev[j] = s[j];
            }
        } else {
            const uint32_t xq = l >> 4;
            // x pass over the 4 quads of the chunk row
            const uint32_t tot = s[3];
            uint32_t inc = tot;
            uint32_t a = (uint32_t)__shfl_up((int)inc, 16);
            inc += xq >= 1 ? a : 0u;
            a = (uint32_t)__shfl_up((int)inc, 32);
            inc += xq >= 2 ? a : 0u;
            const uint32_t left = inc - tot;
            // y pass: the 16 rows of a chunk are the 16 lanes of a DPP row
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                s[j] += left;
                s[j] += dpp_shr_u<1>(s[j]);
                s[j] += dpp_shr_u<2>(s[j]);
                s[j] += dpp_shr_u<4>(s[j]);
                s[j] += dpp_shr_u<8>(s[j]);
            }
        }
        OT v[4];
        dequant4(s, ebx2, v);
        if constexpr (VEC && sizeof(OT) == 4) {
            // one unconditional vector store (absent quads go to the sink);
            // a partial quad (1D tail only) is then written element-wise
            st_nt_f4(nv == 4 ? out + i0 : fd.sink, f32x4{v[0], v[1], v[2], v[3]});
            if (nv > 0 && nv < 4) {
                for (int j = 0; j < nv; ++j) out[i0 + j] = v[j];
            }
        } else {
            store_quad<VEC>(out, i0, nv, v);
        }
    }
}

// Zero codes seen by this workgroup for field fd, added to the field's count
// (checked against the outlier count by k_recon_check).
__device__ __forceinline__ void flush_zeros(const FieldDesc& fd, uint32_t& zeros, uint32_t* s_z)
{
    const uint32_t zs = wave_sum_u32(zeros);
    zeros = 0;
    __syncthreads();
    if (lane_id() == 0) s_z[threadIdx.x / kWave] = zs;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t z = s_z[0] + s_z[1] + s_z[2] + s_z[3];
        if (z) atomicAdd((unsigned long long*)&fd.dyn->zero_count, (unsigned long long)z);
    }
}

// Grid-stride over the workgroup tiles of one (rank, layout) group, with the
// next tile's codes in flight while the current tile is reconstructed (two
// static buffers).  Launched with one workgroup per tile, which measured
// faster than a resident-size grid; the stride loop serves tuned grids.
template <int RANK, bool VEC, class OT>
__global__ __launch_bounds__(kBlock) void k_reconstruct(const FieldDesc* __restrict__ F, int nf,
                                                        uint32_t n_tiles)
{
    __shared__ uint32_t s_z[kWavesPerBlock];
    uint32_t t = blockIdx.x;
    if (t >= n_tiles) return;
    RTile<RANK> A, B;
    int fa = find_field<&FieldDesc::wg_base>(F, nf, t), fb;
    rtile_load<RANK, VEC>(F[fa], t - F[fa].wg_base, A);
    int cur = -1;
    uint32_t zeros = 0;
    for (;;) {
        uint32_t tn = t + gridDim.x;
        const uint32_t tb = tn < n_tiles ? tn : t;
        fb = find_field<&FieldDesc::wg_base>(F, nf, tb);
        if (tn < n_tiles) rtile_load<RANK, VEC>(F[fb], tb - F[fb].wg_base, B);
        {
            const FieldDesc& fd = F[fa];
            const auto* dy = kconst(fd.dyn);
            if (fa != cur) {
                if (cur >= 0) flush_zeros(F[cur], zeros, s_z);
                cur = fa;
            }
            if (dy->status == ST_OK && dy->codec != ARC_CONST)
                rtile_process<RANK, VEC, OT>(fd, t - fd.wg_base, A, dy->ebx2, zeros);
        }
        t = tn;
        if (t >= n_tiles) break;
        tn = t + gridDim.x;
        const uint32_t ta = tn < n_tiles ? tn : t;
        fa = find_field<&FieldDesc::wg_base>(F, nf, ta);
        if (tn < n_tiles) rtile_load<RANK, VEC>(F[fa], ta - F[fa].wg_base, A);
        {
            const FieldDesc& fd = F[fb];
            const auto* dy = kconst(fd.dyn);
            if (fb != cur) {
                if (cur >= 0) flush_zeros(F[cur], zeros, s_z);
                cur = fb;
            }
            if (dy->status == ST_OK && dy->codec != ARC_CONST)
                rtile_process<RANK, VEC, OT>(fd, t - fd.wg_base, B, dy->ebx2, zeros);
        }
        t = tn;
        if (t >= n_tiles) break;
    }
    if (cur >= 0) flush_zeros(F[cur], zeros, s_z);
}

// Bit 15 (bit 31) set iff the low (high) 16-bit code packed in w is 0: with
// each half's top bit forced on, subtracting 1 clears it only in a half that
// was 0, and never borrows across halves (codes are below 2^15).
__device__ __forceinline__ uint32_t zero_half(uint32_t w)
{
    return ~((w | 0x80008000u) - 0x00010001u) & 0x80008000u;
}

// Chunk rows of one wave of the 3D reconstruction (see k_reconstruct3).
// FULL: the wave's 256 x 8 x 8 block lies inside the field and its rows are
// 16-byte aligned, so every row is one load and one store with no per-lane or
// per-row condition, addressed as a wave-uniform row pointer plus the lane's
// offset.  Otherwise rows outside the field are skipped, absent codes read as
// 1 and absent elements are not stored.  Outlier codes (0) enter as 0 - r
// and are only counted here: k_recon3_fix rewrites every chunk that holds
// one.
template <bool FULL, bool VEC, class OT>
__device__ __forceinline__ void recon3_wave(const FieldDesc& fd, uint32_t x0w, uint32_t y0, uint32_t z0,
                                            double ebx2, uint32_t& zeros)
{
    const int l = lane_id();
    const uint32_t nx = fd.nx, ny = fd.ny, nz = fd.nz;
    const uint32_t x0 = x0w + 4 * l;
    const int nvx = x0 < nx ? (int)min<uint32_t>(4, nx - x0) : 0;
    const uint32_t r = fd.n_bins / 2;
    const EBC_G uint16_t* __restrict__ q = fd.q;
    EBC_G OT* __restrict__ out = field_out<OT>(fd);
    // wave-uniform first element of row y of plane iz (x = x0w)
    auto row = [&](int iz, int y) -> uint64_t { return ((uint64_t)(z0 + iz) * ny + y0 + y) * nx + x0w; };
    auto row_ok = [&](int iz, int y) -> bool { return FULL || (y0 + y < ny && z0 + iz < nz); };
    uint32_t zprev[8][4];
#pragma unroll
    for (int y = 0; y < 8; ++y)
#pragma unroll
        for (int k = 0; k < 4; ++k) zprev[y][k] = 0;
    // planes of codes: the next one in flight while this one is processed
    // (fully unrolled, so only those two occupy registers)
    u32x2 raw[8][8];
    auto load_plane = [&](int iz) {
#pragma unroll
        for (int y = 0; y < 8; ++y) {
            if (FULL) {
                raw[iz][y] = *(const EBC_G u32x2*)(q + row(iz, y) + 4 * l);
            } else {
                const bool ok = row_ok(iz, y);
                raw[iz][y] = load_packed<VEC>(q, ok ? row(iz, y) + 4 * l : 0, ok ? nvx : 0);
            }
        }
    };
    load_plane(0);
#pragma unroll
    for (int iz = 0; iz < 8; ++iz) {
        // keep the schedule at one plane of loads ahead: without this fence
        // the compiler hoists every plane's loads and runs out of registers
        __builtin_amdgcn_sched_barrier(0);
        if (iz + 1 < 8) load_plane(iz + 1);
        uint32_t yprev[4] = {0, 0, 0, 0};
#pragma unroll
        for (int y = 0; y < 8; ++y) {
            if (!FULL && !row_ok(iz, y)) continue;  // wave-uniform
            uint32_t c[4], sv[4];
            const u32x2 t = raw[iz][y];
            unpack4(t, c);
#pragma unroll
            for (int k = 0; k < 4; ++k) sv[k] = c[k] - r;
            zeros += __builtin_popcount(zero_half(t.x)) + __builtin_popcount(zero_half(t.y));
            // accumulate in place: a reassociated sum would hold every
            // row's count in a register of its own until the end
            asm volatile("" : "+v"(zeros));
            sv[1] += sv[0], sv[2] += sv[1], sv[3] += sv[2];  // x pass within the quad
            uint32_t left = dpp_shr_u<1>(sv[3]);            // the pair lane's total
            if ((l & 1) == 0) left = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                sv[k] += left;
                sv[k] += yprev[k];  // y pass
                yprev[k] = sv[k];
                sv[k] += zprev[y][k];  // z pass
                zprev[y][k] = sv[k];
            }
            OT v[4];
            dequant4(sv, ebx2, v);
            if constexpr (FULL && sizeof(OT) == 4) {
                st_nt_f4(out + row(iz, y) + 4 * l, f32x4{v[0], v[1], v[2], v[3]});
            } else {
                store_quad<VEC>(out, row(iz, y) + 4 * l, FULL ? 4 : nvx, v);
            }
        }
    }
}

// 3D: a wave owns 256 x (one quad per lane) by one 8x8 chunk layer in y and
// z; a workgroup stacks four waves along y (tile 256 x 32 x 8; the field
// descriptor's nxb/nyb/nzb hold this tiling during decompression).  Per z
// plane a lane holds its quad in each of the 8 rows of the chunk layer: the x
// pass is in-lane plus the total of the pair lane (an 8-wide chunk row is two
// quads), the y pass a running sum over the rows and the z pass a running sum
// over the planes, both in registers.  Every row is one 512-byte code load
// and one 1 KiB store per wave.
//
// Outliers are not read here: a wait for a delta loaded in the middle of the
// stream would also wait for every load and store issued before it.  Instead
// each wave clears its block's chunk flags, which the outlier scatter sets
// afterwards, and k_recon3_fix recomputes the flagged chunks exactly.
template <bool VEC, class OT>
__global__ __launch_bounds__(kBlock) void k_reconstruct3(const FieldDesc* __restrict__ F, int nf)
{
    __shared__ uint32_t s_z[kWavesPerBlock];
    const uint32_t t = blockIdx.x;
    const int f = find_field<&FieldDesc::wg_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    const auto* dy = kconst(fd.dyn);
    if (dy->status != ST_OK || dy->codec == ARC_CONST) return;
    const uint32_t tl = t - fd.wg_base;
    const uint32_t nxb = fd.nxb, nyb = fd.nyb;
    const uint32_t xb = tl % nxb, yb = (tl / nxb) % nyb, zb = tl / (nxb * nyb);
    const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const uint32_t x0w = xb * 256, y0 = yb * 32 + w * 8, z0 = zb * 8;
    const double ebx2 = dy->ebx2;
    uint32_t zeros = 0;
    if (lane_id() == 0) fd.oflag[(zb * (nyb * kWavesPerBlock) + yb * kWavesPerBlock + w) * nxb + xb] = 0;
    if (VEC && x0w + 256 <= fd.nx && y0 + 8 <= fd.ny && z0 + 8 <= fd.nz)
        recon3_wave<true, VEC, OT>(fd, x0w, y0, z0, ebx2, zeros);
    else
        recon3_wave<false, VEC, OT>(fd, x0w, y0, z0, ebx2, zeros);
    const uint32_t zs = wave_sum_u32(zeros);
    if (lane_id() == 0) s_z[w] = zs;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t z = s_z[0] + s_z[1] + s_z[2] + s_z[3];
        if (z) atomicAdd((unsigned long long*)&fd.dyn->zero_count, (unsigned long long)z);
    }
}

// Outlier fix-up of the 3D reconstruction: one wave per 8x8x8 chunk that
// holds an outlier (queued by the outlier scatter), recomputed from its codes
// with the exact deltas substituted.  Lane (yl, zl) = (l % 8, l / 8) owns the
// chunk row of 8 x; the x pass is in-lane, the y pass a scan over the 8 lanes
// of a z layer and the z pass a scan over the 8 layers.  Elements outside
// the field enter as 0 and are not stored.
__global__ __launch_bounds__(kBlock) void k_recon3_fix(const FieldDesc* __restrict__ F, int nf)
{
    const uint32_t t = blockIdx.x;
    const int f = find_field<&FieldDesc::fx_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    const auto* dy = kconst(fd.dyn);
    if (dy->status != ST_OK || dy->codec == ARC_CONST) return;
    const uint32_t g = (t - fd.fx_base) * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    // the queue entry is fetched alongside the count (clamped into the queue)
    const uint32_t cnt = dy->fix_count;
    const uint64_t i = kconst(fd.fixl)[min<uint64_t>(g, fd.n_out_hdr - 1)];
    if (g >= cnt) return;
    const uint32_t nx = fd.nx, ny = fd.ny, nz = fd.nz;
    const uint32_t cx = (uint32_t)(i % nx) & ~7u;
    const uint64_t yz = i / nx;
    const uint32_t cy = (uint32_t)(yz % ny) & ~7u, cz = (uint32_t)(yz / ny) & ~7u;
    const int l = lane_id();
    const uint32_t yl = l & 7, zl = l >> 3;
    const uint32_t yy = cy + yl, zz = cz + zl;
    const bool ok = yy < ny && zz < nz;
    const uint32_t nv = ok ? min<uint32_t>(8, nx - cx) : 0;
    const uint64_t i0 = ok ? ((uint64_t)zz * ny + yy) * nx + cx : 0;
    const uint32_t r = fd.n_bins / 2;
    // codes and deltas loaded together (one round trip)
    uint32_t c[8], dv[8], sv[8];
#pragma unroll
    for (uint32_t e = 0; e < 8; ++e) {
        c[e] = 1, dv[e] = 0;
        if (e < nv) c[e] = fd.q[i0 + e], dv[e] = (uint32_t)fd.dsc[i0 + e];
    }
#pragma unroll
    for (uint32_t e = 0; e < 8; ++e) sv[e] = e < nv ? (c[e] == 0 ? dv[e] : c[e] - r) : 0u;
#pragma unroll
    for (int e = 1; e < 8; ++e) sv[e] += sv[e - 1];  // x pass
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        // y pass: inclusive scan over the 8 lanes of this z layer
        uint32_t a = dpp_shr_u<1>(sv[e]);
        sv[e] += yl >= 1 ? a : 0u;
        a = dpp_shr_u<2>(sv[e]);
        sv[e] += yl >= 2 ? a : 0u;
        a = dpp_shr_u<4>(sv[e]);
        sv[e] += yl >= 4 ? a : 0u;
        // z pass: inclusive scan over the 8 layers (lane strides of 8)
        a = (uint32_t)__shfl_up((int)sv[e], 8);
        sv[e] += zl >= 1 ? a : 0u;
        a = (uint32_t)__shfl_up((int)sv[e], 16);
        sv[e] += zl >= 2 ? a : 0u;
        a = (uint32_t)__shfl_up((int)sv[e], 32);
        sv[e] += zl >= 4 ? a : 0u;
    }
    const double ebx2 = dy->ebx2;
    if (fd.dtype == 1) {
#pragma unroll
        for (uint32_t e = 0; e < 8; ++e)
            if (e < nv) fd.outd[i0 + e] = (double)(int32_t)sv[e] * ebx2;
    } else {
#pragma unroll
        for (uint32_t e = 0; e < 8; ++e)
            if (e < nv) fd.outf[i0 + e] = (float)((double)(int32_t)sv[e] * ebx2);
    }
}

// decompression epilogue: the code-0 count must equal the outlier count
__global__ void k_recon_check(const FieldDesc* __restrict__ F, int nf)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const FieldDesc& fd = F[f];
    EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || fd.codec_hdr == ARC_CONST) return;
    if (dy->zero_count != fd.n_out_hdr) dy->status = ST_ERR_ARCHIVE;
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
    if (fd.dtype == 1) {
        for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock) fd.outd[i] = fd.cval;
    } else {
        for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock) fd.outf[i] = (float)fd.cval;
    }
}

template <class OT>
static void reconstruct_launch(const FieldDesc* F, int nf, int rank, bool vec, uint32_t wg_tiles,
                               uint32_t blocks, hipStream_t s)
{
    const dim3 g(blocks), b(kBlock);
    if (rank == 1) {
        if (vec) hipLaunchKernelGGL((k_reconstruct<1, true, OT>), g, b, 0, s, F, nf, wg_tiles);
        else hipLaunchKernelGGL((k_reconstruct<1, false, OT>), g, b, 0, s, F, nf, wg_tiles);
    } else if (rank == 2) {
        if (vec) hipLaunchKernelGGL((k_reconstruct<2, true, OT>), g, b, 0, s, F, nf, wg_tiles);
        else hipLaunchKernelGGL((k_reconstruct<2, false, OT>), g, b, 0, s, F, nf, wg_tiles);
    } else {
        const dim3 g3(wg_tiles);  // one workgroup per tile
        if (vec) hipLaunchKernelGGL((k_reconstruct3<true, OT>), g3, b, 0, s, F, nf);
        else hipLaunchKernelGGL((k_reconstruct3<false, OT>), g3, b, 0, s, F, nf);
    }
}

hipError_t launch_reconstruct(const FieldDesc* F, int nf, int rank, bool vec, bool f64, uint32_t wg_tiles,
                              uint32_t blocks, hipStream_t s)
{
    if (wg_tiles == 0) return hipSuccess;
    if (f64) reconstruct_launch<double>(F, nf, rank, vec, wg_tiles, blocks, s);
    else reconstruct_launch<float>(F, nf, rank, vec, wg_tiles, blocks, s);
    return hipGetLastError();
}

hipError_t launch_recon_fix(const FieldDesc* F, int nf, uint32_t units, hipStream_t s)
{
    if (!units) return hipSuccess;
    hipLaunchKernelGGL(k_recon3_fix, dim3(units), dim3(kBlock), 0, s, F, nf);
    return hipGetLastError();
}

hipError_t launch_recon_check(const FieldDesc* F, int nf, hipStream_t s)
{
    hipLaunchKernelGGL(k_recon_check, dim3((nf + 63) / 64), dim3(64), 0, s, F, nf);
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
