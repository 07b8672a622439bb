// ebc_dev.h -- device-side wave helpers shared by the HIP kernels.
#pragma once

#include "ebc_types.h"

namespace ebc {

// Largest f with base(F[f]) <= t (fields are ordered by base).
template <uint32_t FieldDesc::*Base>
__device__ __forceinline__ int find_field(const FieldDesc* F, int nf, uint32_t t)
{
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (F[mid].*Base <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// native vector types for streaming (non-temporal) loads and stores
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
// the same vectors at dword alignment: multi-dword global accesses need only
// 4-byte alignment, so rows that are not 16-byte aligned still move a quad in
// one access
typedef f32x4 f32x4_a4 __attribute__((aligned(4)));
typedef u32x2 u32x2_a4 __attribute__((aligned(4)));
__device__ __forceinline__ f32x4 ld_nt_f4(const EBC_G float* p)
{
    return __builtin_nontemporal_load((const EBC_G f32x4*)p);
}
__device__ __forceinline__ u32x2 ld_nt_u2(const EBC_G uint16_t* p)
{
    return __builtin_nontemporal_load((const EBC_G u32x2*)p);
}
__device__ __forceinline__ void st_nt_f4(EBC_G float* p, f32x4 v)
{
    __builtin_nontemporal_store(v, (EBC_G f32x4*)p);
}

// Value of lane (l - K) within a 16-lane DPP row; lanes with l % 16 < K read 0.
template <int K>
__device__ __forceinline__ int dpp_shr(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x110 + K, 0xF, 0xF, true);
}
template <int K>
__device__ __forceinline__ uint32_t dpp_shr_u(uint32_t v)
{
    return (uint32_t)dpp_shr<K>((int)v);
}

// Workgroup-uniform read of data that no kernel writes while this one runs
// (e.g. the per-field scalars written by earlier kernels): through the
// constant address space it becomes a scalar load, which does not count
// against the vector-memory counter and so never waits on loads in flight.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* kconst(const EBC_G T* p)
{
    return (const __attribute__((address_space(4))) T*)p;
}

// Keeps a DPP move as an instruction of its own.  Folded into a following
// subtraction, it became v_subrev_u32_dpp, which returned the negated
// difference on gfx950; additions and masks fold correctly.
__device__ __forceinline__ int dpp_keep(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Inclusive scan across the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v)
{
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t t = __shfl_up(v, d);
        if (l >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Order-preserving map of a finite float to an unsigned key.
__device__ __forceinline__ uint32_t float_key(float f)
{
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key_float(uint32_t k)
{
    uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(b);
}

__device__ __forceinline__ uint64_t align16(uint64_t v) { return (v + 15u) & ~(uint64_t)15u; }

}  // namespace ebc
