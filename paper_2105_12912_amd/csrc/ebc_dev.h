// ebc_dev.h -- device-side types and wave helpers shared by the HIP kernels.
//
// Work decomposition: every kernel covers all fields of a batch in one grid.
// Each field owns a contiguous range of the grid's work units of that kernel
// (FieldDesc::*_base); a workgroup finds its field with a binary search over
// those bases.  A single-field call is simply a batch of one.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ebc {

constexpr int kWave = 64;
constexpr int kBlock = 256;                 // threads per workgroup everywhere
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr uint32_t kHdr = 128;              // archive header bytes
constexpr uint32_t kMaxBins = 4096;         // n_bins this GPU path implements
constexpr uint32_t kMaxHc = 4096;           // Huffman chunk symbols implemented
constexpr uint32_t kRangeUnit = 16384;      // elements per value-range work unit
constexpr uint32_t kRleTile = 4096;         // elements per RLE work unit
constexpr int kLutBits = 10;                // Huffman decode table width
constexpr int kMaxDecodeLen = 60;           // longest code the decoder accepts (N < 2^32 gives <= 46)

enum : int32_t { ARC_HUFFMAN = 0, ARC_RLE = 1, ARC_CONST = 2 };
enum : int32_t { REQ_AUTO = 0, REQ_HUFFMAN = 1, REQ_RLE = 2 };
enum : int32_t { MODE_ABS = 0, MODE_REL = 1 };
enum : int32_t {
    ST_OK = 0,
    ST_ERR_EB_TOO_SMALL = -4,
    ST_ERR_EB = -3,
    ST_ERR_NONFINITE = -6,
    ST_ERR_OUT_TOO_SMALL = -7,
    ST_ERR_ARCHIVE = -9,
    ST_ERR_UNSUPPORTED = -11,
};

// Scalars produced on the device, one record per field.
struct FieldDyn {
    int32_t status;
    int32_t codec;
    float mn, mx;
    double eb_abs, ebx2, inv;
    uint64_t n_out;
    uint64_t n_runs;
    uint64_t n_words;
    uint64_t huff_bits;
    uint64_t total;
    uint64_t off_bits, off_words, off_rlen, off_oidx, off_oval;
    uint32_t max_len;
    uint32_t n_used;  // symbols with a non-zero count
    uint64_t zero_count;
    uint64_t pad[2];
};

// Static description of one field: geometry, buffers, work bases.
struct FieldDesc {
    uint64_t n;
    uint32_t nx, ny, nz;
    int32_t rank;
    uint32_t n_bins;
    uint32_t hc;
    int32_t eb_mode;
    int32_t codec_req;
    double eb;
    // construct / reconstruct wave-tile geometry
    uint32_t lx;             // lanes along x (each lane owns 4 consecutive x)
    uint32_t nxb, nyb, nzb;  // wave-tile grid
    uint32_t n_wave_tiles;
    uint32_t vec;            // 1: rows 16-byte aligned, quads never straddle rows
    // buffers (device)
    const float* in;         // compress input
    float* outf;             // decompress output
    uint8_t* arc;            // archive (compress output / decompress input)
    uint64_t arc_cap;        // compress: capacity; decompress: archive size
    uint16_t* q;             // quant-codes, n
    int32_t* dsc;            // outlier delta scratch, n (dense, sparsely written)
    uint32_t* hist;          // n_bins
    uint32_t* hpart;         // wg_tiles * n_bins partial histograms
    uint32_t* rpart;         // range partials: 3 words per range unit
    uint64_t* code;          // n_bins packed codewords: (len << 56) | code
    uint8_t* len;            // n_bins code lengths
    uint32_t* hbits;         // per Huffman chunk bit counts
    uint32_t* rstart;        // RLE run starts (compress scratch)
    uint32_t* zpart;         // per WG-tile zero counts (decompress validation)
    FieldDyn* dyn;
    // this field's work units in each batch-wide index space
    uint32_t range_units, range_base;  // value range / fill: kRangeUnit elements per WG
    uint32_t wg_tiles, wg_base;        // construct / reconstruct WG tiles (rank group relative)
    uint32_t n_seg, seg_base;          // outlier segments: count-array entries
    uint32_t ow_units, ow_base;        // outlier write: 1024 segments per WG
    uint32_t n_hch, hch_base;          // Huffman chunks: word-count array entries
    uint32_t hwg_units, hwg_base;      // Huffman encode: huff_cpw(hc) chunks per WG
    uint32_t hdwg_units, hdwg_base;    // Huffman decode: 256 chunks per WG
    uint32_t n_rt, rt_base;            // RLE tiles of kRleTile elements (count array / WG)
    uint32_t n_runs_hdr, rle_base;     // decompress: runs in the archive (start array entries)
    uint32_t sc_units, sc_base;        // decompress outlier scatter: 256 outliers per WG
    uint32_t rl_units, rl_base;        // decompress run-length prep: 256 runs per WG
    // decompress: header values
    uint64_t n_out_hdr;
    uint64_t n_words_hdr;
    double ebx2_hdr;
    float cval;
    int32_t codec_hdr;
    uint64_t off_bits, off_words, off_val, off_rlen, off_oidx, off_oval;
};

// Canonical Huffman decoder tables of one field (built by k_dectab).
struct DecTab {
    uint64_t first[65];   // first code of each length
    uint32_t count[65];   // codes of each length
    uint32_t offset[65];  // index of the first symbol of each length in perm
    uint32_t max_len;
    uint32_t pad;
    uint32_t lut[1u << kLutBits];  // (symbol << 8) | length for codes <= kLutBits, else 0
    uint16_t perm[kMaxBins];       // symbols ordered by (length, symbol)
};

// Huffman chunks (one wavefront each) per encode workgroup
__host__ __device__ constexpr uint32_t huff_cpw(uint32_t hc) { return hc <= 1024 ? 4 : 4096 / hc; }

__host__ __device__ constexpr size_t dectab_bytes() { return (sizeof(DecTab) + 255) & ~(size_t)255; }

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
__device__ __forceinline__ f32x4 ld_nt_f4(const float* p)
{
    return __builtin_nontemporal_load((const f32x4*)p);
}
__device__ __forceinline__ u32x2 ld_nt_u2(const uint16_t* p)
{
    return __builtin_nontemporal_load((const u32x2*)p);
}
__device__ __forceinline__ void st_nt_f4(float* p, f32x4 v)
{
    __builtin_nontemporal_store(v, (f32x4*)p);
}

// Value of lane (l - 1) within a 16-lane DPP row; lane 0 of each row reads 0.
__device__ __forceinline__ int dpp_shr1(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);
}
__device__ __forceinline__ int dpp_shr2(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);
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
