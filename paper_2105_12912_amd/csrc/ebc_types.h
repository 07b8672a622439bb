// ebc_types.h -- descriptors shared by the host planner and the HIP kernels.
//
// Work decomposition: every kernel covers all fields of a batch in one grid.
// Each field owns a contiguous range of the grid's work units of that kernel
// (FieldDesc::*_base); a workgroup finds its field with a binary search over
// those bases.  A single-field call is simply a batch of one.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

// Device code sees every buffer pointer of a descriptor in the global address
// space, so accesses compile to global_* instructions (a flat access would
// also count against the LDS wait counter and serialise LDS work behind HBM).
#if defined(__HIP_DEVICE_COMPILE__)
#define EBC_G __attribute__((address_space(1)))
#else
#define EBC_G
#endif

namespace ebc {

constexpr int kWave = 64;
constexpr int kBlock = 256;                 // threads per workgroup everywhere
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr uint32_t kHdr = 128;              // archive header bytes
constexpr uint32_t kMaxBins = 4096;         // n_bins whose per-bin tables fit in LDS ("narrow")
constexpr uint32_t kBinsLimit = 65536;      // largest n_bins of the format (wide above kMaxBins)
constexpr uint32_t kHistWin = 4096;         // wide bins: LDS histogram slots (code 0 + a window
                                            // of codes around the centre; others counted in HBM)
constexpr uint32_t kPassHc = 4096;          // Huffman chunk symbols an encode pass covers
constexpr uint32_t kRangeUnit = 16384;      // elements per value-range work unit
constexpr uint32_t kRleTile = 4096;         // elements per RLE work unit
constexpr uint32_t kPersistentBlocks = 1024; // grid size of the persistent (grid-stride) kernels
constexpr uint32_t kConstructBlocks = 2048;  // construction grid: 8 workgroups per CU
constexpr int kLutBits = 12;                // Huffman decode table width (bits looked up at once)
constexpr int kMaxDecodeLen = 60;          // longest code the decoder accepts (N < 2^32 gives <= 46)
constexpr uint32_t kL2Size = 2048;         // second-level decode table entries
constexpr uint32_t kL2MaxBits = 8;         // bits a second-level table resolves at most
constexpr uint32_t kSubMax = 256;          // Huffman sub-chunk symbols (hs = min(hc, kSubMax))
constexpr uint32_t kDecLanes = 768;        // decode workgroup: one lane per sub-chunk

enum : int32_t { ARC_HUFFMAN = 0, ARC_RLE = 1, ARC_CONST = 2, ARC_RLE_VLE = 3 };
enum : int32_t { REQ_AUTO = 0, REQ_HUFFMAN = 1, REQ_RLE = 2, REQ_RLE_VLE = 3, REQ_AUTO_VLE = 4 };

// A field's symbols go through the Huffman coder: its quant-codes (Huffman
// codec) or its run values (RLE+VLE codec).
__host__ __device__ inline bool huff_codec(int32_t c) { return c == ARC_HUFFMAN || c == ARC_RLE_VLE; }
// A field is run-length coded (with or without a Huffman pass over the values).
__host__ __device__ inline bool rle_codec(int32_t c) { return c == ARC_RLE || c == ARC_RLE_VLE; }
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
    double mn, mx;
    double eb_abs, ebx2, inv;
    uint64_t n_out;
    uint64_t n_runs;
    uint64_t n_words;
    uint64_t huff_bits;
    uint64_t total;
    uint64_t off_sbits, off_words, off_rlen, off_oidx, off_oval;
    uint32_t max_len;
    uint32_t n_used;  // symbols with a non-zero count
    uint64_t zero_count;
    uint32_t fix_count;  // decompress 3D: chunks queued for the outlier fix-up
    uint32_t pad0;
    uint64_t pad[1];
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
    // construct / reconstruct tiling.  2D/3D: a workgroup tile is wx waves
    // along x by 4/wx along y; a wave covers 64 x 16 (2D, four 16x16 chunks)
    // or 32 x 8 x 8 (3D, four 8x8x8 chunks).  1D: a wave covers four chunks.
    uint32_t wx;             // waves along x in a workgroup tile (1, 2 or 4)
    uint32_t xs;             // x extent of a workgroup tile = outlier segment length
    uint32_t nxb, nyb, nzb;  // workgroup-tile grid (2D/3D)
    uint32_t n_wave_tiles;   // 1D wave tiles
    uint32_t vec;            // 1: rows 16-byte aligned, quads never straddle rows
    uint32_t slot;           // position of this field in the caller's arrays
    // buffers (device)
    const EBC_G float* in;   // compress input (fp32 field)
    const EBC_G double* in64;  // compress input (fp64 field)
    EBC_G float* outf;       // decompress output (fp32 archive)
    EBC_G double* outd;      // decompress output (fp64 archive)
    EBC_G float* sink;       // decompress: 256 bytes that absorb stores of absent elements
    EBC_G uint8_t* arc;      // archive (compress output / decompress input)
    uint64_t arc_cap;        // compress: capacity; decompress: archive size
    EBC_G uint16_t* q;       // quant-codes, n
    EBC_G int32_t* dsc;      // outlier delta scratch, n (dense, sparsely written)
    EBC_G uint32_t* hist;    // n_bins
    EBC_G uint32_t* hpart;   // hrows * n_bins partial histograms
    uint32_t hrows;          // construction workgroups visiting this field
    EBC_G uint32_t* rpart;   // range partials: 3 words per range unit (3 x 64 bits for fp64)
    EBC_G uint64_t* code;    // n_bins packed codewords: (len << 56) | code
    EBC_G uint8_t* len;      // n_bins code lengths
    EBC_G uint8_t* cbs;      // wide bins: codebook scratch (codebook_wide_scratch_bytes)
    EBC_G uint32_t* hbits;   // per Huffman chunk bit counts
    EBC_G uint32_t* rstart;  // RLE run starts (compress scratch)
    EBC_G uint16_t* vsym;    // RLE+VLE: run values (compress: source of the Huffman pass;
                             // decompress: its output), n entries at most
    EBC_G uint32_t* vhist;   // RLE+VLE compress: histogram of the run values (n_bins)
    EBC_G uint16_t* hsym;    // decompress: Huffman decoder output (q, or vsym for RLE+VLE)
    const EBC_G uint16_t* rval;  // decompress: run values (archive section, or vsym)
    EBC_G uint32_t* oflag;   // decompress 3D: per wave block, a bit per 8-wide x chunk with outliers
    EBC_G uint32_t* fixl;    // decompress 3D: an outlier index in each flagged chunk (n_out)
    EBC_G FieldDyn* dyn;
    // this field's work units in each batch-wide index space
    uint32_t range_units, range_base;  // value range / fill: kRangeUnit elements per WG
    uint32_t wg_tiles, wg_base;        // construct / reconstruct WG tiles (rank group relative)
    uint32_t n_seg, seg_base;          // outlier segments: count-array entries
    uint32_t ow_units, ow_base;        // outlier write: 1024 segments per WG
    uint32_t n_hch, hch_base;          // Huffman chunks: word-count array entries
    uint32_t hs;                       // Huffman sub-chunk symbols: min(hc, 256)
    uint32_t n_sub, sub_base;          // Huffman sub-chunks: in-chunk start offsets
    uint32_t hwg_units, hwg_base;      // Huffman encode: huff_cpw(hc) chunks per WG
    uint32_t hdwg_units, hdwg_base;    // Huffman decode: kDecLanes sub-chunks per WG
    uint32_t hpwg_units, hpwg_base;    // Huffman decode prologue: kBlock chunks per WG
    uint32_t n_rt, rt_base;            // RLE tiles of kRleTile elements (count array / WG)
    uint32_t n_runs_hdr, rle_base;     // decompress: runs in the archive (start array entries)
    uint32_t sc_units, sc_base;        // decompress outlier scatter: 256 outliers per WG
    uint32_t rl_units, rl_base;        // decompress run-length prep: 256 runs per WG
    uint32_t fx_units, fx_base;        // decompress 3D outlier fix-up: 4 chunks per WG
    // decompress: header values
    uint64_t hn;             // symbols of the Huffman stream (N, or the run count for RLE+VLE)
    uint64_t n_out_hdr;
    uint64_t n_words_hdr;
    double ebx2_hdr;
    double cval;
    int32_t codec_hdr;
    int32_t dtype;           // 0 fp32, 1 fp64 (input at compression, output at decompression)
    uint64_t off_sbits, off_words, off_val, off_rlen, off_oidx, off_oval;
};

// Compressibility estimates of one field (Sec. III-B), written on the device.
constexpr uint32_t kMadoDist = 200;        // largest madogram distance (Sec. III-B.2)
struct EstDev {
    double entropy, p1, r_lo, r_hi;
    uint64_t hist_max;
    int32_t predict;  // 1 run-length, 0 Huffman, 2 undecided
    int32_t pad;
    uint64_t mado_sum[kMadoDist + 1];
    uint64_t mado_cnt[kMadoDist + 1];
};

// Canonical Huffman decoder tables of one field (built by k_dectab).
// lut[p] decodes the next kLutBits stream bits p into up to three whole
// codewords: bits 0-15/16-31/32-47 the symbols (zero when absent), 48-49 how
// many (0 = the first codeword is longer than kLutBits), 50-55 their total
// length, 56-59 and 60-63 the lengths of the first two.  When the first
// codeword is longer, bits 0-15 hold the start of this prefix's block of
// 2^l2k entries in l2 (0xFFFF: none), indexed by the next l2k bits; an l2
// entry is (length << 16) | symbol, or 0 for a codeword longer still.
struct DecTab {
    uint64_t first[65];   // first code of each length
    uint64_t endv[65];    // (first[L] + count[L]) << (64 - L): a left-aligned window w holds a
                          // code of length <= L iff w < endv[L] (defined for L < max_len)
    uint32_t count[65];   // codes of each length
    uint32_t offset[65];  // index of the first symbol of each length in perm
    uint32_t max_len;
    uint32_t l2k;             // bits resolved by the second level (0: no second level)
    uint32_t l2n;             // second-level entries in use
    uint32_t pad;
    uint64_t lut[1u << kLutBits];
    uint32_t l2[kL2Size];
    uint16_t perm[2];         // symbols ordered by (length, symbol): n_bins entries (the
                              // table occupies dectab_bytes(n_bins))
};

// chunks per encode workgroup (one per wave); chunks longer than kPassHc
// symbols are encoded by one wave in passes of kPassHc
__host__ __device__ constexpr uint32_t huff_cpw(uint32_t hc) { return hc <= 1024 ? 4 : hc <= kPassHc ? kPassHc / hc : 1; }

// histogram slots a construction workgroup keeps in LDS for n_bins bins
__host__ __device__ constexpr uint32_t hist_slots(uint32_t nb) { return nb > kMaxBins ? kHistWin : nb; }
// wide bins: the first code of the LDS window (slot 1); slot 0 is code 0
__host__ __device__ constexpr uint32_t hist_win_lo(uint32_t nb) { return nb / 2 - (kHistWin / 2 - 1); }

// decoder table bytes for n_bins symbols (the permutation grows with n_bins)
__host__ __device__ constexpr size_t dectab_bytes(uint32_t nb)
{
    return (offsetof(DecTab, perm) + 2 * (size_t)(nb > 2 ? nb : 2) + 255) & ~(size_t)255;
}

}  // namespace ebc
