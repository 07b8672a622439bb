// ebc_launch.h -- host-side launchers of the HIP kernels (one per kernel
// family); each enqueues on the given stream and returns hipGetLastError().
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ebc_types.h"

namespace ebc {

// Records a failure detail for ebc_last_error() (calling thread) and returns status.
int set_error(int status, const char* fmt, ...);

constexpr int kDescPerLaunch = 8;
struct DescBlob {
    int first;
    int count;
    FieldDesc d[kDescPerLaunch];
};

// scan
uint32_t scan_tmp_words(uint32_t n);
// exclusive scan, total in a[n]; direct_max: tile count up to which each
// tile's workgroup adds the sums of the tiles before it (0: the default),
// above which the tile sums are scanned by one workgroup first
hipError_t launch_scan(uint32_t* a, uint32_t n, uint32_t* tmp, hipStream_t s, uint32_t direct_max = 0);

// quantisation
hipError_t launch_range(const FieldDesc* F, int nf, uint32_t units, bool f64, hipStream_t s);
hipError_t launch_params(const FieldDesc* F, int nf, hipStream_t s);
uint32_t construct_resident_blocks(int rank, bool vec, uint32_t n_bins, bool f64);
hipError_t launch_construct(const FieldDesc* F, int nf, int rank, bool vec, bool f64, uint32_t wg_tiles,
                            uint32_t blocks, uint32_t n_bins, uint32_t* seg_cnt, hipStream_t s);
hipError_t launch_hist_reduce(const FieldDesc* F, int nf, uint32_t n_bins, hipStream_t s);

// codebook
size_t codebook_lds_bytes(uint32_t n_bins);
hipError_t launch_codebook(const FieldDesc* F, int nf, uint32_t n_bins, int pass, hipStream_t s);
hipError_t launch_dectab(const FieldDesc* F, int nf, uint8_t* tabs, size_t stride, uint32_t max_bins,
                         hipStream_t s);
size_t codebook_wide_scratch_bytes(uint32_t n_bins);

// compressibility estimates (histogram bounds; madogram over `samples` pairs)
hipError_t launch_estimate(const FieldDesc* F, int nf, EstDev* est, uint64_t samples, uint64_t seed,
                           hipStream_t s);

// Huffman
size_t huff_write_lds_bytes(uint32_t n_bins, uint32_t hc);
hipError_t launch_huff_bits(const FieldDesc* F, int nf, uint32_t units, uint32_t hc, uint32_t n_bins,
                            uint32_t* wcnt, int which, hipStream_t s);
hipError_t launch_huff_write(const FieldDesc* F, int nf, uint32_t units, uint32_t hc,
                             uint32_t n_bins, const uint32_t* woff, hipStream_t s);
hipError_t launch_words_check(const FieldDesc* F, int nf, const uint32_t* woff, hipStream_t s);
hipError_t launch_huff_prep(const FieldDesc* F, int nf, uint32_t units, uint32_t* wcnt, uint32_t* soff,
                            hipStream_t s);
hipError_t launch_huff_decode(const FieldDesc* F, int nf, uint32_t units, const uint32_t* woff,
                              const uint32_t* soff, const uint8_t* tabs, size_t tab_stride,
                              hipStream_t s);

// RLE
hipError_t launch_rle_count(const FieldDesc* F, int nf, uint32_t units, uint32_t* rcnt, hipStream_t s);
// what: 1 run values into the archive (RLE), 2 run values into the value
// stream (RLE+VLE), 4 run starts
hipError_t launch_rle_write(const FieldDesc* F, int nf, uint32_t units, const uint32_t* roff, int what,
                            hipStream_t s);
// RLE+VLE: run counts, the run-value stream and its histogram
hipError_t launch_rle_vle_prep(const FieldDesc* F, int nf, uint32_t units, const uint32_t* roff,
                               uint32_t n_bins, hipStream_t s);
hipError_t launch_rle_len(const FieldDesc* F, int nf, uint32_t max_units, hipStream_t s);
hipError_t launch_rle_decode(const FieldDesc* F, int nf, uint32_t rl_units, uint32_t rt_units,
                             uint32_t* starts, uint32_t* tmap, uint32_t* tmp, uint32_t n_starts,
                             uint32_t scan_direct, hipStream_t s);

// outliers
uint32_t outlier_write_units(uint32_t n_seg);
hipError_t launch_outlier_write(const FieldDesc* F, int nf, uint32_t units, const uint32_t* soff,
                                hipStream_t s);
hipError_t launch_outlier_scatter(const FieldDesc* F, int nf, uint32_t units, hipStream_t s);

// reconstruction
hipError_t launch_reconstruct(const FieldDesc* F, int nf, int rank, bool vec, bool f64, uint32_t wg_tiles,
                              uint32_t blocks, hipStream_t s);
hipError_t launch_recon_fix(const FieldDesc* F, int nf, uint32_t units, hipStream_t s);
hipError_t launch_recon_check(const FieldDesc* F, int nf, hipStream_t s);
hipError_t launch_dinit(const FieldDesc* F, int nf, hipStream_t s);
hipError_t launch_fill_const(const FieldDesc* F, int nf, uint32_t units, hipStream_t s);

// archive
hipError_t launch_layout(const FieldDesc* F, int nf, const uint32_t* soff, const uint32_t* woff,
                         const uint32_t* roff, hipStream_t s);
hipError_t launch_header(const FieldDesc* F, int nf, hipStream_t s);
hipError_t launch_result(const FieldDesc* F, uint64_t* res, hipStream_t s);
hipError_t launch_status(const FieldDesc* F, int32_t* st, hipStream_t s);
hipError_t launch_batch_results(const FieldDesc* F, int nf, uint64_t* res, hipStream_t s);
hipError_t launch_batch_status(const FieldDesc* F, int nf, int32_t* st, hipStream_t s);
hipError_t upload_descs(const FieldDesc* host, int nf, FieldDesc* dev, hipStream_t s);

}  // namespace ebc
