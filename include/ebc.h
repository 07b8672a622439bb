/*
 * ebc.h -- C ABI of the MI355X (gfx950) error-bounded lossy compressor core.
 *
 * Method: Tian et al., "Optimizing Error-Bounded Lossy Compression for
 * Scientific Data on GPUs" (cuSZ+).  Compression = dual-quantisation with the
 * first-order Lorenzo predictor (Sec. IV-A.1, Algorithm 1 compression half),
 * the modified quantisation scheme with outliers (Sec. IV-B.1), a histogram
 * and canonical Huffman code (Sec. II-A steps 5-8), and the adaptive choice of
 * run-length encoding when the Huffman average bit length is <= 1.09
 * (Sec. I, Sec. III-B).  Decompression = Huffman or RLE decoding, fusing
 * quant-codes with outliers, and Lorenzo reconstruction as an N-D partial sum
 * (Sec. IV-B.2, Algorithm 1 decompression half).
 *
 * Conventions shared by every entry point
 *   - Return value: EBC_OK (0) or a negative EBC_ERR_* status.  No exception
 *     ever crosses the ABI.  ebc_last_error() gives a human-readable detail
 *     for the calling thread's last failure.
 *   - Pointers named d_* are HIP device pointers on the current device; h_*
 *     and all other pointers are host pointers.  The caller owns every
 *     buffer, including the workspace; the library allocates no device memory
 *     in these calls.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *     All device work is enqueued on it in order.  Calls that return a host
 *     value computed on the device (out_size, stats) synchronise that stream
 *     once; the *_async variants never synchronise.
 *   - A field is fp32 (or fp64 with dtype EBC_F64), row-major with x fastest;
 *     dims = {nx, ny, nz}; unused trailing dims must be 1; rank is 1, 2 or 3;
 *     the element count must be < 2^32.  An archive records the element type;
 *     decompression writes elements of that type.
 *   - Calls on distinct workspaces are independent and may run concurrently
 *     on different streams.  The library keeps no mutable global state.
 */
#ifndef EBC_H
#define EBC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EBC_VERSION 1

/* status codes */
#define EBC_OK 0
#define EBC_ERR_ARG (-1)           /* null pointer or invalid enum value */
#define EBC_ERR_DIMS (-2)          /* rank not 1..3, zero dim, unused dim != 1, N >= 2^32 */
#define EBC_ERR_EB (-3)            /* eb <= 0, not finite, or absurdly large */
#define EBC_ERR_EB_TOO_SMALL (-4)  /* bound below what fp32 output can honour (guard step) */
#define EBC_ERR_BINS (-5)          /* n_bins odd, < 4 or > 65536 */
#define EBC_ERR_NONFINITE (-6)     /* NaN or Inf in the field */
#define EBC_ERR_OUT_TOO_SMALL (-7) /* output buffer (or out_elems) too small */
#define EBC_ERR_WS_TOO_SMALL (-8)  /* workspace smaller than the *_workspace_size result */
#define EBC_ERR_ARCHIVE (-9)       /* bad magic/version/size, truncated or inconsistent archive */
#define EBC_ERR_HIP (-10)          /* HIP launch or runtime failure */
#define EBC_ERR_UNSUPPORTED (-11)  /* valid format option this GPU path does not implement */

/* error-bound mode: absolute, or relative to the value range max - min
   (Sec. II-B.1 table caption; Sec. V-B uses 1e-4 relative) */
#define EBC_EB_ABS 0
#define EBC_EB_REL 1

/* codec request: AUTO applies the 1.09-bit rule (Sec. I, Sec. III-B.2) and
   picks the Huffman or the run-length workflow; AUTO_VLE applies the same
   rule, and its run-length branch Huffman-codes the run values as well
   (the workflow "RLE with optional VLE" of Sec. III-A, VLE switched on);
   RLE_VLE forces that branch. */
#define EBC_CODEC_AUTO 0
#define EBC_CODEC_HUFFMAN 1
#define EBC_CODEC_RLE 2
#define EBC_CODEC_RLE_VLE 3
#define EBC_CODEC_AUTO_VLE 4

/* codec recorded in an archive */
#define EBC_ARC_HUFFMAN 0
#define EBC_ARC_RLE 1
#define EBC_ARC_CONST 2
#define EBC_ARC_RLE_VLE 3  /* RLE with the run values Huffman-coded (Sec. III-A) */

/* element type of a field (input of compression, output of decompression) */
#define EBC_F32 0
#define EBC_F64 1 /* fp64 fields through the same integer core (Sec. III: Huffman CR <= 64) */

typedef struct ebc_params {
    int32_t eb_mode;     /* EBC_EB_ABS or EBC_EB_REL */
    int32_t codec;       /* EBC_CODEC_* */
    double eb;           /* error bound (absolute value, or fraction of the range) */
    uint32_t n_bins;     /* quantisation bins (cap = 2 * radius, Algorithm 1); even,
                            4..65536 (above 4096 the per-bin tables live in HBM) */
    uint32_t huff_chunk; /* symbols per Huffman chunk: 0 selects 1024; power of two
                            in 64..65536 */
    int32_t dtype;       /* EBC_F32 or EBC_F64: element type of the field to compress */
    int32_t reserved;    /* 0 */
} ebc_params;

/* stats flags (in ebc_stats.flags) */
#define EBC_STATS_TIMING 1u /* record a hipEvent pair around every kernel stage */

#define EBC_MAX_STAGES 16
typedef struct ebc_stats {
    uint32_t flags;      /* in: EBC_STATS_* */
    int32_t codec;       /* out: EBC_ARC_* chosen */
    uint64_t n_elems;    /* out */
    uint64_t n_outliers; /* out */
    uint64_t n_runs;     /* out: RLE runs (RLE codec) */
    uint64_t n_words;    /* out: Huffman payload words (Huffman codec) */
    uint64_t huff_bits;  /* out: sum over symbols of freq * code length */
    uint64_t out_bytes;  /* out: archive size (compress) */
    double eb_abs;       /* out: absolute error bound */
    double ebx2;         /* out: quantisation step actually used */
    float value_min;     /* out */
    float value_max;     /* out */
    uint32_t n_stages;   /* out: number of valid stage_ms / stage_name entries */
    float stage_ms[EBC_MAX_STAGES];           /* out: per-stage kernel time (TIMING) */
    const char* stage_name[EBC_MAX_STAGES];   /* out: static strings */
    const char* time_only; /* in: with TIMING, NULL times every stage; else only the stage
                              of this name gets an event pair (one stage reported), so
                              that the rest of the call runs uninstrumented */
    /* out (compression): the histogram estimates of Sec. III-B.1, see ebc_estimate */
    double entropy;      /* H of the quant-code histogram, bits per symbol */
    double p1;           /* probability of the most likely code */
    double r_lo, r_hi;   /* Huffman redundancy bounds: H + r_lo <= avg bits <= H + r_hi */
    int32_t predict;     /* workflow the bounds predict: 1 run-length, 0 Huffman, 2 undecided */
    int32_t pad;
} ebc_stats;

/* Compressibility estimates (Sec. III-B) of a field's quant-codes. */
#define EBC_MADO_DMAX 200 /* largest madogram distance (Sec. III-B.2) */
typedef struct ebc_estimates {
    int32_t codec_hint;  /* 1 run-length, 0 Huffman, 2 undecided (the bounds straddle 1.09) */
    int32_t pad;
    double entropy;      /* H = -sum p_i log2 p_i over the code histogram (Sec. III-B.1) */
    double p1;           /* probability of the most likely code */
    double r_lo, r_hi;   /* redundancy bounds: R- = 1 - H(p1, 1-p1) for p1 > 0.4 (else 0;
                            1 for a single code), R+ = p1 + 0.086 */
    double bits_lo, bits_hi; /* H + r_lo and H + r_hi: bounds of the Huffman average bits */
    uint64_t hist_max;   /* count of the most likely code */
    uint64_t n_elems;
    uint64_t samples;    /* madogram samples drawn (pairs past the end are skipped) */
    double roughness;    /* sum of mado_sum / sum of mado_cnt over all distances */
    uint64_t mado_sum[EBC_MADO_DMAX + 1]; /* pairs at distance d whose codes differ */
    uint64_t mado_cnt[EBC_MADO_DMAX + 1]; /* pairs at distance d (index 0 unused) */
} ebc_estimates;

/* Library version (EBC_VERSION) and a static string for a status code. */
int ebc_version(void);
const char* ebc_status_string(int status);
/* Detail of the calling thread's last failure (static storage, never NULL). */
const char* ebc_last_error(void);

/* Upper bound of the archive size for a field (host only, no device work).
   Bound: 128-byte header + max(Huffman, RLE) payload + 8 bytes per element for
   outliers, with 16-byte section alignment. */
int ebc_compress_bound(int rank, const uint64_t dims[3], const ebc_params* p,
                       uint64_t* max_bytes);

/* Device workspace bytes ebc_compress needs for this field (host only). */
int ebc_compress_workspace_size(int rank, const uint64_t dims[3], const ebc_params* p,
                                uint64_t* bytes);

/* Compress one device-resident field into a device-resident archive.
   d_field: N fp32 (device).  d_out: archive bytes (device), out_cap bytes.
   out_size (host, required): archive size; the stream is synchronised once
   to read it.  d_ws/ws_bytes: device workspace of at least
   ebc_compress_workspace_size bytes, contents need not be initialised.
   stats (host, nullable): filled after the synchronisation.
   Errors detected on the device (NaN/Inf, bound too small, output too small)
   are returned after that synchronisation; the output is then undefined. */
int ebc_compress(const void* d_field, int rank, const uint64_t dims[3], const ebc_params* p,
                 void* d_out, uint64_t out_cap, uint64_t* out_size, void* d_ws,
                 uint64_t ws_bytes, void* stream, ebc_stats* stats);

/* As ebc_compress but never synchronises: the archive size (uint64, 0 on a
   device-detected error) and the status (int32) are written to device memory
   d_result[0] and ((int32_t*)(d_result + 1))[0] once the stream reaches them.
   d_result must hold 16 bytes.  Host-detectable argument errors are returned
   immediately. */
int ebc_compress_async(const void* d_field, int rank, const uint64_t dims[3],
                       const ebc_params* p, void* d_out, uint64_t out_cap, uint64_t* d_result,
                       void* d_ws, uint64_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under stream capture,
   tight serving loops, hosts that forbid hipMalloc): ebc_compress_async
   without a workspace argument.  The workspace is a fixed device array of
   EBC_NOALLOC_SCRATCH_BYTES inside this library; each device the call runs
   on holds its own copy until the process ends (its address is resolved on
   the first call on that device, with that device current).  The call
   allocates no device or page-locked memory (host bookkeeping uses the C++
   heap).  Arguments, outputs and results are those of ebc_compress_async; the
   caller still provides d_field, d_out and d_result.
   Limit: a field whose ebc_compress_workspace_size exceeds the array is
   rejected with EBC_ERR_WS_TOO_SMALL before any device work (about 6.7 bytes
   per fp32 element: fields up to roughly 9.5 million values).
   Every call on one device shares that device's array: calls that overlap in
   time on one device (streams not ordered after each other) race and give
   undefined archives.  Calls ordered on one stream are safe. */
#define EBC_NOALLOC_SCRATCH_BYTES (64ull << 20)
int ebc_compress_async_noalloc(const void* d_field, int rank, const uint64_t dims[3],
                               const ebc_params* p, void* d_out, uint64_t out_cap,
                               uint64_t* d_result, void* stream);

/* Parse a host copy of an archive header (at least 128 bytes).  Any output
   pointer may be NULL.  p receives eb mode, eb, n_bins, the Huffman chunk and
   the element type. */
int ebc_archive_info(const void* h_header, uint64_t header_bytes, int* rank, uint64_t dims[3],
                     ebc_params* p, int* codec, uint64_t* total_bytes);

/* Device workspace bytes ebc_decompress needs for this archive (host only). */
int ebc_decompress_workspace_size(const void* h_header, uint64_t header_bytes, uint64_t* bytes);

/* Decompress a device-resident archive (size bytes) into d_out (out_elems
   fp32, device).  Reads the 128-byte header back to the host once, launches
   the decode, and synchronises once more to return the device-side status. */
int ebc_decompress(const void* d_archive, uint64_t size, void* d_out, uint64_t out_elems,
                   void* d_ws, uint64_t ws_bytes, void* stream, ebc_stats* stats);

/* As ebc_decompress with the header supplied by the caller (host copy) and no
   synchronisation; the int32 status lands in d_status (device). */
int ebc_decompress_async(const void* h_header, const void* d_archive, uint64_t size,
                         void* d_out, uint64_t out_elems, void* d_ws, uint64_t ws_bytes,
                         int32_t* d_status, void* stream);

/* ---------------------------------------------------------------------- */
/* Batched path: many fields of mixed rank and size through one sequence of */
/* launches (each kernel covers every field's tiles in one grid).           */
/* ---------------------------------------------------------------------- */
typedef struct ebc_field {
    const void* d_field;  /* input field (device), of the batch's dtype */
    int32_t rank;
    uint32_t reserved;
    uint64_t dims[3];
    void* d_out;          /* archive buffer (device) */
    uint64_t out_cap;
} ebc_field;

typedef struct ebc_result {
    uint64_t out_size; /* archive bytes */
    int32_t status;    /* EBC_OK or a device-detected error for this field */
    int32_t codec;     /* EBC_ARC_* */
} ebc_result;

int ebc_batch_compress_workspace_size(int n, const ebc_field* fields, const ebc_params* p,
                                      uint64_t* bytes);
/* Compress n fields with the same parameters; results[i] (host) is filled
   after one synchronisation.  Returns the first non-OK field status, or the
   host-side validation error. */
int ebc_batch_compress(int n, const ebc_field* fields, const ebc_params* p, ebc_result* results,
                       void* d_ws, uint64_t ws_bytes, void* stream);

/* As ebc_batch_compress without any synchronisation: d_results (device, n
   records of 16 bytes, caller's order) receives {out_size, status, codec}
   when the stream reaches the end of the work.  Only kernel launches are
   enqueued, so the call can be captured into a HIP graph; host-side
   validation errors are returned immediately and enqueue nothing. */
int ebc_batch_compress_async(int n, const ebc_field* fields, const ebc_params* p,
                             ebc_result* d_results, void* d_ws, uint64_t ws_bytes, void* stream);

typedef struct ebc_archive_ref {
    const void* d_archive; /* device */
    uint64_t size;
    const void* h_header;  /* host copy of the first 128 bytes */
    void* d_out;           /* device output, elements of the archive's type */
    uint64_t out_elems;
} ebc_archive_ref;

int ebc_batch_decompress_workspace_size(int n, const ebc_archive_ref* refs, uint64_t* bytes);
/* Decompress n archives; statuses (host, n entries) filled after one sync. */
int ebc_batch_decompress(int n, const ebc_archive_ref* refs, int32_t* statuses, void* d_ws,
                         uint64_t ws_bytes, void* stream);
/* As ebc_batch_decompress without synchronisation: d_statuses (device, n
   int32, caller's order) receives each field's status.  Kernel launches only
   (graph-capturable). */
int ebc_batch_decompress_async(int n, const ebc_archive_ref* refs, int32_t* d_statuses,
                               void* d_ws, uint64_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Tuning: tile shape, grid and scan schedule per (rank, shape class).      */
/* Tuning never changes the output bytes, only the launch geometry.         */
/* ---------------------------------------------------------------------- */
typedef struct ebc_tuning_entry {
    int32_t rank;      /* 1, 2 or 3 */
    uint32_t nx_class; /* ceil(log2(nx)) */
    uint32_t n_class;  /* 0: N < 2^20, 1: N < 2^24, 2: larger */
    uint32_t tile_wx;  /* 2D/3D workgroup tile width in waves along x (1, 2 or 4); the
                          tile is tile_wx * 64 x (4/tile_wx) * 16 in 2D and
                          tile_wx * 32 x (4/tile_wx) * 8 x 8 in 3D; 0 = default */
    uint32_t grid;     /* persistent construction grid in workgroups, 64..16384;
                          0 = default (the workgroups the device holds at once) */
    uint32_t scan_direct; /* scan schedule: a prefix sum of up to this many tiles of
                          4096 items adds each tile's predecessors directly, a longer
                          one scans the tile sums in a workgroup first; 0 = default
                          (1024), at most 2^20.  A call takes the largest value among
                          its fields' entries. */
} ebc_tuning_entry;

/* Replace the library's tuning table (n = 0 clears it).  This table is the
   library's only global state: every later call takes one snapshot of it.
   Calls already running are unaffected.  A workspace size obtained under one
   table may be too small under another (the call then fails with
   EBC_ERR_WS_TOO_SMALL; it never overruns). */
int ebc_set_tuning(const ebc_tuning_entry* entries, int n);

/* Shape class of a field, as used to look up the tuning table. */
int ebc_shape_class(int rank, const uint64_t dims[3], uint32_t* nx_class, uint32_t* n_class);

/* ---------------------------------------------------------------------- */
/* Test / inspection entry points: stop the compression after the          */
/* dual-quantisation step and expose its products.                        */
/* ---------------------------------------------------------------------- */
/* Runs value range, quantisation step, Lorenzo construction and histogram.
   d_q: N uint16 quant-codes; d_hist: n_bins uint32; d_oidx/d_oval: outlier
   indices (ascending) and int32 deltas, capacity N each; n_outliers (host)
   receives the count; ebx2 (host, nullable) the step.  Synchronises once. */
int ebc_debug_construct(const void* d_field, int rank, const uint64_t dims[3],
                        const ebc_params* p, uint16_t* d_q, uint32_t* d_hist, uint32_t* d_oidx,
                        int32_t* d_oval, uint64_t* n_outliers, double* ebx2, void* d_ws,
                        uint64_t ws_bytes, void* stream);

/* Reconstruction alone: from quant-codes and an outlier list to fp32
   (fuse + partial sum + dequantisation).  Synchronises once. */
int ebc_debug_reconstruct(const uint16_t* d_q, const uint32_t* d_oidx, const int32_t* d_oval,
                          uint64_t n_outliers, int rank, const uint64_t dims[3], uint32_t n_bins,
                          double ebx2, float* d_out, void* d_ws, uint64_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* EBC_H */
