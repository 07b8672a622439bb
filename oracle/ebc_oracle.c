/*
 * ebc_oracle.c -- plain CPU oracle for the error-bounded compressor of
 * Tian et al., "Optimizing Error-Bounded Lossy Compression for Scientific
 * Data on GPUs" (arXiv 2105.12912, "cuSZ+").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library; the product path (the HIP
 * library under paper_2105_12912_amd/) never does, and the two share no code,
 * header, table or constant generator.  The archive layout and the status
 * numbers are an interface both sides implement independently.
 *
 * Every step is a plain single-threaded loop in the order the paper gives it;
 * floating point is IEEE binary64 (SSE2, no contraction, no fast-math).
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *   - delta = d - p  (Sec. IV-A.1, "postquant"; Algorithm 1 prints p - d),
 *   - in-range test |delta| < r with r = n_bins/2, code 0 = outlier,
 *   - outliers store the int32 delta, fused by replacement before the
 *     partial sum (Sec. IV-B.1),
 *   - prequant multiplies by the fp64 reciprocal of a slightly shrunken
 *     step 2*eb*(1-eps) and rounds half to even, so |x - xhat| <= eb holds
 *     after the final fp32 rounding (Sec. IV-A.1 states the bound),
 *   - chunks: 256 (1D), 16x16 (2D), 8x8x8 (3D); zero outside a chunk
 *     (Sec. II-A, Sec. IV-B.3),
 *   - canonical Huffman with a deterministic two-queue construction,
 *     leaf wins ties (Sec. II-A step 6 only names "canonical"),
 *   - adaptive choice: RLE iff the Huffman average bit length <= 1.09,
 *     evaluated as the integer test 100*sum(f*len) <= 109*N
 *     (Sec. I contribution list, Sec. III-B.2),
 *   - the workflow "RLE with optional VLE" (Sec. III-A): on request, the run
 *     values are Huffman-coded with a codebook of their own; the run lengths
 *     stay plain (the paper leaves that metadata uncoded by default),
 *   - fp64 fields (Sec. III, where the Huffman ceiling is 64 for double) run
 *     through the same integer core with a guard step sized for fp64 output.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Status numbers: identical values to the C ABI of the product library. */
enum {
    ORA_OK = 0,
    ORA_ERR_ARG = -1,
    ORA_ERR_DIMS = -2,
    ORA_ERR_EB = -3,
    ORA_ERR_EB_TOO_SMALL = -4,
    ORA_ERR_BINS = -5,
    ORA_ERR_NONFINITE = -6,
    ORA_ERR_OUT_TOO_SMALL = -7,
    ORA_ERR_WS_TOO_SMALL = -8,
    ORA_ERR_ARCHIVE = -9,
    ORA_ERR_HIP = -10,
    ORA_ERR_UNSUPPORTED = -11,
    ORA_ERR_NOMEM = -12
};

/* Archive codec byte and API codec request (two different enumerations). */
enum { ARC_HUFFMAN = 0, ARC_RLE = 1, ARC_CONST = 2, ARC_RLE_VLE = 3 };
enum { REQ_AUTO = 0, REQ_HUFFMAN = 1, REQ_RLE = 2, REQ_RLE_VLE = 3, REQ_AUTO_VLE = 4 };
enum { EB_ABS = 0, EB_REL = 1 };
enum { DT_F32 = 0, DT_F64 = 1 };

#define HDR_BYTES 128u

/* ------------------------------------------------------------------------ */
/* C1: value range.  A total order with -0 < +0 so both ends are unique.     */
/* ------------------------------------------------------------------------ */
static int less_total(float a, float b)
{
    if (a < b) return 1;
    if (a == b && a == 0.0f && signbit(a) && !signbit(b)) return 1;
    return 0;
}

int ora_value_range(const float* x, uint64_t n, float* mn, float* mx)
{
    if (!x || !mn || !mx || n == 0) return ORA_ERR_ARG;
    float lo = x[0], hi = x[0];
    for (uint64_t i = 0; i < n; ++i) {
        if (!isfinite(x[i])) return ORA_ERR_NONFINITE;
        if (less_total(x[i], lo)) lo = x[i];
        if (less_total(hi, x[i])) hi = x[i];
    }
    *mn = lo;
    *mx = hi;
    return ORA_OK;
}

/* C1 for fp64 fields: the same total order (-0 < +0). */
static int less_total64(double a, double b)
{
    if (a < b) return 1;
    if (a == b && a == 0.0 && signbit(a) && !signbit(b)) return 1;
    return 0;
}

int ora_value_range64(const double* x, uint64_t n, double* mn, double* mx)
{
    if (!x || !mn || !mx || n == 0) return ORA_ERR_ARG;
    double lo = x[0], hi = x[0];
    for (uint64_t i = 0; i < n; ++i) {
        if (!isfinite(x[i])) return ORA_ERR_NONFINITE;
        if (less_total64(x[i], lo)) lo = x[i];
        if (less_total64(hi, x[i])) hi = x[i];
    }
    *mn = lo;
    *mx = hi;
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* C2: quantisation step with an fp32 guard.                                 */
/* eps = 2^e, e = max(ilogb(M) - ilogb(eb_abs) - 21, -22) (e = -22 if M = 0) */
/* ebx2 = (eb_abs * (1 - eps)) * 2, inv = 1 / ebx2.                          */
/* ------------------------------------------------------------------------ */
int ora_quant_step(double M, double eb_abs, double* ebx2, double* inv, int* e_out)
{
    if (!(eb_abs > 0.0) || !isfinite(eb_abs)) return ORA_ERR_EB_TOO_SMALL;
    if (eb_abs > 0x1p1000) return ORA_ERR_EB;
    int e = -22;
    if (M != 0.0) {
        int k = ilogb(M) - ilogb(eb_abs) - 21;
        if (k > e) e = k;
    }
    if (e > -4) return ORA_ERR_EB_TOO_SMALL;
    double eps = ldexp(1.0, e);
    double step = (eb_abs * (1.0 - eps)) * 2.0;
    if (ebx2) *ebx2 = step;
    if (inv) *inv = 1.0 / step;
    if (e_out) *e_out = e;
    return ORA_OK;
}

/* C2 for fp64 fields.  The output rounding is now 2^-53 relative, so the
   guard needs eps >= 2^-50 (M/eb + 1): eps = 2^max(k - 48, -49) with
   k = ilogb(M) - ilogb(eb_abs).  The codes must also stay far inside int32
   (the 3D Lorenzo difference adds eight of them): k > 27 is rejected as a
   bound too small for this code width. */
int ora_quant_step64(double M, double eb_abs, double* ebx2, double* inv, int* e_out)
{
    if (!(eb_abs > 0.0) || !isfinite(eb_abs)) return ORA_ERR_EB_TOO_SMALL;
    if (eb_abs > 0x1p1000) return ORA_ERR_EB;
    int e = -49;
    if (M != 0.0) {
        int k = ilogb(M) - ilogb(eb_abs);
        if (k > 27) return ORA_ERR_EB_TOO_SMALL;
        if (k - 48 > e) e = k - 48;
    }
    double eps = ldexp(1.0, e);
    double step = (eb_abs * (1.0 - eps)) * 2.0;
    if (ebx2) *ebx2 = step;
    if (inv) *inv = 1.0 / step;
    if (e_out) *e_out = e;
    return ORA_OK;
}

/* C3: prequantisation d = round(x / (2 eb)) as rint(x * inv) (Sec. IV-A.1). */
void ora_prequant(const float* x, uint64_t n, double inv, int32_t* d)
{
    for (uint64_t i = 0; i < n; ++i) d[i] = (int32_t)rint((double)x[i] * inv);
}

void ora_prequant64(const double* x, uint64_t n, double inv, int32_t* d)
{
    for (uint64_t i = 0; i < n; ++i) d[i] = (int32_t)rint(x[i] * inv);
}

/* ------------------------------------------------------------------------ */
/* C4: first-order Lorenzo prediction within chunks (Sec. IV-B.2 formulas).  */
/* A neighbour that lies outside the chunk of (z,y,x) reads as zero.         */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t nx, ny, nz;
    uint32_t cx, cy, cz;
} grid_t;

static int64_t at(const int32_t* d, const grid_t* g, uint64_t z, uint64_t y, uint64_t x,
                  int dz, int dy, int dx)
{
    /* same-chunk test: stepping back by one crosses a chunk edge exactly when
       the coordinate is a multiple of the chunk extent */
    if (dz && z % g->cz == 0) return 0;
    if (dy && y % g->cy == 0) return 0;
    if (dx && x % g->cx == 0) return 0;
    uint64_t zz = z - (uint64_t)dz, yy = y - (uint64_t)dy, xx = x - (uint64_t)dx;
    return d[(zz * g->ny + yy) * g->nx + xx];
}

/* prediction p from already known values, rank-specific formula */
static int64_t lorenzo_pred(const int32_t* d, const grid_t* g, int rank, uint64_t z, uint64_t y,
                            uint64_t x)
{
    if (rank == 1) return at(d, g, z, y, x, 0, 0, 1);
    if (rank == 2)
        return -at(d, g, z, y, x, 0, 1, 1) + at(d, g, z, y, x, 0, 1, 0) + at(d, g, z, y, x, 0, 0, 1);
    return +at(d, g, z, y, x, 1, 1, 1) - at(d, g, z, y, x, 1, 1, 0) - at(d, g, z, y, x, 0, 1, 1) +
           at(d, g, z, y, x, 0, 1, 0) - at(d, g, z, y, x, 1, 0, 1) + at(d, g, z, y, x, 1, 0, 0) +
           at(d, g, z, y, x, 0, 0, 1);
}

static void make_grid(grid_t* g, const uint64_t dims[3], const uint32_t chunk[3])
{
    g->nx = dims[0];
    g->ny = dims[1];
    g->nz = dims[2];
    g->cx = chunk[0];
    g->cy = chunk[1];
    g->cz = chunk[2];
}

/* delta = d - p for every element (postquant input, Sec. IV-A.1) */
void ora_lorenzo(const int32_t* d, int rank, const uint64_t dims[3], const uint32_t chunk[3],
                 int32_t* delta)
{
    grid_t g;
    make_grid(&g, dims, chunk);
    for (uint64_t z = 0; z < g.nz; ++z)
        for (uint64_t y = 0; y < g.ny; ++y)
            for (uint64_t x = 0; x < g.nx; ++x) {
                uint64_t i = (z * g.ny + y) * g.nx + x;
                delta[i] = (int32_t)((int64_t)d[i] - lorenzo_pred(d, &g, rank, z, y, x));
            }
}

/* ------------------------------------------------------------------------ */
/* C5: modified quantisation (Sec. IV-B.1, Algorithm 1 compression half).    */
/* |delta| < r -> q = delta + r; else q = 0 and (i, delta) is an outlier.    */
/* Returns the outlier count; oidx/oval may be NULL to count only.           */
/* ------------------------------------------------------------------------ */
uint64_t ora_postquant(const int32_t* delta, uint64_t n, uint32_t n_bins, uint16_t* q,
                       uint32_t* oidx, int32_t* oval)
{
    int64_t r = (int64_t)(n_bins / 2);
    uint64_t k = 0;
    for (uint64_t i = 0; i < n; ++i) {
        int64_t v = delta[i];
        if (v > -r && v < r) {
            q[i] = (uint16_t)(v + r);
        } else {
            q[i] = 0;
            if (oidx) oidx[k] = (uint32_t)i;
            if (oval) oval[k] = (int32_t)v;
            ++k;
        }
    }
    return k;
}

/* C6: histogram of quant-codes (Sec. II-A step 5). */
void ora_histogram(const uint16_t* q, uint64_t n, uint32_t n_bins, uint64_t* hist)
{
    memset(hist, 0, sizeof(uint64_t) * n_bins);
    for (uint64_t i = 0; i < n; ++i) hist[q[i]] += 1;
}

/* ------------------------------------------------------------------------ */
/* C7: Huffman code lengths, two-queue construction (leaves sorted by        */
/* (frequency, symbol); internal nodes in a FIFO; the leaf wins ties).       */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t w;
    uint32_t sym;
} leaf_t;

static int cmp_leaf(const void* a, const void* b)
{
    const leaf_t* p = (const leaf_t*)a;
    const leaf_t* q = (const leaf_t*)b;
    if (p->w != q->w) return p->w < q->w ? -1 : 1;
    if (p->sym != q->sym) return p->sym < q->sym ? -1 : 1;
    return 0;
}

int ora_huffman_lengths(const uint64_t* hist, uint32_t n_bins, uint8_t* len)
{
    memset(len, 0, n_bins);
    uint32_t m = 0;
    for (uint32_t s = 0; s < n_bins; ++s)
        if (hist[s]) ++m;
    if (m == 0) return ORA_ERR_ARG;
    if (m == 1) {
        for (uint32_t s = 0; s < n_bins; ++s)
            if (hist[s]) len[s] = 1;
        return ORA_OK;
    }
    leaf_t* leaf = (leaf_t*)malloc(sizeof(leaf_t) * m);
    uint64_t* iw = (uint64_t*)malloc(sizeof(uint64_t) * (m - 1));
    uint32_t* parent = (uint32_t*)malloc(sizeof(uint32_t) * (2 * m - 1));
    uint32_t* depth = (uint32_t*)malloc(sizeof(uint32_t) * (2 * m - 1));
    if (!leaf || !iw || !parent || !depth) {
        free(leaf), free(iw), free(parent), free(depth);
        return ORA_ERR_NOMEM;
    }
    uint32_t j = 0;
    for (uint32_t s = 0; s < n_bins; ++s)
        if (hist[s]) leaf[j].w = hist[s], leaf[j].sym = s, ++j;
    qsort(leaf, m, sizeof(leaf_t), cmp_leaf);

    /* node ids: leaves 0..m-1 (sorted order), internal node k is m + k */
    uint32_t li = 0, ih = 0, ni = 0;
    for (uint32_t k = 0; k + 1 < m; ++k) {
        uint32_t pick[2];
        uint64_t w = 0;
        for (int t = 0; t < 2; ++t) {
            if (li < m && (ih == ni || leaf[li].w <= iw[ih])) {
                pick[t] = li;
                w += leaf[li].w;
                ++li;
            } else {
                pick[t] = m + ih;
                w += iw[ih];
                ++ih;
            }
        }
        iw[ni] = w;
        parent[pick[0]] = m + ni;
        parent[pick[1]] = m + ni;
        ++ni;
    }
    /* the root is the last internal node; a parent always has a larger id */
    uint32_t root = 2 * m - 2;
    depth[root] = 0;
    int status = ORA_OK;
    for (int64_t v = (int64_t)root - 1; v >= 0; --v) depth[v] = depth[parent[v]] + 1;
    for (uint32_t i = 0; i < m; ++i) {
        if (depth[i] > 64) status = ORA_ERR_UNSUPPORTED;
        len[leaf[i].sym] = (uint8_t)depth[i];
    }
    free(leaf), free(iw), free(parent), free(depth);
    return status;
}

/* ------------------------------------------------------------------------ */
/* C8: canonical codes.  Symbols with len > 0 sorted by (len, symbol); the   */
/* first code is 0 and code_{k+1} = (code_k + 1) << (len_{k+1} - len_k).     */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t len, sym;
} ls_t;

static int cmp_ls(const void* a, const void* b)
{
    const ls_t* p = (const ls_t*)a;
    const ls_t* q = (const ls_t*)b;
    if (p->len != q->len) return p->len < q->len ? -1 : 1;
    if (p->sym != q->sym) return p->sym < q->sym ? -1 : 1;
    return 0;
}

int ora_canonical_codes(const uint8_t* len, uint32_t n_bins, uint64_t* code)
{
    memset(code, 0, sizeof(uint64_t) * n_bins);
    uint32_t m = 0;
    for (uint32_t s = 0; s < n_bins; ++s)
        if (len[s]) ++m;
    if (m == 0) return ORA_OK;
    ls_t* v = (ls_t*)malloc(sizeof(ls_t) * m);
    if (!v) return ORA_ERR_NOMEM;
    uint32_t j = 0;
    for (uint32_t s = 0; s < n_bins; ++s)
        if (len[s]) v[j].len = len[s], v[j].sym = s, ++j;
    qsort(v, m, sizeof(ls_t), cmp_ls);
    uint64_t c = 0;
    code[v[0].sym] = 0;
    for (uint32_t k = 1; k < m; ++k) {
        c = (c + 1) << (v[k].len - v[k - 1].len);
        code[v[k].sym] = c;
    }
    free(v);
    return ORA_OK;
}

/* C9: adaptive choice, RLE iff <b> <= 1.09 as an exact integer test. */
int ora_choose_rle(const uint64_t* hist, const uint8_t* len, uint32_t n_bins, uint64_t n)
{
    uint64_t bits = 0;
    for (uint32_t s = 0; s < n_bins; ++s) bits += hist[s] * (uint64_t)len[s];
    return 100u * bits <= 109u * n;
}

/* ------------------------------------------------------------------------ */
/* C10a: chunked Huffman encoding.  Chunks of hc symbols; each chunk starts  */
/* on a 32-bit word; code bits are written MSB-first; bit 31 of a chunk's    */
/* first word is its first bit; unused bits are zero.                        */
/*                                                                          */
/* Sub-chunk metadata (container choice, not from the paper): a chunk is cut */
/* into sub-chunks of hs = min(hc, 256) symbols that follow each other in    */
/* the chunk's bits without padding, and the bit count of every sub-chunk   */
/* is stored as a u16 (at most 256 codewords of at most 64 bits: below      */
/* 2^16).  The chunk's bit count is the sum of its sub-chunks', and every   */
/* sub-chunk start is known, so a decoder can start on each one at once.    */
/* Writes sbits for every sub-chunk and, when words != NULL, the words in   */
/* chunk order.  Returns the total word count.                              */
/* ------------------------------------------------------------------------ */
uint32_t ora_sub_chunk(uint32_t hc) { return hc < 256 ? hc : 256; }

uint64_t ora_huffman_encode(const uint16_t* q, uint64_t n, const uint8_t* len,
                            const uint64_t* code, uint32_t hc, uint16_t* sbits, uint32_t* words)
{
    uint32_t hs = ora_sub_chunk(hc);
    uint64_t nch = (n + hc - 1) / hc;
    uint64_t wbase = 0;
    for (uint64_t c = 0; c < nch; ++c) {
        uint64_t lo = c * hc, hi = lo + hc < n ? lo + hc : n;
        uint64_t nb = 0;
        for (uint64_t s0 = lo; s0 < hi; s0 += hs) {
            uint64_t s1 = s0 + hs < hi ? s0 + hs : hi, sb = 0;
            for (uint64_t i = s0; i < s1; ++i) sb += len[q[i]];
            sbits[s0 / hs] = (uint16_t)sb;
            nb += sb;
        }
        uint64_t nw = (nb + 31) / 32;
        if (words) {
            for (uint64_t w = 0; w < nw; ++w) words[wbase + w] = 0;
            uint64_t pos = 0;
            for (uint64_t i = lo; i < hi; ++i) {
                uint32_t l = len[q[i]];
                uint64_t cw = code[q[i]];
                for (uint32_t b = 0; b < l; ++b) {
                    uint32_t bit = (uint32_t)((cw >> (l - 1 - b)) & 1u);
                    if (bit) words[wbase + pos / 32] |= 1u << (31 - pos % 32);
                    ++pos;
                }
            }
        }
        wbase += nw;
    }
    return wbase;
}

/* Canonical decode tables derived from the lengths alone. */
typedef struct {
    uint64_t first[65];
    uint64_t count[65];
    uint32_t offset[65];
    uint32_t* sorted; /* symbols ordered by (len, symbol) */
} canon_t;

static int canon_build(canon_t* t, const uint8_t* len, uint32_t n_bins)
{
    memset(t->first, 0, sizeof(t->first));
    memset(t->count, 0, sizeof(t->count));
    memset(t->offset, 0, sizeof(t->offset));
    t->sorted = (uint32_t*)malloc(sizeof(uint32_t) * (n_bins ? n_bins : 1));
    if (!t->sorted) return ORA_ERR_NOMEM;
    for (uint32_t s = 0; s < n_bins; ++s) {
        if (len[s] > 64) return ORA_ERR_ARCHIVE;
        t->count[len[s]] += 1;
    }
    t->count[0] = 0;
    uint64_t c = 0;
    uint32_t off = 0;
    for (int l = 1; l <= 64; ++l) {
        t->first[l] = c;
        t->offset[l] = off;
        off += (uint32_t)t->count[l];
        c = (c + t->count[l]) << 1;
    }
    uint32_t fill[65];
    memcpy(fill, t->offset, sizeof(fill));
    for (uint32_t s = 0; s < n_bins; ++s)
        if (len[s]) t->sorted[fill[len[s]]++] = s;
    return ORA_OK;
}

/* D2 (Huffman): decode min(hc, remaining) symbols per chunk, bit by bit;  */
/* every sub-chunk must take exactly its stored bit count.                   */
int ora_huffman_decode(const uint16_t* sbits, const uint32_t* words, uint64_t n_words, uint64_t n,
                       uint32_t hc, const uint8_t* len, uint32_t n_bins, uint16_t* q)
{
    canon_t t;
    int st = canon_build(&t, len, n_bins);
    if (st) {
        free(t.sorted);
        return st;
    }
    uint32_t hs = ora_sub_chunk(hc);
    uint64_t nch = (n + hc - 1) / hc;
    uint64_t wbase = 0;
    for (uint64_t c = 0; c < nch && st == ORA_OK; ++c) {
        uint64_t lo = c * hc, hi = lo + hc < n ? lo + hc : n;
        uint64_t nb = 0;
        for (uint64_t s0 = lo; s0 < hi; s0 += hs) nb += sbits[s0 / hs];
        uint64_t nw = (nb + 31) / 32;
        if (wbase + nw > n_words) {
            st = ORA_ERR_ARCHIVE;
            break;
        }
        uint64_t pos = 0, sub_end = 0;
        for (uint64_t i = lo; i < hi; ++i) {
            if ((i - lo) % hs == 0) {
                /* a sub-chunk starts: the previous one must have ended exactly */
                if (pos != sub_end) {
                    st = ORA_ERR_ARCHIVE;
                    break;
                }
                sub_end += sbits[i / hs];
            }
            uint64_t v = 0;
            int l = 0, found = 0;
            while (l < 64) {
                if (pos >= sub_end) break;
                uint32_t bit = (words[wbase + pos / 32] >> (31 - pos % 32)) & 1u;
                ++pos;
                ++l;
                v = (v << 1) | bit;
                if (v >= t.first[l] && v - t.first[l] < t.count[l]) {
                    q[i] = (uint16_t)t.sorted[t.offset[l] + (uint32_t)(v - t.first[l])];
                    found = 1;
                    break;
                }
            }
            if (!found) {
                st = ORA_ERR_ARCHIVE;
                break;
            }
        }
        if (st == ORA_OK && pos != sub_end) st = ORA_ERR_ARCHIVE;
        wbase += nw;
    }
    free(t.sorted);
    return st;
}

/* C10b: run-length encoding, maximal runs in linear order (Sec. III-B). */
uint64_t ora_rle_encode(const uint16_t* q, uint64_t n, uint16_t* val, uint32_t* len)
{
    uint64_t r = 0;
    uint64_t i = 0;
    while (i < n) {
        uint64_t j = i + 1;
        while (j < n && q[j] == q[i]) ++j;
        if (val) val[r] = q[i];
        if (len) len[r] = (uint32_t)(j - i);
        ++r;
        i = j;
    }
    return r;
}

/* D2 (RLE): expand runs; the lengths must add up to n exactly. */
int ora_rle_decode(const uint16_t* val, const uint32_t* len, uint64_t r, uint64_t n, uint16_t* q)
{
    uint64_t pos = 0;
    for (uint64_t k = 0; k < r; ++k) {
        if (len[k] == 0 || pos + len[k] > n) return ORA_ERR_ARCHIVE;
        for (uint32_t j = 0; j < len[k]; ++j) q[pos + j] = val[k];
        pos += len[k];
    }
    return pos == n ? ORA_OK : ORA_ERR_ARCHIVE;
}

/* D3: fuse quant-codes and outliers, q' = q - r then q'[idx] = delta.
   Code 0 is the outlier placeholder (Sec. IV-B.1), so the archive is only
   consistent when the outlier list names every code-0 position exactly once:
   indices ascending, each pointing at a 0, and as many entries as zeros. */
int ora_fuse(const uint16_t* q, uint64_t n, uint32_t n_bins, const uint32_t* oidx,
             const int32_t* oval, uint64_t no, int32_t* qp)
{
    int32_t r = (int32_t)(n_bins / 2);
    uint64_t zeros = 0;
    for (uint64_t i = 0; i < n; ++i) {
        qp[i] = (int32_t)q[i] - r;
        zeros += q[i] == 0;
    }
    if (zeros != no) return ORA_ERR_ARCHIVE;
    for (uint64_t k = 0; k < no; ++k) {
        if (oidx[k] >= n) return ORA_ERR_ARCHIVE;
        if (k > 0 && oidx[k] <= oidx[k - 1]) return ORA_ERR_ARCHIVE;
        if (q[oidx[k]] != 0) return ORA_ERR_ARCHIVE;
        qp[oidx[k]] = oval[k];
    }
    return ORA_OK;
}

/* D4: Lorenzo reconstruction as the sequential recurrence d = p(d) + q' in  */
/* row-major order (the one-by-one scheme of Sec. II-B.2); the paper proves  */
/* that the N-D partial sum of Sec. IV-B.2 yields the same integers.         */
void ora_reconstruct(const int32_t* qp, int rank, const uint64_t dims[3], const uint32_t chunk[3],
                     int32_t* d)
{
    grid_t g;
    make_grid(&g, dims, chunk);
    for (uint64_t z = 0; z < g.nz; ++z)
        for (uint64_t y = 0; y < g.ny; ++y)
            for (uint64_t x = 0; x < g.nx; ++x) {
                uint64_t i = (z * g.ny + y) * g.nx + x;
                d[i] = (int32_t)(lorenzo_pred(d, &g, rank, z, y, x) + (int64_t)qp[i]);
            }
}

/* D5: dequantisation, output = d * (2 eb) rounded once to fp32 (Alg. 1). */
void ora_dequant(const int32_t* d, uint64_t n, double ebx2, float* out)
{
    for (uint64_t i = 0; i < n; ++i) out[i] = (float)((double)d[i] * ebx2);
}

/* D5 for fp64 fields: the product rounded once, in binary64. */
void ora_dequant64(const int32_t* d, uint64_t n, double ebx2, double* out)
{
    for (uint64_t i = 0; i < n; ++i) out[i] = (double)d[i] * ebx2;
}

/* ------------------------------------------------------------------------ */
/* Compressibility estimates (Sec. III-B).                                   */
/*                                                                          */
/* From the histogram (Sec. III-B.1): entropy H = -sum p_i log2 p_i, the    */
/* probability p1 of the most likely symbol, and bounds on the Huffman      */
/* redundancy R = <b> - H: R+ = p1 + 0.086 always, R- = 1 - H(p1, 1 - p1)   */
/* when p1 > 0.4 (else 0), so H + R- <= <b> <= H + R+ without a codebook.   */
/* The workflow they predict: run-length coding when even the upper bound   */
/* of <b> is at most 1.09 bits, Huffman when the lower bound exceeds it,    */
/* undecided otherwise.                                                     */
/* ------------------------------------------------------------------------ */
void ora_estimate_hist(const uint64_t* hist, uint32_t n_bins, uint64_t n, double* H, double* p1,
                       double* r_lo, double* r_hi, int* predict)
{
    uint64_t mx = 0;
    double h = 0.0;
    for (uint32_t s = 0; s < n_bins; ++s) {
        if (!hist[s]) continue;
        double p = (double)hist[s] / (double)n;
        h -= p * log2(p);
        if (hist[s] > mx) mx = hist[s];
    }
    double q = (double)mx / (double)n;
    double lo = 0.0;
    if (q > 0.4 && q < 1.0) lo = 1.0 - (-q * log2(q) - (1.0 - q) * log2(1.0 - q));
    else if (q >= 1.0) lo = 1.0; /* a single symbol: one bit per symbol, H = 0 */
    *H = h;
    *p1 = q;
    *r_lo = lo;
    *r_hi = q + 0.086;
    if (predict) *predict = h + *r_hi <= 1.09 ? 1 : (h + lo > 1.09 ? 0 : 2);
}

/* SplitMix64 as a counter-based generator (Steele, Lea, Flood 2014): the    */
/* k-th output for a seed is the output of a SplitMix64 state that has      */
/* advanced k+1 times from the seed, i.e. mix(seed + (k+1) * golden gamma). */
uint64_t ora_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Sampled binary madogram of the quant-codes (Sec. III-B.2): sample k draws */
/* one 64-bit number; its high half picks a in [0, n) and its low half a    */
/* distance d in [1, dmax] (both by multiply-shift); a pair whose second    */
/* element falls outside the field is skipped.  cnt[d] counts the pairs at  */
/* distance d and sum[d] those whose two codes differ (binary variance).    */
/* v(d) = sum[d] / cnt[d] is the roughness at d, 1 - v(d) the smoothness.   */
void ora_madogram(const uint16_t* q, uint64_t n, uint64_t samples, uint64_t seed, uint32_t dmax,
                  uint64_t* sum, uint64_t* cnt)
{
    for (uint32_t d = 0; d <= dmax; ++d) sum[d] = cnt[d] = 0;
    for (uint64_t k = 0; k < samples; ++k) {
        uint64_t r = ora_splitmix64(seed, k);
        uint64_t a = ((r >> 32) * n) >> 32;
        uint32_t d = 1 + (uint32_t)(((r & 0xFFFFFFFFull) * dmax) >> 32);
        if (a + d >= n) continue;
        cnt[d] += 1;
        sum[d] += q[a] != q[a + d];
    }
}

/* ------------------------------------------------------------------------ */
/* Archive format v2 (little-endian, 128-byte header, 16-byte aligned        */
/* sections, zero padding).                                                  */
/*   0 "EBC1", 4 version u16 = 2, 6 flags u16 = 0,                           */
/*   8 rank, codec, eb_mode, dtype (u8 each), 12 n_bins u32,                 */
/*  16 dims u64 x3, 40 Lorenzo chunk u32 x3, 52 hc u32,                      */
/*  56 eb, eb_abs, ebx2 (f64), 80 constant value f64,                        */
/*  88 n_outliers, 96 n_runs or n_chunks, 104 n_words (u64), 112 total u64,  */
/* 120 hs (Huffman sub-chunk symbols) u32, 124 zero u32.                     */
/* Sections: Huffman  u8 len[n_bins] | u16 sbits[n_sub] | u32 words        */
/*           RLE      u16 val[R] | u32 rlen[R]                               */
/*           RLE+VLE  u8 len[n_bins] | u16 sbits[n_sub(R)] | u32 words |     */
/*                    u32 rlen[R]   (Huffman over the R run values)          */
/*           all      u32 outlier_index[n_out] | i32 outlier_delta[n_out]    */
/* ------------------------------------------------------------------------ */
static uint64_t a16(uint64_t v) { return (v + 15u) & ~(uint64_t)15u; }

static void put_u16(uint8_t* p, uint16_t v) { memcpy(p, &v, 2); }
static void put_u32(uint8_t* p, uint32_t v) { memcpy(p, &v, 4); }
static void put_u64(uint8_t* p, uint64_t v) { memcpy(p, &v, 8); }
static void put_f64(uint8_t* p, double v) { memcpy(p, &v, 8); }
static uint16_t get_u16(const uint8_t* p) { uint16_t v; memcpy(&v, p, 2); return v; }
static uint32_t get_u32(const uint8_t* p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint64_t get_u64(const uint8_t* p) { uint64_t v; memcpy(&v, p, 8); return v; }
static double get_f64(const uint8_t* p) { double v; memcpy(&v, p, 8); return v; }

typedef struct {
    int rank, codec, eb_mode, dtype;
    uint32_t n_bins;
    uint64_t dims[3];
    uint32_t chunk[3];
    uint32_t hc, hs;
    double eb, eb_abs, ebx2;
    double cval;
    uint64_t n_out, n_a, n_words, total;
} hdr_t;

static void write_header(uint8_t* o, const hdr_t* h)
{
    memset(o, 0, HDR_BYTES);
    memcpy(o, "EBC1", 4);
    put_u16(o + 4, 2);
    put_u16(o + 6, 0);
    o[8] = (uint8_t)h->rank;
    o[9] = (uint8_t)h->codec;
    o[10] = (uint8_t)h->eb_mode;
    o[11] = (uint8_t)h->dtype;
    put_u32(o + 12, h->n_bins);
    for (int k = 0; k < 3; ++k) put_u64(o + 16 + 8 * k, h->dims[k]);
    for (int k = 0; k < 3; ++k) put_u32(o + 40 + 4 * k, h->chunk[k]);
    put_u32(o + 52, h->hc);
    put_f64(o + 56, h->eb);
    put_f64(o + 64, h->eb_abs);
    put_f64(o + 72, h->ebx2);
    put_f64(o + 80, h->cval);
    put_u64(o + 88, h->n_out);
    put_u64(o + 96, h->n_a);
    put_u64(o + 104, h->n_words);
    put_u64(o + 112, h->total);
    put_u32(o + 120, h->hs);
}

static int read_header(const uint8_t* a, uint64_t size, hdr_t* h)
{
    if (!a || size < HDR_BYTES) return ORA_ERR_ARCHIVE;
    if (memcmp(a, "EBC1", 4) != 0 || get_u16(a + 4) != 2) return ORA_ERR_ARCHIVE;
    h->rank = a[8];
    h->codec = a[9];
    h->eb_mode = a[10];
    h->dtype = a[11];
    h->n_bins = get_u32(a + 12);
    for (int k = 0; k < 3; ++k) h->dims[k] = get_u64(a + 16 + 8 * k);
    for (int k = 0; k < 3; ++k) h->chunk[k] = get_u32(a + 40 + 4 * k);
    h->hc = get_u32(a + 52);
    h->eb = get_f64(a + 56);
    h->eb_abs = get_f64(a + 64);
    h->ebx2 = get_f64(a + 72);
    h->cval = get_f64(a + 80);
    h->n_out = get_u64(a + 88);
    h->n_a = get_u64(a + 96);
    h->n_words = get_u64(a + 104);
    h->total = get_u64(a + 112);
    h->hs = get_u32(a + 120);
    if (h->rank < 1 || h->rank > 3 || h->codec > 3 || h->dtype > 1) return ORA_ERR_ARCHIVE;
    if (h->total > size) return ORA_ERR_ARCHIVE;
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* C0: argument validation.                                                  */
/* ------------------------------------------------------------------------ */
static int validate(int rank, const uint64_t dims[3], uint32_t n_bins, uint32_t hc, uint64_t* n)
{
    if (!dims) return ORA_ERR_ARG;
    if (rank < 1 || rank > 3) return ORA_ERR_DIMS;
    for (int k = 0; k < 3; ++k) {
        if (dims[k] == 0) return ORA_ERR_DIMS;
        if (k >= rank && dims[k] != 1) return ORA_ERR_DIMS;
        if (dims[k] >= (1ull << 32)) return ORA_ERR_DIMS;
    }
    uint64_t p = dims[0] * dims[1];
    if (p >= (1ull << 32)) return ORA_ERR_DIMS;
    p *= dims[2];
    if (p >= (1ull << 32)) return ORA_ERR_DIMS;
    if (n_bins < 4 || n_bins > 65536 || (n_bins & 1)) return ORA_ERR_BINS;
    if (hc < 64 || hc > 65536 || (hc & (hc - 1))) return ORA_ERR_ARG;
    *n = p;
    return ORA_OK;
}

static void default_chunk(int rank, uint32_t chunk[3])
{
    if (rank == 1) chunk[0] = 256, chunk[1] = 1, chunk[2] = 1;
    else if (rank == 2) chunk[0] = 16, chunk[1] = 16, chunk[2] = 1;
    else chunk[0] = 8, chunk[1] = 8, chunk[2] = 8;
}

static uint32_t ceil_log2(uint32_t v)
{
    uint32_t b = 0;
    while ((1ull << b) < v) ++b;
    return b;
}

/* Bytes of a Huffman-coded stream of m symbols (length table, sub-chunk bit
   counts, words) at most: no more bits than a fixed-length code of
   ceil(log2 n_bins) bits, plus one partial word per chunk. */
static uint64_t huff_stream_bound(uint64_t m, uint32_t n_bins, uint32_t hc)
{
    uint64_t nch = (m + hc - 1) / hc, nsub = (m + ora_sub_chunk(hc) - 1) / ora_sub_chunk(hc);
    return a16(n_bins) + a16(2 * nsub) + a16(4 * ((m * ceil_log2(n_bins) + 31) / 32 + nch));
}

/* Worst case over all codecs: a Huffman stream of N symbols; RLE <= N runs
   of 6 bytes; RLE+VLE <= a Huffman stream of N run values plus N lengths;
   outliers <= N entries of 8 bytes. */
uint64_t ora_compress_bound(int rank, const uint64_t dims[3], uint32_t n_bins, uint32_t hc)
{
    uint64_t n;
    if (validate(rank, dims, n_bins, hc, &n)) return 0;
    uint64_t huff = huff_stream_bound(n, n_bins, hc);
    uint64_t rle = a16(2 * n) + a16(4 * n);
    uint64_t rv = huff + a16(4 * n);
    uint64_t m = huff > rle ? huff : rle;
    if (rv > m) m = rv;
    return HDR_BYTES + m + a16(4 * n) + a16(4 * n);
}

/* Huffman coding of a symbol stream s[m] over n_bins symbols into
   o = len | sbits | words (section offsets from `base`); returns the words.
   Used for the codes themselves (Huffman codec) and for the run values
   (RLE+VLE codec); each stream has a codebook of its own. */
typedef struct {
    uint64_t off_len, off_sbits, off_words, end, n_words;
} hsec_t;

static int huff_stream(const uint16_t* s, uint64_t m, uint32_t n_bins, uint32_t hc, uint64_t base,
                       uint8_t* o, uint64_t cap, hsec_t* sec)
{
    uint64_t* hist = (uint64_t*)malloc(sizeof(uint64_t) * n_bins);
    uint8_t* len = (uint8_t*)malloc(n_bins);
    uint64_t* code = (uint64_t*)malloc(sizeof(uint64_t) * n_bins);
    uint32_t hs = ora_sub_chunk(hc);
    uint64_t nsub = (m + hs - 1) / hs;
    uint16_t* sb = (uint16_t*)malloc(2 * (nsub ? nsub : 1));
    uint32_t* words = NULL;
    int st = ORA_OK;
    if (!hist || !len || !code || !sb) {
        st = ORA_ERR_NOMEM;
        goto out;
    }
    ora_histogram(s, m, n_bins, hist);
    st = ora_huffman_lengths(hist, n_bins, len);
    if (st) goto out;
    ora_canonical_codes(len, n_bins, code);
    sec->n_words = ora_huffman_encode(s, m, len, code, hc, sb, NULL);
    sec->off_len = base;
    sec->off_sbits = a16(base + n_bins);
    sec->off_words = a16(sec->off_sbits + 2 * nsub);
    sec->end = a16(sec->off_words + 4 * sec->n_words);
    if (!o) goto out;
    if (sec->end > cap) {
        st = ORA_ERR_OUT_TOO_SMALL;
        goto out;
    }
    words = (uint32_t*)malloc(4 * (sec->n_words ? sec->n_words : 1));
    if (!words) {
        st = ORA_ERR_NOMEM;
        goto out;
    }
    ora_huffman_encode(s, m, len, code, hc, sb, words);
    memcpy(o + sec->off_len, len, n_bins);
    memcpy(o + sec->off_sbits, sb, 2 * nsub);
    memcpy(o + sec->off_words, words, 4 * sec->n_words);
out:
    free(hist), free(len), free(code), free(sb), free(words);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Whole compression pipeline (C0..C11).  x points at N fp32 (dtype 0) or   */
/* fp64 (dtype 1) values.  chunk == NULL selects the default Lorenzo chunk. */
/* ------------------------------------------------------------------------ */
int ora_compress(const void* x, int dtype, int rank, const uint64_t dims[3], int eb_mode,
                 double eb, uint32_t n_bins, int codec_req, uint32_t hc, const uint32_t* chunk_in,
                 uint8_t* out, uint64_t cap, uint64_t* size)
{
    uint64_t n;
    if (!x || !out || !size) return ORA_ERR_ARG;
    if (dtype != DT_F32 && dtype != DT_F64) return ORA_ERR_ARG;
    int st = validate(rank, dims, n_bins, hc, &n);
    if (st) return st;
    if (!(eb > 0.0) || !isfinite(eb)) return ORA_ERR_EB;
    if (eb_mode != EB_ABS && eb_mode != EB_REL) return ORA_ERR_ARG;
    if (codec_req < REQ_AUTO || codec_req > REQ_AUTO_VLE) return ORA_ERR_ARG;
    uint32_t chunk[3];
    if (chunk_in) memcpy(chunk, chunk_in, sizeof(chunk));
    else default_chunk(rank, chunk);
    for (int k = 0; k < 3; ++k)
        if (chunk[k] == 0 || (k >= rank && chunk[k] != 1)) return ORA_ERR_ARG;

    hdr_t h;
    memset(&h, 0, sizeof(h));
    h.rank = rank;
    h.eb_mode = eb_mode;
    h.dtype = dtype;
    h.n_bins = n_bins;
    memcpy(h.dims, dims, sizeof(h.dims));
    memcpy(h.chunk, chunk, sizeof(h.chunk));
    h.hc = hc;
    h.eb = eb;

    double mn, mx;
    if (dtype == DT_F32) {
        float a, b;
        st = ora_value_range((const float*)x, n, &a, &b);
        mn = a, mx = b;
    } else {
        st = ora_value_range64((const double*)x, n, &mn, &mx);
    }
    if (st) return st;
    double range = mx - mn; /* exact for fp32 ends; rounded once for fp64 ends */
    double M = fabs(mn) > fabs(mx) ? fabs(mn) : fabs(mx);

    if (eb_mode == EB_REL && range == 0.0) {
        h.codec = ARC_CONST;
        h.cval = mn;
        h.total = HDR_BYTES;
        if (cap < HDR_BYTES) return ORA_ERR_OUT_TOO_SMALL;
        write_header(out, &h);
        *size = HDR_BYTES;
        return ORA_OK;
    }
    h.eb_abs = eb_mode == EB_REL ? eb * range : eb;
    double inv;
    st = dtype == DT_F32 ? ora_quant_step(M, h.eb_abs, &h.ebx2, &inv, NULL)
                         : ora_quant_step64(M, h.eb_abs, &h.ebx2, &inv, NULL);
    if (st) return st;

    int32_t* d = (int32_t*)malloc(sizeof(int32_t) * n);
    int32_t* delta = (int32_t*)malloc(sizeof(int32_t) * n);
    uint16_t* q = (uint16_t*)malloc(sizeof(uint16_t) * n);
    uint64_t* hist = (uint64_t*)malloc(sizeof(uint64_t) * n_bins);
    uint8_t* len = (uint8_t*)malloc(n_bins);
    uint32_t* oidx = NULL;
    int32_t* oval = NULL;
    uint16_t* val = NULL;
    uint32_t* rl = NULL;
    if (!d || !delta || !q || !hist || !len) {
        st = ORA_ERR_NOMEM;
        goto done;
    }
    if (dtype == DT_F32) ora_prequant((const float*)x, n, inv, d);
    else ora_prequant64((const double*)x, n, inv, d);
    ora_lorenzo(d, rank, dims, chunk, delta);
    h.n_out = ora_postquant(delta, n, n_bins, q, NULL, NULL);
    oidx = (uint32_t*)malloc(sizeof(uint32_t) * (h.n_out ? h.n_out : 1));
    oval = (int32_t*)malloc(sizeof(int32_t) * (h.n_out ? h.n_out : 1));
    if (!oidx || !oval) {
        st = ORA_ERR_NOMEM;
        goto done;
    }
    ora_postquant(delta, n, n_bins, q, oidx, oval);
    ora_histogram(q, n, n_bins, hist);
    st = ora_huffman_lengths(hist, n_bins, len);
    if (st) goto done;
    {
        int rle = ora_choose_rle(hist, len, n_bins, n);
        switch (codec_req) {
        case REQ_AUTO: h.codec = rle ? ARC_RLE : ARC_HUFFMAN; break;
        case REQ_AUTO_VLE: h.codec = rle ? ARC_RLE_VLE : ARC_HUFFMAN; break;
        case REQ_HUFFMAN: h.codec = ARC_HUFFMAN; break;
        case REQ_RLE: h.codec = ARC_RLE; break;
        default: h.codec = ARC_RLE_VLE; break;
        }
    }
    uint64_t off_o;
    if (h.codec == ARC_HUFFMAN) {
        hsec_t sec;
        h.n_a = (n + hc - 1) / hc;
        h.hs = ora_sub_chunk(hc);
        st = huff_stream(q, n, n_bins, hc, HDR_BYTES, NULL, 0, &sec);
        if (st) goto done;
        h.n_words = sec.n_words;
        off_o = sec.end;
        h.total = a16(a16(off_o + 4 * h.n_out) + 4 * h.n_out);
        if (h.total > cap) {
            st = ORA_ERR_OUT_TOO_SMALL;
            goto done;
        }
        memset(out, 0, h.total);
        st = huff_stream(q, n, n_bins, hc, HDR_BYTES, out, cap, &sec);
        if (st) goto done;
    } else {
        h.n_a = ora_rle_encode(q, n, NULL, NULL);
        val = (uint16_t*)malloc(2 * h.n_a);
        rl = (uint32_t*)malloc(4 * h.n_a);
        if (!val || !rl) {
            st = ORA_ERR_NOMEM;
            goto done;
        }
        ora_rle_encode(q, n, val, rl);
        if (h.codec == ARC_RLE) {
            uint64_t off_len = a16(HDR_BYTES + 2 * h.n_a);
            off_o = a16(off_len + 4 * h.n_a);
            h.total = a16(a16(off_o + 4 * h.n_out) + 4 * h.n_out);
            if (h.total > cap) {
                st = ORA_ERR_OUT_TOO_SMALL;
                goto done;
            }
            memset(out, 0, h.total);
            memcpy(out + HDR_BYTES, val, 2 * h.n_a);
            memcpy(out + off_len, rl, 4 * h.n_a);
        } else {
            /* RLE+VLE: the run values as a Huffman stream of their own */
            hsec_t sec;
            h.hs = ora_sub_chunk(hc);
            st = huff_stream(val, h.n_a, n_bins, hc, HDR_BYTES, NULL, 0, &sec);
            if (st) goto done;
            h.n_words = sec.n_words;
            uint64_t off_len = sec.end;
            off_o = a16(off_len + 4 * h.n_a);
            h.total = a16(a16(off_o + 4 * h.n_out) + 4 * h.n_out);
            if (h.total > cap) {
                st = ORA_ERR_OUT_TOO_SMALL;
                goto done;
            }
            memset(out, 0, h.total);
            st = huff_stream(val, h.n_a, n_bins, hc, HDR_BYTES, out, cap, &sec);
            if (st) goto done;
            memcpy(out + off_len, rl, 4 * h.n_a);
        }
    }
    memcpy(out + off_o, oidx, 4 * h.n_out);
    memcpy(out + a16(off_o + 4 * h.n_out), oval, 4 * h.n_out);
    write_header(out, &h);
    *size = h.total;
done:
    free(d), free(delta), free(q), free(hist), free(len), free(oidx), free(oval), free(val), free(rl);
    return st;
}

/* Header fields for the Python side (n_elems = product of dims). */
int ora_archive_info(const uint8_t* a, uint64_t size, int* rank, uint64_t dims[3], int* codec,
                     uint32_t* n_bins, uint64_t* n_out, uint64_t* n_a, uint64_t* n_words,
                     double* ebx2, int* dtype, uint32_t* hc)
{
    hdr_t h;
    int st = read_header(a, size, &h);
    if (st) return st;
    if (rank) *rank = h.rank;
    if (dims) memcpy(dims, h.dims, sizeof(h.dims));
    if (codec) *codec = h.codec;
    if (n_bins) *n_bins = h.n_bins;
    if (n_out) *n_out = h.n_out;
    if (n_a) *n_a = h.n_a;
    if (n_words) *n_words = h.n_words;
    if (ebx2) *ebx2 = h.ebx2;
    if (dtype) *dtype = h.dtype;
    if (hc) *hc = h.hc;
    return ORA_OK;
}

/* Section offsets of a Huffman stream of m symbols starting at base. */
static void huff_layout(uint64_t m, uint32_t n_bins, uint32_t hc, uint64_t n_words, uint64_t base,
                        hsec_t* sec)
{
    uint64_t nsub = (m + ora_sub_chunk(hc) - 1) / ora_sub_chunk(hc);
    sec->off_len = base;
    sec->off_sbits = a16(base + n_bins);
    sec->off_words = a16(sec->off_sbits + 2 * nsub);
    sec->end = a16(sec->off_words + 4 * n_words);
    sec->n_words = n_words;
}

/* ------------------------------------------------------------------------ */
/* Whole decompression pipeline (D1..D5).  out receives N fp32 or fp64       */
/* values according to the archive's dtype.                                 */
/* ------------------------------------------------------------------------ */
int ora_decompress(const uint8_t* a, uint64_t size, void* out, uint64_t n_out_elems)
{
    hdr_t h;
    int st = read_header(a, size, &h);
    if (st) return st;
    if (h.total > size) return ORA_ERR_ARCHIVE;
    uint64_t n;
    st = validate(h.rank, h.dims, h.n_bins, h.hc, &n);
    if (st) return ORA_ERR_ARCHIVE;
    if (n_out_elems < n || !out) return ORA_ERR_OUT_TOO_SMALL;
    if (h.codec == ARC_CONST) {
        for (uint64_t i = 0; i < n; ++i) {
            if (h.dtype == DT_F32) ((float*)out)[i] = (float)h.cval;
            else ((double*)out)[i] = h.cval;
        }
        return ORA_OK;
    }
    if (h.codec != ARC_RLE && h.hs != ora_sub_chunk(h.hc)) return ORA_ERR_ARCHIVE;
    uint16_t* q = (uint16_t*)malloc(2 * n);
    int32_t* qp = (int32_t*)malloc(4 * n);
    int32_t* d = (int32_t*)malloc(4 * n);
    uint16_t* val = NULL;
    if (!q || !qp || !d) {
        st = ORA_ERR_NOMEM;
        goto done;
    }
    uint64_t off_o;
    if (h.codec == ARC_HUFFMAN) {
        hsec_t sec;
        if (h.n_a != (n + h.hc - 1) / h.hc) {
            st = ORA_ERR_ARCHIVE;
            goto done;
        }
        huff_layout(n, h.n_bins, h.hc, h.n_words, HDR_BYTES, &sec);
        off_o = sec.end;
        if (a16(a16(off_o + 4 * h.n_out) + 4 * h.n_out) > size) {
            st = ORA_ERR_ARCHIVE;
            goto done;
        }
        st = ora_huffman_decode((const uint16_t*)(a + sec.off_sbits), (const uint32_t*)(a + sec.off_words),
                                h.n_words, n, h.hc, a + sec.off_len, h.n_bins, q);
    } else if (h.codec == ARC_RLE) {
        uint64_t off_len = a16(HDR_BYTES + 2 * h.n_a);
        off_o = a16(off_len + 4 * h.n_a);
        if (h.n_a > n || a16(a16(off_o + 4 * h.n_out) + 4 * h.n_out) > size) {
            st = ORA_ERR_ARCHIVE;
            goto done;
        }
        st = ora_rle_decode((const uint16_t*)(a + HDR_BYTES), (const uint32_t*)(a + off_len), h.n_a,
                            n, q);
    } else {
        /* RLE+VLE: decode the run values, then expand the runs */
        hsec_t sec;
        if (h.n_a == 0 || h.n_a > n) {
            st = ORA_ERR_ARCHIVE;
            goto done;
        }
        huff_layout(h.n_a, h.n_bins, h.hc, h.n_words, HDR_BYTES, &sec);
        uint64_t off_len = sec.end;
        off_o = a16(off_len + 4 * h.n_a);
        if (a16(a16(off_o + 4 * h.n_out) + 4 * h.n_out) > size) {
            st = ORA_ERR_ARCHIVE;
            goto done;
        }
        val = (uint16_t*)malloc(2 * h.n_a);
        if (!val) {
            st = ORA_ERR_NOMEM;
            goto done;
        }
        st = ora_huffman_decode((const uint16_t*)(a + sec.off_sbits), (const uint32_t*)(a + sec.off_words),
                                h.n_words, h.n_a, h.hc, a + sec.off_len, h.n_bins, val);
        if (!st) st = ora_rle_decode(val, (const uint32_t*)(a + off_len), h.n_a, n, q);
    }
    if (st) goto done;
    st = ora_fuse(q, n, h.n_bins, (const uint32_t*)(a + off_o),
                  (const int32_t*)(a + a16(off_o + 4 * h.n_out)), h.n_out, qp);
    if (st) goto done;
    ora_reconstruct(qp, h.rank, h.dims, h.chunk, d);
    if (h.dtype == DT_F32) ora_dequant(d, n, h.ebx2, (float*)out);
    else ora_dequant64(d, n, h.ebx2, (double*)out);
done:
    free(q), free(qp), free(d), free(val);
    return st;
}
