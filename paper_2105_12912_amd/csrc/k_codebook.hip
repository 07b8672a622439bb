// k_codebook.hip -- canonical Huffman codebook on the device, one workgroup
// per field, plus the adaptive RLE/Huffman decision and the decoder tables.
//
// Sec. II-A steps 6-7 build a canonical Huffman codebook from the histogram
// (the earlier single-thread build is named as a bottleneck in Sec. I); the
// paper does not fix the construction, so this path uses the deterministic
// two-queue method: leaves ordered by (frequency, symbol), internal nodes in
// a FIFO, the leaf wins ties.  Lengths come from parent pointers by pointer
// jumping; canonical codes are assigned in (length, symbol) order, first
// code 0, code_{k+1} = (code_k + 1) << (len_{k+1} - len_k).
//
// Decision (Sec. I contribution list, Sec. III-B.2): run-length encoding when
// the Huffman average bit length is <= 1.09, i.e. 100 * sum(f*len) <= 109 * N
// in exact integers.
#include "ebc_dev.h"
#include "ebc_launch.h"

namespace ebc {

__host__ __device__ inline uint32_t pow2ceil(uint32_t v)
{
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

size_t codebook_lds_bytes(uint32_t n_bins)
{
    const uint32_t P = max(pow2ceil(n_bins), 512u);
    return (size_t)16 * P;
}

// Rank of every symbol among the symbols of equal length with a smaller index,
// and per-length counts, using wave ballots.  Fills
//   rank_out[k] for the symbols s = 64 * (w + 4k) + lane handled by this wave,
//   cnt[b * 65 + L] = symbols of length L in block b, then prefix over blocks.
// len_s: LDS code lengths.  After return (block-synchronised):
//   cnt[b*65+L] = number of symbols of length L in blocks < b,
//   cntL[L]     = total symbols of length L.
__device__ void canonical_rank(const uint8_t* len_s, uint32_t nb, uint16_t* cnt, uint32_t* cntL,
                               uint32_t rank_out[16])
{
    const int l = lane_id();
    const int w = threadIdx.x / kWave;
    const uint32_t nblk = (nb + 63) / 64;
    for (uint32_t i = threadIdx.x; i < nblk * 65; i += kBlock) cnt[i] = 0;
    __syncthreads();
    int k = 0;
    for (uint32_t b = w; b < nblk; b += kWavesPerBlock, ++k) {
        const uint32_t s = b * 64 + l;
        const uint32_t L = s < nb ? len_s[s] : 0u;
        uint64_t todo = ballot(L != 0);
        uint32_t rk = 0;
        while (todo) {
            const int leader = __ffsll((long long)todo) - 1;
            const uint32_t LL = __shfl(L, leader);
            const uint64_t m = ballot(L == LL);
            if (L == LL) rk = __popcll(m & ((1ull << l) - 1));
            if (l == 0) cnt[b * 65 + LL] = (uint16_t)__popcll(m);
            todo &= ~m;
        }
        rank_out[k] = rk;
    }
    __syncthreads();
    if (threadIdx.x < 65) {
        const uint32_t L = threadIdx.x;
        uint32_t run = 0;
        for (uint32_t b = 0; b < nblk; ++b) {
            const uint32_t c = cnt[b * 65 + L];
            cnt[b * 65 + L] = (uint16_t)run;
            run += c;
        }
        cntL[L] = run;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_codebook(const FieldDesc* __restrict__ F)
{
    const FieldDesc& fd = F[blockIdx.x];
    EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || dy->codec == ARC_CONST) return;
    const uint32_t nb = fd.n_bins;
    const uint32_t P = pow2ceil(nb);
    const uint32_t Pa = max(P, 512u);
    extern __shared__ uint64_t lds64[];
    uint64_t* keys = lds64;                             // R0: 8 Pa bytes
    uint32_t* iw = (uint32_t*)(lds64 + Pa);             // R1: 4 Pa bytes
    uint16_t* parent = (uint16_t*)(iw + Pa);            // R2: 4 Pa bytes
    uint8_t* dep = (uint8_t*)iw;                        // R1 reuse: 2 Pa bytes
    uint8_t* len_s = dep + 2 * Pa;                      // R1 reuse: Pa bytes
    __shared__ uint32_t s_m;
    __shared__ uint32_t s_red[kWavesPerBlock];

    // leaves: key = (freq << 16) | symbol; absent symbols sort last
    uint32_t used = 0;
    for (uint32_t s = threadIdx.x; s < P; s += kBlock) {
        const uint32_t h = s < nb ? fd.hist[s] : 0u;
        keys[s] = h ? (((uint64_t)h << 16) | s) : ~0ull;
        used += h != 0;
    }
    used = wave_sum_u32(used);
    if (lane_id() == 0) s_red[threadIdx.x / kWave] = used;
    __syncthreads();
    if (threadIdx.x == 0) s_m = s_red[0] + s_red[1] + s_red[2] + s_red[3];
    // bitonic sort of P keys, ascending
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < P; i += kBlock) {
                const uint32_t p = i ^ j;
                if (p > i) {
                    const uint64_t a = keys[i], b = keys[p];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) keys[i] = b, keys[p] = a;
                }
            }
        }
    }
    __syncthreads();
    const uint32_t m = s_m;
    if (m == 0) {
        if (threadIdx.x == 0) dy->status = ST_ERR_ARCHIVE;
        return;
    }
    // Two-queue merge in parallel rounds.  Let t be the weight of the next
    // internal node (sum of the two smallest available items).  Every
    // available item of weight <= t is picked before that node and before
    // any later one (ties: leaf before internal node, older internal node
    // before newer), so all of them can be paired in merged order at once;
    // an odd one out waits for the next round.  This reproduces the sequential
    // two-queue picks exactly.
    __shared__ uint32_t s_li, s_ih, s_ni, s_t;
    if (threadIdx.x == 0) s_li = 0, s_ih = 0, s_ni = 0;
    __syncthreads();
    while (m > 1) {
        const uint32_t li = s_li, ih = s_ih, ni = s_ni;
        if (ni + 1 >= m) break;
        if (threadIdx.x == 0) {
            uint32_t a = li, b = ih, t = 0;
            for (int k = 0; k < 2; ++k) {
                const uint32_t lw = a < m ? (uint32_t)(keys[a] >> 16) : 0xFFFFFFFFu;
                if (a < m && (b == ni || lw <= iw[b])) t += lw, ++a;
                else t += iw[b], ++b;
            }
            s_t = t;
        }
        __syncthreads();
        const uint32_t t = s_t;
        // available leaves / internal nodes of weight <= t (both lists sorted)
        uint32_t cl = 0, ci = 0;
        for (uint32_t base = li;; base += kBlock) {
            const uint32_t i = base + threadIdx.x;
            const int c = __syncthreads_count(i < m && (uint32_t)(keys[i] >> 16) <= t);
            cl += c;
            if (c < kBlock) break;
        }
        for (uint32_t base = ih;; base += kBlock) {
            const uint32_t j = base + threadIdx.x;
            const int c = __syncthreads_count(j < ni && iw[j] <= t);
            ci += c;
            if (c < kBlock) break;
        }
        const uint32_t np = (cl + ci) / 2;
        for (uint32_t k = threadIdx.x; k < np; k += kBlock) iw[ni + k] = 0;
        __syncthreads();
        // merged position of every item, then parent and weight of its pair
        for (uint32_t i = threadIdx.x; i < cl; i += kBlock) {
            const uint32_t wi = (uint32_t)(keys[li + i] >> 16);
            uint32_t a = 0, b = ci;  // internal nodes lighter than the leaf
            while (a < b) {
                const uint32_t mid = (a + b) >> 1;
                if (iw[ih + mid] < wi) a = mid + 1;
                else b = mid;
            }
            const uint32_t pos = i + a;
            if (pos < 2 * np) {
                parent[li + i] = (uint16_t)(m + ni + pos / 2);
                atomicAdd(&iw[ni + pos / 2], wi);
            }
        }
        for (uint32_t j = threadIdx.x; j < ci; j += kBlock) {
            const uint32_t wj = iw[ih + j];
            uint32_t a = 0, b = cl;  // leaves not heavier than the node
            while (a < b) {
                const uint32_t mid = (a + b) >> 1;
                if ((uint32_t)(keys[li + mid] >> 16) <= wj) a = mid + 1;
                else b = mid;
            }
            const uint32_t pos = j + a;
            if (pos < 2 * np) {
                parent[m + ih + j] = (uint16_t)(m + ni + pos / 2);
                atomicAdd(&iw[ni + pos / 2], wj);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t dl = cl, di = ci;
            if ((cl + ci) & 1) {
                // the last item in merged order stays: an internal node comes
                // after a leaf of equal weight
                bool last_is_leaf;
                if (ci == 0) last_is_leaf = true;
                else if (cl == 0) last_is_leaf = false;
                else last_is_leaf = (uint32_t)(keys[li + cl - 1] >> 16) > iw[ih + ci - 1];
                if (last_is_leaf) --dl;
                else --di;
            }
            s_li = li + dl, s_ih = ih + di, s_ni = ni + np;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && m > 1) parent[2 * m - 2] = (uint16_t)(2 * m - 2);  // the root points to itself
    __syncthreads();
    // depths by pointer jumping over nodes 0 .. 2m-2 (depth <= 64 < 2^7)
    const uint32_t nn = m > 1 ? 2 * m - 1 : 1;
    const uint32_t root = nn - 1;
    for (uint32_t v = threadIdx.x; v < nn; v += kBlock) dep[v] = v == root ? 0 : 1;
    if (m == 1 && threadIdx.x == 0) dep[0] = 1;  // a lone symbol gets one bit
    __syncthreads();
    if (m > 1) {
        for (int round = 0; round < 7; ++round) {
            uint32_t nd[32], na[32];
            int c = 0;
            for (uint32_t v = threadIdx.x; v < nn; v += kBlock, ++c) {
                const uint32_t a = parent[v];
                nd[c] = dep[v] + (a == v ? 0u : dep[a]);
                na[c] = parent[a];
            }
            __syncthreads();
            c = 0;
            for (uint32_t v = threadIdx.x; v < nn; v += kBlock, ++c) {
                dep[v] = (uint8_t)min(nd[c], 255u);
                parent[v] = (uint16_t)na[c];
            }
            __syncthreads();
        }
    }
    // leaf lengths -> symbols
    for (uint32_t s = threadIdx.x; s < Pa; s += kBlock) len_s[s] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < m; i += kBlock) len_s[keys[i] & 0xFFFFu] = dep[i];
    __syncthreads();

    // canonical codes (R0 reused for the per-block counts)
    uint16_t* cnt = (uint16_t*)keys;
    uint32_t* cntL = (uint32_t*)(((uintptr_t)(cnt + ((nb + 63) / 64) * 65 + 2) + 7) & ~(uintptr_t)7);
    uint64_t* first = (uint64_t*)(((uintptr_t)(cntL + 65) + 7) & ~(uintptr_t)7);
    uint32_t rank[16];
    canonical_rank(len_s, nb, cnt, cntL, rank);
    if (threadIdx.x == 0) {
        uint64_t c = 0;
        uint32_t maxl = 0;
        for (int L = 1; L <= 64; ++L) {
            first[L] = c;
            c = (c + cntL[L]) << 1;
            if (cntL[L]) maxl = L;
        }
        dy->max_len = maxl;
        dy->n_used = m;
    }
    __syncthreads();
    const int l = lane_id();
    const int w = threadIdx.x / kWave;
    uint64_t bits = 0;
    int k = 0;
    for (uint32_t b = w; b < (nb + 63) / 64; b += kWavesPerBlock, ++k) {
        const uint32_t s = b * 64 + l;
        if (s < nb) {
            const uint32_t L = len_s[s];
            uint64_t packed = 0;
            if (L) {
                const uint64_t code = first[L] + cnt[b * 65 + L] + rank[k];
                packed = ((uint64_t)L << 56) | code;
                bits += (uint64_t)fd.hist[s] * L;
            }
            fd.code[s] = packed;
            fd.len[s] = (uint8_t)L;
        }
    }
    bits = wave_sum_u64(bits);
    __shared__ uint64_t s_bits[kWavesPerBlock];
    if (l == 0) s_bits[w] = bits;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint64_t tb = s_bits[0] + s_bits[1] + s_bits[2] + s_bits[3];
        dy->huff_bits = tb;
        int codec;
        if (fd.codec_req == REQ_AUTO) codec = 100ull * tb <= 109ull * fd.n ? ARC_RLE : ARC_HUFFMAN;
        else codec = fd.codec_req == REQ_RLE ? ARC_RLE : ARC_HUFFMAN;
        dy->codec = codec;
        dy->n_out = fd.hist[0];
    }
}

// ------------------------------------------------------- decoder tables
// From the code lengths stored in an archive: per-length counts, first codes
// and offsets, the symbol permutation in (length, symbol) order and a
// kLutBits-wide lookup table.



__global__ __launch_bounds__(kBlock) void k_dectab(const FieldDesc* __restrict__ F,
                                                   uint8_t* __restrict__ tabs)
{
    const FieldDesc& fd = F[blockIdx.x];
    EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || dy->codec != ARC_HUFFMAN) return;
    DecTab* T = (DecTab*)(tabs + (size_t)blockIdx.x * dectab_bytes());
    const uint32_t nb = fd.n_bins;
    __shared__ uint8_t len_s[kMaxBins];
    __shared__ uint16_t cnt[(kMaxBins / 64) * 65 + 2];
    __shared__ uint32_t cntL[65];
    __shared__ uint64_t first[65];
    __shared__ uint32_t offs[65];
    __shared__ int s_bad;
    __shared__ uint32_t s_maxl;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const uint8_t* alen = fd.arc + kHdr;
    for (uint32_t s = threadIdx.x; s < nb; s += kBlock) {
        const uint8_t L = alen[s];
        if (L > kMaxDecodeLen) s_bad = 1;
        len_s[s] = L;
    }
    __syncthreads();
    if (s_bad) {
        if (threadIdx.x == 0) dy->status = ST_ERR_ARCHIVE;
        return;
    }
    uint32_t rank[16];
    canonical_rank(len_s, nb, cnt, cntL, rank);
    if (threadIdx.x == 0) {
        // canonical first codes; the lengths must satisfy Kraft's inequality
        // (first[L] + count[L] <= 2^L at every length), otherwise the archive
        // is corrupt and no table lookup below may be trusted
        uint64_t c = 0;
        uint32_t off = 0, maxl = 0;
        int bad = 0;
        for (int L = 1; L <= 64; ++L) {
            first[L] = c;
            offs[L] = off;
            off += cntL[L];
            if (L <= kMaxDecodeLen && c + cntL[L] > (1ull << L)) bad = 1;
            c = L <= kMaxDecodeLen ? (c + cntL[L]) << 1 : 0;
            if (cntL[L]) maxl = L;
            T->first[L] = first[L];
            T->count[L] = cntL[L];
            T->offset[L] = offs[L];
        }
        T->first[0] = 0, T->count[0] = 0, T->offset[0] = 0;
        T->max_len = maxl;
        s_maxl = maxl;
        if (maxl == 0 || bad) dy->status = ST_ERR_ARCHIVE;
        s_bad = bad | (maxl == 0);
    }
    __syncthreads();
    if (s_bad) return;
    __shared__ uint16_t perm_s[kMaxBins];
    const int l = lane_id();
    const int w = threadIdx.x / kWave;
    int k = 0;
    for (uint32_t b = w; b < (nb + 63) / 64; b += kWavesPerBlock, ++k) {
        const uint32_t s = b * 64 + l;
        if (s < nb) {
            const uint32_t L = len_s[s];
            if (L) perm_s[offs[L] + cnt[b * 65 + L] + rank[k]] = (uint16_t)s;
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nb; i += kBlock) T->perm[i] = perm_s[i];
    // left-aligned ends of the code space of lengths <= L (monotone in L)
    __syncthreads();
    if (threadIdx.x <= 64) {
        const uint32_t L = threadIdx.x;
        const uint32_t maxl = s_maxl;
        uint64_t endv = ~0ull;
        if (L >= 1 && L < maxl) endv = (first[L] + cntL[L]) << (64 - L);
        T->endv[L] = endv;
    }
    // Multi-symbol lookup table in two steps.  t1[p]: the codeword (length
    // <= kLutBits) that a kLutBits-bit window p starts with, by the canonical
    // limit test, as (L << 16) | symbol, or 0.  Then each entry chains up to
    // three t1 lookups; a window with only r valid leading bits (the rest
    // zero) still decodes a codeword of length <= r correctly, because such a
    // codeword depends on its own bits only.
    __shared__ uint32_t t1[1u << kLutBits];
    for (uint32_t p = threadIdx.x; p < (1u << kLutBits); p += kBlock) {
        uint32_t e = 0;
        for (uint32_t l = 1; l <= (uint32_t)kLutBits; ++l) {
            const uint64_t v = p >> (kLutBits - l);
            if (cntL[l] && v < first[l] + cntL[l]) {
                e = (l << 16) | perm_s[offs[l] + (uint32_t)(v - first[l])];
                break;
            }
        }
        t1[p] = e;
    }
    __syncthreads();
    // Second level: number the prefixes that start a longer codeword, give
    // each a block of 2^k entries resolving the next k bits.
    __shared__ uint16_t lslot[1u << kLutBits];
    __shared__ uint16_t lpref[1u << kLutBits];
    __shared__ uint32_t s_wsum[kWavesPerBlock];
    constexpr uint32_t kPer = (1u << kLutBits) / kBlock;
    {
        uint32_t c = 0;
        for (uint32_t i = 0; i < kPer; ++i) c += t1[threadIdx.x * kPer + i] == 0;
        const uint32_t inc = wave_incl_scan_u32(c);
        if (lane_id() == kWave - 1) s_wsum[threadIdx.x / kWave] = inc;
        __syncthreads();
        uint32_t base = inc - c;
        for (uint32_t v = 0; v < threadIdx.x / kWave; ++v) base += s_wsum[v];
        for (uint32_t i = 0; i < kPer; ++i) {
            const uint32_t p = threadIdx.x * kPer + i;
            if (t1[p] == 0) {
                lslot[p] = (uint16_t)base;
                lpref[base] = (uint16_t)p;
                ++base;
            } else {
                lslot[p] = 0xFFFF;
            }
        }
    }
    __syncthreads();
    const uint32_t nlong = s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3];
    const uint32_t maxl = s_maxl;
    uint32_t l2k = 0;
    if (maxl > (uint32_t)kLutBits && nlong > 0) {
        l2k = min(kL2MaxBits, maxl - (uint32_t)kLutBits);
        while (l2k > 0 && (nlong << l2k) > kL2Size) --l2k;
    }
    const uint32_t l2n = l2k ? nlong << l2k : 0u;
    for (uint32_t i = threadIdx.x; i < l2n; i += kBlock) {
        const uint32_t p = lpref[i >> l2k];
        const uint64_t wv = ((uint64_t)p << l2k) | (i & ((1u << l2k) - 1));  // kLutBits + l2k bits
        uint32_t e = 0;
        for (uint32_t l = kLutBits + 1; l <= kLutBits + l2k; ++l) {
            const uint64_t v = wv >> (kLutBits + l2k - l);
            if (cntL[l] && v < first[l] + cntL[l]) {
                e = (l << 16) | perm_s[offs[l] + (uint32_t)(v - first[l])];
                break;
            }
        }
        T->l2[i] = e;
    }
    if (threadIdx.x == 0) T->l2k = l2k, T->l2n = l2n;
    for (uint32_t p = threadIdx.x; p < (1u << kLutBits); p += kBlock) {
        uint64_t e = 0;
        uint32_t pos = 0, n = 0;
        while (n < 3 && pos < (uint32_t)kLutBits) {
            const uint32_t v = t1[(p << pos) & ((1u << kLutBits) - 1)];
            const uint32_t L = v >> 16;
            if (L == 0 || L > (uint32_t)kLutBits - pos) break;
            e |= (uint64_t)(v & 0xFFFFu) << (16 * n);
            if (n < 2) e |= (uint64_t)L << (56 + 4 * n);
            pos += L;
            ++n;
        }
        if (n == 0) e = l2k && lslot[p] != 0xFFFF ? (uint64_t)lslot[p] << l2k : 0xFFFFull;
        e |= (uint64_t)n << 48;
        e |= (uint64_t)pos << 50;
        T->lut[p] = e;
    }
}

hipError_t launch_codebook(const FieldDesc* F, int nf, uint32_t n_bins, hipStream_t s)
{
    hipLaunchKernelGGL(k_codebook, dim3(nf), dim3(kBlock), codebook_lds_bytes(n_bins), s, F);
    return hipGetLastError();
}

hipError_t launch_dectab(const FieldDesc* F, int nf, uint8_t* tabs, hipStream_t s)
{
    hipLaunchKernelGGL(k_dectab, dim3(nf), dim3(kBlock), 0, s, F, tabs);
    return hipGetLastError();
}

}  // namespace ebc
