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

// The codebook and the decoder tables run as one workgroup per field of kCb
// threads: the merge rounds are short and mostly a per-item binary search,
// and the table entries are independent, so one item per thread keeps each
// step to a few dependent LDS reads.
constexpr uint32_t kCb = 1024;
constexpr int kCbWaves = kCb / kWave;

size_t codebook_lds_bytes(uint32_t n_bins)
{
    const uint32_t P = max(pow2ceil(n_bins), 512u);
    return (size_t)16 * P;
}

// Rank of every symbol among the symbols of equal length with a smaller index,
// and per-length counts, using wave ballots.  Fills
//   rank_out[k] for the symbols s = 64 * (w + k NT / 64) + lane handled by wave w of NT threads,
//   cnt[b * 65 + L] = symbols of length L in block b, then prefix over blocks.
// len_s: LDS code lengths.  After return (block-synchronised):
//   cnt[b*65+L] = number of symbols of length L in blocks < b,
//   cntL[L]     = total symbols of length L.
template <uint32_t NT>
__device__ void canonical_rank(const uint8_t* len_s, uint32_t nb, uint16_t* cnt, uint32_t* cntL,
                               uint32_t rank_out[16])
{
    const int l = lane_id();
    const int w = threadIdx.x / kWave;
    const uint32_t nblk = (nb + 63) / 64;
    for (uint32_t i = threadIdx.x; i < nblk * 65; i += NT) cnt[i] = 0;
    __syncthreads();
    int k = 0;
    for (uint32_t b = w; b < nblk; b += (NT / kWave), ++k) {
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

// pass 0: the codebook of the quant-codes and the codec decision; pass 1
// (RLE+VLE fields only): the codebook of the run values, from their own
// histogram, which replaces the first in code / len.
__global__ __launch_bounds__(kCb) void k_codebook(const FieldDesc* __restrict__ F, int pass)
{
    const FieldDesc& fd = F[blockIdx.x];
    EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || dy->codec == ARC_CONST) return;
    if (pass == 1 && dy->codec != ARC_RLE_VLE) return;
    const EBC_G uint32_t* __restrict__ hist = pass == 0 ? fd.hist : fd.vhist;
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
    __shared__ uint32_t s_red[kCbWaves];

    // leaves: key = (freq << 16) | symbol; absent symbols sort last
    uint32_t used = 0;
    for (uint32_t s = threadIdx.x; s < P; s += kCb) {
        const uint32_t h = s < nb ? hist[s] : 0u;
        keys[s] = h ? (((uint64_t)h << 16) | s) : ~0ull;
        used += h != 0;
    }
    used = wave_sum_u32(used);
    if (lane_id() == 0) s_red[threadIdx.x / kWave] = used;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kCbWaves; ++k) t += s_red[k];
        s_m = t;
    }
    // bitonic sort of P keys, ascending
    if (P <= kCb) {
        // one key per thread in a register: partners closer than a wave are
        // exchanged by lane shuffles, farther ones through LDS
        __syncthreads();
        const uint32_t i = threadIdx.x;
        uint64_t v = i < P ? keys[i] : ~0ull;
        for (uint32_t k = 2; k <= P; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                uint64_t u;
                if (j < (uint32_t)kWave) {
                    u = ((uint64_t)(uint32_t)__shfl_xor((int)(v >> 32), (int)j) << 32) |
                        (uint32_t)__shfl_xor((int)(uint32_t)v, (int)j);
                } else {
                    __syncthreads();
                    if (i < P) keys[i] = v;
                    __syncthreads();
                    u = i < P ? keys[i ^ j] : ~0ull;
                }
                // the lower index of an ascending pair keeps the minimum
                const bool lower = (i & j) == 0, up = (i & k) == 0;
                v = (lower == up) ? min(v, u) : max(v, u);
            }
        }
        __syncthreads();
        if (i < P) keys[i] = v;
    } else {
        for (uint32_t k = 2; k <= P; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                __syncthreads();
                for (uint32_t i = threadIdx.x; i < P; i += kCb) {
                    const uint32_t p = i ^ j;
                    if (p > i) {
                        const uint64_t a = keys[i], b = keys[p];
                        const bool up = (i & k) == 0;
                        if ((a > b) == up) keys[i] = b, keys[p] = a;
                    }
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
    // two-queue picks exactly.  The rounds run in one wave: ballots instead of
    // workgroup barriers, and a wave's LDS accesses complete in order, so the
    // new nodes are cleared and then summed with LDS atomics in place.
    if (threadIdx.x < (uint32_t)kWave) {
        const uint32_t lane = lane_id();
        auto lw = [&](uint32_t i) { return (uint32_t)(keys[i] >> 16); };
        uint32_t li = 0, ih = 0, ni = 0;
        while (ni + 1 < m) {
            // the two smallest available items, from the four queue heads
            const uint32_t l0 = li < m ? lw(li) : 0xFFFFFFFFu, l1 = li + 1 < m ? lw(li + 1) : 0xFFFFFFFFu;
            const uint32_t i0 = ih < ni ? iw[ih] : 0xFFFFFFFFu, i1 = ih + 1 < ni ? iw[ih + 1] : 0xFFFFFFFFu;
            uint32_t t, a = li, b = ih;
            {
                const bool f0 = a < m && (b == ni || l0 <= i0);
                t = f0 ? l0 : i0;
                a += f0, b += !f0;
                const uint32_t la = a == li ? l0 : l1, ib = b == ih ? i0 : i1;
                const bool f1 = a < m && (b == ni || la <= ib);
                t += f1 ? la : ib;
            }
            // available leaves / internal nodes of weight <= t (prefixes of sorted lists)
            uint32_t cl = 0, ci = 0;
            for (uint32_t base = li;; base += kWave) {
                const uint32_t i = base + lane;
                const uint32_t c = (uint32_t)__popcll(ballot(i < m && lw(i) <= t));
                cl += c;
                if (c < (uint32_t)kWave) break;
            }
            for (uint32_t base = ih;; base += kWave) {
                const uint32_t j = base + lane;
                const uint32_t c = (uint32_t)__popcll(ballot(j < ni && iw[j] <= t));
                ci += c;
                if (c < (uint32_t)kWave) break;
            }
            const uint32_t np = (cl + ci) / 2;
            for (uint32_t k = lane; k < np; k += kWave) iw[ni + k] = 0;
            // merged position of every item: its parent, and its weight added
            // to that parent's
            for (uint32_t i = lane; i < cl; i += kWave) {
                const uint32_t wi = lw(li + i);
                uint32_t lo = 0, hi = ci;  // internal nodes lighter than the leaf
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (iw[ih + mid] < wi) lo = mid + 1;
                    else hi = mid;
                }
                const uint32_t pos = i + lo;
                if (pos < 2 * np) {
                    parent[li + i] = (uint16_t)(m + ni + pos / 2);
                    atomicAdd(&iw[ni + pos / 2], wi);
                }
            }
            for (uint32_t j = lane; j < ci; j += kWave) {
                const uint32_t wj = iw[ih + j];
                uint32_t lo = 0, hi = cl;  // leaves not heavier than the node
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (lw(li + mid) <= wj) lo = mid + 1;
                    else hi = mid;
                }
                const uint32_t pos = j + lo;
                if (pos < 2 * np) {
                    parent[m + ih + j] = (uint16_t)(m + ni + pos / 2);
                    atomicAdd(&iw[ni + pos / 2], wj);
                }
            }
            uint32_t dl = cl, di = ci;
            if ((cl + ci) & 1) {
                // the last item in merged order stays: an internal node comes
                // after a leaf of equal weight
                bool last_is_leaf;
                if (ci == 0) last_is_leaf = true;
                else if (cl == 0) last_is_leaf = false;
                else last_is_leaf = lw(li + cl - 1) > iw[ih + ci - 1];
                if (last_is_leaf) --dl;
                else --di;
            }
            li += dl, ih += di, ni += np;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && m > 1) parent[2 * m - 2] = (uint16_t)(2 * m - 2);  // the root points to itself
    __syncthreads();
    // depths by pointer jumping over nodes 0 .. 2m-2 (depth <= 64 < 2^7)
    const uint32_t nn = m > 1 ? 2 * m - 1 : 1;
    const uint32_t root = nn - 1;
    for (uint32_t v = threadIdx.x; v < nn; v += kCb) dep[v] = v == root ? 0 : 1;
    if (m == 1 && threadIdx.x == 0) dep[0] = 1;  // a lone symbol gets one bit
    __syncthreads();
    if (m > 1) {
        // at most kNodes nodes per thread (2 * 4096 - 1 nodes, kCb threads),
        // in registers through fully unrolled loops
        constexpr int kNodes = (2 * kMaxBins + kCb - 1) / kCb;
        for (int round = 0; round < 7; ++round) {
            uint32_t nd[kNodes], na[kNodes];
#pragma unroll
            for (int c = 0; c < kNodes; ++c) {
                const uint32_t v = threadIdx.x + c * kCb;
                if (v < nn) {
                    const uint32_t a = parent[v];
                    nd[c] = dep[v] + (a == v ? 0u : dep[a]);
                    na[c] = parent[a];
                }
            }
            __syncthreads();
#pragma unroll
            for (int c = 0; c < kNodes; ++c) {
                const uint32_t v = threadIdx.x + c * kCb;
                if (v < nn) {
                    dep[v] = (uint8_t)min(nd[c], 255u);
                    parent[v] = (uint16_t)na[c];
                }
            }
            __syncthreads();
        }
    }
    // leaf lengths -> symbols
    for (uint32_t s = threadIdx.x; s < Pa; s += kCb) len_s[s] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < m; i += kCb) len_s[keys[i] & 0xFFFFu] = dep[i];
    __syncthreads();

    // canonical codes (R0 reused for the per-block counts)
    uint16_t* cnt = (uint16_t*)keys;
    uint32_t* cntL = (uint32_t*)(((uintptr_t)(cnt + ((nb + 63) / 64) * 65 + 2) + 7) & ~(uintptr_t)7);
    uint64_t* first = (uint64_t*)(((uintptr_t)(cntL + 65) + 7) & ~(uintptr_t)7);
    uint32_t rank[16];
    canonical_rank<kCb>(len_s, nb, cnt, cntL, rank);
    if (threadIdx.x == 0) {
        uint64_t c = 0;
        uint32_t maxl = 0;
        // counts read 16 at a time so that the chain below waits on LDS
        // four times, not 64
        for (int L0 = 1; L0 <= 64; L0 += 16) {
            uint32_t cl[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) cl[u] = cntL[L0 + u];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                first[L0 + u] = c;
                c = (c + cl[u]) << 1;
                if (cl[u]) maxl = L0 + u;
            }
        }
        dy->max_len = maxl;
        dy->n_used = m;
    }
    __syncthreads();
    const int l = lane_id();
    const int w = threadIdx.x / kWave;
    uint64_t bits = 0;
    int k = 0;
    for (uint32_t b = w; b < (nb + 63) / 64; b += kCbWaves, ++k) {
        const uint32_t s = b * 64 + l;
        if (s < nb) {
            const uint32_t L = len_s[s];
            uint64_t packed = 0;
            if (L) {
                const uint64_t code = first[L] + cnt[b * 65 + L] + rank[k];
                packed = ((uint64_t)L << 56) | code;
                bits += (uint64_t)hist[s] * L;
            }
            fd.code[s] = packed;
            fd.len[s] = (uint8_t)L;
        }
    }
    bits = wave_sum_u64(bits);
    __shared__ uint64_t s_bits[kCbWaves];
    if (l == 0) s_bits[w] = bits;
    __syncthreads();
    if (threadIdx.x == 0 && pass == 0) {
        uint64_t tb = 0;
        for (int k = 0; k < kCbWaves; ++k) tb += s_bits[k];
        dy->huff_bits = tb;
        // the 1.09-bit rule picks the run-length workflow; with VLE requested
        // its run values are Huffman-coded as well
        const bool rle = 100ull * tb <= 109ull * fd.n;
        int codec;
        switch (fd.codec_req) {
        case REQ_AUTO: codec = rle ? ARC_RLE : ARC_HUFFMAN; break;
        case REQ_AUTO_VLE: codec = rle ? ARC_RLE_VLE : ARC_HUFFMAN; break;
        case REQ_HUFFMAN: codec = ARC_HUFFMAN; break;
        case REQ_RLE: codec = ARC_RLE; break;
        default: codec = ARC_RLE_VLE; break;
        }
        dy->codec = codec;
        dy->n_out = fd.hist[0];
    }
}

// ------------------------------------------------- wide bins (> kMaxBins)
// The same construction for n_bins up to 65536, whose per-symbol arrays do
// not fit in LDS: keys, internal weights, parents and depths live in a
// per-field scratch of the workspace (codebook_wide_scratch_bytes), one
// workgroup per field, every phase separated by workgroup barriers.  The
// internal weights are summed with atomics, so they are read back with
// atomic loads (the vector L1 is not kept coherent with L2 atomics).

size_t codebook_wide_scratch_bytes(uint32_t n_bins)
{
    const size_t P = pow2ceil(n_bins);
    return 8 * P + 4 * P + 4 * (4 * P) + 4 * (4 * P);  // keys, weights, 2 x 2P parents, 2 x 2P depths
}

__device__ __forceinline__ uint32_t ld_atomic(const EBC_G uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Running per-length ranks over the symbols in blocks of kCb: for symbol s of
// length L (0 = unused) returns the number of symbols of length L below s;
// run[65] (LDS) carries the per-length totals from block to block, wc[16][65]
// is LDS scratch.  Uniform loop; every thread calls it for its symbol.
__device__ __forceinline__ uint32_t blocked_rank(uint32_t L, uint32_t* run, uint32_t (*wc)[65])
{
    const int l = lane_id();
    const int w = threadIdx.x / kWave;
    uint64_t todo = ballot(L != 0);
    uint32_t rk = 0;
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const uint32_t LL = __shfl(L, leader);
        const uint64_t m = ballot(L == LL);
        if (L == LL) rk = __popcll(m & ((1ull << l) - 1));
        if (l == 0) wc[w][LL] = (uint32_t)__popcll(m);
        todo &= ~m;
    }
    __syncthreads();
    uint32_t off = 0;
    if (L) {
        off = run[L];
        for (int v = 0; v < w; ++v) off += wc[v][L];
    }
    __syncthreads();
    if (threadIdx.x < 65) {
        uint32_t t = 0;
        for (int v = 0; v < kCbWaves; ++v) {
            t += wc[v][threadIdx.x];
            wc[v][threadIdx.x] = 0;
        }
        run[threadIdx.x] += t;
    }
    __syncthreads();
    return off + rk;
}

__global__ __launch_bounds__(kCb) void k_codebook_wide(const FieldDesc* __restrict__ F, int pass)
{
    const FieldDesc& fd = F[blockIdx.x];
    EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || dy->codec == ARC_CONST) return;
    if (pass == 1 && dy->codec != ARC_RLE_VLE) return;
    const EBC_G uint32_t* __restrict__ hist = pass == 0 ? fd.hist : fd.vhist;
    const uint32_t nb = fd.n_bins;
    const uint32_t P0 = pow2ceil(nb);
    EBC_G uint64_t* keys = (EBC_G uint64_t*)fd.cbs;
    EBC_G uint32_t* iw = (EBC_G uint32_t*)(keys + P0);
    // nodes: m leaves then m - 1 internal ones, below 2 P0
    EBC_G uint32_t* par[2] = {iw + P0, iw + 3 * P0};
    EBC_G uint32_t* dep[2] = {iw + 5 * P0, iw + 7 * P0};
    __shared__ uint32_t wc[kCbWaves][65];
    __shared__ uint32_t run[65];
    __shared__ uint64_t first[65];
    __shared__ uint32_t s_li, s_ih, s_ni, s_cl, s_ci;
    __shared__ uint64_t s_bits[kCbWaves];
    for (uint32_t i = threadIdx.x; i < kCbWaves * 65; i += kCb) (&wc[0][0])[i] = 0;
    if (threadIdx.x < 65) run[threadIdx.x] = 0;
    __syncthreads();

    // used symbols in symbol order, keyed (freq << 16) | symbol
    for (uint32_t b0 = 0; b0 < nb; b0 += kCb) {
        const uint32_t s = b0 + threadIdx.x;
        const uint32_t h = s < nb ? hist[s] : 0u;
        const uint32_t pos = blocked_rank(h ? 1u : 0u, run, wc);
        if (h) keys[pos] = ((uint64_t)h << 16) | s;
    }
    const uint32_t m = run[1];
    if (m == 0) {
        if (threadIdx.x == 0) dy->status = ST_ERR_ARCHIVE;
        return;
    }
    // ascending bitonic sort of the m keys, padded to a power of two
    const uint32_t P = pow2ceil(m);
    for (uint32_t i = m + threadIdx.x; i < P; i += kCb) keys[i] = ~0ull;
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < P; i += kCb) {
                const uint32_t q = i ^ j;
                if (q > i) {
                    const uint64_t a = keys[i], b = keys[q];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) keys[i] = b, keys[q] = a;
                }
            }
        }
    }
    // two-queue merge in parallel rounds (as in k_codebook): every available
    // item not heavier than the next internal node pairs up in merged order
    if (threadIdx.x == 0) s_li = 0, s_ih = 0, s_ni = 0;
    auto lw = [&](uint32_t i) { return (uint32_t)(keys[i] >> 16); };
    for (;;) {
        __syncthreads();
        const uint32_t li = s_li, ih = s_ih, ni = s_ni;
        if (ni + 1 >= m) break;
        if (threadIdx.x == 0) {
            const uint32_t l0 = li < m ? lw(li) : 0xFFFFFFFFu, l1 = li + 1 < m ? lw(li + 1) : 0xFFFFFFFFu;
            const uint32_t i0 = ih < ni ? ld_atomic(iw + ih) : 0xFFFFFFFFu;
            const uint32_t i1 = ih + 1 < ni ? ld_atomic(iw + ih + 1) : 0xFFFFFFFFu;
            uint32_t t, a = li, b = ih;
            {
                const bool f0 = a < m && (b == ni || l0 <= i0);
                t = f0 ? l0 : i0;
                a += f0, b += !f0;
                const uint32_t la = a == li ? l0 : l1, ib = b == ih ? i0 : i1;
                const bool f1 = a < m && (b == ni || la <= ib);
                t += f1 ? la : ib;
            }
            // both queues are sorted: binary searches for the items <= t
            uint32_t lo = li, hi = m;
            while (lo < hi) {
                const uint32_t md = (lo + hi) >> 1;
                if (lw(md) <= t) lo = md + 1;
                else hi = md;
            }
            s_cl = lo - li;
            lo = ih, hi = ni;
            while (lo < hi) {
                const uint32_t md = (lo + hi) >> 1;
                if (ld_atomic(iw + md) <= t) lo = md + 1;
                else hi = md;
            }
            s_ci = lo - ih;
        }
        __syncthreads();
        const uint32_t cl = s_cl, ci = s_ci, np = (cl + ci) / 2;
        if (np == 0) {
            // cannot happen (the two lightest items always pair); guards the loop
            if (threadIdx.x == 0) dy->status = ST_ERR_ARCHIVE;
            return;
        }
        for (uint32_t k = threadIdx.x; k < np; k += kCb)
            __hip_atomic_store(iw + ni + k, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cl; i += kCb) {
            const uint32_t wi = lw(li + i);
            uint32_t lo = 0, hi = ci;  // internal nodes lighter than the leaf
            while (lo < hi) {
                const uint32_t md = (lo + hi) >> 1;
                if (ld_atomic(iw + ih + md) < wi) lo = md + 1;
                else hi = md;
            }
            const uint32_t pos = i + lo;
            if (pos < 2 * np) {
                par[0][li + i] = m + ni + pos / 2;
                atomicAdd(iw + ni + pos / 2, wi);
            }
        }
        for (uint32_t j = threadIdx.x; j < ci; j += kCb) {
            const uint32_t wj = ld_atomic(iw + ih + j);
            uint32_t lo = 0, hi = cl;  // leaves not heavier than the node
            while (lo < hi) {
                const uint32_t md = (lo + hi) >> 1;
                if (lw(li + md) <= wj) lo = md + 1;
                else hi = md;
            }
            const uint32_t pos = j + lo;
            if (pos < 2 * np) {
                par[0][m + ih + j] = m + ni + pos / 2;
                atomicAdd(iw + ni + pos / 2, wj);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t dl = cl, di = ci;
            if ((cl + ci) & 1) {
                bool last_is_leaf;
                if (ci == 0) last_is_leaf = true;
                else if (cl == 0) last_is_leaf = false;
                else last_is_leaf = lw(li + cl - 1) > ld_atomic(iw + ih + ci - 1);
                if (last_is_leaf) --dl;
                else --di;
            }
            s_li = li + dl, s_ih = ih + di, s_ni = ni + np;
        }
    }
    // depths by pointer jumping (ping-pong buffers); a lone symbol gets one bit
    const uint32_t nn = m > 1 ? 2 * m - 1 : 1;
    const uint32_t root = nn - 1;
    for (uint32_t v = threadIdx.x; v < nn; v += kCb) {
        dep[0][v] = m == 1 ? 1u : (v == root ? 0u : 1u);
        if (v == root) par[0][v] = v;
    }
    int cur = 0;
    if (m > 1) {
        for (int round = 0; round < 7; ++round) {
            __syncthreads();
            for (uint32_t v = threadIdx.x; v < nn; v += kCb) {
                const uint32_t a = par[cur][v];
                dep[cur ^ 1][v] = min(dep[cur][v] + (a == v ? 0u : dep[cur][a]), 255u);
                par[cur ^ 1][v] = par[cur][a];
            }
            cur ^= 1;
        }
    }
    __syncthreads();
    // leaf lengths -> symbols, per-length counts
    for (uint32_t s2 = threadIdx.x; s2 < nb; s2 += kCb) fd.len[s2] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < m; i += kCb) fd.len[keys[i] & 0xFFFFu] = (uint8_t)dep[cur][i];
    if (threadIdx.x < 65) run[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t s2 = threadIdx.x; s2 < nb; s2 += kCb) {
        const uint32_t L = fd.len[s2];
        if (L) atomicAdd(&run[L], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t c = 0;
        uint32_t maxl = 0;
        for (int L = 1; L <= 64; ++L) {
            first[L] = c;
            c = (c + run[L]) << 1;
            if (run[L]) maxl = L;
        }
        dy->max_len = maxl;
        dy->n_used = m;
    }
    __syncthreads();
    if (threadIdx.x < 65) run[threadIdx.x] = 0;
    __syncthreads();
    // canonical codes in (length, symbol) order
    uint64_t bits = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += kCb) {
        const uint32_t s2 = b0 + threadIdx.x;
        const uint32_t L = s2 < nb ? fd.len[s2] : 0u;
        const uint32_t rk = blocked_rank(L, run, wc);
        if (s2 < nb) {
            uint64_t packed = 0;
            if (L) {
                packed = ((uint64_t)L << 56) | (first[L] + rk);
                bits += (uint64_t)hist[s2] * L;
            }
            fd.code[s2] = packed;
        }
    }
    bits = wave_sum_u64(bits);
    if (lane_id() == 0) s_bits[threadIdx.x / kWave] = bits;
    __syncthreads();
    if (threadIdx.x == 0 && pass == 0) {
        uint64_t tb = 0;
        for (int k = 0; k < kCbWaves; ++k) tb += s_bits[k];
        dy->huff_bits = tb;
        const bool rle = 100ull * tb <= 109ull * fd.n;
        int codec;
        switch (fd.codec_req) {
        case REQ_AUTO: codec = rle ? ARC_RLE : ARC_HUFFMAN; break;
        case REQ_AUTO_VLE: codec = rle ? ARC_RLE_VLE : ARC_HUFFMAN; break;
        case REQ_HUFFMAN: codec = ARC_HUFFMAN; break;
        case REQ_RLE: codec = ARC_RLE; break;
        default: codec = ARC_RLE_VLE; break;
        }
        dy->codec = codec;
        dy->n_out = fd.hist[0];
    }
}

// ------------------------------------------------------- decoder tables
// From the code lengths stored in an archive: per-length counts, first codes
// and offsets, the symbol permutation in (length, symbol) order and a
// kLutBits-wide lookup table.



// The lookup tables of a decoder table T from the per-length counts, first
// codes and offsets (LDS) and the (length, symbol) permutation, read through
// perm(i) (LDS for narrow bins, T->perm in HBM for wide ones).  Called by every
// thread of the workgroup after a barrier.
template <class PERM>
__device__ __forceinline__ void dectab_tables(DecTab* T, const uint32_t* cntL, const uint64_t* first,
                                              const uint32_t* offs, uint32_t maxl_in, PERM perm)
{
    // left-aligned ends of the code space of lengths <= L (monotone in L)
    __syncthreads();
    if (threadIdx.x <= 64) {
        const uint32_t L = threadIdx.x;
        const uint32_t maxl = maxl_in;
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
    for (uint32_t p = threadIdx.x; p < (1u << kLutBits); p += kCb) {
        uint32_t e = 0;
        for (uint32_t l = 1; l <= (uint32_t)kLutBits; ++l) {
            const uint64_t v = p >> (kLutBits - l);
            if (cntL[l] && v < first[l] + cntL[l]) {
                e = (l << 16) | perm(offs[l] + (uint32_t)(v - first[l]));
                break;
            }
        }
        t1[p] = e;
    }
    __syncthreads();
    // Second level: number the prefixes that start a longer codeword, give
    // each a block of 2^k entries resolving the next k bits.  Longer codewords
    // are numerically larger (the limit test above), so these prefixes are the
    // top nlong ones and the numbering in prefix order makes a block's start
    // (p - (2^kLutBits - nlong)) << k: the decoder computes the second-level
    // index from the stream bits alone and relies on this order.
    __shared__ uint16_t lslot[1u << kLutBits];
    __shared__ uint16_t lpref[1u << kLutBits];
    __shared__ uint32_t s_wsum[kCbWaves];
    constexpr uint32_t kPer = (1u << kLutBits) / kCb;
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
    uint32_t nlong = 0;
    for (int v = 0; v < kCbWaves; ++v) nlong += s_wsum[v];
    const uint32_t maxl = maxl_in;
    uint32_t l2k = 0;
    if (maxl > (uint32_t)kLutBits && nlong > 0) {
        l2k = min(kL2MaxBits, maxl - (uint32_t)kLutBits);
        while (l2k > 0 && (nlong << l2k) > kL2Size) --l2k;
    }
    const uint32_t l2n = l2k ? nlong << l2k : 0u;
    for (uint32_t i = threadIdx.x; i < l2n; i += kCb) {
        const uint32_t p = lpref[i >> l2k];
        const uint64_t wv = ((uint64_t)p << l2k) | (i & ((1u << l2k) - 1));  // kLutBits + l2k bits
        uint32_t e = 0;
        for (uint32_t l = kLutBits + 1; l <= kLutBits + l2k; ++l) {
            const uint64_t v = wv >> (kLutBits + l2k - l);
            if (cntL[l] && v < first[l] + cntL[l]) {
                e = (l << 16) | perm(offs[l] + (uint32_t)(v - first[l]));
                break;
            }
        }
        T->l2[i] = e;
    }
    if (threadIdx.x == 0) T->l2k = l2k, T->l2n = l2n;
    for (uint32_t p = threadIdx.x; p < (1u << kLutBits); p += kCb) {
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

__global__ __launch_bounds__(kCb) void k_dectab(const FieldDesc* __restrict__ F,
                                                   uint8_t* __restrict__ tabs, size_t stride)
{
    const FieldDesc& fd = F[blockIdx.x];
    EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || !huff_codec(dy->codec) || fd.n_bins > kMaxBins) return;
    DecTab* T = (DecTab*)(tabs + (size_t)blockIdx.x * stride);
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
    for (uint32_t s = threadIdx.x; s < nb; s += kCb) {
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
    canonical_rank<kCb>(len_s, nb, cnt, cntL, rank);
    if (threadIdx.x == 0) {
        // canonical first codes; the lengths must satisfy Kraft's inequality
        // (first[L] + count[L] <= 2^L at every length), otherwise the archive
        // is corrupt and no table lookup below may be trusted
        uint64_t c = 0;
        uint32_t off = 0, maxl = 0;
        int bad = 0;
        // counts read 16 at a time so that the chain waits on LDS four times
        for (int L0 = 1; L0 <= 64; L0 += 16) {
            uint32_t cl[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) cl[u] = cntL[L0 + u];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int L = L0 + u;
                const uint32_t n = cl[u];
                first[L] = c;
                offs[L] = off;
                T->first[L] = c;
                T->count[L] = n;
                T->offset[L] = off;
                off += n;
                if (L <= kMaxDecodeLen && c + n > (1ull << L)) bad = 1;
                c = L <= kMaxDecodeLen ? (c + n) << 1 : 0;
                if (n) maxl = L;
            }
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
    for (uint32_t b = w; b < (nb + 63) / 64; b += kCbWaves, ++k) {
        const uint32_t s = b * 64 + l;
        if (s < nb) {
            const uint32_t L = len_s[s];
            if (L) perm_s[offs[L] + cnt[b * 65 + L] + rank[k]] = (uint16_t)s;
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nb; i += kCb) T->perm[i] = perm_s[i];
    __syncthreads();
    dectab_tables(T, cntL, first, offs, s_maxl, [&](uint32_t i) { return (uint32_t)perm_s[i]; });
}

// Decoder tables for wide bins (n_bins > kMaxBins): the same tables, with the
// per-length counts taken by LDS atomics, the permutation written straight
// to T->perm in blocks of kCb symbols (running per-length ranks) and read
// back from there.
__global__ __launch_bounds__(kCb) void k_dectab_wide(const FieldDesc* __restrict__ F,
                                                        uint8_t* __restrict__ tabs, size_t stride)
{
    const FieldDesc& fd = F[blockIdx.x];
    EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || !huff_codec(dy->codec) || fd.n_bins <= kMaxBins) return;
    DecTab* T = (DecTab*)(tabs + (size_t)blockIdx.x * stride);
    const uint32_t nb = fd.n_bins;
    __shared__ uint32_t cntL[65];
    __shared__ uint64_t first[65];
    __shared__ uint32_t offs[65];
    __shared__ uint32_t run[65];
    __shared__ uint32_t wc[kCbWaves][65];
    __shared__ int s_bad;
    __shared__ uint32_t s_maxl;
    if (threadIdx.x < 65) cntL[threadIdx.x] = 0, run[threadIdx.x] = 0;
    for (uint32_t i = threadIdx.x; i < kCbWaves * 65; i += kCb) (&wc[0][0])[i] = 0;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const uint8_t* alen = fd.arc + kHdr;
    for (uint32_t s = threadIdx.x; s < nb; s += kCb) {
        const uint32_t L = alen[s];
        if (L > kMaxDecodeLen) s_bad = 1;
        else if (L) atomicAdd(&cntL[L], 1u);
    }
    __syncthreads();
    if (s_bad) {
        if (threadIdx.x == 0) dy->status = ST_ERR_ARCHIVE;
        return;
    }
    if (threadIdx.x == 0) {
        // canonical first codes; Kraft's inequality must hold at every length
        uint64_t c = 0;
        uint32_t off = 0, maxl = 0;
        int bad = 0;
        for (int L = 1; L <= 64; ++L) {
            const uint32_t n = cntL[L];
            first[L] = c;
            offs[L] = off;
            T->first[L] = c;
            T->count[L] = n;
            T->offset[L] = off;
            off += n;
            if (L <= kMaxDecodeLen && c + n > (1ull << L)) bad = 1;
            c = L <= kMaxDecodeLen ? (c + n) << 1 : 0;
            if (n) maxl = L;
        }
        T->first[0] = 0, T->count[0] = 0, T->offset[0] = 0;
        T->max_len = maxl;
        s_maxl = maxl;
        if (maxl == 0 || bad) dy->status = ST_ERR_ARCHIVE;
        s_bad = bad | (maxl == 0);
    }
    __syncthreads();
    if (s_bad) return;
    for (uint32_t b0 = 0; b0 < nb; b0 += kCb) {
        const uint32_t s = b0 + threadIdx.x;
        const uint32_t L = s < nb ? alen[s] : 0u;
        const uint32_t rk = blocked_rank(L, run, wc);
        if (L) T->perm[offs[L] + rk] = (uint16_t)s;
    }
    __syncthreads();
    dectab_tables(T, cntL, first, offs, s_maxl, [&](uint32_t i) { return (uint32_t)T->perm[i]; });
}

hipError_t launch_codebook(const FieldDesc* F, int nf, uint32_t n_bins, int pass, hipStream_t s)
{
    if (n_bins > kMaxBins) hipLaunchKernelGGL(k_codebook_wide, dim3(nf), dim3(kCb), 0, s, F, pass);
    else hipLaunchKernelGGL(k_codebook, dim3(nf), dim3(kCb), codebook_lds_bytes(n_bins), s, F, pass);
    return hipGetLastError();
}

hipError_t launch_dectab(const FieldDesc* F, int nf, uint8_t* tabs, size_t stride, uint32_t max_bins,
                         hipStream_t s)
{
    // narrow and wide fields of one batch each skip the other kernel
    hipLaunchKernelGGL(k_dectab, dim3(nf), dim3(kCb), 0, s, F, tabs, stride);
    if (max_bins > kMaxBins) hipLaunchKernelGGL(k_dectab_wide, dim3(nf), dim3(kCb), 0, s, F, tabs, stride);
    return hipGetLastError();
}

}  // namespace ebc
