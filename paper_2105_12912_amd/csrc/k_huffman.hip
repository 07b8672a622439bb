// k_huffman.hip -- chunked canonical Huffman encoding and decoding.
//
// Sec. II-A steps 7-8: encode the quant-codes with the codebook and
// concatenate ("deflate") the codewords.  The stream is cut into chunks of hc
// symbols so both directions run chunk-parallel; each chunk starts on a 32-bit
// word, bits are packed MSB-first, and the per-chunk bit counts are stored so
// a decoder can locate every chunk (Sec. III-B.2 mentions the chunk-wise
// metadata).  Sec. V-C notes that writing a word only once it is full saves
// DRAM stores: here every chunk is assembled in LDS and leaves with
// coalesced full-word stores.
//
// Encode: one wavefront per chunk (k_huff_bits counts bits; after a scan of
// the word counts k_huff_write packs with LDS atomic ORs and copies out).
// Decode: one lane per chunk; a kLutBits-wide table yields up to three short
// codewords per lookup, longer codewords use the canonical limit test.
#include "ebc_dev.h"
#include "ebc_launch.h"

namespace ebc {


size_t huff_write_lds_bytes(uint32_t n_bins, uint32_t hc)
{
    return (size_t)n_bins * 8 + (size_t)huff_cpw(hc) * 2 * hc * 4;
}

// symbols [lo, lo + S) of a chunk, S = hc / 64, owned by one lane
template <uint32_t S>
__device__ __forceinline__ void load_syms(const EBC_G uint16_t* __restrict__ q, uint64_t lo, uint64_t n,
                                          uint16_t* out)
{
    if (S >= 8 && lo + S <= n) {
#pragma unroll
        for (uint32_t k = 0; k < S; k += 8) {
            const uint4 t = *(const EBC_G uint4*)(q + lo + k);
            out[k + 0] = t.x & 0xFFFF, out[k + 1] = t.x >> 16;
            out[k + 2] = t.y & 0xFFFF, out[k + 3] = t.y >> 16;
            out[k + 4] = t.z & 0xFFFF, out[k + 5] = t.z >> 16;
            out[k + 6] = t.w & 0xFFFF, out[k + 7] = t.w >> 16;
        }
    } else {
#pragma unroll
        for (uint32_t k = 0; k < S; ++k) out[k] = lo + k < n ? q[lo + k] : 0;
    }
}

// Both encode kernels are persistent: a workgroup walks groups of
// huff_cpw(hc) chunks with a grid stride and reloads the code table in LDS
// only when it moves to another field.
template <uint32_t S>
__global__ __launch_bounds__(kBlock) void k_huff_bits(const FieldDesc* __restrict__ F, int nf,
                                                      uint32_t* __restrict__ wcnt, uint32_t units)
{
    __shared__ uint8_t len_s[kMaxBins];
    int cur = -1;
    for (uint32_t t = blockIdx.x; t < units; t += gridDim.x) {
        const int f = find_field<&FieldDesc::hwg_base>(F, nf, t);
        const FieldDesc& fd = F[f];
        const EBC_G FieldDyn* dy = fd.dyn;
        if (dy->status != ST_OK || dy->codec != ARC_HUFFMAN) continue;
        if (f != cur) {
            __syncthreads();
            for (uint32_t s = threadIdx.x; s < fd.n_bins; s += blockDim.x) len_s[s] = fd.len[s];
            __syncthreads();
            cur = f;
        }
        const uint32_t c = (t - fd.hwg_base) * (blockDim.x / kWave) + threadIdx.x / kWave;
        if (c >= fd.n_hch) continue;
        const uint64_t lo = (uint64_t)c * fd.hc + (uint64_t)lane_id() * S;
        uint16_t sym[S];
        load_syms<S>(fd.q, lo, fd.n, sym);
        uint32_t bits = 0;
#pragma unroll
        for (uint32_t k = 0; k < S; ++k)
            if (lo + k < fd.n) bits += len_s[sym[k]];
        bits = wave_sum_u32(bits);
        if (lane_id() == 0) {
            fd.hbits[c] = bits;
            wcnt[fd.hch_base + c] = (bits + 31) / 32;
        }
    }
}

// append the low `take` (<= 32) bits of v to a window that starts on a word
// boundary; full words are ORed into the chunk's LDS word buffer
__device__ __forceinline__ void put_bits(uint64_t& acc, uint32_t& nacc, uint32_t& w, uint32_t* wbuf,
                                         uint64_t v, uint32_t take)
{
    acc |= v << (64 - nacc - take);
    nacc += take;
    if (nacc >= 32) {
        atomicOr(&wbuf[w], (uint32_t)(acc >> 32));
        ++w;
        acc <<= 32;
        nacc -= 32;
    }
}

template <uint32_t S>
__global__ __launch_bounds__(kBlock) void k_huff_write(const FieldDesc* __restrict__ F, int nf,
                                                       const uint32_t* __restrict__ woff,
                                                       uint32_t units)
{
    extern __shared__ uint64_t lds64[];
    int cur = -1;
    for (uint32_t t = blockIdx.x; t < units; t += gridDim.x) {
        const int f = find_field<&FieldDesc::hwg_base>(F, nf, t);
        const FieldDesc& fd = F[f];
        const EBC_G FieldDyn* dy = fd.dyn;
        if (dy->status != ST_OK || dy->codec != ARC_HUFFMAN) continue;
        const uint32_t nb = fd.n_bins, hc = fd.hc;
        uint64_t* code_s = lds64;
        uint32_t* wbuf = (uint32_t*)(lds64 + nb) + (threadIdx.x / kWave) * 2 * hc;
        __syncthreads();  // previous chunk's words are out of the buffers
        if (f != cur) {
            for (uint32_t s = threadIdx.x; s < nb; s += blockDim.x) code_s[s] = fd.code[s];
            cur = f;
        }
        const uint32_t c = (t - fd.hwg_base) * (blockDim.x / kWave) + threadIdx.x / kWave;
        const bool live = c < fd.n_hch;
        const uint32_t cbits = live ? fd.hbits[c] : 0u;
        const uint32_t nw = (cbits + 31) / 32;
        for (uint32_t i = lane_id(); i < nw; i += kWave) wbuf[i] = 0;
        __syncthreads();
        if (live) {
            const uint64_t lo = (uint64_t)c * hc + (uint64_t)lane_id() * S;
            uint16_t sym[S];
            load_syms<S>(fd.q, lo, fd.n, sym);
            uint32_t mybits = 0;
#pragma unroll
            for (uint32_t k = 0; k < S; ++k)
                if (lo + k < fd.n) mybits += (uint32_t)(code_s[sym[k]] >> 56);
            const uint32_t b0 = wave_incl_scan_u32(mybits) - mybits;
            uint32_t w = b0 >> 5, nacc = b0 & 31;
            uint64_t acc = 0;
#pragma unroll
            for (uint32_t k = 0; k < S; ++k) {
                if (lo + k >= fd.n) continue;
                const uint64_t e = code_s[sym[k]];
                const uint32_t L = (uint32_t)(e >> 56);
                const uint64_t cw = e & ((1ull << 56) - 1);
                if (L > 32) put_bits(acc, nacc, w, wbuf, cw >> 32, L - 32);  // rare long code
                const uint32_t low = L > 32 ? 32u : L;
                put_bits(acc, nacc, w, wbuf, cw & (low == 32 ? 0xFFFFFFFFull : ((1ull << low) - 1)), low);
            }
            if (nacc) atomicOr(&wbuf[w], (uint32_t)(acc >> 32));
        }
        __syncthreads();
        if (live) {
            EBC_G uint8_t* arc = fd.arc;
            const uint32_t wo = woff[fd.hch_base + c] - woff[fd.hch_base];
            EBC_G uint32_t* dst = (EBC_G uint32_t*)(arc + dy->off_words) + wo;
            for (uint32_t i = lane_id(); i < nw; i += kWave) dst[i] = wbuf[i];
            if (lane_id() == 0) ((EBC_G uint32_t*)(arc + dy->off_bits))[c] = cbits;
        }
    }
}

// ------------------------------------------------------------- decoding


__device__ __forceinline__ uint32_t word_at(const EBC_G uint32_t* __restrict__ w, uint32_t nw, uint32_t i)
{
    return i < nw ? w[i] : 0u;
}

// 64 stream bits starting at bit `pos` (zero beyond the chunk's words)
__device__ __forceinline__ uint64_t window_at(const EBC_G uint32_t* __restrict__ w, uint32_t nw,
                                              uint32_t pos)
{
    const uint32_t k = pos >> 5, s = pos & 31;
    uint64_t a = ((uint64_t)word_at(w, nw, k) << 32) | word_at(w, nw, k + 1);
    if (s) a = (a << s) | (word_at(w, nw, k + 2) >> (32 - s));
    return a;
}

// Per-lane ring of the chunk's 32-bit stream words in LDS.  Words reach the
// ring in 16-byte blocks: a block is loaded into registers and written to the
// ring at the next wave-uniform refill point, kRefillEvery iterations later,
// so its load has long completed when it is waited for.  Bit refills then
// read LDS; a lane that outruns its ring reads global memory directly.
constexpr uint32_t kRingWords = 32;
constexpr uint32_t kRingStride = kRingWords + 1;  // odd stride: no bank conflicts across lanes
constexpr uint32_t kRefillEvery = 4;

struct WordRing {
    uint32_t* ring;                        // this lane's slots in LDS
    const EBC_G uint4* __restrict__ blk;   // aligned 16-byte blocks of the stream
    const EBC_G uint32_t* __restrict__ words;
    uint32_t nw, o, nblk;  // words, offset of word 0 inside block 0, blocks
    uint32_t rd;           // next chunk word to hand out
    uint32_t wr;           // block-coordinate words [wr - kRingWords, wr) are in the ring
    uint32_t jn;           // block held in `pend`
    uint4 pend;
    __device__ __forceinline__ uint4 fetch(uint32_t j) const
    {
        if (j < nblk) {
            const uint4 v = blk[j];
            return v;
        }
        return make_uint4(0u, 0u, 0u, 0u);
    }
    // Stream word i.  The value always comes out of the ring slot, so the
    // common path never waits on global memory; a lane that outran the ring
    // first copies the word into the (already consumed) slot.
    __device__ __forceinline__ uint32_t get(uint32_t i)
    {
        const uint32_t a = i + o;
        const uint32_t slot = a % kRingWords;
        if (!(a < wr && a + kRingWords >= wr)) ring[slot] = i < nw ? words[i] : 0u;
        return ring[slot];
    }
    __device__ __forceinline__ void init(uint32_t* r, const EBC_G uint32_t* __restrict__ w, uint32_t n)
    {
        ring = r;
        words = w;
        nw = n;
        const uintptr_t a = (uintptr_t)w;
        o = (uint32_t)((a & 15u) >> 2);
        blk = (const EBC_G uint4*)(a & ~(uintptr_t)15u);
        nblk = (o + nw + 3) / 4;
        for (uint32_t j = 0; j < kRingWords / 4; ++j) {
            const uint4 b = fetch(j);
            ring[4 * j + 0] = b.x, ring[4 * j + 1] = b.y, ring[4 * j + 2] = b.z, ring[4 * j + 3] = b.w;
        }
        wr = kRingWords;
        jn = kRingWords / 4;
        pend = fetch(jn);
        rd = 0;
    }
    __device__ __forceinline__ uint32_t pop() { return get(rd++); }
    // wave-uniform refill point: move the pending block in if its slots are consumed
    __device__ __forceinline__ void refill()
    {
        if (jn < nblk && wr + 4 <= rd + o + kRingWords) {
            uint32_t* d = ring + (wr % kRingWords);
            d[0] = pend.x, d[1] = pend.y, d[2] = pend.z, d[3] = pend.w;
            wr += 4;
            ++jn;
            pend = fetch(jn);
        }
    }
};

// Output accumulator: up to 7 pending 16-bit symbols in a0/a1 plus overflow
// in a2; appending up to three symbols is branch-free, and every full group
// of 8 leaves as one aligned 16-byte store (chunks start at multiples of 8).
struct SymAcc {
    uint64_t a0 = 0, a1 = 0, a2 = 0;
    uint32_t cnt = 0, base = 0;
    __device__ __forceinline__ void append(EBC_G uint16_t* __restrict__ out, uint64_t syms, uint32_t n)
    {
        const uint32_t s = 16 * cnt;  // 0..112
        const uint32_t s0 = s & 63;
        const uint64_t lo = syms << s0;
        const uint64_t hi = s0 ? syms >> (64 - s0) : 0ull;
        if (s < 64) {
            a0 |= lo;
            a1 |= hi;
        } else {
            a1 |= lo;
            a2 |= hi;
        }
        cnt += n;
        if (cnt >= 8) {
            *(EBC_G uint4*)(out + base) =
                make_uint4((uint32_t)a0, (uint32_t)(a0 >> 32), (uint32_t)a1, (uint32_t)(a1 >> 32));
            base += 8;
            cnt -= 8;
            a0 = a2;
            a1 = 0;
            a2 = 0;
        }
    }
    __device__ __forceinline__ void flush(EBC_G uint16_t* __restrict__ out)
    {
        for (uint32_t k = 0; k < cnt; ++k)
            out[base + k] = (uint16_t)((k < 4 ? a0 >> (16 * k) : a1 >> (16 * (k - 4))) & 0xFFFF);
    }
};

// One codeword longer than kLutBits at the head of a window: its length is
// kLutBits + 1 plus the number of code-space ends the window lies at or above.
// Returns the length (0 if the bits are not a codeword) and the symbol.
struct LongCode {
    const uint64_t* ev;  // ends of lengths kLutBits+1 .. kLutBits+kLongLens (wave-uniform)
    uint32_t nlong, maxl;
    const uint64_t* s_endv;
    const uint64_t* s_first;
    const uint32_t* s_off;
    const uint16_t* perm;
    __device__ __forceinline__ uint32_t decode(uint64_t w, uint32_t& sym) const
    {
        uint32_t L = kLutBits + 1;
#pragma unroll
        for (int k = 0; k < kLongLens; ++k)
            if ((uint32_t)k < nlong) L += w >= ev[k] ? 1u : 0u;
        for (uint32_t l = kLutBits + 1 + kLongLens; l < maxl; ++l) L += w >= s_endv[l] ? 1u : 0u;
        // the window is at or above the first length-L code by construction;
        // it must also be below the end of the length-L codes
        const uint64_t d = (w >> (64 - L)) - s_first[L];
        if (d >= (uint64_t)(s_off[L + 1] - s_off[L])) return 0;
        sym = perm[s_off[L] + (uint32_t)d];
        return L;
    }
};

__global__ __launch_bounds__(kBlock) void k_huff_decode(const FieldDesc* __restrict__ F, int nf,
                                                        const uint32_t* __restrict__ woff,
                                                        const uint8_t* __restrict__ tabs,
                                                        size_t tab_stride)
{
    __shared__ uint64_t lut[1u << kLutBits];
    __shared__ uint16_t perm[kMaxBins];
    __shared__ uint64_t s_first[65];
    __shared__ uint64_t s_endv[65];
    __shared__ uint32_t s_off[65];
    __shared__ uint32_t s_ring[kBlock * kRingStride];
    const uint32_t t = blockIdx.x;
    const int f = find_field<&FieldDesc::hdwg_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || dy->codec != ARC_HUFFMAN) return;
    const DecTab* __restrict__ T = (const DecTab*)(tabs + (size_t)f * tab_stride);
    for (uint32_t i = threadIdx.x; i < (1u << kLutBits); i += kBlock) lut[i] = T->lut[i];
    for (uint32_t i = threadIdx.x; i < fd.n_bins; i += kBlock) perm[i] = T->perm[i];
    if (threadIdx.x < 65) {
        s_first[threadIdx.x] = T->first[threadIdx.x];
        s_endv[threadIdx.x] = T->endv[threadIdx.x];
        s_off[threadIdx.x] = T->offset[threadIdx.x];
    }
    const uint32_t maxl = T->max_len;
    uint64_t ev[kLongLens];
#pragma unroll
    for (int k = 0; k < kLongLens; ++k) ev[k] = T->endv[kLutBits + 1 + k];
    __syncthreads();
    const uint32_t c = (t - fd.hdwg_base) * kBlock + threadIdx.x;
    if (c >= fd.n_hch) return;
    const EBC_G uint8_t* arc = fd.arc;
    const uint32_t nbits = ((const EBC_G uint32_t*)(arc + fd.off_bits))[c];
    const uint32_t nw = (nbits + 31) / 32;
    const uint32_t wo = woff[fd.hch_base + c] - woff[fd.hch_base];
    if ((uint64_t)wo + nw > fd.n_words_hdr) {
        atomicMin(&dy->status, ST_ERR_ARCHIVE);
        return;
    }
    const EBC_G uint32_t* __restrict__ words = (const EBC_G uint32_t*)(arc + fd.off_words) + wo;
    const uint32_t hc = fd.hc;
    const uint64_t lo = (uint64_t)c * hc;
    const uint32_t nsym = (uint32_t)min<uint64_t>(hc, fd.n - lo);
    EBC_G uint16_t* __restrict__ out = fd.q + lo;
    const LongCode lc{ev, maxl > kLutBits + 1 ? maxl - kLutBits - 1 : 0u, maxl,
                      s_endv, s_first, s_off, perm};

    WordRing wr;
    wr.init(s_ring + threadIdx.x * kRingStride, words, nw);
    uint64_t buf = (uint64_t)wr.pop() << 32;
    buf |= wr.pop();
    uint32_t valid = 64, pos = 0, j = 0, it = 0;
    bool bad = false;
    SymAcc acc;
    // main loop: at least three symbols left, so whole table entries are used
    while (j + 3 <= nsym) {
        if ((++it & (kRefillEvery - 1)) == 0) wr.refill();
        if (valid < 32) {
            buf |= (uint64_t)wr.pop() << (32 - valid);
            valid += 32;
        }
        const uint64_t e = lut[(uint32_t)(buf >> (64 - kLutBits))];
        uint32_t n = (uint32_t)(e >> 48) & 3u;
        uint32_t tl = (uint32_t)(e >> 50) & 63u;
        uint64_t syms = e & 0xFFFFFFFFFFFFull;
        if (n == 0) {
            uint32_t sym = 0;
            uint32_t L = lc.decode(buf, sym);
            if (L == 0 || L > valid) {
                // longer than the buffered bits (only codes > 32 bits): exact window
                L = lc.decode(window_at(words, nw, pos), sym);
                if (L == 0) {
                    bad = true;
                    break;
                }
            }
            n = 1;
            tl = L;
            syms = sym;
        }
        acc.append(out, syms, n);
        j += n;
        pos += tl;
        if (tl <= valid) {
            buf <<= tl;
            valid -= tl;
        } else {
            const uint32_t kk = pos >> 5, s = pos & 31;
            buf = (((uint64_t)wr.get(kk) << 32) | wr.get(kk + 1)) << s;
            wr.rd = kk + 2;
            valid = 64 - s;
        }
    }
    // tail: one codeword at a time
    while (!bad && j < nsym) {
        if ((++it & (kRefillEvery - 1)) == 0) wr.refill();
        if (valid < 32) {
            buf |= (uint64_t)wr.pop() << (32 - valid);
            valid += 32;
        }
        const uint64_t e = lut[(uint32_t)(buf >> (64 - kLutBits))];
        uint32_t sym = (uint32_t)e & 0xFFFFu;
        uint32_t L = (uint32_t)(e >> 56) & 15u;
        if (((e >> 48) & 3u) == 0) {
            L = lc.decode(buf, sym);
            if (L == 0 || L > valid) {
                L = lc.decode(window_at(words, nw, pos), sym);
                if (L == 0) {
                    bad = true;
                    break;
                }
            }
        }
        acc.append(out, sym, 1);
        j += 1;
        pos += L;
        if (L <= valid) {
            buf <<= L;
            valid -= L;
        } else {
            const uint32_t kk = pos >> 5, s = pos & 31;
            buf = (((uint64_t)wr.get(kk) << 32) | wr.get(kk + 1)) << s;
            wr.rd = kk + 2;
            valid = 64 - s;
        }
    }
    if (!bad) acc.flush(out);
    if (bad || pos > nbits) atomicMin(&dy->status, ST_ERR_ARCHIVE);
}

// Huffman decompression prologue: word counts of every chunk into the
// batch-wide array (scanned next into word offsets).
__global__ __launch_bounds__(kBlock) void k_huff_prep(const FieldDesc* __restrict__ F, int nf,
                                                      uint32_t* __restrict__ wcnt)
{
    const uint32_t t = blockIdx.x;
    const int f = find_field<&FieldDesc::hdwg_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    const uint32_t c = (t - fd.hdwg_base) * kBlock + threadIdx.x;
    if (fd.dyn->codec != ARC_HUFFMAN || c >= fd.n_hch) return;
    const uint32_t nbits = ((const EBC_G uint32_t*)(fd.arc + fd.off_bits))[c];
    wcnt[fd.hch_base + c] = (nbits + 31) / 32;
}

#define EBC_HC_DISPATCH(KERNEL, ...)                                                        \
    switch (hc) {                                                                           \
    case 64: hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__); break;                             \
    case 128: hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__); break;                            \
    case 256: hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__); break;                            \
    case 512: hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__); break;                            \
    case 1024: hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__); break;                          \
    case 2048: hipLaunchKernelGGL(KERNEL<32>, __VA_ARGS__); break;                          \
    case 4096: hipLaunchKernelGGL(KERNEL<64>, __VA_ARGS__); break;                          \
    default: return hipErrorInvalidValue;                                                   \
    }

// decompression: the scanned word counts must add up to the header's count
__global__ void k_words_check(const FieldDesc* __restrict__ F, int nf, const uint32_t* __restrict__ woff)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const FieldDesc& fd = F[f];
    if (fd.codec_hdr != ARC_HUFFMAN) return;
    const uint32_t tot = woff[fd.hch_base + fd.n_hch] - woff[fd.hch_base];
    if ((uint64_t)tot != fd.n_words_hdr) atomicMin(&fd.dyn->status, (int32_t)ST_ERR_ARCHIVE);
}

hipError_t launch_words_check(const FieldDesc* F, int nf, const uint32_t* woff, hipStream_t s)
{
    hipLaunchKernelGGL(k_words_check, dim3((nf + 63) / 64), dim3(64), 0, s, F, nf, woff);
    return hipGetLastError();
}

// persistent grid: enough workgroups to fill the device several times over
static uint32_t persistent_grid(uint32_t units) { return units < kPersistentBlocks ? units : kPersistentBlocks; }

hipError_t launch_huff_bits(const FieldDesc* F, int nf, uint32_t units, uint32_t hc, uint32_t* wcnt,
                            hipStream_t s)
{
    if (!units) return hipSuccess;
    EBC_HC_DISPATCH(k_huff_bits, dim3(persistent_grid(units)), dim3(kWave * huff_cpw(hc)), 0, s, F, nf,
                    wcnt, units)
    return hipGetLastError();
}

hipError_t launch_huff_write(const FieldDesc* F, int nf, uint32_t units, uint32_t hc,
                             uint32_t n_bins, const uint32_t* woff, hipStream_t s)
{
    if (!units) return hipSuccess;
    EBC_HC_DISPATCH(k_huff_write, dim3(persistent_grid(units)), dim3(kWave * huff_cpw(hc)),
                    huff_write_lds_bytes(n_bins, hc), s, F, nf, woff, units)
    return hipGetLastError();
}

hipError_t launch_huff_prep(const FieldDesc* F, int nf, uint32_t units, uint32_t* wcnt, hipStream_t s)
{
    if (!units) return hipSuccess;
    hipLaunchKernelGGL(k_huff_prep, dim3(units), dim3(kBlock), 0, s, F, nf, wcnt);
    return hipGetLastError();
}

hipError_t launch_huff_decode(const FieldDesc* F, int nf, uint32_t units, const uint32_t* woff,
                              const uint8_t* tabs, size_t tab_stride, hipStream_t s)
{
    if (!units) return hipSuccess;
    hipLaunchKernelGGL(k_huff_decode, dim3(units), dim3(kBlock), 0, s, F, nf, woff, tabs, tab_stride);
    return hipGetLastError();
}

}  // namespace ebc
