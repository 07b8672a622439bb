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

template <uint32_t S>
__global__ __launch_bounds__(kBlock) void k_huff_bits(const FieldDesc* __restrict__ F, int nf, uint32_t* __restrict__ wcnt)
{
    __shared__ uint8_t len_s[kMaxBins];
    const uint32_t t = blockIdx.x;
    const int f = find_field<&FieldDesc::hwg_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    const EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || dy->codec != ARC_HUFFMAN) return;
    for (uint32_t s = threadIdx.x; s < fd.n_bins; s += blockDim.x) len_s[s] = fd.len[s];
    __syncthreads();
    const uint32_t c = (t - fd.hwg_base) * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (c >= fd.n_hch) return;
    const uint32_t hc = fd.hc;
    const uint64_t lo = (uint64_t)c * hc + (uint64_t)lane_id() * S;
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

template <uint32_t S>
__global__ __launch_bounds__(kBlock) void k_huff_write(const FieldDesc* __restrict__ F, int nf,
                             const uint32_t* __restrict__ woff)
{
    extern __shared__ uint64_t lds64[];
    const uint32_t t = blockIdx.x;
    const int f = find_field<&FieldDesc::hwg_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    const EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || dy->codec != ARC_HUFFMAN) return;
    const uint32_t nb = fd.n_bins, hc = fd.hc;
    uint64_t* code_s = lds64;
    uint32_t* wbuf = (uint32_t*)(lds64 + nb) + (threadIdx.x / kWave) * 2 * hc;
    for (uint32_t s = threadIdx.x; s < nb; s += blockDim.x) code_s[s] = fd.code[s];
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
        // accumulate into a 64-bit window that always starts on a word boundary
        uint32_t w = b0 >> 5;
        uint32_t nacc = b0 & 31;
        uint64_t acc = 0;
#pragma unroll
        for (uint32_t k = 0; k < S; ++k) {
            if (lo + k >= fd.n) continue;
            const uint64_t e = code_s[sym[k]];
            const uint32_t L = (uint32_t)(e >> 56);
            const uint64_t cw = e & ((1ull << 56) - 1);
            // emit in pieces of at most 32 bits: high part first
            uint32_t rem = L;
            while (rem) {
                const uint32_t take = rem > 32 ? rem - 32 : rem;
                const uint64_t piece = (cw >> (rem - take)) & ((1ull << take) - 1);
                acc |= piece << (64 - nacc - take);
                nacc += take;
                rem -= take;
                if (nacc >= 32) {
                    atomicOr(&wbuf[w], (uint32_t)(acc >> 32));
                    ++w;
                    acc <<= 32;
                    nacc -= 32;
                }
            }
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

// In-order stream of a chunk's 32-bit words, fetched as aligned 16-byte
// blocks one block ahead of use: each lane issues one vector load per four
// words consumed, so the wait at a refill rarely finds the load outstanding.
struct WordQueue {
    const EBC_G uint4* __restrict__ blk;  // aligned 16-byte blocks covering the chunk
    uint32_t nblk, jn, have;
    uint32_t q0, q1, q2, q3, q4, q5, q6, q7;
    __device__ __forceinline__ uint4 fetch(uint32_t j) const
    {
        if (j < nblk) {
            const uint4 v = blk[j];
            return v;
        }
        return make_uint4(0u, 0u, 0u, 0u);
    }
    __device__ __forceinline__ void init(const EBC_G uint32_t* __restrict__ words, uint32_t nw)
    {
        const uintptr_t a = (uintptr_t)words;
        const uint32_t o = (uint32_t)((a & 15u) >> 2);
        blk = (const EBC_G uint4*)(a & ~(uintptr_t)15u);
        nblk = (o + nw + 3) / 4;
        const uint4 b0 = fetch(0), b1 = fetch(1);
        q0 = b0.x, q1 = b0.y, q2 = b0.z, q3 = b0.w, q4 = b1.x, q5 = b1.y, q6 = b1.z, q7 = b1.w;
        jn = 2;
        have = 8;
        for (uint32_t i = 0; i < o; ++i) pop();
    }
    __device__ __forceinline__ uint32_t pop()
    {
        const uint32_t w = q0;
        q0 = q1, q1 = q2, q2 = q3, q3 = q4, q4 = q5, q5 = q6, q6 = q7;
        if (--have == 4) {
            const uint4 b = fetch(jn++);
            q4 = b.x, q5 = b.y, q6 = b.z, q7 = b.w;
            have = 8;
        }
        return w;
    }
};

// Appends symbols to a 128-bit register pack and stores every 8 (16 bytes,
// aligned because chunks start at multiples of 8 symbols).
struct SymPack {
    uint64_t lo = 0, hi = 0;
    uint32_t cnt = 0, base = 0;
    __device__ __forceinline__ void push(EBC_G uint16_t* __restrict__ out, uint32_t s)
    {
        if (cnt < 4) lo |= (uint64_t)s << (16 * cnt);
        else hi |= (uint64_t)s << (16 * (cnt - 4));
        if (++cnt == 8) {
            *(EBC_G uint4*)(out + base) =
                make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
            base += 8;
            lo = hi = 0;
            cnt = 0;
        }
    }
    __device__ __forceinline__ void flush(EBC_G uint16_t* __restrict__ out)
    {
        for (uint32_t k = 0; k < cnt; ++k)
            out[base + k] = (uint16_t)((k < 4 ? lo >> (16 * k) : hi >> (16 * (k - 4))) & 0xFFFF);
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
    // ends of the first kLongLens long lengths, wave-uniform (scalar registers)
    uint64_t ev[kLongLens];
    const uint32_t nlong = maxl > kLutBits + 1 ? maxl - kLutBits - 1 : 0;
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

    // 64-bit window fed from the block queue
    WordQueue wq;
    wq.init(words, nw);
    uint64_t buf = (uint64_t)wq.pop() << 32;
    buf |= wq.pop();
    uint32_t valid = 64, pos = 0, j = 0;
    bool bad = false;
    SymPack pk;
    while (j < nsym) {
        if (valid < 32) {
            buf |= (uint64_t)wq.pop() << (32 - valid);
            valid += 32;
        }
        const uint64_t e = lut[(uint32_t)(buf >> (64 - kLutBits))];
        uint32_t n = (uint32_t)(e >> 48) & 3u;
        const bool slow = n == 0;
        if (!slow) {
            const uint32_t rem = nsym - j;
            uint32_t tl = (uint32_t)(e >> 50) & 63u;
            if (n > rem) {
                n = rem;
                tl = (uint32_t)(e >> 36) & 15u;
                if (n == 2) tl += (uint32_t)(e >> 40) & 15u;
            }
            pk.push(out, (uint32_t)e & 0xFFFu);
            if (n > 1) pk.push(out, (uint32_t)(e >> 12) & 0xFFFu);
            if (n > 2) pk.push(out, (uint32_t)(e >> 24) & 0xFFFu);
            buf <<= tl;
            valid -= tl;
            pos += tl;
            j += n;
        }
        if (slow) {
            // codeword longer than kLutBits: its length is kLutBits + 1 plus the
            // number of longer code-space ends the window lies at or above
            uint32_t L = kLutBits + 1;
#pragma unroll
            for (int k = 0; k < kLongLens; ++k)
                if ((uint32_t)k < nlong) L += buf >= ev[k] ? 1u : 0u;
            for (uint32_t l = kLutBits + 1 + kLongLens; l < maxl; ++l) L += buf >= s_endv[l] ? 1u : 0u;
            if (L <= valid) {
                // the window is at or above the start of the length-L codes by
                // construction; it must also lie below their end
                const uint64_t d = (buf >> (64 - L)) - s_first[L];
                if (d >= (uint64_t)(s_off[L + 1] - s_off[L])) {
                    bad = true;
                    break;
                }
                pk.push(out, perm[s_off[L] + (uint32_t)d]);
                buf <<= L;
                valid -= L;
                pos += L;
                j += 1;
            } else {
                // longer than the buffered bits (> 32-bit codes) or invalid:
                // exact window from memory, then resynchronise the buffer
                const uint64_t win = window_at(words, nw, pos);
                L = kLutBits + 1;
                for (uint32_t l = kLutBits + 1; l < maxl; ++l) L += win >= s_endv[l] ? 1u : 0u;
                const uint64_t d = (win >> (64 - L)) - s_first[L];
                if (d >= (uint64_t)(s_off[L + 1] - s_off[L])) {
                    bad = true;
                    break;
                }
                pk.push(out, perm[s_off[L] + (uint32_t)d]);
                pos += L;
                j += 1;
                const uint32_t kk = pos >> 5, s = pos & 31;
                wq.init(words + kk, nw > kk ? nw - kk : 0u);
                buf = (uint64_t)wq.pop() << 32;
                buf |= wq.pop();
                buf <<= s;
                valid = 64 - s;
            }
        }
    }
    if (!bad) pk.flush(out);
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

hipError_t launch_huff_bits(const FieldDesc* F, int nf, uint32_t units, uint32_t hc, uint32_t* wcnt,
                            hipStream_t s)
{
    if (!units) return hipSuccess;
    EBC_HC_DISPATCH(k_huff_bits, dim3(units), dim3(kWave * huff_cpw(hc)), 0, s, F, nf, wcnt)
    return hipGetLastError();
}

hipError_t launch_huff_write(const FieldDesc* F, int nf, uint32_t units, uint32_t hc,
                             uint32_t n_bins, const uint32_t* woff, hipStream_t s)
{
    if (!units) return hipSuccess;
    EBC_HC_DISPATCH(k_huff_write, dim3(units), dim3(kWave * huff_cpw(hc)),
                    huff_write_lds_bytes(n_bins, hc), s, F, nf, woff)
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
