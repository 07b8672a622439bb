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
    // code table (none for wide bins, whose table stays in HBM), then per
    // wave a word buffer of 2 * hc words (one pass of kPassHc symbols for
    // longer chunks)
    const uint32_t span = hc <= kPassHc ? hc : kPassHc;
    return (size_t)(n_bins > kMaxBins ? 0 : n_bins) * 8 + (size_t)huff_cpw(hc) * 2 * span * 4;
}

// The writer's table entry for symbol s (see write_entry), for wide bins
// built from the codebook in HBM on every lookup.
__device__ __forceinline__ uint64_t write_entry(uint64_t packed);

// Symbols [lo, lo + S) of a chunk (S = hc / 64, owned by one lane), kept as
// raw 16-byte blocks so that the loads can be issued one work unit ahead and
// unpacked only when the unit is processed.
template <uint32_t S>
struct SymRaw {
    static constexpr uint32_t NV = S >= 8 ? S / 8 : 1;
    uint4 v[NV];
    __device__ __forceinline__ uint32_t at(uint32_t k) const
    {
        const uint4& b = v[k / 8];
        const uint32_t h = (k % 8) / 2;
        const uint32_t w = h == 0 ? b.x : h == 1 ? b.y : h == 2 ? b.z : b.w;
        return (w >> (16 * (k & 1))) & 0xFFFFu;
    }
};

template <uint32_t S>
__device__ __forceinline__ void load_raw(const EBC_G uint16_t* __restrict__ q, uint64_t lo, uint64_t n,
                                         SymRaw<S>& r)
{
    if (S >= 8 && lo + S <= n) {
#pragma unroll
        for (uint32_t k = 0; k < SymRaw<S>::NV; ++k) r.v[k] = *(const EBC_G uint4*)(q + lo + 8 * k);
    } else {  // short chunks and the field's tail: assembled here
        uint32_t w[4 * SymRaw<S>::NV];
#pragma unroll
        for (uint32_t k = 0; k < 4 * SymRaw<S>::NV; ++k) w[k] = 0;
#pragma unroll
        for (uint32_t k = 0; k < S; ++k)
            if (lo + k < n) w[k / 2] |= (uint32_t)q[lo + k] << (16 * (k & 1));
#pragma unroll
        for (uint32_t k = 0; k < SymRaw<S>::NV; ++k)
            r.v[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
    }
}

// One encode work unit: huff_cpw(hc) chunks, one per wavefront.  The coded
// stream is a field's quant-codes (Huffman codec) or its run values (RLE+VLE
// codec, as many as the run count found on the device); `which` selects the
// codecs a launch covers: 0 Huffman, 1 RLE+VLE, 2 both.
struct EncUnit {
    int f;
    uint32_t c;                      // this wave's chunk
    bool ok;                         // field is being Huffman-coded by this launch
    const EBC_G uint16_t* src;       // symbols of the stream
    uint64_t cnt;                    // symbols in the stream
    uint32_t nch, nsub;              // its chunks and sub-chunks
};

template <uint32_t S>
__device__ __forceinline__ EncUnit enc_unit(const FieldDesc* __restrict__ F, int nf, uint32_t t, int which)
{
    EncUnit u;
    u.f = find_field<&FieldDesc::hwg_base>(F, nf, t);
    const FieldDesc& fd = F[u.f];
    const auto* dk = kconst(fd.dyn);
    const int32_t codec = dk->codec;
    u.ok = dk->status == ST_OK &&
           (which == 0 ? codec == ARC_HUFFMAN : which == 1 ? codec == ARC_RLE_VLE : huff_codec(codec));
    const bool vle = codec == ARC_RLE_VLE;
    u.src = vle ? fd.vsym : fd.q;
    u.cnt = vle ? dk->n_runs : fd.n;
    u.nch = vle ? (uint32_t)((u.cnt + fd.hc - 1) / fd.hc) : fd.n_hch;
    u.nsub = vle ? (uint32_t)((u.cnt + fd.hs - 1) / fd.hs) : fd.n_sub;
    // blockDim = 64 * cpw; the chunk index is wave-uniform (scalar)
    u.c = (t - fd.hwg_base) * huff_cpw(64 * S) + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    return u;
}

// For S >= 8 the loads are unconditional (a lane with nothing to load reads
// the start of the stream instead), so every pipeline stage issues the same
// number of loads and the compiler's wait counts never have to assume a stage
// without them.  Symbols past the stream's end are masked by the users; the
// tail chunk's last lane may read up to 30 bytes past the stream, which the
// workspace always follows with other scratch.
template <uint32_t S>
__device__ __forceinline__ void enc_issue(const FieldDesc* __restrict__ F, const EncUnit& u, SymRaw<S>& r)
{
    const FieldDesc& fd = F[u.f];
    const uint64_t lo = (uint64_t)u.c * fd.hc + (uint64_t)lane_id() * S;
    const bool live = u.ok && u.c < u.nch && lo < u.cnt;
    if (S >= 8) {
        const EBC_G uint16_t* p = u.src + (live ? lo : 0);
#pragma unroll
        for (uint32_t k = 0; k < SymRaw<S>::NV; ++k) r.v[k] = *(const EBC_G uint4*)(p + 8 * k);
    } else if (live) {
        load_raw<S>(u.src, lo, u.cnt, r);
    }
}

// Grid-stride walk over the work units with the next unit's symbols in
// flight while the current one is processed (two static buffers, so no
// register copy ever waits on a load).  proc(unit, symbols) must treat the
// workgroup uniformly (it may synchronise).
template <uint32_t S, class Proc>
__device__ __forceinline__ void enc_pipeline(const FieldDesc* __restrict__ F, int nf, uint32_t units,
                                             int which, Proc& proc)
{
    uint32_t t = blockIdx.x;
    if (t >= units) return;
    SymRaw<S> A, B;
    EncUnit ua = enc_unit<S>(F, nf, t, which), ub;
    enc_issue<S>(F, ua, A);
    for (;;) {
        // the next stage's loads are always issued (a dead unit past the end)
        uint32_t tn = t + gridDim.x;
        ub = enc_unit<S>(F, nf, tn < units ? tn : t, which);
        if (tn >= units) ub.ok = false;
        enc_issue<S>(F, ub, B);
        proc(ua, A);
        t = tn;
        if (t >= units) break;
        tn = t + gridDim.x;
        ua = enc_unit<S>(F, nf, tn < units ? tn : t, which);
        if (tn >= units) ua.ok = false;
        enc_issue<S>(F, ua, A);
        proc(ub, B);
        t = tn;
        if (t >= units) break;
    }
}

// Both encode kernels are persistent: a workgroup walks groups of
// huff_cpw(hc) chunks with a grid stride and reloads the code table in LDS
// only when it moves to another field.
// W: wide bins (n_bins > kMaxBins), whose lengths are read from HBM
template <uint32_t S, bool W>
struct BitsProc {
    const FieldDesc* F;
    uint32_t* wcnt;
    uint8_t* len_s;
    int cur;
    __device__ __forceinline__ void operator()(const EncUnit& u, const SymRaw<S>& r)
    {
        if (!u.ok) return;
        const FieldDesc& fd = F[u.f];
        if (!W && u.f != cur) {
            __syncthreads();
            for (uint32_t s = threadIdx.x; s < fd.n_bins; s += kWave * huff_cpw(64 * S)) len_s[s] = fd.len[s];
            __syncthreads();
            cur = u.f;
        }
        if (u.c >= u.nch) return;
        const uint64_t lo = (uint64_t)u.c * fd.hc + (uint64_t)lane_id() * S;
        // symbols past the stream's end count zero bits; every lookup is
        // issued before any is used
        const uint32_t m = lo < u.cnt ? (uint32_t)min<uint64_t>(S, u.cnt - lo) : 0u;
        uint32_t bits = 0;
        if (__all(m == S)) {
            // every lane holds S symbols (all chunks but a field's last)
#pragma unroll
            for (uint32_t k = 0; k < S; ++k) bits += W ? fd.len[r.at(k)] : len_s[r.at(k)];
        } else {
#pragma unroll
            for (uint32_t k = 0; k < S; ++k) {
                const uint32_t L = W ? fd.len[k < m ? r.at(k) : 0u] : len_s[k < m ? r.at(k) : 0u];
                bits += k < m ? L : 0u;
            }
        }
        bits = wave_sum_u32(bits);
        if (lane_id() == 0) {
            fd.hbits[u.c] = bits;
            wcnt[fd.hch_base + u.c] = (bits + 31) / 32;
        }
    }
};

template <uint32_t S, bool W>
__global__ __launch_bounds__(kBlock) void k_huff_bits(const FieldDesc* __restrict__ F, int nf,
                                                      uint32_t* __restrict__ wcnt, uint32_t units,
                                                      int which)
{
    __shared__ uint8_t len_s[W ? 1 : kMaxBins];
    BitsProc<S, W> proc{F, wcnt, len_s, -1};
    enc_pipeline<S>(F, nf, units, which, proc);
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

// The writer's LDS copy of the codebook: a codeword of at most 32 bits sits
// left-aligned in the high word with its length in the low byte, so that
// appending it is one shift and one OR; a longer codeword keeps only its
// length here and is read from the codebook itself.
__device__ __forceinline__ uint64_t write_entry(uint64_t packed)
{
    const uint32_t L = (uint32_t)(packed >> 56);
    if (L == 0 || L > 32) return L;
    return ((uint64_t)((uint32_t)packed << (32 - L)) << 32) | L;
}

// append a codeword of L <= 32 bits given left-aligned in cw
__device__ __forceinline__ void put_left(uint64_t& acc, uint32_t& nacc, uint32_t& w, uint32_t* wbuf,
                                         uint32_t cw, uint32_t L)
{
    acc |= (uint64_t)cw << (32 - nacc);
    nacc += L;
    if (nacc >= 32) {
        atomicOr(&wbuf[w], (uint32_t)(acc >> 32));
        ++w;
        acc <<= 32;
        nacc -= 32;
    }
}

template <uint32_t S, bool W>
struct WriteProc {
    const FieldDesc* F;
    const uint32_t* woff;
    uint64_t* lds64;
    int cur;
    __device__ __forceinline__ uint64_t entry(const FieldDesc& fd, const uint64_t* code_s, uint32_t sym) const
    {
        return W ? write_entry(fd.code[sym]) : code_s[sym];
    }
    // up to 16 symbols per lane keep their table entries in registers between
    // the bit count and the packing; wider lanes look them up twice
    static constexpr bool kKeep = S <= 16;
    __device__ __forceinline__ void operator()(const EncUnit& u, const SymRaw<S>& r)
    {
        if (!u.ok) return;
        const FieldDesc& fd = F[u.f];
        const auto* dy = kconst(fd.dyn);
        const uint32_t nb = fd.n_bins, hc = fd.hc;
        uint64_t* code_s = lds64;
        // Each wave packs its chunk in a word buffer of its own, and a wave's
        // LDS accesses complete in order, so clearing, packing and copying
        // out need no barrier; only a new field's code table (shared by the
        // workgroup, whose waves all work on one field) does.
        uint32_t* wbuf = (uint32_t*)(lds64 + (W ? 0 : nb)) + (threadIdx.x / kWave) * 2 * hc;
        if (!W && u.f != cur) {
            __syncthreads();
            for (uint32_t s = threadIdx.x; s < nb; s += kWave * huff_cpw(64 * S))
                code_s[s] = write_entry(fd.code[s]);
            __syncthreads();
            cur = u.f;
        }
        const bool live = u.c < u.nch;
        const uint32_t cbits = live ? kconst(fd.hbits)[u.c] : 0u;
        const uint32_t nw = (cbits + 31) / 32;
        const uint64_t lo = (uint64_t)u.c * hc + (uint64_t)lane_id() * S;
        // symbols past the stream's end take the empty entry
        const uint32_t m = live && lo < u.cnt ? (uint32_t)min<uint64_t>(S, u.cnt - lo) : 0u;
        uint64_t e[kKeep ? S : 1];
        uint32_t mybits = 0, lmax = 0;
        if (__all(m == S)) {
            // every lane holds S symbols (all chunks but a field's last)
#pragma unroll
            for (uint32_t k = 0; k < S; ++k) {
                const uint64_t v = entry(fd, code_s, r.at(k));
                if (kKeep) e[kKeep ? k : 0] = v;
                const uint32_t L = (uint32_t)v & 0xFFu;
                mybits += L;
                lmax = max(lmax, L);
            }
        } else {
#pragma unroll
            for (uint32_t k = 0; k < S; ++k) {
                const uint64_t v0 = entry(fd, code_s, k < m ? r.at(k) : 0u);
                const uint64_t v = k < m ? v0 : 0ull;
                if (kKeep) e[kKeep ? k : 0] = v;
                const uint32_t L = (uint32_t)v & 0xFFu;
                mybits += L;
                lmax = max(lmax, L);
            }
        }
        for (uint32_t i = lane_id(); i < nw; i += kWave) wbuf[i] = 0;
        uint32_t sb = 0;
        if (live) {
            const uint32_t incl = wave_incl_scan_u32(mybits);
            const uint32_t b0 = incl - mybits;
            // bit count of the sub-chunk that starts at this lane (lanes_per_sub
            // lanes of S symbols each): the scan at its last lane minus b0
            constexpr uint32_t kLps = kSubMax / S < 64 ? kSubMax / S : 64u;
            sb = (uint32_t)__shfl((int)incl, (int)min<uint32_t>(lane_id() + kLps - 1, 63)) - b0;
            uint32_t w = b0 >> 5, nacc = b0 & 31;
            uint64_t acc = 0;
            if (!__any(lmax > 32)) {
#pragma unroll
                for (uint32_t k = 0; k < S; ++k) {
                    const uint64_t v = kKeep ? e[kKeep ? k : 0] : (k < m ? entry(fd, code_s, r.at(k)) : 0ull);
                    put_left(acc, nacc, w, wbuf, (uint32_t)(v >> 32), (uint32_t)v & 0xFFu);
                }
            } else {  // a codeword longer than 32 bits somewhere in the chunk
#pragma unroll
                for (uint32_t k = 0; k < S; ++k) {
                    const uint64_t v = k < m ? entry(fd, code_s, r.at(k)) : 0ull;
                    const uint32_t L = (uint32_t)v & 0xFFu;
                    if (L <= 32) {
                        put_left(acc, nacc, w, wbuf, (uint32_t)(v >> 32), L);
                    } else {
                        const uint64_t cw = fd.code[r.at(k)] & ((1ull << 56) - 1);
                        put_bits(acc, nacc, w, wbuf, cw >> 32, L - 32);
                        put_bits(acc, nacc, w, wbuf, cw & 0xFFFFFFFFull, 32);
                    }
                }
            }
            if (nacc) atomicOr(&wbuf[w], (uint32_t)(acc >> 32));
        }
        if (live) {
            EBC_G uint8_t* arc = fd.arc;
            const auto* wk = (const __attribute__((address_space(4))) uint32_t*)woff;
            const uint32_t wo = wk[fd.hch_base + u.c] - wk[fd.hch_base];
            EBC_G uint32_t* dst = (EBC_G uint32_t*)(arc + dy->off_words) + wo;
            for (uint32_t i = lane_id(); i < nw; i += kWave) dst[i] = wbuf[i];
            // sub-chunk bit counts (u16): one per kSubMax symbols of the
            // chunk, or one for the whole chunk when it is shorter
            constexpr uint32_t kLps = kSubMax / S < 64 ? kSubMax / S : 64u;
            const uint32_t hs = fd.hs;
            const uint64_t sub = (uint64_t)u.c * (hc / hs) + lane_id() / kLps;
            if (lane_id() % kLps == 0 && lo < u.cnt && sub < u.nsub)
                ((EBC_G uint16_t*)(arc + dy->off_sbits))[sub] = (uint16_t)sb;
        }
    }
};

template <uint32_t S, bool W>
__global__ __launch_bounds__(kBlock) void k_huff_write(const FieldDesc* __restrict__ F, int nf,
                                                       const uint32_t* __restrict__ woff,
                                                       uint32_t units)
{
    extern __shared__ uint64_t lds64[];
    WriteProc<S, W> proc{F, woff, lds64, -1};
    enc_pipeline<S>(F, nf, units, 2, proc);
}

// ------------------------------------------------ chunks longer than kPassHc
// One wave per chunk, in passes of kPassHc symbols (64 per lane).  The bit
// count pass sums code lengths per sub-chunk (4 lanes) and per chunk; the
// write pass packs each pass into an LDS word buffer starting at the bit
// offset the previous passes reached (its partial last word carried over as
// the buffer's first word), copies out the complete words and keeps the
// partial one for the next pass.
constexpr uint32_t kPassPerLane = kPassHc / kWave;  // 64 symbols
static_assert(kSubMax % kPassPerLane == 0, "a sub-chunk is a whole number of lanes");

__device__ __forceinline__ void load_pass(const EncUnit& u, uint64_t lo, uint32_t sym[kPassPerLane])
{
    const uint64_t i0 = lo + (uint64_t)lane_id() * kPassPerLane;
    if (i0 + kPassPerLane <= u.cnt) {
#pragma unroll
        for (uint32_t k = 0; k < kPassPerLane / 8; ++k) {
            const uint4 v = *(const EBC_G uint4*)(u.src + i0 + 8 * k);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) sym[8 * k + 2 * h] = w[h] & 0xFFFF, sym[8 * k + 2 * h + 1] = w[h] >> 16;
        }
    } else {
#pragma unroll
        for (uint32_t k = 0; k < kPassPerLane; ++k) sym[k] = i0 + k < u.cnt ? u.src[i0 + k] : 0xFFFFFFFFu;
    }
}

template <bool W>
__global__ __launch_bounds__(kWave) void k_huff_bits_long(const FieldDesc* __restrict__ F, int nf,
                                                          uint32_t* __restrict__ wcnt, uint32_t units,
                                                          int which)
{
    __shared__ uint8_t len_s[W ? 1 : kMaxBins];
    int cur = -1;
    for (uint32_t t = blockIdx.x; t < units; t += gridDim.x) {
        const EncUnit u = enc_unit<kPassPerLane>(F, nf, t, which);
        if (!u.ok) continue;
        const FieldDesc& fd = F[u.f];
        if (!W && u.f != cur) {
            for (uint32_t s = threadIdx.x; s < fd.n_bins; s += kWave) len_s[s] = fd.len[s];
            cur = u.f;
        }
        if (u.c >= u.nch) continue;
        uint64_t bits = 0;
        for (uint32_t p = 0; p < fd.hc / kPassHc; ++p) {
            const uint64_t lo = (uint64_t)u.c * fd.hc + (uint64_t)p * kPassHc;
            if (lo >= u.cnt) break;
            uint32_t sym[kPassPerLane];
            load_pass(u, lo, sym);
            uint32_t b = 0;
#pragma unroll
            for (uint32_t k = 0; k < kPassPerLane; ++k)
                b += sym[k] == 0xFFFFFFFFu ? 0u : (W ? fd.len[sym[k]] : len_s[sym[k]]);
            bits += wave_sum_u32(b);
        }
        if (lane_id() == 0) {
            fd.hbits[u.c] = (uint32_t)bits;
            wcnt[fd.hch_base + u.c] = (uint32_t)((bits + 31) / 32);
        }
    }
}

template <bool W>
__global__ __launch_bounds__(kWave) void k_huff_write_long(const FieldDesc* __restrict__ F, int nf,
                                                           const uint32_t* __restrict__ woff,
                                                           uint32_t units)
{
    extern __shared__ uint64_t lds64[];
    int cur = -1;
    for (uint32_t t = blockIdx.x; t < units; t += gridDim.x) {
        const EncUnit u = enc_unit<kPassPerLane>(F, nf, t, 2);
        if (!u.ok) continue;
        const FieldDesc& fd = F[u.f];
        const auto* dy = kconst(fd.dyn);
        const uint32_t nb = fd.n_bins;
        uint64_t* code_s = lds64;
        uint32_t* wbuf = (uint32_t*)(lds64 + (W ? 0 : nb));
        if (!W && u.f != cur) {
            for (uint32_t s = threadIdx.x; s < nb; s += kWave) code_s[s] = write_entry(fd.code[s]);
            cur = u.f;
        }
        auto entry = [&](uint32_t sym) { return W ? write_entry(fd.code[sym]) : code_s[sym]; };
        if (u.c >= u.nch) continue;
        const uint32_t wo = woff[fd.hch_base + u.c] - woff[fd.hch_base];
        EBC_G uint32_t* dst = (EBC_G uint32_t*)(fd.arc + dy->off_words) + wo;
        EBC_G uint16_t* sbits = (EBC_G uint16_t*)(fd.arc + dy->off_sbits);
        uint64_t done = 0;      // bits of the chunk already packed
        uint32_t carry = 0;     // the partial word at bit (done & ~31)
        uint32_t words_out = 0; // complete words stored
        for (uint32_t p = 0; p < fd.hc / kPassHc; ++p) {
            const uint64_t lo = (uint64_t)u.c * fd.hc + (uint64_t)p * kPassHc;
            if (lo >= u.cnt) break;
            uint32_t sym[kPassPerLane];
            load_pass(u, lo, sym);
            uint32_t mybits = 0;
#pragma unroll
            for (uint32_t k = 0; k < kPassPerLane; ++k)
                mybits += sym[k] == 0xFFFFFFFFu ? 0u : (uint32_t)entry(sym[k]) & 0xFFu;
            const uint32_t incl = wave_incl_scan_u32(mybits);
            const uint32_t pass_bits = (uint32_t)__shfl((int)incl, kWave - 1);
            // sub-chunk counts: 4 lanes of 64 symbols per 256-symbol sub-chunk
            constexpr uint32_t kLps = kSubMax / kPassPerLane;
            const uint32_t sb = (uint32_t)__shfl((int)incl, (int)min<uint32_t>(lane_id() + kLps - 1, 63)) -
                                (incl - mybits);
            const uint64_t sub = lo / fd.hs + lane_id() / kLps;
            const uint64_t l0 = lo + (uint64_t)lane_id() * kPassPerLane;
            if (lane_id() % kLps == 0 && l0 < u.cnt) sbits[sub] = (uint16_t)sb;
            // buffer word 0 holds the carried partial word
            const uint32_t head = (uint32_t)(done & 31);
            const uint32_t nbw = (head + pass_bits + 31) / 32;
            for (uint32_t i = lane_id(); i < nbw + 1; i += kWave) wbuf[i] = i == 0 ? carry : 0u;
            const uint32_t b0 = head + incl - mybits;
            uint32_t w = b0 >> 5, nacc = b0 & 31;
            uint64_t acc = 0;
#pragma unroll
            for (uint32_t k = 0; k < kPassPerLane; ++k) {
                if (sym[k] == 0xFFFFFFFFu) continue;
                const uint64_t v = entry(sym[k]);
                const uint32_t L = (uint32_t)v & 0xFFu;
                if (L <= 32) {
                    put_left(acc, nacc, w, wbuf, (uint32_t)(v >> 32), L);
                } else {
                    const uint64_t cw = fd.code[sym[k]] & ((1ull << 56) - 1);
                    put_bits(acc, nacc, w, wbuf, cw >> 32, L - 32);
                    put_bits(acc, nacc, w, wbuf, cw & 0xFFFFFFFFull, 32);
                }
            }
            if (nacc) atomicOr(&wbuf[w], (uint32_t)(acc >> 32));
            // complete words leave; the last partial one is carried
            const uint32_t full = (head + pass_bits) / 32;
            for (uint32_t i = lane_id(); i < full; i += kWave) dst[words_out + i] = wbuf[i];
            carry = wbuf[full];  // a wave's LDS accesses complete in order
            words_out += full;
            done += pass_bits;
        }
        if ((done & 31) && lane_id() == 0) dst[words_out] = carry;
    }
}

// ------------------------------------------------------------- decoding

__device__ __forceinline__ uint32_t word_at(const EBC_G uint32_t* __restrict__ w, uint32_t nw, uint32_t i)
{
    return i < nw ? w[i] : 0u;
}

// 64 stream bits starting at bit `pos` (zero beyond the lane's words)
__device__ __forceinline__ uint64_t window_at(const EBC_G uint32_t* __restrict__ w, uint32_t nw,
                                              uint32_t pos)
{
    const uint32_t k = pos >> 5, s = pos & 31;
    uint64_t a = ((uint64_t)word_at(w, nw, k) << 32) | word_at(w, nw, k + 1);
    if (s) a = (a << s) | (word_at(w, nw, k + 2) >> (32 - s));
    return a;
}

// Per-lane ring of a stream's 32-bit words in LDS, in two halves of one
// 16-byte block each.  The next block is always in flight in registers: at a
// wave-uniform refill point, every kRefillEvery steps, a lane whose reader
// has entered the newer half writes the loaded block over the older half and
// issues the load of the following one, so a load has a whole refill period
// to land and bit top-ups read LDS only.  A step takes at most one word, so
// between two refill points a reader advances at most kRefillEvery <=
// kHalfWords words and never leaves the ring.
constexpr uint32_t kRingWords = 8;
constexpr uint32_t kHalfWords = kRingWords / 2;
constexpr uint32_t kRingStride = kRingWords + 1;  // odd stride: no bank conflicts across lanes
constexpr uint32_t kRefillEvery = 4;              // steps between refill points (<= kHalfWords)
static_assert(kRefillEvery <= kHalfWords, "a reader must not outrun the ring between refills");

struct WordRing {
    uint32_t* ring;                       // this lane's slots in LDS
    const EBC_G uint4* __restrict__ blk;  // aligned 16-byte blocks of the stream
    uint32_t o, nblk;  // offset of the lane's word 0 inside block 0, blocks
    uint32_t rd;       // next stream word to hand out
    uint32_t wr;       // block-coordinate words [wr - kRingWords, wr) are in the ring
    uint4 p;           // block wr / 4, in flight
    __device__ __forceinline__ uint4 fetch(uint32_t j) const
    {
        if (j < nblk) {
            const uint4 v = blk[j];
            return v;
        }
        return make_uint4(0u, 0u, 0u, 0u);
    }
    // stream word rd (in the ring by the refill schedule); past the stream's
    // end the slot holds zeros or stale words, which a valid stream never uses
    __device__ __forceinline__ uint32_t peek() const { return ring[(rd + o) % kRingWords]; }
    __device__ __forceinline__ void put(uint32_t* d, uint4 v)
    {
        d[0] = v.x, d[1] = v.y, d[2] = v.z, d[3] = v.w;
    }
    __device__ __forceinline__ void init(uint32_t* r, const EBC_G uint32_t* __restrict__ w, uint32_t nw)
    {
        ring = r;
        const uintptr_t a = (uintptr_t)w;
        o = (uint32_t)((a & 15u) >> 2);
        blk = (const EBC_G uint4*)(a & ~(uintptr_t)15u);
        nblk = (o + nw + 3) / 4;
        put(ring, fetch(0));
        put(ring + 4, fetch(1));
        wr = kRingWords;
        p = fetch(2);
        rd = 0;
    }
    // wave-uniform refill point
    __device__ __forceinline__ void refill()
    {
        if (wr < 4 * nblk && rd + o >= wr - kHalfWords) {
            put(ring + (wr % kRingWords), p);
            wr += kHalfWords;
            p = fetch(wr / 4);
        }
    }
};

// One codeword longer than kLutBits at the head of a window: its length is
// kLutBits + 1 plus the number of code-space ends the window lies at or above.
// Returns the length (0 if the bits are not a codeword) and the symbol.
struct LongCode {
    uint32_t maxl;
    const uint64_t* s_endv;
    const uint64_t* s_first;
    const uint32_t* s_off;
    const uint16_t* perm;  // global: only codewords longer than both table levels get here
    __device__ __forceinline__ uint32_t decode(uint64_t w, uint32_t& sym) const
    {
        uint32_t L = kLutBits + 1;
        for (uint32_t l = kLutBits + 1; l < maxl; ++l) L += w >= s_endv[l] ? 1u : 0u;
        // the window is at or above the first length-L code by construction;
        // it must also be below the end of the length-L codes
        const uint64_t d = (w >> (64 - L)) - s_first[L];
        if (d >= (uint64_t)(s_off[L + 1] - s_off[L])) return 0;
        sym = perm[s_off[L] + (uint32_t)d];
        // wait for the symbol here: where the paths merge, a wait would also
        // cover every stream load and output store in flight
        asm volatile("" ::"v"(sym));
        return L;
    }
};

// Output staging: each lane collects its decoded symbols in an LDS row and
// the wave moves them to HBM in blocks of kFlush symbols per lane.  A block
// leaves when every lane still decoding holds one; the copy is transposed
// (four consecutive threads write one lane's 64-byte block), so a store
// instruction writes sixteen whole 64-byte segments.  A lane that runs
// kCap - 3 symbols ahead of its last flush waits (its steps are empty)
// until the slower lanes have caught up, which never delays the wave: the
// waiting lane is ahead of the slowest one.
constexpr uint32_t kFlush = 32;
constexpr uint32_t kCap = kFlush + 14;            // symbols a row holds; a step needs 3 free slots
constexpr uint32_t kStageWords = ((kCap + 4) / 2) | 1;  // row stride (odd): kCap + 3 slots and more
constexpr uint32_t kParts = kFlush / 8;           // 16-byte pieces of a flushed block
constexpr uint32_t kCheckEvery = 4;               // steps between flush checks
static_assert(2 * kStageWords >= kCap + 3, "the three slots of a step stay inside the row");
static_assert(kCap - 2 > kFlush, "a waiting lane always holds a whole block");
static_assert(kRefillEvery == kCheckEvery, "refill and flush checks share the step loop");

// One lane per sub-chunk (hs = min(hc, 256) symbols, its bit count and its
// start from the archive's sub-chunk counts), kDecLanes lanes per workgroup.
// The decoded stream is the field's quant-codes, or its run values (RLE+VLE).
// The main loop runs passes of kCheckEvery steps behind one refill point and
// one flush check.  A step tops the bit buffer up to at least 32 bits
// (branch-free, with the next stream word read from the ring one step
// ahead), takes one kLutBits table entry (up to three codewords) and writes
// its three symbol slots into the lane's row; only the decoded ones count.
// Codewords longer than the table go through a second-level table or the
// canonical limit test; longer than 32 bits, the lane leaves for an exact
// path that reads windows straight from the stream.
__global__ __launch_bounds__(kDecLanes) void k_huff_decode(const FieldDesc* __restrict__ F, int nf,
                                                          const uint32_t* __restrict__ woff,
                                                          const uint32_t* __restrict__ soff,
                                                          const uint8_t* __restrict__ tabs,
                                                          size_t tab_stride)
{
    // one block so that the table sits at LDS address 0 (its index needs no base)
    struct Lds {
        uint64_t lut[1u << kLutBits];
        uint64_t first[65];
        uint64_t endv[65];
        uint32_t l2s[kL2Size];
        uint32_t off[65];
        uint32_t ring[kDecLanes * kRingStride];
        uint32_t stage[kDecLanes * kStageWords];
    };
    __shared__ Lds sm;
    uint64_t* const lut = sm.lut;
    uint32_t* const l2s = sm.l2s;
    uint64_t* const s_first = sm.first;
    uint64_t* const s_endv = sm.endv;
    uint32_t* const s_off = sm.off;
    uint32_t* const s_ring = sm.ring;
    uint32_t* const s_stage = sm.stage;
    const uint32_t t = blockIdx.x;
    const int f = find_field<&FieldDesc::hdwg_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    EBC_G FieldDyn* dy = fd.dyn;
    if (dy->status != ST_OK || !huff_codec(dy->codec)) return;
    const DecTab* __restrict__ T = (const DecTab*)(tabs + (size_t)f * tab_stride);
    for (uint32_t i = threadIdx.x; i < (1u << kLutBits); i += kDecLanes) lut[i] = T->lut[i];
    const uint32_t l2k = T->l2k, l2n = T->l2n;
    const uint32_t l2sub = (1u << (kLutBits + l2k)) - l2n;  // first long prefix << l2k
    for (uint32_t i = threadIdx.x; i < l2n; i += kDecLanes) l2s[i] = T->l2[i];
    if (threadIdx.x < 65) {
        s_first[threadIdx.x] = T->first[threadIdx.x];
        s_endv[threadIdx.x] = T->endv[threadIdx.x];
        s_off[threadIdx.x] = T->offset[threadIdx.x];
    }
    const uint32_t maxl = T->max_len;
    __syncthreads();
    const uint32_t lane = lane_id();
    const uint32_t sub0 = (t - fd.hdwg_base) * kDecLanes + (threadIdx.x & ~(uint32_t)(kWave - 1));
    if (sub0 >= fd.n_sub) return;  // whole wave past the field's sub-chunks
    const uint32_t sub = sub0 + lane;
    const bool live = sub < fd.n_sub;
    const uint32_t hs = fd.hs, per = fd.hc / hs;
    const uint32_t c = live ? sub / per : 0;
    const EBC_G uint8_t* arc = fd.arc;
    const uint32_t nbits = live ? ((const EBC_G uint16_t*)(arc + fd.off_sbits))[sub] : 0u;
    // start bit of the sub-chunk inside the field's word stream
    const uint64_t b0 = live ? (uint64_t)(woff[fd.hch_base + c] - woff[fd.hch_base]) * 32 +
                                   soff[fd.sub_base + sub]
                             : 0ull;
    const uint64_t lo = (uint64_t)sub * hs;
    const uint32_t want = live ? (uint32_t)min<uint64_t>(hs, fd.hn - lo) : 0u;
    const uint32_t w0 = (uint32_t)(b0 >> 5);
    const uint32_t skip = (uint32_t)(b0 & 31);
    const uint32_t nwl = live ? (skip + nbits + 31) / 32 : 0u;  // words the lane may read
    // the chunk words were checked against the archive's word count, and a
    // sub-chunk ends inside its chunk by construction of the offsets
    const EBC_G uint32_t* __restrict__ words = (const EBC_G uint32_t*)(arc + fd.off_words) + w0;
    EBC_G uint16_t* __restrict__ out = fd.hsym + lo;
    const LongCode lc{maxl, s_endv, s_first, s_off, T->perm};
    uint32_t* row = s_stage + threadIdx.x * kStageWords;
    uint16_t* row16 = (uint16_t*)row;
    const uint32_t* wave_rows = s_stage + (threadIdx.x - lane) * kStageWords;

    WordRing wr;
    wr.init(s_ring + threadIdx.x * kRingStride, words, nwl);
    uint64_t buf = (uint64_t)wr.peek() << 32;
    ++wr.rd;
    buf |= wr.peek();
    ++wr.rd;
    buf <<= skip;
    uint32_t valid = 64 - skip;
    uint32_t j = 0, sp = 0, flushed = 0;
    uint32_t nflush = 0;  // flushes the wave has made
    bool slow = false;
    bool act = want > 0;
    uint32_t nxt = wr.peek();
    // a block of kFlush symbols leaves when every lane still decoding has one
    auto flush = [&]() {
        if (__all(sp >= kFlush || !act)) {
            // every lane holding a block has taken part in every flush so far
            // (a lane left out had stopped decoding with fewer than kFlush
            // symbols and never gains more), so its offset is wave-uniform
            const uint64_t has = ballot(sp >= kFlush);
            const uint32_t flw = (uint32_t)__builtin_amdgcn_readfirstlane((int)(nflush * kFlush));
#pragma unroll
            for (uint32_t k = 0; k < kParts; ++k) {
                const uint32_t piece = k * kWave + lane;
                const uint32_t L = piece / kParts, part = piece % kParts;
                if ((has >> L) & 1u) {
                    const uint32_t* src = wave_rows + L * kStageWords + part * 4;
                    const uint4 v = make_uint4(src[0], src[1], src[2], src[3]);
                    *(EBC_G uint4*)(fd.hsym + (uint64_t)(sub0 + L) * hs + flw + part * 8) = v;
                }
            }
            ++nflush;
            if (sp >= kFlush) {
                // the symbols past the block (at most kCap - kFlush) move to
                // the front of the row
#pragma unroll
                for (uint32_t w = 0; w < (kCap - kFlush + 1) / 2; ++w) row[w] = row[kFlush / 2 + w];
                sp -= kFlush;
                flushed += kFlush;
            }
        }
    };
    while (__any(act)) {
        wr.refill();
#pragma unroll
        for (uint32_t u = 0; u < kCheckEvery; ++u) {
            {
                const bool need = valid < 32;
                buf |= need ? ((uint64_t)nxt << ((32u - valid) & 63u)) : 0ull;
                valid += need ? 32u : 0u;
                wr.rd += need ? 1u : 0u;
                // only lanes that took a word read the next one (fewer LDS bank
                // accesses; the word at rd is in the ring by the refill schedule)
                if (need) nxt = wr.peek();
            }
            // the prefixes that start a codeword longer than the table are the
            // top nlong ones and own consecutive blocks in prefix order, so the
            // second-level index follows from the bits alone and its read
            // overlaps the table's (clamped: other lanes read entry 0)
            uint32_t i2 = ((uint32_t)(buf >> 32) >> (32 - kLutBits - l2k)) - l2sub;
            i2 = i2 < l2n ? i2 : 0u;
            const uint32_t v2 = l2s[i2];
            const uint64_t e = lut[(uint32_t)(buf >> (64 - kLutBits))];
            const uint32_t eh = (uint32_t)(e >> 32);
            // keeps the read above the branch; LDS reads return in order, so
            // the wait for the table entry covers it
            asm volatile("" ::"v"(v2), "v"(eh));
            uint32_t n = (eh >> 16) & 3u;
            uint32_t tl = (eh >> 18) & 63u;
            uint32_t s01 = (uint32_t)e, s2 = eh & 0xFFFFu;
            if (act && n == 0) {
                // second level, then the canonical search for longer codewords
                uint32_t sym = 0, L = 0;
                const uint32_t base = (uint32_t)e & 0xFFFFu;
                if (base != 0xFFFFu) {
                    const uint32_t v = v2;
                    L = v >> 16;
                    sym = v & 0xFFFFu;
                }
                if (L == 0) L = lc.decode(buf, sym);
                if (L == 0 || L > 32) {
                    slow = true;
                    act = false;
                }
                n = 1;
                tl = L;
                s01 = sym;
            }
            // the step's three symbol slots (only the decoded ones are kept;
            // sp <= kCap) in two LDS stores: the dword at halfword
            // (sp + 1) & ~1 and the halfword left over.  The LDS pipe, not the
            // VALU, bounds this loop: three halfword stores took 14% longer at
            // rel 1e-4, and one store of two dwords (with the previous symbol
            // kept in a register) was no faster than three.
            {
                const bool odd = (sp & 1u) != 0;
                // the halfword sits just before (odd sp) or just after the dword
                uint32_t* const dw = (uint32_t*)((char*)row + ((2 * sp + 2) & ~3u));
                *dw = odd ? (s01 >> 16) | (s2 << 16) : s01;
                *(uint16_t*)((char*)dw + (odd ? -2 : 4)) = (uint16_t)(odd ? s01 : s2);
            }
            const uint32_t left = want - j;
            if (__builtin_expect(act && n > left, 0)) {
                // the lane's last symbols take only the leading codewords (the
                // bit count is checked against the sub-chunk's); a branch taken
                // once per lane, kept out of the step by the empty asm
                tl = ((eh >> 24) & 15u) + (left == 2 ? eh >> 28 : 0u);
                n = left;
                asm volatile("" ::: "memory");
            }
            const bool go = act && sp + 3 <= kCap;
            n = go ? n : 0u;
            tl = go ? tl : 0u;
            j += n;
            sp += n;
            buf <<= tl;
            valid -= tl;
            act = act && j < want;
        }
        flush();
    }
    // exact path, one codeword at a time from a window read straight from the
    // stream (lanes that met a codeword longer than 32 bits)
    bool bad = false;
    uint32_t pos = 32 * wr.rd - valid;  // bits consumed, counted from word w0
    while (slow && j < want) {
        const uint64_t w = window_at(words, nwl, pos);
        const uint64_t e = lut[(uint32_t)(w >> (64 - kLutBits))];
        uint32_t sym = (uint32_t)e & 0xFFFFu;
        uint32_t L = (uint32_t)(e >> 56) & 15u;
        if (((e >> 48) & 3u) == 0) {
            L = 0;
            const uint32_t base = (uint32_t)e & 0xFFFFu;
            if (base != 0xFFFFu) {
                const uint32_t v = l2s[base + (uint32_t)((w << kLutBits) >> (64 - l2k))];
                L = v >> 16;
                sym = v & 0xFFFFu;
            }
            if (L == 0) L = lc.decode(w, sym);
            if (L == 0) {
                bad = true;
                break;
            }
        }
        row16[sp++] = (uint16_t)sym;
        ++j;
        pos += L;
        if (sp >= kCap) {
            // a full row: its leading block goes straight to HBM
            for (uint32_t k = 0; k < kFlush; ++k) out[flushed + k] = row16[k];
            for (uint32_t w = 0; w < kStageWords - kFlush / 2; ++w) row[w] = row[kFlush / 2 + w];
            sp -= kFlush;
            flushed += kFlush;
        }
    }
    if (!bad && live) {
        // what is left in the row: whole 16-byte groups, then single symbols
        uint32_t k = 0;
        for (; k + 8 <= sp; k += 8)
            *(EBC_G uint4*)(out + flushed + k) = make_uint4(row[k / 2], row[k / 2 + 1], row[k / 2 + 2],
                                                             row[k / 2 + 3]);
        for (; k < sp; ++k) out[flushed + k] = row16[k];
    }
    // the sub-chunk must take exactly its stored bit count
    if (live && (bad || pos != skip + nbits)) atomicMin(&dy->status, ST_ERR_ARCHIVE);
}

// Huffman decompression prologue, one thread per chunk: the in-chunk start
// bit of each of its sub-chunks (the running sum of the stored sub-chunk bit
// counts) and the chunk's word count (scanned next into word offsets).
__global__ __launch_bounds__(kBlock) void k_huff_prep(const FieldDesc* __restrict__ F, int nf,
                                                      uint32_t* __restrict__ wcnt,
                                                      uint32_t* __restrict__ soff)
{
    const uint32_t t = blockIdx.x;
    const int f = find_field<&FieldDesc::hpwg_base>(F, nf, t);
    const FieldDesc& fd = F[f];
    const uint32_t c = (t - fd.hpwg_base) * kBlock + threadIdx.x;
    if (!huff_codec(fd.dyn->codec) || c >= fd.n_hch) return;
    const uint32_t per = fd.hc / fd.hs;
    const uint32_t s0 = c * per, s1 = min(s0 + per, fd.n_sub);
    const EBC_G uint16_t* sb = (const EBC_G uint16_t*)(fd.arc + fd.off_sbits);
    uint32_t run = 0;
    for (uint32_t k = s0; k < s1; ++k) {
        soff[fd.sub_base + k] = run;
        run += sb[k];
    }
    wcnt[fd.hch_base + c] = (run + 31) / 32;
}

#define EBC_HC_DISPATCH(KERNEL, W, ...)                                                     \
    switch (hc) {                                                                           \
    case 64: hipLaunchKernelGGL((KERNEL<1, W>), __VA_ARGS__); break;                        \
    case 128: hipLaunchKernelGGL((KERNEL<2, W>), __VA_ARGS__); break;                       \
    case 256: hipLaunchKernelGGL((KERNEL<4, W>), __VA_ARGS__); break;                       \
    case 512: hipLaunchKernelGGL((KERNEL<8, W>), __VA_ARGS__); break;                       \
    case 1024: hipLaunchKernelGGL((KERNEL<16, W>), __VA_ARGS__); break;                     \
    case 2048: hipLaunchKernelGGL((KERNEL<32, W>), __VA_ARGS__); break;                     \
    case 4096: hipLaunchKernelGGL((KERNEL<64, W>), __VA_ARGS__); break;                     \
    default: return hipErrorInvalidValue;                                                   \
    }

// decompression: the scanned word counts must add up to the header's count
__global__ void k_words_check(const FieldDesc* __restrict__ F, int nf, const uint32_t* __restrict__ woff)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const FieldDesc& fd = F[f];
    if (!huff_codec(fd.codec_hdr)) return;
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

hipError_t launch_huff_bits(const FieldDesc* F, int nf, uint32_t units, uint32_t hc, uint32_t n_bins,
                            uint32_t* wcnt, int which, hipStream_t s)
{
    if (!units) return hipSuccess;
    const bool wide = n_bins > kMaxBins;
    const dim3 g(persistent_grid(units));
    if (hc > kPassHc) {
        if (wide) hipLaunchKernelGGL(k_huff_bits_long<true>, g, dim3(kWave), 0, s, F, nf, wcnt, units, which);
        else hipLaunchKernelGGL(k_huff_bits_long<false>, g, dim3(kWave), 0, s, F, nf, wcnt, units, which);
        return hipGetLastError();
    }
    const dim3 b(kWave * huff_cpw(hc));
    if (wide) {
        EBC_HC_DISPATCH(k_huff_bits, true, g, b, 0, s, F, nf, wcnt, units, which)
    } else {
        EBC_HC_DISPATCH(k_huff_bits, false, g, b, 0, s, F, nf, wcnt, units, which)
    }
    return hipGetLastError();
}

hipError_t launch_huff_write(const FieldDesc* F, int nf, uint32_t units, uint32_t hc,
                             uint32_t n_bins, const uint32_t* woff, hipStream_t s)
{
    if (!units) return hipSuccess;
    const bool wide = n_bins > kMaxBins;
    const dim3 g(persistent_grid(units));
    const size_t sh = huff_write_lds_bytes(n_bins, hc);
    if (hc > kPassHc) {
        if (wide) hipLaunchKernelGGL(k_huff_write_long<true>, g, dim3(kWave), sh, s, F, nf, woff, units);
        else hipLaunchKernelGGL(k_huff_write_long<false>, g, dim3(kWave), sh, s, F, nf, woff, units);
        return hipGetLastError();
    }
    const dim3 b(kWave * huff_cpw(hc));
    if (wide) {
        EBC_HC_DISPATCH(k_huff_write, true, g, b, sh, s, F, nf, woff, units)
    } else {
        EBC_HC_DISPATCH(k_huff_write, false, g, b, sh, s, F, nf, woff, units)
    }
    return hipGetLastError();
}

hipError_t launch_huff_prep(const FieldDesc* F, int nf, uint32_t units, uint32_t* wcnt, uint32_t* soff,
                            hipStream_t s)
{
    if (!units) return hipSuccess;
    hipLaunchKernelGGL(k_huff_prep, dim3(units), dim3(kBlock), 0, s, F, nf, wcnt, soff);
    return hipGetLastError();
}

hipError_t launch_huff_decode(const FieldDesc* F, int nf, uint32_t units, const uint32_t* woff,
                              const uint32_t* soff, const uint8_t* tabs, size_t tab_stride,
                              hipStream_t s)
{
    if (!units) return hipSuccess;
    hipLaunchKernelGGL(k_huff_decode, dim3(units), dim3(kDecLanes), 0, s, F, nf, woff, soff, tabs,
                       tab_stride);
    return hipGetLastError();
}

}  // namespace ebc
