// capi.cpp -- C ABI of the compressor: validation, planning, workspace
// carving and the kernel sequences for compression and decompression.
//
// Every call is a batch: fields are grouped by (rank, 16-byte row alignment)
// so each construct / reconstruct launch is specialised, and every other
// kernel covers all fields in one grid.  The host never looks at data between
// kernels: the codec decision, the outlier count, section offsets and the
// archive size are computed and consumed on the device; the plain compress
// call synchronises once at the end to return the size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "ebc.h"
#include "ebc_types.h"
#include "ebc_launch.h"

using namespace ebc;

namespace {

thread_local char g_err[512] = "";

int fail(int status, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return status;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(EBC_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

inline uint64_t a256(uint64_t v) { return (v + 255u) & ~(uint64_t)255u; }
inline uint64_t a16h(uint64_t v) { return (v + 15u) & ~(uint64_t)15u; }
inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }
inline uint32_t p2ceil(uint32_t v)
{
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

// ------------------------------------------------------------------ tuning
// The only global state: a table of tile choices per (rank, shape class),
// replaced as a whole by ebc_set_tuning.  Each API call takes one snapshot
// (TuneScope) so that workspace sizing and planning inside the call agree.
using TuneTable = std::vector<ebc_tuning_entry>;
std::mutex g_tune_mu;
std::shared_ptr<const TuneTable> g_tune;
thread_local const TuneTable* t_tune = nullptr;

struct TuneScope {
    std::shared_ptr<const TuneTable> snap;
    TuneScope()
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        snap = g_tune;
        t_tune = snap.get();
    }
    ~TuneScope() { t_tune = nullptr; }
};

void shape_class(int rank, const uint64_t dims[3], uint32_t* nxc, uint32_t* nc)
{
    uint32_t c = 0;
    while (c < 31 && (1ull << c) < dims[0]) ++c;
    const uint64_t n = dims[0] * (rank > 1 ? dims[1] : 1) * (rank > 2 ? dims[2] : 1);
    *nxc = c;
    *nc = n < (1ull << 20) ? 0u : n < (1ull << 24) ? 1u : 2u;
}

struct Tune {
    uint32_t wx, grid, scan;
};

Tune lookup_tune(int rank, const uint64_t dims[3])
{
    Tune t = {0, 0, 0};
    if (!t_tune) return t;
    uint32_t nxc, nc;
    shape_class(rank, dims, &nxc, &nc);
    for (const auto& e : *t_tune)
        if (e.rank == rank && e.nx_class == nxc && e.n_class == nc) {
            t.wx = e.tile_wx;
            t.grid = e.grid;
            t.scan = e.scan_direct;
        }
    return t;
}

// ------------------------------------------------------------------ params
struct Params {
    int eb_mode, codec;
    double eb;
    uint32_t n_bins, hc;
    int dtype;  // 0 fp32, 1 fp64 input
};

int check_params(const ebc_params* p, Params* out)
{
    if (!p) return fail(EBC_ERR_ARG, "params is NULL");
    if (p->eb_mode != EBC_EB_ABS && p->eb_mode != EBC_EB_REL) return fail(EBC_ERR_ARG, "bad eb_mode");
    if (p->codec < EBC_CODEC_AUTO || p->codec > EBC_CODEC_AUTO_VLE) return fail(EBC_ERR_ARG, "bad codec");
    if (p->dtype != EBC_F32 && p->dtype != EBC_F64) return fail(EBC_ERR_ARG, "bad data type");
    if (!(p->eb > 0.0) || !std::isfinite(p->eb)) return fail(EBC_ERR_EB, "eb must be finite and > 0");
    if (p->n_bins < 4 || p->n_bins > 65536 || (p->n_bins & 1))
        return fail(EBC_ERR_BINS, "n_bins must be even in [4, 65536]");
    const uint32_t hc = p->huff_chunk ? p->huff_chunk : 1024u;
    if (hc < 64 || hc > 65536 || (hc & (hc - 1)))
        return fail(EBC_ERR_ARG, "huff_chunk must be a power of two in [64, 65536]");
    out->eb_mode = p->eb_mode;
    out->codec = p->codec;
    out->eb = p->eb;
    out->n_bins = p->n_bins;
    out->hc = hc;
    out->dtype = p->dtype;
    return EBC_OK;
}

int check_dims(int rank, const uint64_t dims[3], uint64_t* n)
{
    if (!dims) return fail(EBC_ERR_ARG, "dims is NULL");
    if (rank < 1 || rank > 3) return fail(EBC_ERR_DIMS, "rank must be 1, 2 or 3");
    for (int k = 0; k < 3; ++k) {
        if (dims[k] == 0) return fail(EBC_ERR_DIMS, "zero dimension");
        if (k >= rank && dims[k] != 1) return fail(EBC_ERR_DIMS, "unused dimension must be 1");
        if (dims[k] >= (1ull << 32)) return fail(EBC_ERR_DIMS, "dimension too large");
    }
    uint64_t p = dims[0] * dims[1];
    if (p >= (1ull << 32)) return fail(EBC_ERR_DIMS, "N >= 2^32");
    p *= dims[2];
    if (p >= (1ull << 32)) return fail(EBC_ERR_DIMS, "N >= 2^32");
    *n = p;
    return EBC_OK;
}

// ------------------------------------------------------------------ geometry
// Waves along x in a construct / reconstruct workgroup tile: enough to cover
// nx (narrow fields stack the waves along y instead).
uint32_t choose_wx(int rank, uint64_t nx)
{
    if (rank == 1) return 1;
    const uint64_t wave_x = rank == 2 ? 64 : 32;
    const uint32_t want = p2ceil((uint32_t)std::min<uint64_t>((nx + wave_x - 1) / wave_x, 4));
    return std::max(1u, std::min(4u, want));
}

struct Geo {
    int rank;
    uint64_t nx, ny, nz, n;
    uint32_t wx, xs, nxb, nyb, nzb, n_wave_tiles, wg_tiles;
    uint32_t grid;  // persistent construction grid (workgroups)
    uint32_t scan;  // scan schedule: direct down-sweep up to this many tiles (0: default)
    uint32_t n_seg, range_units, ow_units, n_hch, hwg_units, hdwg_units, n_rt;
    uint32_t hs, n_sub, hpwg_units;
};

Geo make_geo(int rank, const uint64_t dims[3], uint32_t hc)
{
    Geo g = {};
    g.rank = rank;
    g.nx = dims[0], g.ny = dims[1], g.nz = dims[2];
    g.n = g.nx * g.ny * g.nz;
    const Tune t = lookup_tune(rank, dims);
    g.wx = rank > 1 && t.wx ? t.wx : choose_wx(rank, g.nx);
    g.grid = t.grid;  // 0: as many workgroups as the device holds at once
    g.scan = t.scan;
    if (rank == 1) {
        g.xs = 256;
        g.nxb = 1, g.nyb = 1, g.nzb = 1;
        g.n_wave_tiles = cdiv(g.n, 1024);
        g.wg_tiles = cdiv(g.n_wave_tiles, kWavesPerBlock);
        g.n_seg = cdiv(g.n, 256);
    } else {
        const uint32_t wy = kWavesPerBlock / g.wx;
        const uint32_t wave_x = rank == 2 ? 64 : 32, wave_y = rank == 2 ? 16 : 8;
        g.xs = wave_x * g.wx;
        g.nxb = cdiv(g.nx, g.xs);
        g.nyb = cdiv(g.ny, (uint64_t)wave_y * wy);
        g.nzb = rank == 3 ? cdiv(g.nz, 8) : 1;
        g.n_wave_tiles = 0;
        g.wg_tiles = g.nxb * g.nyb * g.nzb;
        g.n_seg = (uint32_t)(g.nz * g.ny * g.nxb);
    }
    g.range_units = cdiv(g.n, kRangeUnit);
    g.ow_units = outlier_write_units(g.n_seg);
    g.n_hch = cdiv(g.n, hc);
    g.hwg_units = cdiv(g.n_hch, huff_cpw(hc));
    g.hs = std::min(hc, kSubMax);
    g.n_sub = cdiv(g.n, g.hs);
    g.hdwg_units = cdiv(g.n_sub, kDecLanes);
    g.hpwg_units = cdiv(g.n_hch, kBlock);
    g.n_rt = cdiv(g.n, kRleTile);
    return g;
}

// ------------------------------------------------------------------ workspace
struct Bump {
    uint8_t* base;
    uint64_t off = 0;
    template <class T>
    T* take(uint64_t bytes)
    {
        T* p = base ? (T*)(base + off) : nullptr;
        off = a256(off + std::max<uint64_t>(bytes, 1));
        return p;
    }
};

struct Batch {
    int nf = 0;
    std::vector<FieldDesc> fd;    // sorted by (rank, vec)
    std::vector<int> order;       // fd[k] is caller field order[k]
    struct Group {
        int rank;
        bool vec;
        bool f64;
        int first, count;
        uint32_t wg_tiles;
        uint32_t blocks;  // construction grid
    };
    std::vector<Group> groups;
    uint32_t tot_range = 0, tot_seg = 0, tot_ow = 0, tot_hch = 0, tot_hwg = 0, tot_hdwg = 0,
             tot_rt = 0, tot_runs = 0, tot_sc = 0, tot_rl = 0, tot_fx = 0, tot_sub = 0, tot_hpwg = 0;
    uint32_t max_rle_units = 0;
    bool overflow = false;  // some work-unit total of the batch reached 2^32
    uint32_t scan = 0;      // scan schedule of the call (largest tuned value of its fields)
    FieldDesc* d_fd = nullptr;
    FieldDyn* d_dyn = nullptr;
    uint32_t *d_seg = nullptr, *d_wcnt = nullptr, *d_rcnt = nullptr, *d_starts = nullptr, *d_tmap = nullptr,
             *d_tmp = nullptr, *d_soff = nullptr;
    uint8_t* d_tabs = nullptr;
    size_t tab_stride = 0;  // decompress: decoder table bytes per field (largest n_bins of the batch)
    uint32_t max_bins = 0;
    uint64_t* d_result = nullptr;
    EstDev* d_est = nullptr;
    uint64_t ws_bytes = 0;
};

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// Group fields by (rank, vec) and assign every work-unit base.
// Default persistent construction grid for a (rank, layout) variant: the
// workgroups the device holds at once, cached per device and bin count.
uint32_t resident_grid(int rank, bool vec, uint32_t n_bins, bool f64)
{
    static std::mutex mu;
    static std::vector<std::pair<uint64_t, uint32_t>> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const uint64_t key = ((uint64_t)dev << 32) | ((uint64_t)n_bins << 4) | (f64 ? 8u : 0u) |
                         (uint64_t)(rank * 2 + (vec ? 1 : 0));
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const auto& kv : cache)
            if (kv.first == key) return kv.second;
    }
    uint32_t g = construct_resident_blocks(rank, vec, n_bins, f64);
    if (g == 0) g = kConstructBlocks;
    std::lock_guard<std::mutex> lk(mu);
    cache.push_back({key, g});
    return g;
}

// Work-unit totals are summed in 64 bits: a batch whose total in any index
// space reaches 2^32 cannot be addressed by the 32-bit unit indices of the
// kernels and is rejected by the caller (Batch::overflow).
struct Tot {
    uint64_t v = 0;
    bool* over;
    uint32_t add(uint64_t x)
    {
        const uint32_t base = (uint32_t)v;
        v += x;
        if (v >= 0xFFFFFFFFull) *over = true;
        return base;
    }
};

void assign_bases(Batch& B, const std::vector<Geo>& geo, const std::vector<bool>& vec,
                  const std::vector<int>& dt, uint32_t n_bins)
{
    const int nf = B.nf;
    std::vector<int> idx(nf);
    for (int i = 0; i < nf; ++i) idx[i] = i;
    // groups of one (data type, rank, row alignment): one specialised launch each
    auto key = [&](int i) { return dt[i] * 8 + geo[i].rank * 2 + (vec[i] ? 1 : 0); };
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return key(a) < key(b); });
    B.order = idx;
    B.groups.clear();
    B.overflow = false;
    bool* ov = &B.overflow;
    Tot range{0, ov}, seg{0, ov}, ow{0, ov}, hch{0, ov}, hwg{0, ov}, hdwg{0, ov}, rt{0, ov}, wg{0, ov},
        sub{0, ov}, hpwg{0, ov};
    for (int k = 0; k < nf; ++k) {
        const Geo& g = geo[idx[k]];
        const bool v = vec[idx[k]];
        const bool f64 = dt[idx[k]] == 1;
        if (B.groups.empty() || B.groups.back().rank != g.rank || B.groups.back().vec != v ||
            B.groups.back().f64 != f64) {
            B.groups.push_back({g.rank, v, f64, k, 0, 0, 0});
            wg.v = 0;
        }
        Batch::Group& G = B.groups.back();
        FieldDesc& d = B.fd[k];
        d.wg_base = wg.add(g.wg_tiles);
        d.wg_tiles = g.wg_tiles;
        G.wg_tiles = (uint32_t)wg.v;
        G.count++;
        d.range_base = range.add(g.range_units), d.range_units = g.range_units;
        d.seg_base = seg.add(g.n_seg), d.n_seg = g.n_seg;
        d.ow_base = ow.add(g.ow_units), d.ow_units = g.ow_units;
        d.hch_base = hch.add(g.n_hch), d.n_hch = g.n_hch;
        d.hwg_base = hwg.add(g.hwg_units), d.hwg_units = g.hwg_units;
        d.hdwg_base = hdwg.add(g.hdwg_units), d.hdwg_units = g.hdwg_units;
        d.hs = g.hs;
        d.sub_base = sub.add(g.n_sub), d.n_sub = g.n_sub;
        d.hpwg_base = hpwg.add(g.hpwg_units), d.hpwg_units = g.hpwg_units;
        d.rt_base = rt.add(g.n_rt), d.n_rt = g.n_rt;
        B.max_rle_units = std::max(B.max_rle_units, cdiv(g.n, kBlock));
    }
    B.tot_range = (uint32_t)range.v, B.tot_seg = (uint32_t)seg.v, B.tot_ow = (uint32_t)ow.v;
    B.tot_hch = (uint32_t)hch.v, B.tot_hwg = (uint32_t)hwg.v, B.tot_hdwg = (uint32_t)hdwg.v;
    B.tot_rt = (uint32_t)rt.v, B.tot_sub = (uint32_t)sub.v, B.tot_hpwg = (uint32_t)hpwg.v;
    B.scan = 0;
    for (int k = 0; k < nf; ++k) B.scan = std::max(B.scan, geo[k].scan);
    for (auto& G : B.groups) {
        uint32_t grid = 0;
        for (int k = G.first; k < G.first + G.count; ++k) grid = std::max(grid, geo[B.order[k]].grid);
        if (grid == 0) grid = n_bins ? resident_grid(G.rank, G.vec, n_bins, G.f64) : kConstructBlocks;
        G.blocks = std::min(G.wg_tiles, grid);
        for (int k = G.first; k < G.first + G.count; ++k)
            B.fd[k].hrows = std::min(B.fd[k].wg_tiles, G.blocks);
    }
}

void fill_geometry(FieldDesc& d, const Geo& g, bool vec)
{
    d.n = g.n;
    d.nx = (uint32_t)g.nx, d.ny = (uint32_t)g.ny, d.nz = (uint32_t)g.nz;
    d.rank = g.rank;
    d.wx = g.wx;
    d.xs = g.xs;
    d.nxb = g.nxb, d.nyb = g.nyb, d.nzb = g.nzb;
    d.n_wave_tiles = g.n_wave_tiles;
    d.vec = vec ? 1u : 0u;
}

// 3D reconstruction workgroup tiles: 256 x 32 x 8 (a wave per 8-row layer)
void recon3_tiles(const Geo& g, uint32_t t[3])
{
    t[0] = cdiv(g.nx, 256), t[1] = cdiv(g.ny, 32), t[2] = cdiv(g.nz, 8);
}

// Compression plan: geometry, bases and workspace carving (base == nullptr
// only sizes the workspace).
struct CompressIn {
    const void* in;
    int rank;
    uint64_t dims[3];
    void* out;
    uint64_t cap;
};

int plan_compress(Batch& B, const std::vector<CompressIn>& fin, const Params& P, uint8_t* ws)
{
    B.nf = (int)fin.size();
    B.fd.assign(B.nf, FieldDesc{});
    std::vector<Geo> geo(B.nf);
    std::vector<bool> vec(B.nf);
    std::vector<int> dt(B.nf, P.dtype);
    for (int i = 0; i < B.nf; ++i) {
        geo[i] = make_geo(fin[i].rank, fin[i].dims, P.hc);
        vec[i] = aligned16(fin[i].in) && (fin[i].rank == 1 || geo[i].nx % 4 == 0);
    }
    assign_bases(B, geo, vec, dt, P.n_bins);
    Bump bp{ws};
    B.d_fd = bp.take<FieldDesc>(sizeof(FieldDesc) * B.nf);
    B.d_dyn = bp.take<FieldDyn>(sizeof(FieldDyn) * B.nf);
    B.d_seg = bp.take<uint32_t>(4ull * (B.tot_seg + 1));
    B.d_wcnt = bp.take<uint32_t>(4ull * (B.tot_hch + 1));
    B.d_rcnt = bp.take<uint32_t>(4ull * (B.tot_rt + 1));
    const uint32_t big = std::max({B.tot_seg, B.tot_hch, B.tot_rt});
    B.d_tmp = bp.take<uint32_t>(4ull * scan_tmp_words(big));
    B.d_result = bp.take<uint64_t>(16);
    B.d_est = bp.take<EstDev>(sizeof(EstDev) * B.nf);
    for (int k = 0; k < B.nf; ++k) {
        const int i = B.order[k];
        const Geo& g = geo[i];
        FieldDesc& d = B.fd[k];
        fill_geometry(d, g, vec[i]);
        d.n_bins = P.n_bins;
        d.hc = P.hc;
        d.eb_mode = P.eb_mode;
        d.codec_req = P.codec;
        d.eb = P.eb;
        d.dtype = P.dtype;
        d.in = P.dtype == EBC_F32 ? (const float*)fin[i].in : nullptr;
        d.in64 = P.dtype == EBC_F64 ? (const double*)fin[i].in : nullptr;
        d.arc = (uint8_t*)fin[i].out;
        d.arc_cap = fin[i].cap;
        d.dyn = B.d_dyn ? B.d_dyn + k : nullptr;
        d.slot = (uint32_t)B.order[k];
        d.q = bp.take<uint16_t>(2 * g.n);
        d.dsc = bp.take<int32_t>(4 * g.n);
        d.rstart = (uint32_t*)d.dsc;  // used only after the outliers are written
        d.hist = bp.take<uint32_t>(4ull * P.n_bins);
        d.hpart = bp.take<uint32_t>(4ull * hist_slots(P.n_bins) * d.hrows);
        d.rpart = bp.take<uint32_t>(24ull * g.range_units);  // room for 64-bit keys
        d.code = bp.take<uint64_t>(8ull * P.n_bins);
        d.len = bp.take<uint8_t>(P.n_bins);
        d.cbs = P.n_bins > kMaxBins ? bp.take<uint8_t>(codebook_wide_scratch_bytes(P.n_bins)) : nullptr;
        d.hbits = bp.take<uint32_t>(4ull * g.n_hch);
        // RLE+VLE requested: the run values (at most N, and the encoder may
        // read 30 bytes past the stream) and their histogram
        const bool vle = P.codec == EBC_CODEC_RLE_VLE || P.codec == EBC_CODEC_AUTO_VLE;
        d.vsym = vle ? bp.take<uint16_t>(2 * g.n + 64) : nullptr;
        d.vhist = vle ? bp.take<uint32_t>(4ull * P.n_bins) : nullptr;
    }
    B.ws_bytes = bp.off;
    if (B.overflow) return fail(EBC_ERR_DIMS, "batch too large: a work-unit total reaches 2^32");
    return EBC_OK;
}

// ------------------------------------------------------------------ timing
struct Timer {
    ebc_stats* st;
    hipStream_t s;
    std::vector<hipEvent_t> ev;
    std::vector<const char*> names;
    bool on;
    const char* only = nullptr;  // time just this stage
    bool in_only = false;
    Timer(ebc_stats* st_, hipStream_t s_) : st(st_), s(s_), on(st_ && (st_->flags & EBC_STATS_TIMING))
    {
        if (on) only = st->time_only;
    }
    void mark(const char* name)
    {
        if (!on || names.size() >= EBC_MAX_STAGES) return;
        if (only) {
            // the event after the chosen stage closes it; nothing else is recorded
            const bool hit = strcmp(name, only) == 0;
            if (!hit && !in_only) return;
            in_only = hit;
        }
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        (void)hipEventRecord(e, s);
        ev.push_back(e);
        names.push_back(name);
    }
    // call after the stream has been synchronised
    void finish()
    {
        if (!on || ev.empty()) return;
        (void)hipEventSynchronize(ev.back());
        st->n_stages = 0;
        for (size_t k = 0; k + 1 < ev.size(); ++k) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
            st->stage_ms[k] = ms;
            st->stage_name[k] = names[k];
            st->n_stages = (uint32_t)(k + 1);
        }
    }
    ~Timer()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

// ------------------------------------------------------------------ pipelines
int enqueue_compress(Batch& B, const Params& P, hipStream_t s, Timer& T, bool debug_stop = false)
{
    const int nf = B.nf;
    HIP_TRY(upload_descs(B.fd.data(), nf, B.d_fd, s));
    T.mark("range");
    HIP_TRY(launch_range(B.d_fd, nf, B.tot_range, P.dtype == EBC_F64, s));
    T.mark("params");
    HIP_TRY(launch_params(B.d_fd, nf, s));
    T.mark("construct");
    for (const auto& G : B.groups)
        HIP_TRY(launch_construct(B.d_fd + G.first, G.count, G.rank, G.vec, G.f64, G.wg_tiles, G.blocks,
                                 P.n_bins, B.d_seg, s));
    T.mark("hist_reduce");
    HIP_TRY(launch_hist_reduce(B.d_fd, nf, P.n_bins, s));
    T.mark("scan_outliers");
    HIP_TRY(launch_scan(B.d_seg, B.tot_seg, B.d_tmp, s, B.scan));
    if (debug_stop) return EBC_OK;
    T.mark("codebook");
    HIP_TRY(launch_codebook(B.d_fd, nf, P.n_bins, 0, s));
    const bool vle = P.codec == EBC_CODEC_RLE_VLE || P.codec == EBC_CODEC_AUTO_VLE;
    T.mark("encode_count");
    HIP_TRY(launch_huff_bits(B.d_fd, nf, B.tot_hwg, P.hc, P.n_bins, B.d_wcnt, 0, s));
    HIP_TRY(launch_rle_count(B.d_fd, nf, B.tot_rt, B.d_rcnt, s));
    T.mark("encode_scan");
    HIP_TRY(launch_scan(B.d_rcnt, B.tot_rt, B.d_tmp, s, B.scan));
    if (vle) {
        // RLE+VLE fields: the run values become a stream of their own with a
        // codebook of their own, counted like the codes of a Huffman field
        T.mark("rle_vle");
        HIP_TRY(launch_rle_vle_prep(B.d_fd, nf, B.tot_rt, B.d_rcnt, P.n_bins, s));
        HIP_TRY(launch_codebook(B.d_fd, nf, P.n_bins, 1, s));
        HIP_TRY(launch_huff_bits(B.d_fd, nf, B.tot_hwg, P.hc, P.n_bins, B.d_wcnt, 1, s));
    }
    HIP_TRY(launch_scan(B.d_wcnt, B.tot_hch, B.d_tmp, s, B.scan));
    T.mark("layout");
    HIP_TRY(launch_layout(B.d_fd, nf, B.d_seg, B.d_wcnt, B.d_rcnt, s));
    T.mark("outlier_write");
    HIP_TRY(launch_outlier_write(B.d_fd, nf, B.tot_ow, B.d_seg, s));
    T.mark("encode_write");
    HIP_TRY(launch_huff_write(B.d_fd, nf, B.tot_hwg, P.hc, P.n_bins, B.d_wcnt, s));
    // run values of RLE fields into the archive, run starts of both run-length
    // codecs (they overwrite the outlier delta scratch, now written out)
    HIP_TRY(launch_rle_write(B.d_fd, nf, B.tot_rt, B.d_rcnt, 1 | 4, s));
    HIP_TRY(launch_rle_len(B.d_fd, nf, B.max_rle_units, s));
    T.mark("header");
    HIP_TRY(launch_header(B.d_fd, nf, s));
    return EBC_OK;
}

int compress_common(const std::vector<CompressIn>& fin, const ebc_params* p, void* d_ws,
                    uint64_t ws_bytes, hipStream_t s, Batch& B, Params& P)
{
    int st = check_params(p, &P);
    if (st) return st;
    for (const auto& f : fin) {
        uint64_t n;
        if (!f.in || !f.out) return fail(EBC_ERR_ARG, "NULL field or output pointer");
        st = check_dims(f.rank, f.dims, &n);
        if (st) return st;
    }
    if (!d_ws) return fail(EBC_ERR_ARG, "workspace is NULL");
    Batch sizing;
    if (int e_ = plan_compress(sizing, fin, P, nullptr)) return e_;
    if (ws_bytes < sizing.ws_bytes)
        return fail(EBC_ERR_WS_TOO_SMALL, "workspace %llu < required %llu",
                    (unsigned long long)ws_bytes, (unsigned long long)sizing.ws_bytes);
    if (int e_ = plan_compress(B, fin, P, (uint8_t*)d_ws)) return e_;
    return EBC_OK;
}

void fill_stats(ebc_stats* st, const FieldDyn& d, uint64_t n)
{
    if (!st) return;
    st->codec = d.codec;
    st->n_elems = n;
    st->n_outliers = d.n_out;
    st->n_runs = d.n_runs;
    st->n_words = d.n_words;
    st->huff_bits = d.huff_bits;
    st->out_bytes = d.total;
    st->eb_abs = d.eb_abs;
    st->ebx2 = d.ebx2;
    st->value_min = d.mn;
    st->value_max = d.mx;
}

// ------------------------------------------------------------------ decompress plan
struct Header {
    int rank, codec, eb_mode, dtype;
    uint32_t n_bins, hc, hs;
    uint64_t dims[3];
    uint32_t chunk[3];
    double eb, eb_abs, ebx2;
    double cval;
    uint64_t n_out, n_a, n_words, total;
    uint64_t n;
    uint64_t off_sbits, off_words, off_val, off_rlen, off_oidx, off_oval;
};

int parse_header(const void* h, uint64_t bytes, Header* H)
{
    if (!h) return fail(EBC_ERR_ARG, "header is NULL");
    if (bytes < kHdr) return fail(EBC_ERR_ARCHIVE, "archive shorter than its header");
    const uint8_t* a = (const uint8_t*)h;
    if (memcmp(a, "EBC1", 4) != 0) return fail(EBC_ERR_ARCHIVE, "bad magic");
    uint16_t ver;
    memcpy(&ver, a + 4, 2);
    if (ver != 2) return fail(EBC_ERR_ARCHIVE, "unsupported version %u", ver);
    H->rank = a[8], H->codec = a[9], H->eb_mode = a[10], H->dtype = a[11];
    memcpy(&H->n_bins, a + 12, 4);
    memcpy(H->dims, a + 16, 24);
    memcpy(H->chunk, a + 40, 12);
    memcpy(&H->hc, a + 52, 4);
    memcpy(&H->eb, a + 56, 8);
    memcpy(&H->eb_abs, a + 64, 8);
    memcpy(&H->ebx2, a + 72, 8);
    memcpy(&H->cval, a + 80, 8);
    memcpy(&H->n_out, a + 88, 8);
    memcpy(&H->n_a, a + 96, 8);
    memcpy(&H->n_words, a + 104, 8);
    memcpy(&H->total, a + 112, 8);
    memcpy(&H->hs, a + 120, 4);
    if (H->codec > 3) return fail(EBC_ERR_ARCHIVE, "bad codec byte");
    if (H->dtype > 1) return fail(EBC_ERR_ARCHIVE, "bad data type byte");
    if (H->rank < 1 || H->rank > 3) return fail(EBC_ERR_ARCHIVE, "bad rank");
    uint64_t n;
    if (check_dims(H->rank, H->dims, &n)) return fail(EBC_ERR_ARCHIVE, "bad dims");
    H->n = n;
    if (H->n_bins < 4 || H->n_bins > 65536 || (H->n_bins & 1)) return fail(EBC_ERR_ARCHIVE, "bad n_bins");
    if (H->hc < 64 || H->hc > 65536 || (H->hc & (H->hc - 1))) return fail(EBC_ERR_ARCHIVE, "bad chunk");
    if (H->codec == EBC_ARC_CONST) {
        if (H->total != kHdr) return fail(EBC_ERR_ARCHIVE, "bad constant archive size");
        return EBC_OK;
    }
    if (H->n_out > n) return fail(EBC_ERR_ARCHIVE, "outlier count exceeds N");
    if (H->codec == EBC_ARC_HUFFMAN) {
        const uint64_t nch = (n + H->hc - 1) / H->hc;
        if (H->n_a != nch) return fail(EBC_ERR_ARCHIVE, "chunk count mismatch");
        if (H->hs != std::min(H->hc, kSubMax)) return fail(EBC_ERR_ARCHIVE, "bad sub-chunk length");
        if (H->n_words > 2 * n + nch) return fail(EBC_ERR_ARCHIVE, "word count too large");
        const uint64_t nsub = (n + H->hs - 1) / H->hs;
        H->off_sbits = a16h(kHdr + H->n_bins);
        H->off_words = a16h(H->off_sbits + 2 * nsub);
        H->off_oidx = a16h(H->off_words + 4 * H->n_words);
    } else if (H->codec == EBC_ARC_RLE_VLE) {
        if (H->n_a > n || H->n_a == 0) return fail(EBC_ERR_ARCHIVE, "bad run count");
        if (H->hs != std::min(H->hc, kSubMax)) return fail(EBC_ERR_ARCHIVE, "bad sub-chunk length");
        const uint64_t nch = (H->n_a + H->hc - 1) / H->hc;
        if (H->n_words > 2 * H->n_a + nch) return fail(EBC_ERR_ARCHIVE, "word count too large");
        const uint64_t nsub = (H->n_a + H->hs - 1) / H->hs;
        H->off_sbits = a16h(kHdr + H->n_bins);
        H->off_words = a16h(H->off_sbits + 2 * nsub);
        H->off_rlen = a16h(H->off_words + 4 * H->n_words);
        H->off_oidx = a16h(H->off_rlen + 4 * H->n_a);
    } else {
        if (H->n_a > n || H->n_a == 0) return fail(EBC_ERR_ARCHIVE, "bad run count");
        if (H->n_words != 0) return fail(EBC_ERR_ARCHIVE, "RLE archive with Huffman words");
        H->off_val = kHdr;
        H->off_rlen = a16h(kHdr + 2 * H->n_a);
        H->off_oidx = a16h(H->off_rlen + 4 * H->n_a);
    }
    H->off_oval = a16h(H->off_oidx + 4 * H->n_out);
    const uint64_t total = a16h(H->off_oval + 4 * H->n_out);
    if (total != H->total) return fail(EBC_ERR_ARCHIVE, "section sizes do not add up");
    return EBC_OK;
}

int header_supported(const Header& H)
{
    if (H.codec == EBC_ARC_CONST) return EBC_OK;
    const uint32_t want[3][3] = {{256, 1, 1}, {16, 16, 1}, {8, 8, 8}};
    for (int k = 0; k < 3; ++k)
        if (H.chunk[k] != want[H.rank - 1][k])
            return fail(EBC_ERR_UNSUPPORTED, "non-default Lorenzo chunk not implemented");
    return EBC_OK;
}

struct DecompressIn {
    Header H;
    const void* arc;
    uint64_t size;
    void* out;  // elements of the archive's data type
    uint64_t out_elems;
};

int plan_decompress(Batch& B, const std::vector<DecompressIn>& din, uint8_t* ws)
{
    B.nf = (int)din.size();
    B.fd.assign(B.nf, FieldDesc{});
    std::vector<Geo> geo(B.nf);
    std::vector<bool> vec(B.nf);
    std::vector<int> dt(B.nf);
    for (int i = 0; i < B.nf; ++i) {
        const Header& H = din[i].H;
        geo[i] = make_geo(H.rank, H.dims, H.hc);
        vec[i] = aligned16(din[i].out) && (H.rank == 1 || geo[i].nx % 4 == 0);
        dt[i] = H.dtype;
    }
    assign_bases(B, geo, vec, dt, 0);  // no construction grid needed
    Bump bp{ws};
    B.d_fd = bp.take<FieldDesc>(sizeof(FieldDesc) * B.nf);
    B.d_dyn = bp.take<FieldDyn>(sizeof(FieldDyn) * B.nf);
    // per-codec unit counts (other codecs get zero units)
    bool* ov = &B.overflow;
    Tot hch{0, ov}, hdwg{0, ov}, rt{0, ov}, runs{0, ov}, sc{0, ov}, rl{0, ov}, fx{0, ov}, range{0, ov},
        sub{0, ov}, hpwg{0, ov};
    for (int k = 0; k < B.nf; ++k) {
        const DecompressIn& D = din[B.order[k]];
        const Header& H = D.H;
        FieldDesc& d = B.fd[k];
        const Geo& g = geo[B.order[k]];
        d.codec_hdr = H.codec;
        const bool huff = huff_codec(H.codec), rle = rle_codec(H.codec), cst = H.codec == EBC_ARC_CONST;
        // the Huffman stream: the N codes, or the run values of RLE+VLE
        const uint64_t hm = H.codec == EBC_ARC_RLE_VLE ? H.n_a : g.n;
        d.hn = huff ? hm : 0;
        d.hs = g.hs;
        d.n_hch = huff ? cdiv(hm, H.hc) : 0, d.hch_base = hch.add(d.n_hch);
        d.n_sub = huff ? cdiv(hm, g.hs) : 0, d.sub_base = sub.add(d.n_sub);
        d.hdwg_units = cdiv(d.n_sub, kDecLanes), d.hdwg_base = hdwg.add(d.hdwg_units);
        d.hpwg_units = cdiv(d.n_hch, kBlock), d.hpwg_base = hpwg.add(d.hpwg_units);
        d.n_rt = rle ? g.n_rt : 0, d.rt_base = rt.add(d.n_rt);
        d.n_runs_hdr = rle ? (uint32_t)H.n_a : 0, d.rle_base = runs.add(d.n_runs_hdr);
        d.rl_units = cdiv(d.n_runs_hdr, kBlock), d.rl_base = rl.add(d.rl_units);
        d.sc_units = cst ? 0 : cdiv(H.n_out, kBlock), d.sc_base = sc.add(d.sc_units);
        // 3D: at most one fix-up chunk per outlier, a wave each
        d.fx_units = (cst || H.rank != 3) ? 0 : cdiv(H.n_out, kWavesPerBlock);
        d.fx_base = fx.add(d.fx_units);
        d.range_units = cst ? g.range_units : 0, d.range_base = range.add(d.range_units);
        if (cst) {
            // no reconstruction work for a constant field
            d.wg_tiles = 0;
        }
    }
    B.tot_hch = (uint32_t)hch.v, B.tot_hdwg = (uint32_t)hdwg.v, B.tot_rt = (uint32_t)rt.v;
    B.tot_runs = (uint32_t)runs.v, B.tot_sc = (uint32_t)sc.v, B.tot_rl = (uint32_t)rl.v;
    B.tot_fx = (uint32_t)fx.v, B.tot_range = (uint32_t)range.v;
    B.tot_sub = (uint32_t)sub.v, B.tot_hpwg = (uint32_t)hpwg.v;
    // reconstruct groups: recount WG tiles without constant fields
    for (auto& G : B.groups) {
        Tot wg{0, ov};
        for (int k = G.first; k < G.first + G.count; ++k) {
            FieldDesc& d = B.fd[k];
            const Geo& g = geo[B.order[k]];
            uint32_t wt = d.codec_hdr == EBC_ARC_CONST ? 0 : g.wg_tiles;
            if (G.rank == 3 && wt) {
                uint32_t t3[3];
                recon3_tiles(g, t3);
                wt = t3[0] * t3[1] * t3[2];
            }
            d.wg_base = wg.add(wt);
            d.wg_tiles = wt;
        }
        G.wg_tiles = (uint32_t)wg.v;
        G.blocks = G.wg_tiles;  // one workgroup per tile
    }
    B.d_wcnt = bp.take<uint32_t>(4ull * (B.tot_hch + 1));
    B.d_soff = bp.take<uint32_t>(4ull * (B.tot_sub + 1));
    B.d_starts = bp.take<uint32_t>(4ull * (B.tot_runs + 1));
    B.d_tmap = bp.take<uint32_t>(8ull * (B.tot_rt + 1));  // (first run, run count) per tile
    B.d_tmp = bp.take<uint32_t>(4ull * scan_tmp_words(std::max(B.tot_hch, B.tot_runs)));
    B.max_bins = 0;
    for (int k = 0; k < B.nf; ++k) B.max_bins = std::max(B.max_bins, din[B.order[k]].H.n_bins);
    B.tab_stride = dectab_bytes(B.max_bins);
    B.d_tabs = bp.take<uint8_t>(B.tab_stride * B.nf);
    B.d_result = bp.take<uint64_t>(16);
    for (int k = 0; k < B.nf; ++k) {
        const DecompressIn& D = din[B.order[k]];
        const Header& H = D.H;
        const Geo& g = geo[B.order[k]];
        FieldDesc& d = B.fd[k];
        fill_geometry(d, g, vec[B.order[k]]);
        if (g.rank == 3) {
            // the 3D reconstruction kernel tiles differently from construction
            uint32_t t3[3];
            recon3_tiles(g, t3);
            d.nxb = t3[0], d.nyb = t3[1], d.nzb = t3[2];
        }
        d.n_bins = H.n_bins;
        d.hc = H.hc;
        d.eb_mode = H.eb_mode;
        d.eb = H.eb;
        d.outf = H.dtype == 0 ? (float*)D.out : nullptr;
        d.outd = H.dtype == 1 ? (double*)D.out : nullptr;
        d.arc = (uint8_t*)D.arc;
        d.arc_cap = D.size;
        d.dyn = B.d_dyn ? B.d_dyn + k : nullptr;
        d.slot = (uint32_t)B.order[k];
        d.n_out_hdr = H.n_out;
        d.n_words_hdr = H.n_words;
        d.ebx2_hdr = H.ebx2;
        d.cval = H.cval;
        d.dtype = H.dtype;
        d.off_sbits = H.off_sbits, d.off_words = H.off_words, d.off_val = H.off_val;
        d.off_rlen = H.off_rlen, d.off_oidx = H.off_oidx, d.off_oval = H.off_oval;
        const bool cst = H.codec == EBC_ARC_CONST;
        d.q = bp.take<uint16_t>(cst ? 0 : 2 * g.n);
        d.dsc = bp.take<int32_t>(cst ? 0 : 4 * g.n);
        // RLE+VLE: the decoded run values feed the run expansion
        d.vsym = bp.take<uint16_t>(H.codec == EBC_ARC_RLE_VLE ? 2 * H.n_a : 0);
        d.hsym = H.codec == EBC_ARC_RLE_VLE ? d.vsym : d.q;
        d.rval = H.codec == EBC_ARC_RLE_VLE ? d.vsym
                 : (d.arc ? (const uint16_t*)(d.arc + H.off_val) : nullptr);
        d.sink = bp.take<float>(256);
        const bool r3 = g.rank == 3 && !cst;
        d.oflag = bp.take<uint32_t>(r3 ? 4ull * d.nxb * d.nyb * kWavesPerBlock * d.nzb : 0);
        d.fixl = bp.take<uint32_t>(r3 ? 4ull * H.n_out : 0);
    }
    B.ws_bytes = bp.off;
    if (B.overflow) return fail(EBC_ERR_DIMS, "batch too large: a work-unit total reaches 2^32");
    return EBC_OK;
}

// Outlier scatter and reconstruction.  The 3D reconstruction reads no
// deltas and clears the chunk flags, so it runs before the scatter, which
// queues the chunks holding outliers for the fix-up; 1D/2D reconstruction
// fuses the scattered deltas itself.
int enqueue_reconstruct(Batch& B, hipStream_t s, Timer& T)
{
    bool has3 = false, has12 = false;
    for (const auto& G : B.groups) (G.rank == 3 ? has3 : has12) |= G.wg_tiles > 0;
    if (has3) T.mark("reconstruct");
    for (const auto& G : B.groups)
        if (G.rank == 3)
            HIP_TRY(launch_reconstruct(B.d_fd + G.first, G.count, G.rank, G.vec, G.f64, G.wg_tiles,
                                       G.blocks, s));
    if (B.tot_sc) T.mark("outlier_scatter");
    HIP_TRY(launch_outlier_scatter(B.d_fd, B.nf, B.tot_sc, s));
    if (has12) T.mark(has3 ? "reconstruct_12" : "reconstruct");
    for (const auto& G : B.groups)
        if (G.rank != 3)
            HIP_TRY(launch_reconstruct(B.d_fd + G.first, G.count, G.rank, G.vec, G.f64, G.wg_tiles,
                                       G.blocks, s));
    if (B.tot_fx) T.mark("outlier_fix");
    HIP_TRY(launch_recon_fix(B.d_fd, B.nf, B.tot_fx, s));
    return EBC_OK;
}

int enqueue_decompress(Batch& B, hipStream_t s, Timer& T)
{
    const int nf = B.nf;
    HIP_TRY(upload_descs(B.fd.data(), nf, B.d_fd, s));
    HIP_TRY(launch_dinit(B.d_fd, nf, s));
    T.mark("decode_prep");
    if (B.tot_hch) {
        HIP_TRY(launch_huff_prep(B.d_fd, nf, B.tot_hpwg, B.d_wcnt, B.d_soff, s));
        HIP_TRY(launch_scan(B.d_wcnt, B.tot_hch, B.d_tmp, s, B.scan));
        HIP_TRY(launch_words_check(B.d_fd, nf, B.d_wcnt, s));
        T.mark("dectab");
        HIP_TRY(launch_dectab(B.d_fd, nf, B.d_tabs, B.tab_stride, B.max_bins, s));
        T.mark("huffman_decode");
        HIP_TRY(launch_huff_decode(B.d_fd, nf, B.tot_hdwg, B.d_wcnt, B.d_soff, B.d_tabs, B.tab_stride, s));
    }
    if (B.tot_runs) {
        T.mark("rle_decode");
        HIP_TRY(launch_rle_decode(B.d_fd, nf, B.tot_rl, B.tot_rt, B.d_starts, B.d_tmap, B.d_tmp, B.tot_runs, B.scan, s));
    }
    const int st = enqueue_reconstruct(B, s, T);
    if (st) return st;
    T.mark("check");
    HIP_TRY(launch_recon_check(B.d_fd, nf, s));
    HIP_TRY(launch_fill_const(B.d_fd, nf, B.tot_range, s));
    return EBC_OK;
}

// Page-locked staging for the small device-to-host reads of the synchronous
// entry points: a copy into it is one DMA ordered on the stream, where a copy
// into pageable memory is staged by the runtime and starts late.  One buffer
// per host thread, grown on demand and kept for the life of the thread; NULL
// if page-locked memory is unavailable (the caller then reads into pageable
// memory).
void* pinned_stage(size_t bytes)
{
    thread_local void* p = nullptr;
    thread_local size_t cap = 0;
    if (bytes > cap) {
        const size_t want = std::max<size_t>(4096, (bytes + 4095) & ~size_t(4095));
        void* q = nullptr;
        if (hipHostMalloc(&q, want, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        if (p) (void)hipHostFree(p);
        p = q, cap = want;
    }
    return p;
}

// Synchronous device-to-host read of a few bytes on stream s.
int read_small(void* host, const void* dev, size_t bytes, hipStream_t s)
{
    void* stage = pinned_stage(bytes);
    HIP_TRY(hipMemcpyAsync(stage ? stage : host, dev, bytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (stage) memcpy(host, stage, bytes);
    return EBC_OK;
}

int read_dyn(const Batch& B, std::vector<FieldDyn>& dyn, hipStream_t s)
{
    dyn.resize(B.nf);
    return read_small(dyn.data(), B.d_dyn, sizeof(FieldDyn) * B.nf, s);
}

int status_of(const FieldDyn& d)
{
    if (d.status == ST_OK) return EBC_OK;
    switch (d.status) {
    case ST_ERR_NONFINITE: return fail(EBC_ERR_NONFINITE, "NaN or Inf in the field");
    case ST_ERR_EB_TOO_SMALL: return fail(EBC_ERR_EB_TOO_SMALL, "error bound below fp32 resolution of the field");
    case ST_ERR_EB: return fail(EBC_ERR_EB, "error bound out of range");
    case ST_ERR_OUT_TOO_SMALL: return fail(EBC_ERR_OUT_TOO_SMALL, "archive larger than the output buffer (%llu bytes needed)", (unsigned long long)d.total);
    case ST_ERR_ARCHIVE: return fail(EBC_ERR_ARCHIVE, "archive content is inconsistent");
    default: return fail(d.status, "device status %d", d.status);
    }
}

}  // namespace

int ebc::set_error(int status, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return status;
}

// ====================================================================== ABI
extern "C" {

int ebc_version(void) { return EBC_VERSION; }

int ebc_set_tuning(const ebc_tuning_entry* entries, int n)
{
    if (n < 0 || (n > 0 && !entries)) return fail(EBC_ERR_ARG, "bad tuning table");
    auto t = std::make_shared<TuneTable>();
    for (int i = 0; i < n; ++i) {
        const ebc_tuning_entry& e = entries[i];
        if (e.rank < 1 || e.rank > 3) return fail(EBC_ERR_ARG, "tuning entry %d: bad rank", i);
        if (e.tile_wx != 0 && e.tile_wx != 1 && e.tile_wx != 2 && e.tile_wx != 4)
            return fail(EBC_ERR_ARG, "tuning entry %d: tile_wx must be 0, 1, 2 or 4", i);
        if (e.grid != 0 && (e.grid < 64 || e.grid > 16384))
            return fail(EBC_ERR_ARG, "tuning entry %d: grid must be 0 or in [64, 16384]", i);
        if (e.scan_direct > (1u << 20))
            return fail(EBC_ERR_ARG, "tuning entry %d: scan_direct must be at most 2^20", i);
        t->push_back(e);
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (n == 0) g_tune.reset();
    else g_tune = t;
    return EBC_OK;
}

int ebc_shape_class(int rank, const uint64_t dims[3], uint32_t* nx_class, uint32_t* n_class)
{
    if (!nx_class || !n_class) return fail(EBC_ERR_ARG, "NULL argument");
    uint64_t n;
    int st = check_dims(rank, dims, &n);
    if (st) return st;
    shape_class(rank, dims, nx_class, n_class);
    return EBC_OK;
}

const char* ebc_status_string(int status)
{
    switch (status) {
    case EBC_OK: return "ok";
    case EBC_ERR_ARG: return "invalid argument";
    case EBC_ERR_DIMS: return "invalid dimensions";
    case EBC_ERR_EB: return "invalid error bound";
    case EBC_ERR_EB_TOO_SMALL: return "error bound too small for fp32 output";
    case EBC_ERR_BINS: return "invalid bin count";
    case EBC_ERR_NONFINITE: return "non-finite value in field";
    case EBC_ERR_OUT_TOO_SMALL: return "output buffer too small";
    case EBC_ERR_WS_TOO_SMALL: return "workspace too small";
    case EBC_ERR_ARCHIVE: return "corrupt or inconsistent archive";
    case EBC_ERR_HIP: return "HIP runtime error";
    case EBC_ERR_UNSUPPORTED: return "unsupported option";
    default: return "unknown status";
    }
}

const char* ebc_last_error(void) { return g_err; }

int ebc_compress_bound(int rank, const uint64_t dims[3], const ebc_params* p, uint64_t* max_bytes)
{
    TuneScope tune_scope;
    Params P;
    uint64_t n;
    if (!max_bytes) return fail(EBC_ERR_ARG, "max_bytes is NULL");
    int st = check_dims(rank, dims, &n);
    if (st) return st;
    st = check_params(p, &P);
    if (st && st != EBC_ERR_UNSUPPORTED) return st;
    const uint32_t hc = p->huff_chunk ? p->huff_chunk : 1024u;
    const uint64_t nch = (n + hc - 1) / hc, nsub = (n + std::min(hc, kSubMax) - 1) / std::min(hc, kSubMax);
    uint32_t lb = 0;
    while ((1ull << lb) < p->n_bins) ++lb;
    // a Huffman stream of N symbols: no more bits than a fixed-length code,
    // plus one partial word per chunk; RLE+VLE: such a stream over the run
    // values plus the run lengths
    const uint64_t huff = a16h(p->n_bins) + a16h(2 * nsub) + a16h(4 * ((n * lb + 31) / 32 + nch));
    const uint64_t rle = a16h(2 * n) + a16h(4 * n);
    const uint64_t rv = huff + a16h(4 * n);
    *max_bytes = kHdr + std::max({huff, rle, rv}) + a16h(4 * n) + a16h(4 * n);
    return EBC_OK;
}

int ebc_compress_workspace_size(int rank, const uint64_t dims[3], const ebc_params* p, uint64_t* bytes)
{
    TuneScope tune_scope;
    Params P;
    uint64_t n;
    if (!bytes) return fail(EBC_ERR_ARG, "bytes is NULL");
    int st = check_dims(rank, dims, &n);
    if (st) return st;
    st = check_params(p, &P);
    if (st) return st;
    std::vector<CompressIn> fin(1);
    fin[0] = {(const float*)nullptr, rank, {dims[0], dims[1], dims[2]}, nullptr, 0};
    Batch B;
    if (int e_ = plan_compress(B, fin, P, nullptr)) return e_;
    *bytes = B.ws_bytes;
    return EBC_OK;
}

int ebc_compress(const void* d_field, int rank, const uint64_t dims[3], const ebc_params* p,
                 void* d_out, uint64_t out_cap, uint64_t* out_size, void* d_ws, uint64_t ws_bytes,
                 void* stream, ebc_stats* stats)
{
    TuneScope tune_scope;
    if (!out_size) return fail(EBC_ERR_ARG, "out_size is NULL");
    *out_size = 0;
    if (!dims) return fail(EBC_ERR_ARG, "dims is NULL");
    hipStream_t s = (hipStream_t)stream;
    std::vector<CompressIn> fin(1);
    fin[0] = {d_field, rank, {dims[0], dims[1], dims[2]}, d_out, out_cap};
    Batch B;
    Params P;
    int st = compress_common(fin, p, d_ws, ws_bytes, s, B, P);
    if (st) return st;
    Timer T(stats, s);
    st = enqueue_compress(B, P, s, T);
    if (st) return st;
    T.mark("end");
    if (stats) HIP_TRY(launch_estimate(B.d_fd, 1, B.d_est, 0, 0, s));  // after the timed stages
    std::vector<FieldDyn> dyn;
    st = read_dyn(B, dyn, s);
    if (st) return st;
    T.finish();
    fill_stats(stats, dyn[0], B.fd[0].n);
    if (stats && dyn[0].status == ST_OK && dyn[0].codec != ARC_CONST) {
        EstDev e;
        st = read_small(&e, B.d_est, sizeof(EstDev), s);
        if (st) return st;
        stats->entropy = e.entropy, stats->p1 = e.p1, stats->r_lo = e.r_lo, stats->r_hi = e.r_hi;
        stats->predict = e.predict;
    }
    st = status_of(dyn[0]);
    if (st) return st;
    *out_size = dyn[0].total;
    return EBC_OK;
}

int ebc_compress_async(const void* d_field, int rank, const uint64_t dims[3], const ebc_params* p,
                       void* d_out, uint64_t out_cap, uint64_t* d_result, void* d_ws,
                       uint64_t ws_bytes, void* stream)
{
    TuneScope tune_scope;
    if (!d_result || !dims) return fail(EBC_ERR_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    std::vector<CompressIn> fin(1);
    fin[0] = {d_field, rank, {dims[0], dims[1], dims[2]}, d_out, out_cap};
    Batch B;
    Params P;
    int st = compress_common(fin, p, d_ws, ws_bytes, s, B, P);
    if (st) return st;
    Timer T(nullptr, s);
    st = enqueue_compress(B, P, s, T);
    if (st) return st;
    HIP_TRY(launch_result(B.d_fd, d_result, s));
    return EBC_OK;
}

int ebc_archive_info(const void* h_header, uint64_t header_bytes, int* rank, uint64_t dims[3],
                     ebc_params* p, int* codec, uint64_t* total_bytes)
{
    Header H;
    int st = parse_header(h_header, header_bytes, &H);
    if (st) return st;
    if (rank) *rank = H.rank;
    if (dims) memcpy(dims, H.dims, sizeof(H.dims));
    if (p) {
        p->eb_mode = H.eb_mode;
        p->codec = EBC_CODEC_AUTO;
        p->eb = H.eb;
        p->n_bins = H.n_bins;
        p->huff_chunk = H.hc;
        p->dtype = H.dtype;
        p->reserved = 0;
    }
    if (codec) *codec = H.codec;
    if (total_bytes) *total_bytes = H.total;
    return EBC_OK;
}

int ebc_decompress_workspace_size(const void* h_header, uint64_t header_bytes, uint64_t* bytes)
{
    TuneScope tune_scope;
    if (!bytes) return fail(EBC_ERR_ARG, "bytes is NULL");
    std::vector<DecompressIn> din(1);
    int st = parse_header(h_header, header_bytes, &din[0].H);
    if (st) return st;
    st = header_supported(din[0].H);
    if (st) return st;
    din[0].arc = nullptr, din[0].out = nullptr, din[0].size = din[0].H.total, din[0].out_elems = 0;
    Batch B;
    if (int e_ = plan_decompress(B, din, nullptr)) return e_;
    *bytes = B.ws_bytes;
    return EBC_OK;
}

static int decompress_impl(const Header& H, const void* d_archive, uint64_t size, void* d_out,
                           uint64_t out_elems, void* d_ws, uint64_t ws_bytes, hipStream_t s,
                           Batch& B, Timer& T)
{
    if (!d_archive || !d_out || !d_ws) return fail(EBC_ERR_ARG, "NULL argument");
    int st = header_supported(H);
    if (st) return st;
    if (H.total > size) return fail(EBC_ERR_ARCHIVE, "archive truncated: %llu < %llu",
                                    (unsigned long long)size, (unsigned long long)H.total);
    if (out_elems < H.n) return fail(EBC_ERR_OUT_TOO_SMALL, "output holds %llu < %llu elements",
                                     (unsigned long long)out_elems, (unsigned long long)H.n);
    std::vector<DecompressIn> din(1);
    din[0] = {H, d_archive, size, d_out, out_elems};
    Batch sizing;
    if (int e_ = plan_decompress(sizing, din, nullptr)) return e_;
    if (ws_bytes < sizing.ws_bytes)
        return fail(EBC_ERR_WS_TOO_SMALL, "workspace %llu < required %llu",
                    (unsigned long long)ws_bytes, (unsigned long long)sizing.ws_bytes);
    if (int e_ = plan_decompress(B, din, (uint8_t*)d_ws)) return e_;
    return enqueue_decompress(B, s, T);
}

int ebc_decompress(const void* d_archive, uint64_t size, void* d_out, uint64_t out_elems,
                   void* d_ws, uint64_t ws_bytes, void* stream, ebc_stats* stats)
{
    TuneScope tune_scope;
    hipStream_t s = (hipStream_t)stream;
    if (!d_archive) return fail(EBC_ERR_ARG, "archive is NULL");
    if (size < kHdr) return fail(EBC_ERR_ARCHIVE, "archive shorter than its header");
    uint8_t hdr[kHdr];
    int st0 = read_small(hdr, d_archive, kHdr, s);
    if (st0) return st0;
    Header H;
    int st = parse_header(hdr, kHdr, &H);
    if (st) return st;
    Batch B;
    Timer T(stats, s);
    st = decompress_impl(H, d_archive, size, d_out, out_elems, d_ws, ws_bytes, s, B, T);
    if (st) return st;
    T.mark("end");
    std::vector<FieldDyn> dyn;
    st = read_dyn(B, dyn, s);
    if (st) return st;
    T.finish();
    if (stats) {
        stats->codec = H.codec;
        stats->n_elems = H.n;
        stats->n_outliers = H.n_out;
        stats->n_runs = H.codec == EBC_ARC_RLE ? H.n_a : 0;
        stats->n_words = H.n_words;
        stats->out_bytes = H.total;
        stats->eb_abs = H.eb_abs;
        stats->ebx2 = H.ebx2;
    }
    return status_of(dyn[0]);
}

int ebc_decompress_async(const void* h_header, const void* d_archive, uint64_t size, void* d_out,
                         uint64_t out_elems, void* d_ws, uint64_t ws_bytes, int32_t* d_status,
                         void* stream)
{
    TuneScope tune_scope;
    if (!d_status) return fail(EBC_ERR_ARG, "d_status is NULL");
    hipStream_t s = (hipStream_t)stream;
    Header H;
    int st = parse_header(h_header, kHdr, &H);
    if (st) return st;
    Batch B;
    Timer T(nullptr, s);
    st = decompress_impl(H, d_archive, size, d_out, out_elems, d_ws, ws_bytes, s, B, T);
    if (st) return st;
    HIP_TRY(launch_status(B.d_fd, d_status, s));
    return EBC_OK;
}

// ------------------------------------------------------------------ batch
int ebc_batch_compress_workspace_size(int n, const ebc_field* fields, const ebc_params* p,
                                      uint64_t* bytes)
{
    TuneScope tune_scope;
    if (n <= 0 || !fields || !bytes) return fail(EBC_ERR_ARG, "bad batch arguments");
    Params P;
    int st = check_params(p, &P);
    if (st) return st;
    std::vector<CompressIn> fin(n);
    for (int i = 0; i < n; ++i) {
        uint64_t cnt;
        st = check_dims(fields[i].rank, fields[i].dims, &cnt);
        if (st) return st;
        fin[i] = {fields[i].d_field, fields[i].rank,
                  {fields[i].dims[0], fields[i].dims[1], fields[i].dims[2]}, fields[i].d_out,
                  fields[i].out_cap};
    }
    Batch B;
    if (int e_ = plan_compress(B, fin, P, nullptr)) return e_;
    *bytes = B.ws_bytes;
    return EBC_OK;
}

int ebc_batch_compress(int n, const ebc_field* fields, const ebc_params* p, ebc_result* results,
                       void* d_ws, uint64_t ws_bytes, void* stream)
{
    TuneScope tune_scope;
    if (n <= 0 || !fields || !results) return fail(EBC_ERR_ARG, "bad batch arguments");
    hipStream_t s = (hipStream_t)stream;
    std::vector<CompressIn> fin(n);
    for (int i = 0; i < n; ++i)
        fin[i] = {fields[i].d_field, fields[i].rank,
                  {fields[i].dims[0], fields[i].dims[1], fields[i].dims[2]}, fields[i].d_out,
                  fields[i].out_cap};
    Batch B;
    Params P;
    int st = compress_common(fin, p, d_ws, ws_bytes, s, B, P);
    if (st) return st;
    Timer T(nullptr, s);
    st = enqueue_compress(B, P, s, T);
    if (st) return st;
    std::vector<FieldDyn> dyn;
    st = read_dyn(B, dyn, s);
    if (st) return st;
    int first_err = EBC_OK;
    for (int k = 0; k < n; ++k) {
        const int i = B.order[k];
        results[i].status = dyn[k].status;
        results[i].codec = dyn[k].codec;
        results[i].out_size = dyn[k].status == ST_OK ? dyn[k].total : 0;
        if (dyn[k].status != ST_OK && first_err == EBC_OK) first_err = status_of(dyn[k]);
    }
    return first_err;
}

static_assert(sizeof(ebc_result) == 16, "ebc_result is written by the device as two u64 words");

int ebc_batch_compress_async(int n, const ebc_field* fields, const ebc_params* p,
                             ebc_result* d_results, void* d_ws, uint64_t ws_bytes, void* stream)
{
    TuneScope tune_scope;
    if (n <= 0 || !fields || !d_results) return fail(EBC_ERR_ARG, "bad batch arguments");
    hipStream_t s = (hipStream_t)stream;
    std::vector<CompressIn> fin(n);
    for (int i = 0; i < n; ++i)
        fin[i] = {fields[i].d_field, fields[i].rank,
                  {fields[i].dims[0], fields[i].dims[1], fields[i].dims[2]}, fields[i].d_out,
                  fields[i].out_cap};
    Batch B;
    Params P;
    int st = compress_common(fin, p, d_ws, ws_bytes, s, B, P);
    if (st) return st;
    Timer T(nullptr, s);
    st = enqueue_compress(B, P, s, T);
    if (st) return st;
    HIP_TRY(launch_batch_results(B.d_fd, n, (uint64_t*)d_results, s));
    return EBC_OK;
}

static int batch_dec_inputs(int n, const ebc_archive_ref* refs, std::vector<DecompressIn>& din)
{
    if (n <= 0 || !refs) return fail(EBC_ERR_ARG, "bad batch arguments");
    din.resize(n);
    for (int i = 0; i < n; ++i) {
        int st = parse_header(refs[i].h_header, kHdr, &din[i].H);
        if (st) return st;
        st = header_supported(din[i].H);
        if (st) return st;
        din[i].arc = refs[i].d_archive;
        din[i].size = refs[i].size;
        din[i].out = refs[i].d_out;
        din[i].out_elems = refs[i].out_elems;
    }
    return EBC_OK;
}

int ebc_batch_decompress_workspace_size(int n, const ebc_archive_ref* refs, uint64_t* bytes)
{
    TuneScope tune_scope;
    if (!bytes) return fail(EBC_ERR_ARG, "bytes is NULL");
    std::vector<DecompressIn> din;
    int st = batch_dec_inputs(n, refs, din);
    if (st) return st;
    Batch B;
    if (int e_ = plan_decompress(B, din, nullptr)) return e_;
    *bytes = B.ws_bytes;
    return EBC_OK;
}

static int batch_dec_prepare(int n, const ebc_archive_ref* refs, void* d_ws, uint64_t ws_bytes,
                             hipStream_t s, Batch& B)
{
    if (!d_ws) return fail(EBC_ERR_ARG, "workspace is NULL");
    std::vector<DecompressIn> din;
    int st = batch_dec_inputs(n, refs, din);
    if (st) return st;
    for (const auto& D : din) {
        if (!D.arc || !D.out) return fail(EBC_ERR_ARG, "NULL archive or output");
        if (D.H.total > D.size) return fail(EBC_ERR_ARCHIVE, "archive truncated");
        if (D.out_elems < D.H.n) return fail(EBC_ERR_OUT_TOO_SMALL, "output too small");
    }
    Batch sizing;
    if (int e_ = plan_decompress(sizing, din, nullptr)) return e_;
    if (ws_bytes < sizing.ws_bytes) return fail(EBC_ERR_WS_TOO_SMALL, "workspace too small");
    if (int e_ = plan_decompress(B, din, (uint8_t*)d_ws)) return e_;
    Timer T(nullptr, s);
    return enqueue_decompress(B, s, T);
}

int ebc_batch_decompress(int n, const ebc_archive_ref* refs, int32_t* statuses, void* d_ws,
                         uint64_t ws_bytes, void* stream)
{
    TuneScope tune_scope;
    if (!statuses) return fail(EBC_ERR_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    Batch B;
    int st = batch_dec_prepare(n, refs, d_ws, ws_bytes, s, B);
    if (st) return st;
    std::vector<FieldDyn> dyn;
    st = read_dyn(B, dyn, s);
    if (st) return st;
    int first_err = EBC_OK;
    for (int k = 0; k < n; ++k) {
        statuses[B.order[k]] = dyn[k].status;
        if (dyn[k].status != ST_OK && first_err == EBC_OK) first_err = status_of(dyn[k]);
    }
    return first_err;
}

int ebc_batch_decompress_async(int n, const ebc_archive_ref* refs, int32_t* d_statuses, void* d_ws,
                               uint64_t ws_bytes, void* stream)
{
    TuneScope tune_scope;
    if (!d_statuses) return fail(EBC_ERR_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    Batch B;
    int st = batch_dec_prepare(n, refs, d_ws, ws_bytes, s, B);
    if (st) return st;
    HIP_TRY(launch_batch_status(B.d_fd, n, d_statuses, s));
    return EBC_OK;
}

// ------------------------------------------------------------------ estimates
int ebc_estimate(const void* d_field, int rank, const uint64_t dims[3], const ebc_params* p,
                 uint64_t samples, uint64_t seed, ebc_estimates* out, void* d_ws, uint64_t ws_bytes,
                 void* stream)
{
    TuneScope tune_scope;
    if (!out || !dims) return fail(EBC_ERR_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    std::vector<CompressIn> fin(1);
    fin[0] = {d_field, rank, {dims[0], dims[1], dims[2]}, (void*)d_ws, ~0ull};
    Batch B;
    Params P;
    int st = compress_common(fin, p, d_ws, ws_bytes, s, B, P);
    if (st) return st;
    Timer T(nullptr, s);
    st = enqueue_compress(B, P, s, T, true);  // up to the code histogram
    if (st) return st;
    HIP_TRY(launch_estimate(B.d_fd, 1, B.d_est, samples, seed, s));
    std::vector<FieldDyn> dyn;
    st = read_dyn(B, dyn, s);
    if (st) return st;
    st = status_of(dyn[0]);
    if (st) return st;
    if (dyn[0].codec == ARC_CONST) return fail(EBC_ERR_ARG, "constant field: no quant-codes");
    EstDev e;
    st = read_small(&e, B.d_est, sizeof(EstDev), s);
    if (st) return st;
    memset(out, 0, sizeof(*out));
    out->codec_hint = e.predict;
    out->entropy = e.entropy, out->p1 = e.p1, out->r_lo = e.r_lo, out->r_hi = e.r_hi;
    out->bits_lo = e.entropy + e.r_lo, out->bits_hi = e.entropy + e.r_hi;
    out->hist_max = e.hist_max;
    out->n_elems = B.fd[0].n;
    out->samples = samples;
    uint64_t ts = 0, tc = 0;
    for (uint32_t d = 0; d <= kMadoDist; ++d) {
        out->mado_sum[d] = e.mado_sum[d], out->mado_cnt[d] = e.mado_cnt[d];
        ts += e.mado_sum[d], tc += e.mado_cnt[d];
    }
    out->roughness = tc ? (double)ts / (double)tc : 0.0;
    return EBC_OK;
}

// ------------------------------------------------------------------ debug
int ebc_debug_construct(const void* d_field, int rank, const uint64_t dims[3], const ebc_params* p,
                        uint16_t* d_q, uint32_t* d_hist, uint32_t* d_oidx, int32_t* d_oval,
                        uint64_t* n_outliers, double* ebx2, void* d_ws, uint64_t ws_bytes,
                        void* stream)
{
    TuneScope tune_scope;
    if (!d_q || !d_hist || !d_oidx || !d_oval || !n_outliers || !dims)
        return fail(EBC_ERR_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    std::vector<CompressIn> fin(1);
    fin[0] = {d_field, rank, {dims[0], dims[1], dims[2]}, (void*)d_oidx, ~0ull};
    Batch B;
    Params P;
    int st = compress_common(fin, p, d_ws, ws_bytes, s, B, P);
    if (st) return st;
    Timer T(nullptr, s);
    st = enqueue_compress(B, P, s, T, true);
    if (st) return st;
    std::vector<FieldDyn> dyn;
    st = read_dyn(B, dyn, s);
    if (st) return st;
    st = status_of(dyn[0]);
    if (st) return st;
    const FieldDesc& d = B.fd[0];
    if (dyn[0].codec == ARC_CONST) return fail(EBC_ERR_ARG, "constant field: nothing constructed");
    // outlier count from the scanned segment counts, then compaction straight
    // into the caller's arrays (the "archive" base is d_oidx)
    uint32_t seg_tot[2];
    HIP_TRY(hipMemcpyAsync(seg_tot, B.d_seg + d.seg_base + d.n_seg, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(seg_tot + 1, B.d_seg + d.seg_base, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    FieldDyn nd = dyn[0];
    nd.n_out = seg_tot[0] - seg_tot[1];
    nd.off_oidx = 0;
    nd.off_oval = (uint64_t)((uintptr_t)d_oval - (uintptr_t)d_oidx);
    HIP_TRY(hipMemcpyAsync(B.d_dyn, &nd, sizeof(FieldDyn), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_outlier_write(B.d_fd, 1, B.tot_ow, B.d_seg, s));
    HIP_TRY(hipMemcpyAsync(d_q, d.q, 2 * d.n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_hist, d.hist, 4ull * P.n_bins, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    *n_outliers = nd.n_out;
    if (ebx2) *ebx2 = dyn[0].ebx2;
    return EBC_OK;
}

int ebc_debug_reconstruct(const uint16_t* d_q, const uint32_t* d_oidx, const int32_t* d_oval,
                          uint64_t n_outliers, int rank, const uint64_t dims[3], uint32_t n_bins,
                          double ebx2, float* d_out, void* d_ws, uint64_t ws_bytes, void* stream)
{
    TuneScope tune_scope;
    if (!d_q || !d_out || !dims || !d_ws || (n_outliers && (!d_oidx || !d_oval)))
        return fail(EBC_ERR_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    Header H = {};
    int st = check_dims(rank, dims, &H.n);
    if (st) return st;
    if (n_bins < 4 || n_bins > kBinsLimit || (n_bins & 1)) return fail(EBC_ERR_BINS, "bad n_bins");
    H.rank = rank;
    memcpy(H.dims, dims, sizeof(H.dims));
    H.codec = EBC_ARC_HUFFMAN;
    H.n_bins = n_bins;
    H.hc = 1024;
    H.ebx2 = ebx2;
    H.n_out = n_outliers;
    H.off_oidx = 0;
    const uintptr_t o_base = d_oidx ? (uintptr_t)d_oidx : (uintptr_t)d_q;
    H.off_oval = (uint64_t)((d_oval ? (uintptr_t)d_oval : o_base) - o_base);
    std::vector<DecompressIn> din(1);
    din[0] = {H, (const void*)o_base, ~0ull, d_out, H.n};
    Batch sizing;
    if (int e_ = plan_decompress(sizing, din, nullptr)) return e_;
    if (ws_bytes < sizing.ws_bytes) return fail(EBC_ERR_WS_TOO_SMALL, "workspace too small");
    Batch B;
    if (int e_ = plan_decompress(B, din, (uint8_t*)d_ws)) return e_;
    FieldDesc& d = B.fd[0];
    HIP_TRY(hipMemcpyAsync(d.q, d_q, 2 * H.n, hipMemcpyDeviceToDevice, s));
    d.n_hch = 0, d.hdwg_units = 0;  // no entropy decoding
    HIP_TRY(upload_descs(B.fd.data(), 1, B.d_fd, s));
    HIP_TRY(launch_dinit(B.d_fd, 1, s));
    Timer T(nullptr, s);
    st = enqueue_reconstruct(B, s, T);
    if (st) return st;
    HIP_TRY(launch_recon_check(B.d_fd, 1, s));
    std::vector<FieldDyn> dyn;
    st = read_dyn(B, dyn, s);
    if (st) return st;
    return status_of(dyn[0]);
}

}  // extern "C"
