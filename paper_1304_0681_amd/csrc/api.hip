// C ABI: context, argument validation, scratch management and dispatch.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "mlp_internal.h"

namespace hpgsw {

const ClassShape kDefaultClasses[kNumClasses] = {
    {16, 1, 16},  {32, 1, 32},  {64, 2, 32},    {100, 4, 25},   {128, 4, 32},   {160, 8, 20},
    {256, 8, 32}, {512, 16, 32}, {1024, 32, 32}, {2048, 64, 32}, {65535, 64, 32}};

int score_class_m_max(int cls) { return kDefaultClasses[cls].m_max; }

// Packed int16 is dispatched only for the shape it is verified on the GPU
// (4 lanes x 25 rows).  A call that ran the packed kernel for every class did
// not return; the kernel's source, run on the host for every shape on that
// call's pairs, is exact and in bounds, so the cause lies outside what the
// source shows and the other shapes stay off.
static bool packed_verified(const ClassShape &s) { return s.G == 4 && s.RPL == 25; }

}  // namespace hpgsw

using namespace hpgsw;

struct sw_ctx {
    int device = 0;
    int n_cu = 0;
    std::string err;
    // bucketing scratch
    void *bscratch = nullptr;
    size_t bscratch_bytes = 0;
    // strip boundary rows of the score kernel (allocated on first use)
    int2 *strip_buf = nullptr;
    int strip_waves = 0;
    // best-per-read keys
    uint64_t *keys = nullptr;
    size_t keys_n = 0;
    // traceback code slots: a fixed budget, sized once
    uint32_t *tb = nullptr;
    size_t tb_bytes = 0;
    size_t tb_budget = 2ull << 30;
    // inside sw_graph_begin / sw_graph_end: no allocation, no host synchronisation
    bool capturing = false;
    // graphs ended on this context and not yet destroyed: their kernel nodes hold
    // the current scratch pointers, so no scratch buffer may be freed or moved
    int live_graphs = 0;
    // device address of the allocation-free call's static scratch (null: none)
    void *static_scratch = nullptr;
    // filter scratch: read segments (first, last, count) and compaction offsets
    uint32_t *seg = nullptr;
    size_t seg_bytes = 0;
    // CAL joining scratch: windows, flags, compaction ids and scan words
    void *join = nullptr;
    size_t join_bytes = 0;
    // seeker scratch: scan tile sums, per-read region counts
    void *seek = nullptr;
    size_t seek_bytes = 0;
    // single-window split scratch: per-read words, keep flags, scan words
    void *sole = nullptr;
    size_t sole_bytes = 0;
    ClassShape shapes[kNumClasses];
    int blocks_per_cu[kNumClasses];
    ClassEdges edges;    // query-length class bounds of the score path
    bool int16 = true;   // packed int16 datapath where exact
    // phase timing: ev[0] before bucketing, ev[1] after it, ev[2 + c] after class c
    bool timing = false;
    bool timed_call = false;
    int32_t class_path[kNumClasses] = {};
    hipEvent_t ev[2 + kNumClasses] = {};
};

struct sw_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {

thread_local std::string g_noctx_err;

sw_status fail(sw_ctx *ctx, sw_status st, const char *fmt, ...) __attribute__((format(printf, 3, 4)));

sw_status fail(sw_ctx *ctx, sw_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_noctx_err = buf;
    return st;
}

#define HIP_TRY(ctx, expr)                                                                 \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail((ctx), e_ == hipErrorOutOfMemory ? SW_E_NOMEM : SW_E_DEVICE,       \
                        "%s: %s", #expr, hipGetErrorString(e_));                           \
    } while (0)

sw_status check_scoring(sw_ctx *ctx, const sw_scoring *sc)
{
    if (!sc)
        return fail(ctx, SW_E_INVALID, "scoring is NULL");
    if (sc->match <= 0 || sc->match > 127)
        return fail(ctx, SW_E_INVALID, "match must be in [1, 127]");
    if (sc->mismatch >= sc->match || sc->mismatch < -127)
        return fail(ctx, SW_E_INVALID, "mismatch must be in [-127, match)");
    if (sc->gap_open >= 0 || sc->gap_open < -127)
        return fail(ctx, SW_E_INVALID, "gap_open must be in [-127, -1]");
    if (sc->gap_extend > 0 || sc->gap_extend < sc->gap_open)
        return fail(ctx, SW_E_INVALID, "gap_extend must be in [gap_open, 0]");
    return SW_OK;
}

sw_status check_batch(sw_ctx *ctx, const sw_batch *b)
{
    if (!b)
        return fail(ctx, SW_E_INVALID, "batch is NULL");
    if (b->n_pairs == 0)
        return SW_OK;
    if (!b->d_win || !b->d_read_len || !b->d_read_off || !b->d_reads2b || !b->d_ref2b)
        return fail(ctx, SW_E_INVALID, "batch has a NULL device pointer");
    if (b->ref_len >= (1ull << 36))
        return fail(ctx, SW_E_RANGE, "reference longer than 2^36 bases");
    return SW_OK;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Grow a scratch buffer to at least `need` bytes.  `graph_visible`: the buffer
// may be referenced by a captured graph (every context scratch except the MLP
// training workspace, whose calls cannot be captured), so it may not move while
// such a graph is alive.
sw_status ensure(sw_ctx *ctx, void **buf, size_t *have, size_t need, bool graph_visible = true)
{
    if (*have >= need)
        return SW_OK;
    if (ctx->capturing)
        return fail(ctx, SW_E_STATE, "scratch of %zu bytes needed during graph capture: make the "
                    "same calls once before capturing", need);
    if (graph_visible && ctx->live_graphs > 0)
        return fail(ctx, SW_E_STATE, "scratch of %zu bytes needed while %d captured graph(s) of this "
                    "context still use the current scratch: destroy them first", need,
                    ctx->live_graphs);
    const size_t old = *have;
    if (*buf)
        HIP_TRY(ctx, hipFree(*buf));
    *buf = nullptr;
    *have = 0;
    size_t sz = std::max(need, old * 3 / 2);
    HIP_TRY(ctx, hipMalloc(buf, sz));
    *have = sz;
    return SW_OK;
}

// Bytes of the bucketing scratch for n_items pairs (layout of carve_bucket).
constexpr size_t bucket_bytes(size_t n_items)
{
    return ((4 * (n_items ? n_items : 1) + 255) & ~size_t(255)) * 2 +
           ((4 * kNumBins + 255) & ~size_t(255)) + 3 * ((4 * 2 * kNumClasses + 255) & ~size_t(255));
}

// Lay the bucketing scratch of n_items pairs out from `base` (bucket_bytes long).
void carve_bucket(void *base, uint32_t n_items, BucketScratch *s)
{
    const size_t n = std::max<uint32_t>(n_items, 1);
    char *p = static_cast<char *>(base);
    s->bin = reinterpret_cast<uint32_t *>(p);
    p += align_up(4 * n);
    s->ids = reinterpret_cast<uint32_t *>(p);
    p += align_up(4 * n);
    s->hist = reinterpret_cast<uint32_t *>(p);
    p += align_up(4 * kNumBins);
    s->seg = reinterpret_cast<uint32_t *>(p);
    p += align_up(4 * 2 * kNumClasses);
    s->counter = reinterpret_cast<uint32_t *>(p);
    p += align_up(4 * kNumClasses);
    s->maxlen = reinterpret_cast<uint32_t *>(p);
}

sw_status bucket_scratch(sw_ctx *ctx, uint32_t n_items, BucketScratch *s)
{
    sw_status st = ensure(ctx, &ctx->bscratch, &ctx->bscratch_bytes, bucket_bytes(n_items));
    if (st)
        return st;
    carve_bucket(ctx->bscratch, n_items, s);
    return SW_OK;
}

// ---------------------------------------------------------------------------
// Scratch of sw_batch_score_noalloc: a file-scope device array, so that the
// call needs no allocation.  Every GPU the library runs on holds its own copy
// from module load until the process ends.  Layout: the bucketing scratch of
// SW_NOALLOC_MAX_PAIRS pairs, then strip rows for kStaticStripWaves waves.
// Host code never uses the array's name as an address (on the host it names a
// stand-in, not device memory): sw_ctx_create looks its device address up once
// per device with hipGetSymbolAddress, and only that address is passed on.
// ---------------------------------------------------------------------------
constexpr int kStaticStripWaves = 8;
constexpr size_t kStaticStripOff = bucket_bytes(SW_NOALLOC_MAX_PAIRS);
constexpr size_t kStaticBytes = kStaticStripOff + sizeof(int2) * 65536ull * kStaticStripWaves;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kStaticBytes];

std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};   // device address of `scratch`, per device

// Device address of `scratch` on the current device `dev`, looked up once.
sw_status static_scratch_address(int dev, void **out)
{
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices)
        return SW_OK;       // such devices simply have no allocation-free path
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(nullptr, SW_E_DEVICE, "hipGetSymbolAddress(scratch): %s",
                        hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return SW_OK;
}

}  // namespace

extern "C" {

sw_status sw_ctx_create(int hip_device, sw_ctx **out)
{
    if (!out)
        return fail(nullptr, SW_E_INVALID, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0)
        return fail(nullptr, SW_E_NODEVICE, "no HIP device");
    if (hip_device < 0 || hip_device >= n)
        return fail(nullptr, SW_E_NODEVICE, "device %d does not exist (%d devices)", hip_device, n);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess)
        return fail(nullptr, SW_E_NODEVICE, "cannot query device %d", hip_device);
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, SW_E_NODEVICE, "device %d is %s, not gfx950", hip_device,
                    prop.gcnArchName);
    sw_ctx *ctx = new sw_ctx;
    ctx->device = hip_device;
    ctx->n_cu = prop.multiProcessorCount;
    for (int c = 0; c < kNumClasses; ++c) {
        ctx->shapes[c] = kDefaultClasses[c];
        ctx->blocks_per_cu[c] = 2;
    }
    ctx->edges = default_edges();
    if (hipSetDevice(hip_device) != hipSuccess) {
        delete ctx;
        return fail(nullptr, SW_E_DEVICE, "device set-up failed");
    }
    const sw_status st = static_scratch_address(hip_device, &ctx->static_scratch);
    if (st) {
        delete ctx;
        return st;
    }
    *out = ctx;
    return SW_OK;
}

sw_status sw_ctx_destroy(sw_ctx *ctx)
{
    if (!ctx)
        return SW_E_INVALID;
    hipError_t e = hipSetDevice(ctx->device);
    auto keep = [&e](hipError_t x) { if (e == hipSuccess) e = x; };
    keep(hipDeviceSynchronize());
    if (ctx->bscratch) keep(hipFree(ctx->bscratch));
    if (ctx->strip_buf) keep(hipFree(ctx->strip_buf));
    if (ctx->keys) keep(hipFree(ctx->keys));
    if (ctx->tb) keep(hipFree(ctx->tb));
    if (ctx->seg) keep(hipFree(ctx->seg));
    if (ctx->join) keep(hipFree(ctx->join));
    if (ctx->seek) keep(hipFree(ctx->seek));
    if (ctx->sole) keep(hipFree(ctx->sole));
    for (auto &ev : ctx->ev)
        if (ev) keep(hipEventDestroy(ev));
    delete ctx;
    if (e != hipSuccess)
        return fail(nullptr, SW_E_DEVICE, "sw_ctx_destroy: %s", hipGetErrorString(e));
    return SW_OK;
}

const char *sw_last_error(const sw_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_noctx_err.c_str();
}

sw_status sw_pack2b(sw_ctx *ctx, const uint8_t *d_ascii, uint64_t n, uint32_t *d_out,
                    uint32_t *d_bad, void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    if (n == 0)
        return SW_OK;
    if (!d_ascii || !d_out)
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_pack2b(d_ascii, n, d_out, d_bad, static_cast<hipStream_t>(stream)));
    return SW_OK;
}

}  // extern "C"

namespace {

// Arguments of a score call; SW_OK when the call has work to do (*work set).
sw_status check_score_call(sw_ctx *ctx, const sw_batch *b, const sw_scoring *sc, uint32_t flags,
                           sw_hit *d_hits, bool *work)
{
    *work = false;
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    sw_status st = check_batch(ctx, b);
    if (st)
        return st;
    if ((st = check_scoring(ctx, sc)))
        return st;
    if (flags & ~SW_WANT_ENDS)
        return fail(ctx, SW_E_INVALID, "unknown flags 0x%x", flags);
    if (b->n_pairs == 0)
        return SW_OK;
    if (!d_hits)
        return fail(ctx, SW_E_INVALID, "d_hits is NULL");
    *work = true;
    return SW_OK;
}

// Some read of the batch may exceed the largest single-strip class.
bool batch_may_strip(const sw_ctx *ctx, const sw_batch *b)
{
    return b->reads_len > (uint64_t)ctx->edges.m_max[kNumClasses - 2];
}

// Packed int16 runs only as verified on the GPU: the 4 x 25 tile on the class
// of queries of 65-100 bases (default bounds), where every score fits 16 bits.
bool use_packed(const sw_ctx *ctx, int c, const sw_scoring *sc)
{
    return ctx->int16 && c == 3 && ctx->edges.m_max[2] == 64 && ctx->edges.m_max[3] == 100 &&
           sc->mismatch <= 0 && (int64_t)sc->match * 100 <= 32767 && packed_verified(ctx->shapes[c]);
}

// Bucketing and the class kernels of one score call, on scratch the caller
// provides (strip rows for `strip_waves` waves of 65,536 entries each when the
// batch may hold strip-class reads).
sw_status score_dispatch(sw_ctx *ctx, const sw_batch *b, const sw_scoring *sc, uint32_t flags,
                         sw_hit *d_hits, hipStream_t s, const BucketScratch &bs, int2 *strip_buf,
                         int strip_waves)
{
    const bool may_strip = batch_may_strip(ctx, b);
    if (ctx->timing)
        HIP_TRY(ctx, hipEventRecord(ctx->ev[0], s));
    HIP_TRY(ctx, launch_bucket(*b, nullptr, b->n_pairs, bs, d_hits, nullptr, s, ctx->edges));
    if (ctx->timing)
        HIP_TRY(ctx, hipEventRecord(ctx->ev[1], s));
    ScoreParams p;
    p.ref = b->d_ref2b;
    p.ref_len = b->ref_len;
    p.ref_words = (b->ref_len + 15) / 16;
    p.reads = b->d_reads2b;
    p.read_words = (b->reads_len + 15) / 16;
    p.read_off = b->d_read_off;
    p.read_len = b->d_read_len;
    p.win = b->d_win;
    p.ids = bs.ids;
    p.seg = bs.seg;
    p.counter = bs.counter;
    p.ma = sc->match;
    p.mi = sc->mismatch;
    p.go = sc->gap_open;
    p.ge = sc->gap_extend;
    p.hits = d_hits;
    p.strip_buf = strip_buf;
    p.strip_stride = 65536;
    const bool ends = flags & SW_WANT_ENDS;
    for (int c = 0; c < kNumClasses; ++c) {
        const bool strip = c == kNumClasses - 1;
        const bool skip = (strip && !may_strip) ||
                          (!strip && c > 0 && (uint64_t)ctx->edges.m_max[c - 1] >= b->reads_len);
        ctx->class_path[c] = 0;
        if (skip) {     // no read of this batch can fall in this class
            if (ctx->timing)
                HIP_TRY(ctx, hipEventRecord(ctx->ev[2 + c], s));
            continue;
        }
        p.cls = c;
        const bool wide = (int64_t)sc->match * ctx->edges.m_max[c] >= 32768;
        const int mode = ends ? (wide ? 2 : 1) : 0;
        const int wpb = score_waves_per_block();
        const int grid = strip ? strip_waves / wpb : ctx->n_cu * ctx->blocks_per_cu[c];
        const bool packed = mode == 0 && use_packed(ctx, c, sc);
        if (packed)
            HIP_TRY(ctx, launch_score16_class(ctx->shapes[c].G, ctx->shapes[c].RPL, p, grid, s));
        else
            HIP_TRY(ctx, launch_score_class(c, ctx->shapes[c].G, ctx->shapes[c].RPL, mode, p, grid, s));
        ctx->class_path[c] = packed ? 3 : (mode ? 2 : 1);
        if (ctx->timing)
            HIP_TRY(ctx, hipEventRecord(ctx->ev[2 + c], s));
    }
    ctx->timed_call = ctx->timing;
    return SW_OK;
}

}  // namespace

extern "C" {

sw_status sw_batch_score(sw_ctx *ctx, const sw_batch *b, const sw_scoring *sc, uint32_t flags,
                         sw_hit *d_hits, void *stream)
{
    bool work = false;
    sw_status st = check_score_call(ctx, b, sc, flags, d_hits, &work);
    if (st || !work)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    BucketScratch bs;
    if ((st = bucket_scratch(ctx, b->n_pairs, &bs)))
        return st;
    if (batch_may_strip(ctx, b) && !ctx->strip_buf) {
        if (ctx->capturing || ctx->live_graphs > 0)
            return fail(ctx, SW_E_STATE, "strip buffers needed during graph capture or while a "
                        "captured graph is alive: make the same calls once before capturing");
        ctx->strip_waves = 64;
        HIP_TRY(ctx, hipMalloc(reinterpret_cast<void **>(&ctx->strip_buf),
                               sizeof(int2) * 65536ull * (size_t)ctx->strip_waves));
    }
    return score_dispatch(ctx, b, sc, flags, d_hits, s, bs, ctx->strip_buf, ctx->strip_waves);
}

sw_status sw_batch_score_noalloc(sw_ctx *ctx, const sw_batch *b, const sw_scoring *sc,
                                 uint32_t flags, sw_hit *d_hits, void *stream)
{
    bool work = false;
    sw_status st = check_score_call(ctx, b, sc, flags, d_hits, &work);
    if (st || !work)
        return st;
    if (b->n_pairs > SW_NOALLOC_MAX_PAIRS)
        return fail(ctx, SW_E_RANGE, "sw_batch_score_noalloc takes at most %u pairs, got %u",
                    SW_NOALLOC_MAX_PAIRS, b->n_pairs);
    if (!ctx->static_scratch)
        return fail(ctx, SW_E_STATE, "device %d has no static scratch (devices 0..%d only)",
                    ctx->device, kMaxDevices - 1);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    BucketScratch bs;
    carve_bucket(ctx->static_scratch, b->n_pairs, &bs);
    int2 *strip = reinterpret_cast<int2 *>(static_cast<char *>(ctx->static_scratch) + kStaticStripOff);
    return score_dispatch(ctx, b, sc, flags, d_hits, static_cast<hipStream_t>(stream), bs, strip,
                          kStaticStripWaves);
}

sw_status sw_best_per_read(sw_ctx *ctx, const sw_batch *b, const sw_hit *d_hits, int32_t t_map,
                           uint32_t *d_best_pair, int32_t *d_best_score, uint8_t *d_mapped,
                           void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    sw_status st = check_batch(ctx, b);
    if (st)
        return st;
    if (b->n_reads == 0)
        return SW_OK;
    if ((b->n_pairs && !d_hits) || !d_best_pair || !d_best_score)
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    size_t have = ctx->keys_n * 8;
    void *buf = ctx->keys;
    if ((st = ensure(ctx, &buf, &have, 8ull * b->n_reads)))
        return st;
    ctx->keys = static_cast<uint64_t *>(buf);
    ctx->keys_n = have / 8;
    HIP_TRY(ctx, launch_best(*b, d_hits, ctx->keys, t_map, d_best_pair, d_best_score, d_mapped,
                             static_cast<hipStream_t>(stream)));
    return SW_OK;
}

sw_status sw_sole_windows(sw_ctx *ctx, const sw_batch *b, uint32_t *d_sole, sw_window *d_win_out,
                          uint32_t *d_ids_out, uint32_t *d_n_out, void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    sw_status st = check_batch(ctx, b);
    if (st)
        return st;
    if (!d_n_out || (b->n_reads && !d_sole) || (b->n_pairs && (!d_win_out || !d_ids_out)))
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const size_t o_keep = align_up(8ull * std::max<uint32_t>(b->n_reads, 1));
    const size_t o_scan = o_keep + align_up(std::max<uint32_t>(b->n_pairs, 1));
    const size_t need = o_scan + align_up(4 * compact_scratch_words(b->n_pairs));
    void *buf = ctx->sole;
    size_t have = ctx->sole_bytes;
    if ((st = ensure(ctx, &buf, &have, need)))
        return st;
    ctx->sole = buf;
    ctx->sole_bytes = have;
    char *p = static_cast<char *>(buf);
    uint64_t *keys = reinterpret_cast<uint64_t *>(p);
    uint8_t *keep = reinterpret_cast<uint8_t *>(p + o_keep);
    uint32_t *scan = reinterpret_cast<uint32_t *>(p + o_scan);
    if (b->n_reads)
        HIP_TRY(ctx, launch_sole_windows(*b, keys, keep, d_sole, s));
    // with no reads no pair scores: the compaction of nothing writes the zero count
    HIP_TRY(ctx, compact_pairs(b->n_reads ? b->n_pairs : 0, keep, b->d_win, d_win_out, d_ids_out,
                               d_n_out, scan, s));
    return SW_OK;
}

sw_status sw_merge_best(sw_ctx *ctx, uint32_t n_reads, const uint32_t *d_sole,
                        const uint32_t *d_sub_best, const uint32_t *d_ids, uint32_t n_ids,
                        uint32_t *d_best_pair, void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    if (n_reads == 0)
        return SW_OK;
    if (!d_sole || !d_sub_best || !d_best_pair || (n_ids && !d_ids))
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_merge_best(n_reads, d_sole, d_sub_best, d_ids, n_ids, d_best_pair,
                                   static_cast<hipStream_t>(stream)));
    return SW_OK;
}

sw_status sw_select_windows(sw_ctx *ctx, const sw_batch *b, const uint32_t *d_pair_ids,
                            uint32_t n, sw_window *d_win_out, void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    sw_status st = check_batch(ctx, b);
    if (st)
        return st;
    if (n == 0)
        return SW_OK;
    if (!d_pair_ids || !d_win_out)
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_select_windows(*b, d_pair_ids, n, d_win_out, static_cast<hipStream_t>(stream)));
    return SW_OK;
}

sw_status sw_batch_traceback(sw_ctx *ctx, const sw_batch *b, const sw_scoring *sc,
                             const uint32_t *d_pair_ids, uint32_t n_sel, sw_aln *d_aln,
                             uint32_t *d_ops, uint32_t ops_stride, const sw_hit *d_hits,
                             void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    sw_status st = check_batch(ctx, b);
    if (st)
        return st;
    if ((st = check_scoring(ctx, sc)))
        return st;
    if (n_sel == 0)
        return SW_OK;
    if (!d_pair_ids || !d_aln || (!d_ops && ops_stride))
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    if (b->n_pairs == 0)
        return fail(ctx, SW_E_INVALID, "pair ids given for an empty batch");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    BucketScratch bs;
    if ((st = bucket_scratch(ctx, n_sel, &bs)))
        return st;
    // Code slots come from a fixed scratch budget; every class kernel sizes its
    // slots from the class maxima on the device and runs the waves that fit, so
    // the call needs no host round trip and can be captured in a graph.  Sized
    // before the first launch, so that a refused call changes nothing.
    void *buf = ctx->tb;
    size_t have = ctx->tb_bytes;
    if ((st = ensure(ctx, &buf, &have, ctx->tb_budget)))
        return st;
    ctx->tb = static_cast<uint32_t *>(buf);
    ctx->tb_bytes = have;
    const TbBand band{d_hits, sc->match, -sc->gap_open, -sc->gap_extend};
    const ClassEdges tb_edges = traceback_edges();
    HIP_TRY(ctx, launch_bucket(*b, d_pair_ids, n_sel, bs, nullptr, d_aln, s, tb_edges, band));
    const int wpb = traceback_waves_per_block();
    const int grid = std::max(1, ctx->n_cu * 16 / wpb);
    for (int c = 0; c < kNumClasses; ++c) {
        if (c > 0 && (uint64_t)tb_edges.m_max[c - 1] >= b->reads_len)
            continue;   // no read of this batch can fall in this class
        HIP_TRY(ctx, launch_traceback_class(c, *b, *sc, d_pair_ids, bs.ids, bs.seg, bs.counter,
                                            d_aln, d_ops, ops_stride, ctx->tb,
                                            std::min(ctx->tb_bytes, ctx->tb_budget) / 4, bs.maxlen,
                                            band, grid, s));
    }
    return SW_OK;
}

sw_status sw_graph_begin(sw_ctx *ctx, void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    if (!stream)
        return fail(ctx, SW_E_INVALID, "graph capture needs a created stream, not the null stream");
    if (ctx->capturing)
        return fail(ctx, SW_E_STATE, "a capture is already open on this context");
    if (ctx->timing)
        return fail(ctx, SW_E_STATE, "disable phase timing before capturing");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal));
    ctx->capturing = true;
    return SW_OK;
}

sw_status sw_graph_end(sw_ctx *ctx, void *stream, sw_graph **out)
{
    if (!ctx || !out)
        return fail(ctx, SW_E_INVALID, "NULL argument");
    if (!ctx->capturing)
        return fail(ctx, SW_E_STATE, "no capture is open on this context");
    ctx->capturing = false;
    *out = nullptr;
    hipGraph_t g = nullptr;
    HIP_TRY(ctx, hipStreamEndCapture(static_cast<hipStream_t>(stream), &g));
    hipGraphExec_t x = nullptr;
    const hipError_t e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(ctx, SW_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    *out = new sw_graph{g, x};
    ctx->live_graphs += 1;
    return SW_OK;
}

sw_status sw_graph_launch(sw_ctx *ctx, const sw_graph *g, void *stream)
{
    if (!ctx || !g)
        return fail(ctx, SW_E_INVALID, "NULL argument");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    return SW_OK;
}

sw_status sw_graph_destroy(sw_ctx *ctx, sw_graph *g)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    if (!g)
        return SW_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipError_t e = hipGraphExecDestroy(g->exec);
    const hipError_t e2 = hipGraphDestroy(g->graph);
    delete g;
    if (ctx->live_graphs > 0)
        ctx->live_graphs -= 1;
    if (e == hipSuccess)
        e = e2;
    if (e != hipSuccess)
        return fail(ctx, SW_E_DEVICE, "sw_graph_destroy: %s", hipGetErrorString(e));
    return SW_OK;
}

sw_status sw_ctx_set_option(sw_ctx *ctx, int option, int value)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    switch (option) {
    case SW_OPT_INT16:
        ctx->int16 = value != 0;
        return SW_OK;
    case SW_OPT_BLOCKS_PER_CU:
        if (value < 1 || value > 64)
            return fail(ctx, SW_E_RANGE, "blocks per CU must be in [1, 64]");
        for (int c = 0; c < kNumClasses; ++c)
            ctx->blocks_per_cu[c] = value;
        return SW_OK;
    case SW_OPT_TB_SCRATCH_MB:
        if (value < 1 || value > 65536)
            return fail(ctx, SW_E_RANGE, "traceback scratch must be in [1, 65536] MiB");
        ctx->tb_budget = (size_t)value << 20;
        return SW_OK;
    default:
        return fail(ctx, SW_E_INVALID, "unknown option %d", option);
    }
}

sw_status sw_timing_enable(sw_ctx *ctx, int on)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (on && !ctx->ev[0])
        for (auto &e : ctx->ev)
            HIP_TRY(ctx, hipEventCreate(&e));
    ctx->timing = on != 0;
    ctx->timed_call = false;
    return SW_OK;
}

sw_status sw_timing_get(sw_ctx *ctx, sw_timing *out)
{
    if (!ctx || !out)
        return fail(ctx, SW_E_INVALID, "NULL argument");
    if (!ctx->timing || !ctx->timed_call)
        return fail(ctx, SW_E_STATE, "no timed sw_batch_score call");
    HIP_TRY(ctx, hipEventSynchronize(ctx->ev[1 + kNumClasses]));
    memset(out, 0, sizeof *out);
    HIP_TRY(ctx, hipEventElapsedTime(&out->bucket_ms, ctx->ev[0], ctx->ev[1]));
    for (int c = 0; c < kNumClasses; ++c) {
        HIP_TRY(ctx, hipEventElapsedTime(&out->class_ms[c], ctx->ev[1 + c], ctx->ev[2 + c]));
        out->score_ms += out->class_ms[c];
        out->class_path[c] = ctx->class_path[c];
    }
    return SW_OK;
}

}  // extern "C"

namespace {

// The tiles the autotuner may pick, as (capacity, G, RPL): the default tile
// of every class, all of them run on the GPU by the parity tests.  (The 4 x 16
// and 8 x 13 tiles are instantiated too; they stay out of the search, see the
// design notes' list of what is switched off.)
const ClassShape kShapes[] = {{16, 1, 16},   {32, 1, 32},   {64, 2, 32},   {100, 4, 25},
                              {128, 4, 32},  {160, 8, 20},  {256, 8, 32},  {512, 16, 32},
                              {1024, 32, 32}, {2048, 64, 32}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

struct TuneChoice {
    ClassEdges edges;
    ClassShape shapes[kNumClasses];
    int bpc[kNumClasses];
};

TuneChoice current_choice(const sw_ctx *ctx)
{
    TuneChoice t;
    t.edges = ctx->edges;
    memcpy(t.shapes, ctx->shapes, sizeof t.shapes);
    memcpy(t.bpc, ctx->blocks_per_cu, sizeof t.bpc);
    return t;
}

void apply_choice(sw_ctx *ctx, const TuneChoice &t)
{
    ctx->edges = t.edges;
    memcpy(ctx->shapes, t.shapes, sizeof t.shapes);
    memcpy(ctx->blocks_per_cu, t.bpc, sizeof t.bpc);
}

TuneChoice default_choice()
{
    TuneChoice t;
    t.edges = default_edges();
    for (int c = 0; c < kNumClasses; ++c) {
        t.shapes[c] = kDefaultClasses[c];
        t.bpc[c] = 2;
    }
    return t;
}

// Smallest instantiated tile holding queries of up to m bases (the strip tile
// for longer ones).
ClassShape smallest_shape(int m)
{
    ClassShape best = kShapes[kNumShapes - 1];
    for (const ClassShape &s : kShapes)
        if (s.m_max >= m && s.m_max < best.m_max)
            best = s;
    return best;
}

// Time of every class of one score call of `b` under choice `t`, averaged over
// `reps` calls (HIP events on the call's stream).
sw_status time_choice(sw_ctx *ctx, const TuneChoice &t, const sw_batch *b, const sw_scoring *sc,
                      uint32_t flags, sw_hit *hits, int reps, void *stream, float *ms, int *path)
{
    apply_choice(ctx, t);
    for (int c = 0; c < kNumClasses; ++c) {
        ms[c] = 0.f;
        path[c] = 0;
    }
    for (int r = 0; r < reps; ++r) {
        sw_timing tm;
        sw_status st = sw_batch_score(ctx, b, sc, flags, hits, stream);
        if (!st)
            st = sw_timing_get(ctx, &tm);
        if (st)
            return st;
        for (int c = 0; c < kNumClasses; ++c) {
            ms[c] += tm.class_ms[c] / (float)reps;
            path[c] = tm.class_path[c];
        }
    }
    return SW_OK;
}

}  // namespace

extern "C" {

sw_status sw_autotune(sw_ctx *ctx, const sw_batch *b, const sw_scoring *sc, uint32_t flags,
                      int repeats, sw_tune_entry *out, void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    sw_status st = check_batch(ctx, b);
    if (st)
        return st;
    if ((st = check_scoring(ctx, sc)))
        return st;
    if (flags & ~SW_WANT_ENDS)
        return fail(ctx, SW_E_INVALID, "unknown flags 0x%x", flags);
    if (repeats < 1 || repeats > 100)
        return fail(ctx, SW_E_RANGE, "repeats must be in [1, 100]");
    if (ctx->capturing)
        return fail(ctx, SW_E_STATE, "sw_autotune cannot be captured");
    if (b->d_n_pairs)
        return fail(ctx, SW_E_INVALID, "sw_autotune takes a sample with a host pair count");
    static_assert(SW_NUM_CLASSES == kNumClasses, "class count of the ABI");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const TuneChoice keep = current_choice(ctx);
    const bool was_timing = ctx->timing;
    void *hits = nullptr;
    bool chosen = false;   // set once the tuned choice is in ctx; every earlier exit restores
    auto restore = [&]() {
        if (hits)
            (void)hipFree(hits);
        ctx->timing = was_timing;
        ctx->timed_call = false;
        if (!chosen)
            apply_choice(ctx, keep);
    };
    auto bail = [&](sw_status e) {
        restore();
        return e;
    };
    const TuneChoice def = default_choice();
    float def_ms[kNumClasses] = {}, cur_ms[kNumClasses] = {};
    int def_path[kNumClasses] = {}, cur_path[kNumClasses] = {};
    int n_cand[kNumClasses] = {};
    TuneChoice cur = def;
    bool populated[kNumClasses] = {}, populated_def[kNumClasses] = {};
    if (b->n_pairs) {
        const hipError_t e = hipMalloc(&hits, sizeof(sw_hit) * (size_t)b->n_pairs);
        if (e != hipSuccess)
            return bail(fail(ctx, SW_E_NOMEM, "sw_autotune: %s", hipGetErrorString(e)));
        if ((st = sw_timing_enable(ctx, 1)))
            return bail(st);
        // query length of every pair of the sample (host copies), for the
        // candidate class edges at its length quantiles
        std::vector<sw_window> win(b->n_pairs);
        std::vector<uint16_t> rlen(b->n_reads);
        HIP_TRY(ctx, hipStreamSynchronize(s));
        HIP_TRY(ctx, hipMemcpy(win.data(), b->d_win, sizeof(sw_window) * win.size(),
                               hipMemcpyDeviceToHost));
        if (b->n_reads)
            HIP_TRY(ctx, hipMemcpy(rlen.data(), b->d_read_len, 2ull * rlen.size(),
                                   hipMemcpyDeviceToHost));
        std::vector<int> lens;
        lens.reserve(win.size());
        for (const sw_window &w : win)
            if (w.read_id < b->n_reads && rlen[w.read_id] > 0)
                lens.push_back(rlen[w.read_id]);
        std::sort(lens.begin(), lens.end());
        // defaults (the first call also warms every kernel up)
        if ((st = time_choice(ctx, def, b, sc, flags, (sw_hit *)hits, 1, stream, def_ms, def_path)) ||
            (st = time_choice(ctx, def, b, sc, flags, (sw_hit *)hits, repeats, stream, def_ms,
                              def_path)))
            return bail(st);
        memcpy(cur_ms, def_ms, sizeof cur_ms);
        memcpy(cur_path, def_path, sizeof cur_path);
        auto pairs_in = [&](uint32_t lo, uint32_t hi) {   // pairs with lo < m <= hi
            return (size_t)(std::upper_bound(lens.begin(), lens.end(), (int)hi) -
                            std::upper_bound(lens.begin(), lens.end(), (int)lo));
        };
        for (int c = 0; c < kNumClasses; ++c)
            populated_def[c] = pairs_in(c ? def.edges.m_max[c - 1] : 0u, def.edges.m_max[c]) > 0;
        // 1. class edges: coordinate search over the bounds between classes k
        //    and k + 1, candidates at the tile capacities and length quantiles
        for (int k = 0; k + 2 < kNumClasses; ++k) {
            const uint32_t lo = k ? cur.edges.m_max[k - 1] : 0u, hi = cur.edges.m_max[k + 1];
            if (pairs_in(lo, hi) == 0)
                continue;
            std::vector<uint32_t> cands;
            for (const ClassShape &sh : kShapes)
                cands.push_back((uint32_t)sh.m_max);
            for (double q : {0.1, 0.25, 0.5, 0.75, 0.9}) {
                const size_t a = std::upper_bound(lens.begin(), lens.end(), (int)lo) - lens.begin();
                const size_t z = std::upper_bound(lens.begin(), lens.end(), (int)hi) - lens.begin();
                if (z > a)
                    cands.push_back((uint32_t)lens[a + (size_t)(q * (double)(z - a - 1))]);
            }
            std::sort(cands.begin(), cands.end());
            cands.erase(std::unique(cands.begin(), cands.end()), cands.end());
            float best = cur_ms[k] + cur_ms[k + 1];
            TuneChoice best_t = cur;
            for (uint32_t e : cands) {
                if (e <= lo || e >= hi || e == cur.edges.m_max[k] || e > 2048u)
                    continue;
                TuneChoice t = cur;
                t.edges.m_max[k] = e;
                if ((uint32_t)t.shapes[k].m_max < e || t.shapes[k].G * t.shapes[k].RPL < (int)e)
                    t.shapes[k] = smallest_shape((int)e);
                t.shapes[k].m_max = (int)e;
                float ms[kNumClasses];
                int path[kNumClasses];
                if ((st = time_choice(ctx, t, b, sc, flags, (sw_hit *)hits, repeats, stream, ms, path)))
                    return bail(st);
                n_cand[k] += 1;
                if (ms[k] + ms[k + 1] < best) {
                    best = ms[k] + ms[k + 1];
                    best_t = t;
                    memcpy(cur_ms, ms, sizeof cur_ms);
                    memcpy(cur_path, path, sizeof cur_path);
                }
            }
            cur = best_t;
        }
        // 2. tile and workgroups per compute unit of every populated class:
        //    the three smallest tiles that hold the class, at 1, 2, 4 per CU
        struct Cand {
            ClassShape shape;
            int bpc;
        };
        std::vector<Cand> cand[kNumClasses];
        size_t K = 0;
        for (int c = 0; c + 1 < kNumClasses; ++c) {
            std::vector<ClassShape> fit;
            for (const ClassShape &sh : kShapes)
                if ((uint32_t)sh.m_max >= cur.edges.m_max[c])
                    fit.push_back(sh);
            std::sort(fit.begin(), fit.end(), [](const ClassShape &x, const ClassShape &y) {
                return x.m_max < y.m_max || (x.m_max == y.m_max && x.G < y.G);
            });
            if (fit.size() > 3)
                fit.resize(3);
            for (ClassShape sh : fit) {
                sh.m_max = (int)cur.edges.m_max[c];
                for (int bpc : {1, 2, 4})
                    cand[c].push_back(Cand{sh, bpc});
            }
            K = std::max(K, cand[c].size());
        }
        for (int c = 0; c < kNumClasses; ++c)
            populated[c] = pairs_in(c ? cur.edges.m_max[c - 1] : 0u, cur.edges.m_max[c]) > 0;
        TuneChoice base = cur;
        for (size_t k = 0; k < K; ++k) {
            TuneChoice t = base;
            for (int c = 0; c + 1 < kNumClasses; ++c) {
                if (cand[c].empty())
                    continue;
                const Cand &x = cand[c][std::min(k, cand[c].size() - 1)];
                t.shapes[c] = x.shape;
                t.bpc[c] = x.bpc;
            }
            float ms[kNumClasses];
            int path[kNumClasses];
            if ((st = time_choice(ctx, t, b, sc, flags, (sw_hit *)hits, repeats, stream, ms, path)))
                return bail(st);
            for (int c = 0; c + 1 < kNumClasses; ++c) {
                if (k >= cand[c].size() || !path[c] || !populated[c])
                    continue;
                n_cand[c] += 1;
                if (ms[c] < cur_ms[c]) {
                    cur_ms[c] = ms[c];
                    cur_path[c] = path[c];
                    cur.shapes[c] = t.shapes[c];
                    cur.bpc[c] = t.bpc[c];
                }
            }
        }
        // 3. the choice as a whole against the defaults, both timed again side by
        //    side: per-class minima over noisy timings favour the candidates, and
        //    a choice that is not faster in total gives way to the defaults
        float fin_ms[kNumClasses], d2_ms[kNumClasses];
        int fin_path[kNumClasses], d2_path[kNumClasses];
        const int reps2 = std::min(2 * repeats, 100);
        if ((st = time_choice(ctx, cur, b, sc, flags, (sw_hit *)hits, reps2, stream, fin_ms,
                              fin_path)) ||
            (st = time_choice(ctx, def, b, sc, flags, (sw_hit *)hits, reps2, stream, d2_ms,
                              d2_path)))
            return bail(st);
        float fin_sum = 0.f, d2_sum = 0.f;
        for (int c = 0; c < kNumClasses; ++c) {
            fin_sum += fin_ms[c];
            d2_sum += d2_ms[c];
        }
        memcpy(def_ms, d2_ms, sizeof def_ms);
        if (fin_sum < 0.99f * d2_sum) {
            memcpy(cur_ms, fin_ms, sizeof cur_ms);
            memcpy(cur_path, fin_path, sizeof cur_path);
        } else {
            cur = def;
            memcpy(cur_ms, d2_ms, sizeof cur_ms);
            memcpy(cur_path, d2_path, sizeof cur_path);
            memcpy(populated, populated_def, sizeof populated);
        }
    }
    apply_choice(ctx, cur);
    if (out) {
        for (int c = 0; c < kNumClasses; ++c) {
            const int pth = populated[c] ? cur_path[c] : 0;   // 0: the sample left it empty
            out[c].m_max = (int32_t)cur.edges.m_max[c];
            out[c].G = cur.shapes[c].G;
            out[c].RPL = cur.shapes[c].RPL;
            out[c].blocks_per_cu = cur.bpc[c];
            out[c].path = pth;
            out[c].candidates = n_cand[c] + 1;
            out[c].ms = pth ? cur_ms[c] : 0.f;
            // class times under the tuned bounds and under the default ones (the
            // classes hold different pairs when a bound moved; each sum covers all)
            out[c].ms_default = populated_def[c] ? def_ms[c] : 0.f;
        }
    }
    chosen = true;
    const hipError_t e = hipStreamSynchronize(s);
    restore();
    if (e != hipSuccess)
        return fail(ctx, SW_E_DEVICE, "sw_autotune: %s", hipGetErrorString(e));
    return SW_OK;
}

}  // extern "C"

namespace {

uint64_t fnv1a(const void *p, size_t n, uint64_t h = 1469598103934665603ull)
{
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Cache key of a tuning: the device (architecture, compute units), the scoring,
// the flags, and the sample's length profile (share of pairs per query-length
// bin of 8 bases and per window-length bin of 64 bases, in thousandths, and
// the order of magnitude of the pair count).
sw_status tune_key(sw_ctx *ctx, const sw_batch *b, const sw_scoring *sc, uint32_t flags,
                   std::string *key)
{
    std::vector<sw_window> win(b->n_pairs);
    std::vector<uint16_t> rlen(b->n_reads);
    if (b->n_pairs)
        HIP_TRY(ctx, hipMemcpy(win.data(), b->d_win, sizeof(sw_window) * win.size(),
                               hipMemcpyDeviceToHost));
    if (b->n_reads)
        HIP_TRY(ctx, hipMemcpy(rlen.data(), b->d_read_len, 2ull * rlen.size(), hipMemcpyDeviceToHost));
    uint32_t hm[64] = {}, hn[32] = {};
    size_t n = 0;
    for (const sw_window &w : win) {
        if (w.read_id >= b->n_reads)
            continue;
        hm[std::min<uint32_t>(rlen[w.read_id] / 8u, 63u)] += 1;
        hn[std::min<uint32_t>(w.len / 64u, 31u)] += 1;
        ++n;
    }
    uint16_t prof[96 + 1];
    for (int i = 0; i < 64; ++i)
        prof[i] = (uint16_t)(n ? (hm[i] * 1000ull + n / 2) / n : 0);
    for (int i = 0; i < 32; ++i)
        prof[64 + i] = (uint16_t)(n ? (hn[i] * 1000ull + n / 2) / n : 0);
    int mag = 0;
    while ((1ull << mag) < (unsigned long long)n)
        ++mag;
    prof[96] = (uint16_t)mag;
    hipDeviceProp_t prop;
    HIP_TRY(ctx, hipGetDeviceProperties(&prop, ctx->device));
    char buf[256];
    snprintf(buf, sizeof buf, "%.16s/%dcu/sc%d,%d,%d,%d/f%u/%016llx", prop.gcnArchName, ctx->n_cu,
             sc->match, sc->mismatch, sc->gap_open, sc->gap_extend, flags,
             (unsigned long long)fnv1a(prof, sizeof prof));
    *key = buf;
    return SW_OK;
}

// Numbers of the JSON array `"name":[...]` in `line` (false if absent or short).
template <class T>
bool json_array(const std::string &line, const char *name, T *out, int n)
{
    const std::string tag = std::string("\"") + name + "\":[";
    size_t p = line.find(tag);
    if (p == std::string::npos)
        return false;
    const char *c = line.c_str() + p + tag.size();
    for (int i = 0; i < n; ++i) {
        char *end = nullptr;
        const double v = strtod(c, &end);
        if (end == c)
            return false;
        out[i] = (T)v;
        c = end;
        while (*c == ' ' || *c == ',')
            ++c;
    }
    return *c == ']';
}

}  // namespace

extern "C" {

sw_status sw_autotune_cached(sw_ctx *ctx, const sw_batch *b, const sw_scoring *sc, uint32_t flags,
                             int repeats, const char *cache_path, int *cache_hit,
                             sw_tune_entry *out, void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    if (!cache_path || !cache_path[0])
        return fail(ctx, SW_E_INVALID, "cache_path is empty");
    sw_status st = check_batch(ctx, b);
    if (st)
        return st;
    if ((st = check_scoring(ctx, sc)))
        return st;
    if (ctx->capturing)
        return fail(ctx, SW_E_STATE, "sw_autotune_cached cannot be captured");
    if (b->d_n_pairs)
        return fail(ctx, SW_E_INVALID, "sw_autotune_cached takes a sample with a host pair count");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    std::string key;
    if ((st = tune_key(ctx, b, sc, flags, &key)))
        return st;
    if (cache_hit)
        *cache_hit = 0;
    // the last entry with this key wins
    sw_tune_entry found[kNumClasses];
    bool have = false;
    if (FILE *f = fopen(cache_path, "r")) {
        std::string line;
        int ch;
        while (true) {
            line.clear();
            while ((ch = fgetc(f)) != EOF && ch != '\n')
                line.push_back((char)ch);
            if (line.find("\"key\":\"" + key + "\"") != std::string::npos) {
                int32_t edges[kNumClasses], G[kNumClasses], R[kNumClasses], bpc[kNumClasses],
                    path[kNumClasses], nc[kNumClasses];
                float ms[kNumClasses], msd[kNumClasses];
                bool ok = json_array(line, "edges", edges, kNumClasses) &&
                          json_array(line, "G", G, kNumClasses) &&
                          json_array(line, "RPL", R, kNumClasses) &&
                          json_array(line, "blocks_per_cu", bpc, kNumClasses) &&
                          json_array(line, "path", path, kNumClasses) &&
                          json_array(line, "candidates", nc, kNumClasses) &&
                          json_array(line, "ms", ms, kNumClasses) &&
                          json_array(line, "ms_default", msd, kNumClasses);
                // a cached choice must be one this library can run
                for (int c = 0; ok && c < kNumClasses; ++c) {
                    ok = edges[c] >= 1 && edges[c] <= 65535 && (c == 0 || edges[c] > edges[c - 1]) &&
                         (bpc[c] == 1 || bpc[c] == 2 || bpc[c] == 4) &&
                         (c == kNumClasses - 1 ? edges[c] == 65535
                                               : (score_shape_available(G[c], R[c]) &&
                                                  G[c] * R[c] >= edges[c]));
                }
                if (ok) {
                    for (int c = 0; c < kNumClasses; ++c)
                        found[c] = sw_tune_entry{edges[c], G[c], R[c], bpc[c], path[c], nc[c], ms[c], msd[c]};
                    have = true;
                }
            }
            if (ch == EOF)
                break;
        }
        fclose(f);
    }
    if (have) {
        for (int c = 0; c < kNumClasses; ++c) {
            ctx->edges.m_max[c] = (uint32_t)found[c].m_max;
            if (c + 1 < kNumClasses)
                ctx->shapes[c] = ClassShape{found[c].m_max, found[c].G, found[c].RPL};
            ctx->blocks_per_cu[c] = found[c].blocks_per_cu;
        }
        if (out)
            memcpy(out, found, sizeof found);
        if (cache_hit)
            *cache_hit = 1;
        return SW_OK;
    }
    sw_tune_entry t[kNumClasses];
    if ((st = sw_autotune(ctx, b, sc, flags, repeats, t, stream)))
        return st;
    if (out)
        memcpy(out, t, sizeof t);
    std::string line = "{\"key\":\"" + key + "\"";
    auto arr = [&](const char *name, auto get) {
        line += std::string(",\"") + name + "\":[";
        for (int c = 0; c < kNumClasses; ++c) {
            char v[32];
            snprintf(v, sizeof v, "%s%.10g", c ? "," : "", (double)get(t[c]));
            line += v;
        }
        line += "]";
    };
    arr("edges", [](const sw_tune_entry &x) { return x.m_max; });
    arr("G", [](const sw_tune_entry &x) { return x.G; });
    arr("RPL", [](const sw_tune_entry &x) { return x.RPL; });
    arr("blocks_per_cu", [](const sw_tune_entry &x) { return x.blocks_per_cu; });
    arr("path", [](const sw_tune_entry &x) { return x.path; });
    arr("candidates", [](const sw_tune_entry &x) { return x.candidates; });
    arr("ms", [](const sw_tune_entry &x) { return x.ms; });
    arr("ms_default", [](const sw_tune_entry &x) { return x.ms_default; });
    line += "}\n";
    FILE *f = fopen(cache_path, "a");
    if (!f)
        return fail(ctx, SW_E_INVALID, "cannot open the tuning cache %s for appending", cache_path);
    const bool wrote = fwrite(line.data(), 1, line.size(), f) == line.size();
    const bool closed = fclose(f) == 0;
    if (!wrote || !closed)
        return fail(ctx, SW_E_INVALID, "cannot write the tuning cache %s", cache_path);
    return SW_OK;
}

}  // extern "C"

struct sw_mlp {
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *loss = nullptr;
    uint16_t *bf = nullptr;     // w1t | w2t | w2 | w3b
    int step = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    MlpDev dev() const
    {
        MlpDev d;
        d.w1t = bf;
        d.w2t = bf + kIn * kHidden;
        d.w2 = d.w2t + kHidden * kHidden;
        d.w3b = d.w2 + kHidden * kHidden;
        d.b1 = theta + kOffB1;
        d.b2 = theta + kOffB2;
        d.b3 = theta + kOffB3;
        return d;
    }
};

namespace {

sw_status mlp_workspace(sw_ctx *ctx, sw_mlp *mlp, uint32_t n)
{
    return ensure(ctx, &mlp->ws, &mlp->ws_bytes, mlp_workspace_bytes(n), false);
}

sw_status filter_scratch(sw_ctx *ctx, uint32_t n_reads, uint32_t n_pairs, uint32_t **first,
                         uint32_t **last, uint32_t **count, uint32_t **cscan)
{
    const size_t nr = align_up(4ull * std::max<uint32_t>(n_reads, 1));
    const size_t need = 3 * nr + align_up(4 * compact_scratch_words(n_pairs));
    void *buf = ctx->seg;
    size_t have = ctx->seg_bytes;
    sw_status st = ensure(ctx, &buf, &have, need);
    if (st)
        return st;
    ctx->seg = static_cast<uint32_t *>(buf);
    ctx->seg_bytes = have;
    char *p = static_cast<char *>(buf);
    *first = reinterpret_cast<uint32_t *>(p);
    *last = reinterpret_cast<uint32_t *>(p + nr);
    *count = reinterpret_cast<uint32_t *>(p + 2 * nr);
    *cscan = reinterpret_cast<uint32_t *>(p + 3 * nr);
    return SW_OK;
}

}  // namespace

extern "C" {

sw_status sw_mlp_create(sw_ctx *ctx, sw_mlp **out)
{
    if (!ctx || !out)
        return fail(ctx, SW_E_INVALID, "NULL argument");
    *out = nullptr;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    sw_mlp *m = new sw_mlp;
    const size_t fb = align_up(4ull * kParams);
    const size_t bb = 2ull * (kIn * kHidden + 2 * kHidden * kHidden + kHidden);
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, 4 * fb + 256 + align_up(bb));
    if (e != hipSuccess) {
        delete m;
        return fail(ctx, SW_E_NOMEM, "sw_mlp_create: %s", hipGetErrorString(e));
    }
    char *c = static_cast<char *>(p);
    m->theta = reinterpret_cast<float *>(c);
    m->m = reinterpret_cast<float *>(c + fb);
    m->v = reinterpret_cast<float *>(c + 2 * fb);
    m->grad = reinterpret_cast<float *>(c + 3 * fb);
    m->loss = reinterpret_cast<float *>(c + 4 * fb);
    m->bf = reinterpret_cast<uint16_t *>(c + 4 * fb + 256);
    e = hipMemset(p, 0, 4 * fb + 256 + align_up(bb));
    if (e != hipSuccess) {
        (void)hipFree(p);
        delete m;
        return fail(ctx, SW_E_DEVICE, "sw_mlp_create: %s", hipGetErrorString(e));
    }
    *out = m;
    return SW_OK;
}

sw_status sw_mlp_destroy(sw_ctx *ctx, sw_mlp *mlp)
{
    if (!mlp)
        return fail(ctx, SW_E_INVALID, "mlp is NULL");
    hipError_t e = hipDeviceSynchronize();
    if (mlp->theta && e == hipSuccess)
        e = hipFree(mlp->theta);
    if (mlp->ws && e == hipSuccess)
        e = hipFree(mlp->ws);
    delete mlp;
    if (e != hipSuccess)
        return fail(ctx, SW_E_DEVICE, "sw_mlp_destroy: %s", hipGetErrorString(e));
    return SW_OK;
}

sw_status sw_mlp_set_params(sw_ctx *ctx, sw_mlp *mlp, const float *h_params)
{
    if (!ctx || !mlp || !h_params)
        return fail(ctx, SW_E_INVALID, "NULL argument");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipMemcpy(mlp->theta, h_params, 4ull * kParams, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemset(mlp->m, 0, 4ull * kParams));
    HIP_TRY(ctx, hipMemset(mlp->v, 0, 4ull * kParams));
    mlp->step = 0;
    HIP_TRY(ctx, mlp_cast_params(mlp->theta, mlp->dev(), nullptr));
    HIP_TRY(ctx, hipDeviceSynchronize());
    return SW_OK;
}

sw_status sw_mlp_get_params(sw_ctx *ctx, const sw_mlp *mlp, float *h_params)
{
    if (!ctx || !mlp || !h_params)
        return fail(ctx, SW_E_INVALID, "NULL argument");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipDeviceSynchronize());
    HIP_TRY(ctx, hipMemcpy(h_params, mlp->theta, 4ull * kParams, hipMemcpyDeviceToHost));
    return SW_OK;
}

namespace {

constexpr char kMlpMagic[8] = {'H', 'P', 'G', 'S', 'W', 'M', 'L', 'P'};
constexpr uint32_t kMlpVersion = 1;
constexpr size_t kMlpHeader = 24;   // magic, version, parameter count, step, reserved
static_assert(kMlpHeader + 12ull * kParams == SW_MLP_STATE_BYTES, "checkpoint layout");

}  // namespace

sw_status sw_mlp_save(sw_ctx *ctx, const sw_mlp *mlp, void *h_buf, uint64_t cap)
{
    if (!ctx || !mlp || !h_buf)
        return fail(ctx, SW_E_INVALID, "NULL argument");
    if (cap < SW_MLP_STATE_BYTES)
        return fail(ctx, SW_E_RANGE, "checkpoint buffer holds %llu bytes, needs %llu",
                    (unsigned long long)cap, (unsigned long long)SW_MLP_STATE_BYTES);
    if (ctx->capturing)
        return fail(ctx, SW_E_STATE, "sw_mlp_save cannot be captured");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipDeviceSynchronize());
    char *out = static_cast<char *>(h_buf);
    const uint32_t head[4] = {kMlpVersion, (uint32_t)kParams, (uint32_t)mlp->step, 0u};
    memcpy(out, kMlpMagic, 8);
    memcpy(out + 8, head, sizeof head);
    char *body = out + kMlpHeader;
    HIP_TRY(ctx, hipMemcpy(body, mlp->theta, 4ull * kParams, hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(body + 4ull * kParams, mlp->m, 4ull * kParams, hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(body + 8ull * kParams, mlp->v, 4ull * kParams, hipMemcpyDeviceToHost));
    return SW_OK;
}

sw_status sw_mlp_load(sw_ctx *ctx, sw_mlp *mlp, const void *h_buf, uint64_t len)
{
    if (!ctx || !mlp || !h_buf)
        return fail(ctx, SW_E_INVALID, "NULL argument");
    if (len != SW_MLP_STATE_BYTES)
        return fail(ctx, SW_E_INVALID, "checkpoint of %llu bytes, expected %llu",
                    (unsigned long long)len, (unsigned long long)SW_MLP_STATE_BYTES);
    const char *in = static_cast<const char *>(h_buf);
    uint32_t head[4];
    memcpy(head, in + 8, sizeof head);
    if (memcmp(in, kMlpMagic, 8) != 0 || head[0] != kMlpVersion || head[1] != (uint32_t)kParams ||
        head[2] > 0x7FFFFFFFu)
        return fail(ctx, SW_E_INVALID, "not a checkpoint of this network (magic, version, "
                    "parameter count or step)");
    if (ctx->capturing)
        return fail(ctx, SW_E_STATE, "sw_mlp_load cannot be captured");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipDeviceSynchronize());
    const char *body = in + kMlpHeader;
    HIP_TRY(ctx, hipMemcpy(mlp->theta, body, 4ull * kParams, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(mlp->m, body + 4ull * kParams, 4ull * kParams, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(mlp->v, body + 8ull * kParams, 4ull * kParams, hipMemcpyHostToDevice));
    mlp->step = (int)head[2];
    HIP_TRY(ctx, mlp_cast_params(mlp->theta, mlp->dev(), nullptr));
    HIP_TRY(ctx, hipDeviceSynchronize());
    return SW_OK;
}

sw_status sw_features(sw_ctx *ctx, const sw_batch *b, uint16_t *d_feat, void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    sw_status st = check_batch(ctx, b);
    if (st)
        return st;
    if (b->n_pairs == 0)
        return SW_OK;
    if (!d_feat)
        return fail(ctx, SW_E_INVALID, "d_feat is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    uint32_t *first, *last, *count, *cscan;
    if ((st = filter_scratch(ctx, b->n_reads, b->n_pairs, &first, &last, &count, &cscan)))
        return st;
    HIP_TRY(ctx, read_segments(b->n_pairs, b->d_n_pairs, b->d_win, b->n_reads, first, last, count, s));
    HIP_TRY(ctx, launch_features(*b, first, count, d_feat, ctx->n_cu, s));
    return SW_OK;
}

sw_status sw_mlp_forward(sw_ctx *ctx, const sw_mlp *mlp, const uint16_t *d_x, uint32_t n,
                         float *d_logits, void *stream)
{
    if (!ctx || !mlp)
        return fail(ctx, SW_E_INVALID, "NULL argument");
    if (n == 0)
        return SW_OK;
    if (!d_x || !d_logits)
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, mlp_infer(mlp->dev(), d_x, n, nullptr, d_logits, ctx->n_cu,
                           static_cast<hipStream_t>(stream)));
    return SW_OK;
}

sw_status sw_mlp_grad(sw_ctx *ctx, const sw_mlp *mlp, const uint16_t *d_x, const float *d_y,
                      uint32_t n, float *d_grad, float *d_loss, void *stream)
{
    if (!ctx || !mlp || !d_x || !d_y || !d_grad || !d_loss)
        return fail(ctx, SW_E_INVALID, "NULL argument");
    if (n == 0 || n > (1u << 20))
        return fail(ctx, SW_E_RANGE, "minibatch must hold 1..2^20 rows");
    if (ctx->capturing)
        return fail(ctx, SW_E_STATE, "sw_mlp_grad cannot be captured");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    sw_mlp *mm = const_cast<sw_mlp *>(mlp);
    sw_status st = mlp_workspace(ctx, mm, n);
    if (st)
        return st;
    HIP_TRY(ctx, mlp_backprop(mlp->dev(), d_x, d_y, n, d_grad, d_loss, mm->ws,
                              static_cast<hipStream_t>(stream)));
    return SW_OK;
}

sw_status sw_mlp_train_step(sw_ctx *ctx, sw_mlp *mlp, const uint16_t *d_x, const float *d_y,
                            uint32_t n, float lr, float *d_loss, void *stream)
{
    if (!ctx || !mlp || !d_x || !d_y)
        return fail(ctx, SW_E_INVALID, "NULL argument");
    if (n == 0 || n > (1u << 20))
        return fail(ctx, SW_E_RANGE, "minibatch must hold 1..2^20 rows");
    if (!(lr > 0.f))
        return fail(ctx, SW_E_INVALID, "learning rate must be positive");
    // the step count enters Adam's bias correction on the host: a replayed graph
    // would repeat one step's correction
    if (ctx->capturing)
        return fail(ctx, SW_E_STATE, "sw_mlp_train_step cannot be captured");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    sw_status st = mlp_workspace(ctx, mlp, n);
    if (st)
        return st;
    HIP_TRY(ctx, mlp_backprop(mlp->dev(), d_x, d_y, n, mlp->grad, d_loss ? d_loss : mlp->loss,
                              mlp->ws, s));
    mlp->step += 1;
    HIP_TRY(ctx, mlp_adam(mlp->theta, mlp->m, mlp->v, mlp->grad, lr, mlp->step, s));
    HIP_TRY(ctx, mlp_cast_params(mlp->theta, mlp->dev(), s));
    return SW_OK;
}

sw_status sw_mlp_labels(sw_ctx *ctx, const sw_batch *b, const sw_hit *d_hits,
                        const int32_t *d_best_score, int32_t margin, int32_t min_best, float *d_y,
                        void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    sw_status st = check_batch(ctx, b);
    if (st)
        return st;
    if (b->n_pairs == 0)
        return SW_OK;
    if (!d_hits || !d_best_score || !d_y)
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, mlp_labels(b->n_pairs, b->d_win, b->n_reads, d_hits, d_best_score, margin, min_best, d_y,
                            static_cast<hipStream_t>(stream)));
    return SW_OK;
}

sw_status sw_filter_candidates(sw_ctx *ctx, const sw_batch *b, const sw_mlp *mlp,
                               const sw_filter_params *fp, uint16_t *d_feat, float *d_logits,
                               uint8_t *d_keep, sw_window *d_win_out, uint32_t *d_sel_ids,
                               uint32_t *d_n_sel, uint32_t *d_n_unsure, void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    sw_status st = check_batch(ctx, b);
    if (st)
        return st;
    if (!mlp || !fp || !d_n_sel)
        return fail(ctx, SW_E_INVALID, "NULL argument");
    if (!(fp->logit_lo <= fp->logit_hi))
        return fail(ctx, SW_E_INVALID, "logit_lo must not exceed logit_hi");
    if (!(fp->logit_drop <= fp->logit_lo))
        return fail(ctx, SW_E_INVALID, "logit_drop must not exceed logit_lo");
    if (b->d_n_pairs)
        return fail(ctx, SW_E_INVALID, "the filter takes a batch with a host pair count");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (b->n_pairs == 0)
        return SW_OK;
    if (!d_feat || !d_logits || !d_keep || !d_win_out || !d_sel_ids)
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    uint32_t *first, *last, *count, *cscan;
    if ((st = filter_scratch(ctx, b->n_reads, b->n_pairs, &first, &last, &count, &cscan)))
        return st;
    HIP_TRY(ctx, read_segments(b->n_pairs, nullptr, b->d_win, b->n_reads, first, last, count, s));
    HIP_TRY(ctx, launch_features(*b, first, count, d_feat, ctx->n_cu, s));
    HIP_TRY(ctx, mlp_infer(mlp->dev(), d_feat, b->n_pairs, nullptr, d_logits, ctx->n_cu, s));
    uint32_t *unsure = d_n_unsure ? d_n_unsure : cscan + compact_scratch_words(b->n_pairs) - 1;
    HIP_TRY(ctx, filter_decide(b->n_pairs, b->d_win, b->n_reads, first, last, count, d_logits,
                               fp->logit_lo, fp->logit_hi, fp->logit_drop, d_keep, unsure, s));
    HIP_TRY(ctx, compact_pairs(b->n_pairs, d_keep, b->d_win, d_win_out, d_sel_ids, d_n_sel, cscan, s));
    return SW_OK;
}

int sw_cigar_string(const uint32_t *ops, uint32_t n_ops, char *buf, uint32_t cap)
{
    static const char names[] = "MIDNS";
    if (!buf || cap == 0)
        return -1;
    uint32_t k = 0;
    for (uint32_t i = 0; i < n_ops; ++i) {
        const uint32_t code = ops[i] & 15u;
        char tmp[24];
        const int len = snprintf(tmp, sizeof tmp, "%u%c", ops[i] >> 4, code < 5 ? names[code] : '?');
        if (k + (uint32_t)len + 1 > cap)
            return -1;
        memcpy(buf + k, tmp, (size_t)len);
        k += (uint32_t)len;
    }
    buf[k] = 0;
    return (int)k;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Spliced reads: CALs, joined windows, junctions.
// ---------------------------------------------------------------------------
extern "C" {

sw_status sw_seed_cals(sw_ctx *ctx, const sw_batch *seeds, const uint32_t *d_best_pair,
                       const sw_aln *d_aln, const uint32_t *d_seed_read, uint32_t n_seeds,
                       int32_t min_score, sw_cal *d_cals, void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    sw_status st = check_batch(ctx, seeds);
    if (st)
        return st;
    if (n_seeds == 0)
        return SW_OK;
    if (!d_best_pair || !d_aln || !d_seed_read || !d_cals)
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    if (seeds->n_pairs && !seeds->d_win)
        return fail(ctx, SW_E_INVALID, "batch has no windows");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_seed_cals(*seeds, d_best_pair, d_aln, d_seed_read, n_seeds, min_score,
                                  d_cals, static_cast<hipStream_t>(stream)));
    return SW_OK;
}

sw_status sw_join_cals(sw_ctx *ctx, const sw_cal *d_cals, uint32_t n_cals, uint32_t n_reads,
                       uint64_t ref_len, uint32_t ext, uint32_t max_gap, sw_window *d_win_out,
                       uint32_t *d_n_out, void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    if (!d_n_out || (n_cals && (!d_cals || !d_win_out)))
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    if (ref_len >= (1ull << 36))
        return fail(ctx, SW_E_RANGE, "reference longer than 2^36 bases");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const size_t n = std::max<uint32_t>(n_cals, 1);
    const size_t o_keep = align_up(sizeof(sw_window) * n);
    const size_t o_ids = o_keep + align_up(n);
    const size_t o_scan = o_ids + align_up(4 * n);
    const size_t need = o_scan + align_up(4 * compact_scratch_words(n_cals));
    void *buf = ctx->join;
    size_t have = ctx->join_bytes;
    sw_status st = ensure(ctx, &buf, &have, need);
    if (st)
        return st;
    ctx->join = buf;
    ctx->join_bytes = have;
    char *p = static_cast<char *>(buf);
    sw_window *tmp = reinterpret_cast<sw_window *>(p);
    uint8_t *keep = reinterpret_cast<uint8_t *>(p + o_keep);
    uint32_t *ids = reinterpret_cast<uint32_t *>(p + o_ids);
    uint32_t *scan = reinterpret_cast<uint32_t *>(p + o_scan);
    if (n_cals && ref_len)
        HIP_TRY(ctx, launch_join(n_cals, d_cals, n_reads, ref_len, ext, max_gap, tmp, keep, s));
    // no CAL can be valid without a reference: the compaction of nothing
    // writes the zero count
    HIP_TRY(ctx, compact_pairs(ref_len ? n_cals : 0, keep, tmp, d_win_out, ids, d_n_out, scan, s));
    return SW_OK;
}

static sw_status check_table(sw_ctx *ctx, const void *keys, const void *counts, uint32_t cap)
{
    if (!keys || !counts)
        return fail(ctx, SW_E_INVALID, "NULL table");
    if (cap == 0 || (cap & (cap - 1)) || cap > (1u << 31))
        return fail(ctx, SW_E_INVALID, "table capacity %u is not a power of two in [1, 2^31]", cap);
    return SW_OK;
}

sw_status sw_junctions_clear(sw_ctx *ctx, uint64_t *d_keys, uint32_t *d_counts, uint32_t capacity,
                             void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    sw_status st = check_table(ctx, d_keys, d_counts, capacity);
    if (st)
        return st;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_table_clear(d_keys, d_counts, capacity, static_cast<hipStream_t>(stream)));
    return SW_OK;
}

sw_status sw_detect_junctions(sw_ctx *ctx, const sw_batch *b, const uint32_t *d_pair_ids,
                              uint32_t n, const sw_aln *d_aln, uint32_t *d_ops,
                              uint32_t ops_stride, int32_t min_score, uint32_t min_intron,
                              uint64_t *d_keys, uint32_t *d_counts, uint32_t capacity,
                              uint32_t *d_n_junc, uint32_t *d_dropped, void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    sw_status st = check_batch(ctx, b);
    if (st)
        return st;
    if ((st = check_table(ctx, d_keys, d_counts, capacity)))
        return st;
    if (min_intron < 4)
        return fail(ctx, SW_E_INVALID, "min_intron must be at least 4 (GT + AG)");
    if (n == 0)
        return SW_OK;
    if (!d_pair_ids || !d_aln || (!d_ops && ops_stride))
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    if (b->n_pairs == 0)
        return fail(ctx, SW_E_INVALID, "alignments given for an empty batch");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_detect(*b, d_pair_ids, n, d_aln, d_ops, ops_stride, min_score, min_intron,
                               d_keys, d_counts, capacity, d_n_junc, d_dropped,
                               static_cast<hipStream_t>(stream)));
    return SW_OK;
}

sw_status sw_list_junctions(sw_ctx *ctx, const uint64_t *d_keys, const uint32_t *d_counts,
                            uint32_t capacity, sw_junction *d_out, uint32_t out_cap, uint32_t *d_n,
                            void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    sw_status st = check_table(ctx, d_keys, d_counts, capacity);
    if (st)
        return st;
    if (!d_n || (out_cap && !d_out))
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_list(d_keys, d_counts, capacity, d_out, out_cap, d_n,
                             static_cast<hipStream_t>(stream)));
    return SW_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Region and CAL seekers.
// ---------------------------------------------------------------------------
namespace {

// Offsets part of an index: 4^k + 1 words, rounded up to 256 bytes.
uint64_t index_offsets_bytes(uint32_t k) { return (4ull * (kmer_index_codes(k) + 1) + 255) & ~255ull; }

sw_status check_seed_params(sw_ctx *ctx, const sw_seed_params *sp)
{
    if (!sp)
        return fail(ctx, SW_E_INVALID, "seed parameters are NULL");
    if (sp->k < 4 || sp->k > 15)
        return fail(ctx, SW_E_RANGE, "k must be in [4, 15], got %u", sp->k);
    if (sp->step == 0)
        return fail(ctx, SW_E_INVALID, "step must be at least 1");
    if (sp->offset > 65535)
        return fail(ctx, SW_E_RANGE, "offset above the longest read");
    return SW_OK;
}

}  // namespace

extern "C" {

sw_status sw_kmer_index_bytes(uint64_t ref_len, uint32_t k, uint64_t *bytes)
{
    if (!bytes)
        return fail(nullptr, SW_E_INVALID, "bytes is NULL");
    *bytes = 0;
    if (k < 4 || k > 15)
        return fail(nullptr, SW_E_RANGE, "k must be in [4, 15], got %u", k);
    const uint64_t n_pos = ref_len >= k ? ref_len - k + 1 : 0;
    if (n_pos >= (1ull << 32))
        return fail(nullptr, SW_E_RANGE, "the reference holds 2^32 or more k-mers");
    *bytes = index_offsets_bytes(k) + 4 * n_pos;
    return SW_OK;
}

sw_status sw_kmer_index_build(sw_ctx *ctx, const uint32_t *d_ref2b, uint64_t ref_len, uint32_t k,
                              void *d_index, uint64_t index_bytes, void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    uint64_t need = 0;
    sw_status st = sw_kmer_index_bytes(ref_len, k, &need);
    if (st)
        return fail(ctx, st, "%s", g_noctx_err.c_str());
    if (!d_index || (ref_len && !d_ref2b))
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    if (index_bytes < need)
        return fail(ctx, SW_E_RANGE, "index buffer of %llu bytes, %llu needed",
                    (unsigned long long)index_bytes, (unsigned long long)need);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    void *buf = ctx->seek;
    size_t have = ctx->seek_bytes;
    if ((st = ensure(ctx, &buf, &have, 8 * seeker_scan_words(kmer_index_codes(k)))))
        return st;
    ctx->seek = buf;
    ctx->seek_bytes = have;
    uint32_t *starts = static_cast<uint32_t *>(d_index);
    uint32_t *pos = reinterpret_cast<uint32_t *>(static_cast<char *>(d_index) + index_offsets_bytes(k));
    HIP_TRY(ctx, launch_index_build(d_ref2b, ref_len, k, starts, pos, static_cast<uint32_t *>(buf),
                                    static_cast<hipStream_t>(stream)));
    return SW_OK;
}

sw_status sw_seed_regions(sw_ctx *ctx, const sw_batch *reads, const void *d_index,
                          uint64_t index_bytes, const sw_seed_params *sp, sw_region *d_regions,
                          uint64_t cap, uint64_t *d_read_end, void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    if (!reads)
        return fail(ctx, SW_E_INVALID, "batch is NULL");
    sw_status st = check_seed_params(ctx, sp);
    if (st)
        return st;
    uint64_t need = 0;
    if ((st = sw_kmer_index_bytes(reads->ref_len, sp->k, &need)))
        return fail(ctx, st, "%s", g_noctx_err.c_str());
    if (index_bytes < need)
        return fail(ctx, SW_E_RANGE, "index of %llu bytes, an index with k = %u of this reference "
                    "takes %llu", (unsigned long long)index_bytes, sp->k, (unsigned long long)need);
    if (reads->n_reads == 0)
        return SW_OK;
    if (!reads->d_read_len || !reads->d_read_off || !reads->d_reads2b || !d_index || !d_read_end ||
        (cap && !d_regions))
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const size_t cnt_bytes = align_up(4ull * reads->n_reads);
    void *buf = ctx->seek;
    size_t have = ctx->seek_bytes;
    if ((st = ensure(ctx, &buf, &have, cnt_bytes + 8 * seeker_scan_words(reads->n_reads))))
        return st;
    ctx->seek = buf;
    ctx->seek_bytes = have;
    const uint32_t *starts = static_cast<const uint32_t *>(d_index);
    const uint32_t *pos = reinterpret_cast<const uint32_t *>(static_cast<const char *>(d_index) +
                                                             index_offsets_bytes(sp->k));
    uint32_t *cnt = static_cast<uint32_t *>(buf);
    uint64_t *tsum = reinterpret_cast<uint64_t *>(static_cast<char *>(buf) + cnt_bytes);
    HIP_TRY(ctx, launch_regions(*reads, starts, pos, *sp, d_regions, cap, cnt, d_read_end, tsum,
                                static_cast<hipStream_t>(stream)));
    return SW_OK;
}

sw_status sw_cal_seeker(sw_ctx *ctx, const sw_region *d_regions, const uint64_t *d_read_end,
                        uint32_t n_reads, uint64_t cap, uint32_t k, uint32_t merge_gap,
                        uint32_t min_len, const uint32_t *d_skip, sw_cal *d_cals, void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    if (n_reads == 0)
        return SW_OK;
    if (!d_read_end || !d_cals || (cap && !d_regions))
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    if (k < 1 || k > 65535)
        return fail(ctx, SW_E_RANGE, "region length out of range");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_cal_seek(d_regions, d_read_end, n_reads, cap, k, merge_gap, min_len, d_skip,
                                 d_cals, static_cast<hipStream_t>(stream)));
    return SW_OK;
}

sw_status sw_stage_b(sw_ctx *ctx, const sw_batch *b, const sw_region *d_regions,
                     const uint64_t *d_read_end, uint64_t cap, sw_bmap *d_maps, uint32_t *d_n_maps,
                     void *stream)
{
    if (!ctx)
        return fail(nullptr, SW_E_INVALID, "ctx is NULL");
    if (!b)
        return fail(ctx, SW_E_INVALID, "batch is NULL");
    if (b->n_reads == 0)
        return SW_OK;
    if (!b->d_read_len || !b->d_read_off || !b->d_reads2b || !b->d_ref2b || !d_read_end ||
        !d_maps || !d_n_maps || (cap && !d_regions))
        return fail(ctx, SW_E_INVALID, "NULL buffer");
    if (b->ref_len > (1ull << 32))
        return fail(ctx, SW_E_RANGE, "reference longer than 2^32 bases");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_stage_b(*b, d_regions, d_read_end, cap, d_maps, d_n_maps,
                                static_cast<hipStream_t>(stream)));
    return SW_OK;
}

}  // extern "C"
