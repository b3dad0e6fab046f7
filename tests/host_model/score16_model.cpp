// Host model of the packed int16 scoring kernel's wave (test infrastructure).
//
// Compiles the kernel's own wave body (score16_body.h) for the CPU with the
// wave's cross-lane and special instructions emulated, and runs it on a
// caller's batch with every input array placed against an inaccessible guard
// page, so that any read or write outside an array stops the process.
//
// Lanes are threads; the 64 lanes of a wave meet at a barrier around every
// cross-lane operation (each lane publishes its value, the barrier completes,
// each lane reads its source lane, a second barrier completes), which is the
// lockstep the hardware gives.  DPP row_shr:1 and wave_shr:1 with bound_ctrl
// off keep `old` in lanes without a source (the first lane of a row or wave).
// v_perm_b32 follows the instruction's byte selection on the 8 bytes
// {hi, lo}: selectors 0-7 pick a byte (lo holds bytes 0-3), 8-11 replicate the
// sign bit of byte 1, 3, 5 or 7, 12 gives 0x00 and 13-255 give 0xFF.
#include <stdint.h>
#include <string.h>
#include <sys/mman.h>
#include <unistd.h>

#include <atomic>
#include <thread>
#include <vector>

#include "hpgsw.h"
#include "score16_body.h"

namespace {

struct Params {   // the fields the wave body reads, as in the kernel's parameters
    const uint32_t *ref;
    uint64_t ref_len, ref_words;
    const uint32_t *reads;
    const uint64_t *read_off;
    const uint16_t *read_len;
    const sw_window *win;
    const uint32_t *ids;
    const uint32_t *seg;
    uint32_t *counter;
    int cls;
    int ma, mi, go, ge;
    sw_hit *hits;
};

// Sense-reversing barrier of the 64 lanes of a wave: spins, yielding the CPU,
// since the lanes outnumber the host's cores.
struct LaneBarrier {
    std::atomic<int> count{64};
    std::atomic<int> sense{0};
    void arrive_and_wait()
    {
        const int s = sense.load(std::memory_order_relaxed);
        if (count.fetch_sub(1, std::memory_order_acq_rel) == 1) {
            count.store(64, std::memory_order_relaxed);
            sense.store(s ^ 1, std::memory_order_release);
        } else {
            while (sense.load(std::memory_order_acquire) == s)
                std::this_thread::yield();
        }
    }
};

struct Wave {
    LaneBarrier bar;
    int ex[64];
};

thread_local int t_lane;
thread_local Wave *t_wave;

int exchange(int x, int src, bool has_src, int old)
{
    Wave &w = *t_wave;
    w.ex[t_lane] = x;
    w.bar.arrive_and_wait();
    const int r = has_src ? w.ex[src] : old;
    w.bar.arrive_and_wait();
    return r;
}

uint8_t perm_byte(uint64_t d, uint32_t sel)
{
    sel &= 0xFF;
    if (sel >= 13) return 0xFF;
    if (sel == 12) return 0x00;
    if (sel >= 8) {
        const int b = 2 * (int)(sel - 8) + 1;            // bytes 1, 3, 5, 7
        return ((d >> (8 * b + 7)) & 1) ? 0xFF : 0x00;
    }
    return (uint8_t)(d >> (8 * sel));
}

struct HostWave {
    static int lane() { return t_lane; }
    static int dpp_row_shr1(int old, int x) { return exchange(x, t_lane - 1, (t_lane & 15) != 0, old); }
    static int dpp_wave_shr1(int old, int x) { return exchange(x, t_lane - 1, t_lane != 0, old); }
    static int shfl(int v, int src) { return exchange(v, src & 63, true, 0); }
    static int shfl_xor(int v, int mask) { return exchange(v, (t_lane ^ mask) & 63, true, 0); }
    static uint32_t atomic_add(uint32_t *p, uint32_t v)
    {
        return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
    }
    static uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel)
    {
        const uint64_t d = ((uint64_t)hi << 32) | lo;
        uint32_t r = 0;
        for (int k = 0; k < 4; ++k)
            r |= (uint32_t)perm_byte(d, sel >> (8 * k)) << (8 * k);
        return r;
    }
    static uint32_t alignbit(uint32_t hi, uint32_t lo, uint32_t sh)
    {
        return (uint32_t)(((((uint64_t)hi) << 32) | lo) >> (sh & 31));
    }
};

// A copy of `bytes` bytes placed against a guard page: after the end
// (at_end) or before the start.
struct Guarded {
    char *base = nullptr;
    size_t len = 0;
    void *data = nullptr;
    Guarded(const void *src, size_t bytes, bool at_end)
    {
        const size_t pg = (size_t)sysconf(_SC_PAGESIZE);
        const size_t body = (bytes + pg - 1) / pg * pg + pg;
        len = body + 2 * pg;
        base = static_cast<char *>(mmap(nullptr, len, PROT_READ | PROT_WRITE,
                                        MAP_PRIVATE | MAP_ANONYMOUS, -1, 0));
        mprotect(base, pg, PROT_NONE);
        mprotect(base + pg + body, pg, PROT_NONE);
        char *p = at_end ? base + pg + body - bytes : base + pg;
        if (bytes)
            memcpy(p, src, bytes);
        data = p;
    }
    ~Guarded() { munmap(base, len); }
};

template <int G, int RPL>
void run_wave(const Params &P, int lane, Wave *w)
{
    t_lane = lane;
    t_wave = w;
    hpgsw::sw16::wave_body<G, RPL, HostWave>(P);
}

#define HPGSW_MODEL_SHAPES(X) \
    X(1, 16) X(1, 32) X(2, 32) X(4, 16) X(4, 25) X(4, 32) X(8, 13) X(8, 20) X(8, 32) X(16, 32) \
    X(32, 32) X(64, 32)

}  // namespace

extern "C" {

// Scores of the pairs ids[0..n_ids) (one query-length class) with the packed
// kernel body of shape (G, RPL), `waves` waves sharing the task counter.
// Returns 0, or -1 for a shape the kernel is not instantiated with.
int model_score16(int G, int RPL, int waves, int at_end, const uint32_t *ref, uint64_t ref_len,
                  const uint32_t *reads, uint64_t read_words, const uint64_t *read_off,
                  const uint16_t *read_len, uint32_t n_reads, const sw_window *win,
                  uint32_t n_pairs, const uint32_t *ids, uint32_t n_ids, const int32_t *sc,
                  sw_hit *hits_out)
{
    const uint64_t ref_words = (ref_len + 15) / 16;
    Guarded g_ref(ref, 4 * ref_words, at_end), g_reads(reads, 4 * read_words, at_end);
    Guarded g_off(read_off, 8ull * n_reads, at_end), g_len(read_len, 2ull * n_reads, at_end);
    Guarded g_win(win, sizeof(sw_window) * n_pairs, at_end), g_ids(ids, 4ull * n_ids, at_end);
    const uint32_t seg_h[2] = {0, n_ids};
    Guarded g_seg(seg_h, sizeof seg_h, at_end);
    uint32_t zero = 0;
    Guarded g_cnt(&zero, 4, at_end);
    std::vector<sw_hit> init(n_pairs, sw_hit{-7, -7, -7});
    Guarded g_hits(init.data(), sizeof(sw_hit) * n_pairs, at_end);
    Params P;
    P.ref = static_cast<const uint32_t *>(g_ref.data);
    P.ref_len = ref_len;
    P.ref_words = ref_words;
    P.reads = static_cast<const uint32_t *>(g_reads.data);
    P.read_off = static_cast<const uint64_t *>(g_off.data);
    P.read_len = static_cast<const uint16_t *>(g_len.data);
    P.win = static_cast<const sw_window *>(g_win.data);
    P.ids = static_cast<const uint32_t *>(g_ids.data);
    P.seg = static_cast<const uint32_t *>(g_seg.data);
    P.counter = static_cast<uint32_t *>(g_cnt.data);
    P.cls = 0;
    P.ma = sc[0];
    P.mi = sc[1];
    P.go = sc[2];
    P.ge = sc[3];
    P.hits = static_cast<sw_hit *>(g_hits.data);
    void (*fn)(const Params &, int, Wave *) = nullptr;
#define X(g, r) if (G == g && RPL == r) fn = run_wave<g, r>;
    HPGSW_MODEL_SHAPES(X)
#undef X
    if (!fn)
        return -1;
    std::vector<Wave> wv(waves);
    std::vector<std::thread> th;
    for (int w = 0; w < waves; ++w)
        for (int l = 0; l < 64; ++l)
            th.emplace_back(fn, std::cref(P), l, &wv[w]);
    for (auto &t : th)
        t.join();
    memcpy(hits_out, g_hits.data, sizeof(sw_hit) * n_pairs);
    return 0;
}

}  // extern "C"
