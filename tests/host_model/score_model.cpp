// Host model of the score kernels (test infrastructure).
//
// Compiles the unmodified kernel source (paper_1304_0681_amd/csrc/score.hip)
// as C++ for the CPU, against the stand-in HIP header in hip_stub/, and runs
// any instantiation of the packed int16 kernel or the int32 kernel on a
// caller's batch.  Every input array lies against an inaccessible guard page
// (after its end, or before its start), so an access outside an array stops
// the process.
//
// Lanes are threads.  The 64 lanes of a wave meet at a barrier around every
// cross-lane operation (each lane publishes its value, the barrier completes,
// each lane reads its source lane, a second barrier completes): the lockstep
// the hardware gives.  The instructions are emulated from their definitions:
//   DPP row_shr:1 (0x111) / wave_shr:1 (0x138), all rows and banks, bound_ctrl
//     off: lane l takes lane l - 1 (within its 16-lane row for row_shr), and a
//     lane without a source keeps `old`;
//   v_perm_b32: each result byte selects from the 8 bytes {hi, lo} (lo holds
//     bytes 0-3): 0-7 a byte, 8-11 the sign of byte 1, 3, 5 or 7 spread over
//     the byte, 12 the byte 0x00, 13-255 the byte 0xFF;
//   v_alignbit_b32: ({hi, lo} >> (shift & 31)) low 32 bits;
//   v_bfe_i32: the sign-extended `width` bits of src from bit `offset` (0 when
//     the width is 0).
#include <stdint.h>
#include <string.h>
#include <sys/mman.h>
#include <unistd.h>

#include <atomic>
#include <cstdlib>
#include <thread>
#include <vector>

#include "../../paper_1304_0681_amd/csrc/score.hip"

thread_local ModelIdx threadIdx, blockIdx;

namespace {

// Sense-reversing barrier of the 64 lanes of a wave; spins, yielding the CPU,
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
    uint64_t ex[64];
};

thread_local Wave *t_wave;

int lane_id() { return (int)(threadIdx.x & 63u); }

uint64_t exchange(uint64_t x, int src, bool has_src, uint64_t old)
{
    Wave &w = *t_wave;
    w.ex[lane_id()] = x;
    w.bar.arrive_and_wait();
    const uint64_t r = has_src ? w.ex[src & 63] : old;
    w.bar.arrive_and_wait();
    return r;
}

uint8_t perm_byte(uint64_t d, uint32_t sel)
{
    sel &= 0xFF;
    if (sel >= 13) return 0xFF;
    if (sel == 12) return 0x00;
    if (sel >= 8) return ((d >> (8 * (2 * (sel - 8) + 1) + 7)) & 1) ? 0xFF : 0x00;
    return (uint8_t)(d >> (8 * sel));
}

}  // namespace

int model_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl)
{
    if (row_mask != 0xF || bank_mask != 0xF || bound_ctrl)
        abort();
    const int l = lane_id();
    if (ctrl == 0x111)
        return (int)exchange((uint32_t)src, l - 1, (l & 15) != 0, (uint32_t)old);
    if (ctrl == 0x138)
        return (int)exchange((uint32_t)src, l - 1, l != 0, (uint32_t)old);
    abort();
}

int __shfl(int v, int src, int) { return (int)exchange((uint32_t)v, src, true, 0); }
int __shfl_xor(int v, int mask, int) { return (int)exchange((uint32_t)v, lane_id() ^ mask, true, 0); }
uint64_t __shfl_xor(uint64_t v, int mask, int) { return exchange(v, lane_id() ^ mask, true, 0); }
uint32_t atomicAdd(uint32_t *p, uint32_t v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }

uint32_t model_perm(uint32_t hi, uint32_t lo, uint32_t sel)
{
    const uint64_t d = ((uint64_t)hi << 32) | lo;
    uint32_t r = 0;
    for (int k = 0; k < 4; ++k)
        r |= (uint32_t)perm_byte(d, sel >> (8 * k)) << (8 * k);
    return r;
}

uint32_t model_alignbit(uint32_t hi, uint32_t lo, uint32_t shift)
{
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> (shift & 31));
}

int model_sbfe(int src, int offset, int width)
{
    offset &= 31;
    width &= 31;
    if (width == 0)
        return 0;
    const uint32_t u = (uint32_t)src >> offset;
    const uint32_t m = width == 32 ? 0xFFFFFFFFu : ((1u << width) - 1u);
    const uint32_t v = u & m;
    const uint32_t sign = 1u << (width - 1);
    return (int)((v ^ sign) - sign);
}

namespace {

// A copy of `bytes` bytes against a guard page: after its end (at_end) or
// before its start.
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

using KernelFn = void (*)(hpgsw::ScoreParams);

template <int G, int RPL>
void packed(hpgsw::ScoreParams P) { hpgsw::k_sw_score16<G, RPL>(P); }

template <int G, int RPL, int MODE, bool STRIP>
void int32k(hpgsw::ScoreParams P) { hpgsw::k_sw_score<G, RPL, MODE, STRIP>(P); }

KernelFn pick(int packed16, int G, int RPL, int mode, int strip)
{
    if (strip) {
        if (G != 64 || RPL != 32 || packed16) return nullptr;
        return mode == 0 ? int32k<64, 32, 0, true> : mode == 1 ? int32k<64, 32, 1, true>
                                                               : int32k<64, 32, 2, true>;
    }
#define X(g, r)                                                                              \
    if (G == g && RPL == r)                                                                  \
        return packed16 ? packed<g, r>                                                       \
                        : (mode == 0 ? int32k<g, r, 0, false>                                \
                                     : mode == 1 ? int32k<g, r, 1, false> : int32k<g, r, 2, false>);
    HPGSW_SHAPES(X)
#undef X
    return nullptr;
}

}  // namespace

extern "C" {

// Results of the pairs ids[0..n_ids) (one query-length class) scored by one
// kernel instantiation: packed16 (int16 x 2, score only) or int32 with `mode`
// (0 score, 1 ends with 16-bit keys, 2 ends), `strip` (queries in strips),
// `waves` waves sharing the task counter.  Returns 0, or -1 for a kernel that
// is not instantiated.
int model_score(int packed16, int G, int RPL, int mode, int strip, int waves, int at_end,
                const uint32_t *ref, uint64_t ref_len, const uint32_t *reads, uint64_t read_words,
                const uint64_t *read_off, const uint16_t *read_len, uint32_t n_reads,
                const sw_window *win, uint32_t n_pairs, const uint32_t *ids, uint32_t n_ids,
                const int32_t *sc, sw_hit *hits_out)
{
    const KernelFn fn = pick(packed16, G, RPL, mode, strip);
    if (!fn || waves < 1 || waves > 4)
        return -1;
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
    const uint32_t strip_stride = 65536;
    std::vector<int2> strip_init(strip ? (size_t)waves * strip_stride : 1, int2{0, 0});
    Guarded g_strip(strip_init.data(), sizeof(int2) * strip_init.size(), at_end);
    hpgsw::ScoreParams P;
    P.ref = static_cast<const uint32_t *>(g_ref.data);
    P.ref_len = ref_len;
    P.ref_words = ref_words;
    P.reads = static_cast<const uint32_t *>(g_reads.data);
    P.read_words = read_words;
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
    P.strip_buf = strip ? static_cast<int2 *>(g_strip.data) : nullptr;
    P.strip_stride = strip_stride;
    // one block: waves 0..waves-1 of block 0 (wave index = threadIdx.x >> 6)
    std::vector<Wave> wv(waves);
    std::vector<std::thread> th;
    for (int w = 0; w < waves; ++w)
        for (int l = 0; l < 64; ++l)
            th.emplace_back([&, w, l]() {
                threadIdx = ModelIdx{(unsigned)(64 * w + l), 0, 0};
                blockIdx = ModelIdx{0, 0, 0};
                t_wave = &wv[w];
                fn(P);
            });
    for (auto &t : th)
        t.join();
    memcpy(hits_out, g_hits.data, sizeof(sw_hit) * n_pairs);
    return 0;
}

}  // extern "C"
