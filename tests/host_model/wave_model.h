// Lockstep model of one AMD wave on the host (test infrastructure), for the
// host models of the wavefront score and traceback kernels (score_model.cpp,
// traceback_model.cpp).  Cross-lane operations meet the whole wave, or, for a
// lane whose t_group is below 64, only its lane group (a kernel whose groups
// run divergent code that never reads across groups).  Lanes are threads.  The 64 lanes of a wave meet at a
// barrier around every cross-lane operation (each lane publishes its value, the
// barrier completes, each lane reads its source lane, a second barrier
// completes): the lockstep the hardware gives.  The instructions are emulated
// from their definitions:
//   DPP row_shr:1 (0x111) / wave_shr:1 (0x138), all rows and banks, bound_ctrl
//     off: lane l takes lane l - 1 (within its 16-lane row for row_shr), and a
//     lane without a source keeps `old`;
//   v_perm_b32: each result byte selects from the 8 bytes {hi, lo} (lo holds
//     bytes 0-3): 0-7 a byte, 8-11 the sign of byte 1, 3, 5 or 7 spread over
//     the byte, 12 the byte 0x00, 13-255 the byte 0xFF;
//   v_alignbit_b32: ({hi, lo} >> (shift & 31)) low 32 bits;
//   v_bfe_i32: the sign-extended `width` bits of src from bit `offset` (0 when
//     the width is 0);
//   ballot: the OR of every lane's predicate bit; shfl_up within groups of
//     `width` lanes: lane l takes lane l - delta when it stays in its group,
//     else keeps its own value.
// Every input array of a model run lies against an inaccessible guard page
// (Guarded), so an access outside an array stops the process.
#pragma once

#include <stdint.h>
#include <string.h>
#include <sys/mman.h>
#include <unistd.h>

#include <atomic>
#include <cstdlib>
#include <thread>
#include <vector>

namespace wave_model {

// Sense-reversing barrier of `n` lanes (the 64 of a wave, or one lane group);
// spins, yielding the CPU, since the lanes outnumber the host's cores.
struct LaneBarrier {
    int n = 64;
    std::atomic<int> count{64};
    std::atomic<int> sense{0};
    void reset(int lanes)
    {
        n = lanes;
        count.store(lanes);
    }
    void arrive_and_wait()
    {
        const int s = sense.load(std::memory_order_relaxed);
        if (count.fetch_sub(1, std::memory_order_acq_rel) == 1) {
            count.store(n, std::memory_order_relaxed);
            sense.store(s ^ 1, std::memory_order_release);
        } else {
            while (sense.load(std::memory_order_acquire) == s)
                std::this_thread::yield();
        }
    }
};

// gbar: one barrier per lane group, for kernels whose lane groups run
// divergent code (set_groups); a lane whose t_group is below 64 meets only the
// lanes of its group at a cross-lane operation.
struct Wave {
    LaneBarrier bar;
    LaneBarrier gbar[32];
    std::atomic<uint64_t> ex[64];
    void set_groups(int g)
    {
        for (auto &b : gbar)
            b.reset(g);
    }
};

inline thread_local Wave *t_wave;
inline thread_local int t_group = 64;          // lanes in the current scope
inline thread_local void (*t_op_hook)(bool dpp) = nullptr;   // before each cross-lane op

inline int lane_id() { return (int)(threadIdx.x & 63u); }

inline LaneBarrier &scope_barrier(bool dpp)
{
    if (t_op_hook)
        t_op_hook(dpp);
    Wave &w = *t_wave;
    return t_group >= 64 ? w.bar : w.gbar[lane_id() / t_group];
}

inline uint64_t exchange(uint64_t x, int src, bool has_src, uint64_t old, bool dpp = false)
{
    Wave &w = *t_wave;
    LaneBarrier &b = scope_barrier(dpp);
    w.ex[lane_id()].store(x);
    b.arrive_and_wait();
    const uint64_t r = has_src ? w.ex[src & 63].load() : old;
    b.arrive_and_wait();
    return r;
}

inline uint8_t perm_byte(uint64_t d, uint32_t sel)
{
    sel &= 0xFF;
    if (sel >= 13) return 0xFF;
    if (sel == 12) return 0x00;
    if (sel >= 8) return ((d >> (8 * (2 * (sel - 8) + 1) + 7)) & 1) ? 0xFF : 0x00;
    return (uint8_t)(d >> (8 * sel));
}

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
        if (bytes && src)
            memcpy(p, src, bytes);
        data = p;
    }
    ~Guarded() { munmap(base, len); }
    template <class T> T *as() { return static_cast<T *>(data); }
};

// Run fn on `waves` waves of one block (wave index = threadIdx.x >> 6); `group`:
// lanes per group for the barriers of a group's scope.
template <class F> void run_waves(int waves, F fn, int group = 64)
{
    std::vector<Wave> wv(waves);
    for (auto &w : wv)
        w.set_groups(group);
    std::vector<std::thread> th;
    for (int w = 0; w < waves; ++w)
        for (int l = 0; l < 64; ++l)
            th.emplace_back([&, w, l]() {
                threadIdx = ModelIdx{(unsigned)(64 * w + l), 0, 0};
                blockIdx = ModelIdx{0, 0, 0};
                t_wave = &wv[w];
                fn();
            });
    for (auto &t : th)
        t.join();
}

}  // namespace wave_model

int model_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl)
{
    using namespace wave_model;
    if (row_mask != 0xF || bank_mask != 0xF || bound_ctrl)
        abort();
    const int l = lane_id();
    if (ctrl == 0x111)
        return (int)exchange((uint32_t)src, l - 1, (l & 15) != 0, (uint32_t)old, true);
    if (ctrl == 0x138)
        return (int)exchange((uint32_t)src, l - 1, l != 0, (uint32_t)old, true);
    abort();
}

int __shfl(int v, int src, int) { return (int)wave_model::exchange((uint32_t)v, src, true, 0); }
int __shfl_xor(int v, int mask, int)
{
    return (int)wave_model::exchange((uint32_t)v, wave_model::lane_id() ^ mask, true, 0);
}
uint64_t __shfl_xor(uint64_t v, int mask, int)
{
    return wave_model::exchange(v, wave_model::lane_id() ^ mask, true, 0);
}
int __shfl_up(int v, unsigned delta, int width)
{
    const int l = wave_model::lane_id();
    const bool has = (l % width) >= (int)delta;
    return (int)wave_model::exchange((uint32_t)v, l - (int)delta, has, (uint32_t)v);
}
uint64_t __ballot(int pred)
{
    // every lane's bit through the exchange slots, OR-ed by each lane
    // (in a group's scope only the group's bits are gathered, the others are 0)
    using namespace wave_model;
    Wave &w = *t_wave;
    LaneBarrier &b = scope_barrier(false);
    const int g0 = t_group >= 64 ? 0 : lane_id() / t_group * t_group;
    const int g1 = t_group >= 64 ? 64 : g0 + t_group;
    w.ex[lane_id()].store(pred ? 1u : 0u);
    b.arrive_and_wait();
    uint64_t r = 0;
    for (int l = g0; l < g1; ++l)
        r |= (w.ex[l].load() ? 1ull : 0ull) << l;
    b.arrive_and_wait();
    return r;
}
uint32_t atomicAdd(uint32_t *p, uint32_t v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }

uint32_t model_perm(uint32_t hi, uint32_t lo, uint32_t sel)
{
    const uint64_t d = ((uint64_t)hi << 32) | lo;
    uint32_t r = 0;
    for (int k = 0; k < 4; ++k)
        r |= (uint32_t)wave_model::perm_byte(d, sel >> (8 * k)) << (8 * k);
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
