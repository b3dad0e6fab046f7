// Host model of the region and CAL seeker kernels (test infrastructure).
//
// Compiles the unmodified kernel source (paper_1304_0681_amd/csrc/seeker.hip)
// as C++ for the CPU against the stand-in HIP header in hip_stub/, and runs
// its kernels in the launchers' order: the blocks of a launch one after
// another, the lanes of a block as threads.  __syncthreads is a barrier of
// the block's threads, the wave barrier one of the wave's 64 threads, atomics
// are the host's.  Every array lies against an inaccessible guard page (after
// its end, or before its start), so an access outside an array stops the
// process.
#include <stdint.h>
#include <string.h>
#include <sys/mman.h>
#include <unistd.h>

#include <atomic>
#include <memory>
#include <thread>
#include <vector>

#include "../../paper_1304_0681_amd/csrc/seeker.hip"

thread_local ModelIdx threadIdx, blockIdx, gridDim, blockDim;

namespace {

// Sense-reversing barrier of n threads; spins, yielding the CPU.
struct SpinBarrier {
    explicit SpinBarrier(int n_) : n(n_), count(n_) {}
    int n;
    std::atomic<int> count;
    std::atomic<int> sense{0};
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

thread_local SpinBarrier *t_block, *t_wave;
thread_local uint64_t *t_ballot;   // the wave's ballot word

// Every block of a launch of `fn` with `block` threads, one block at a time.
template <class F> void launch(unsigned grid, unsigned block, F fn)
{
    for (unsigned bx = 0; bx < grid; ++bx) {
        SpinBarrier bb((int)block);
        std::vector<std::unique_ptr<SpinBarrier>> wb;
        for (unsigned w = 0; w < (block + 63) / 64; ++w)
            wb.emplace_back(new SpinBarrier((int)std::min(64u, block - 64 * w)));
        std::vector<uint64_t> ballots((block + 63) / 64, 0);
        std::vector<std::thread> th;
        for (unsigned t = 0; t < block; ++t)
            th.emplace_back([&, t]() {
                threadIdx = ModelIdx{t, 0, 0};
                blockIdx = ModelIdx{bx, 0, 0};
                gridDim = ModelIdx{grid, 1, 1};
                blockDim = ModelIdx{block, 1, 1};
                t_block = &bb;
                t_wave = wb[t / 64].get();
                t_ballot = &ballots[t / 64];
                fn();
            });
        for (auto &x : th)
            x.join();
    }
}

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

template <class T> void scan(const uint32_t *in, uint64_t n, T *out, bool at_end)
{
    const uint64_t nt = (n + hpgsw::kTile - 1) / hpgsw::kTile;
    if (!nt)
        return;
    Guarded g_ts(nullptr, sizeof(T) * nt, at_end);
    T *ts = g_ts.as<T>();
    launch((unsigned)nt, 256, [&] { hpgsw::k_tile_sums<T>(in, n, ts); });
    launch(1, 1024, [&] { hpgsw::k_tile_offsets<T>((uint32_t)nt, ts); });
    launch((unsigned)nt, 256, [&] { hpgsw::k_tile_scan<T>(in, n, ts, out); });
}

}  // namespace

void __syncthreads() { t_block->arrive_and_wait(); }

// every lane sets its bit, the wave meets, reads the word, meets again, and the
// last lane out clears it for the next ballot
uint64_t __ballot(int pred)
{
    const unsigned lane = threadIdx.x & 63u;
    if (pred)
        __atomic_fetch_or(t_ballot, 1ull << lane, __ATOMIC_SEQ_CST);
    t_wave->arrive_and_wait();
    const uint64_t v = __atomic_load_n(t_ballot, __ATOMIC_SEQ_CST);
    t_wave->arrive_and_wait();
    if (lane == 0)
        __atomic_store_n(t_ballot, 0ull, __ATOMIC_SEQ_CST);
    t_wave->arrive_and_wait();
    return v;
}
void model_wave_barrier() { t_wave->arrive_and_wait(); }
uint32_t atomicAdd(uint32_t *p, uint32_t v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
uint32_t atomicSub(uint32_t *p, uint32_t v) { return __atomic_fetch_sub(p, v, __ATOMIC_SEQ_CST); }
uint32_t model_alignbit(uint32_t hi, uint32_t lo, uint32_t shift)
{
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> (shift & 31));
}

extern "C" {

// Index of ref2b (ceil(ref_len / 16) words): starts[4^k + 1], pos[ref_len - k + 1].
void model_index(int at_end, const uint32_t *ref2b, uint64_t ref_len, uint32_t k, uint32_t *starts_out,
                 uint32_t *pos_out)
{
    const uint64_t n_codes = hpgsw::kmer_index_codes(k);
    const uint64_t n_pos = ref_len >= k ? ref_len - k + 1 : 0;
    const uint64_t ref_words = (ref_len + 15) / 16;
    const uint32_t mask = (1u << (2 * k)) - 1u;
    Guarded g_ref(ref2b, 4 * ref_words, at_end);
    Guarded g_st(nullptr, 4 * (n_codes + 1), at_end), g_pos(nullptr, 4 * n_pos, at_end);
    const uint32_t *ref = g_ref.as<uint32_t>();
    uint32_t *starts = g_st.as<uint32_t>(), *pos = g_pos.as<uint32_t>();
    // the launcher's grids, capped at 65535 blocks; one block stands for them here
    // (the loops are grid-strided)
    launch(1, 256, [&] { hpgsw::k_fill32(n_codes + 1, starts); });
    if (n_pos) {
        launch(1, 256, [&] { hpgsw::k_kmer_hist(ref, ref_words, n_pos, mask, starts); });
        scan<uint32_t>(starts, n_codes, starts, at_end);
        launch(1, 256, [&] { hpgsw::k_kmer_scatter(ref, ref_words, n_pos, mask, starts, pos); });
    }
    launch(1, 64, [&] { hpgsw::k_set_last(starts, n_codes, (uint32_t)n_pos); });
    memcpy(starts_out, starts, 4 * (n_codes + 1));
    memcpy(pos_out, pos, 4 * n_pos);
}

// Regions of the reads against an index (starts, pos); read_end[n_reads].
void model_regions(int at_end, const uint32_t *reads2b, uint64_t reads_len, const uint64_t *read_off,
                   const uint16_t *read_len, uint32_t n_reads, const uint32_t *starts_in,
                   const uint32_t *pos_in, uint64_t n_pos, uint32_t k, uint32_t step,
                   uint32_t offset, uint32_t max_occ, sw_region *out, uint64_t cap,
                   uint64_t *read_end_out)
{
    const uint64_t n_codes = hpgsw::kmer_index_codes(k);
    const uint64_t read_words = (reads_len + 15) / 16;
    Guarded g_reads(reads2b, 4 * read_words, at_end), g_off(read_off, 8ull * n_reads, at_end);
    Guarded g_len(read_len, 2ull * n_reads, at_end);
    Guarded g_st(starts_in, 4 * (n_codes + 1), at_end), g_pos(pos_in, 4 * n_pos, at_end);
    Guarded g_out(nullptr, sizeof(sw_region) * cap, at_end), g_end(nullptr, 8ull * n_reads, at_end);
    Guarded g_cnt(nullptr, 4ull * n_reads, at_end);
    hpgsw::SeedParams P;
    P.reads = g_reads.as<uint32_t>();
    P.read_words = read_words;
    P.read_off = g_off.as<uint64_t>();
    P.read_len = g_len.as<uint16_t>();
    P.n_reads = n_reads;
    P.reads_len = reads_len;
    P.starts = g_st.as<uint32_t>();
    P.pos = g_pos.as<uint32_t>();
    P.k = k;
    P.step = step;
    P.offset = offset;
    P.max_occ = max_occ;
    P.mask = (1u << (2 * k)) - 1u;
    uint32_t *cnt = g_cnt.as<uint32_t>();
    uint64_t *read_end = g_end.as<uint64_t>();
    launch(1, 256, [&] { hpgsw::k_region_count(P, cnt); });
    scan<uint64_t>(cnt, n_reads, read_end, at_end);
    launch(1, 256, [&] { hpgsw::k_region_write(P, read_end, g_out.as<sw_region>(), cap); });
    memcpy(out, g_out.data, sizeof(sw_region) * cap);
    memcpy(read_end_out, read_end, 8ull * n_reads);
}

void model_cal_seek(int at_end, const sw_region *reg, uint64_t n_reg, const uint64_t *read_end,
                    uint32_t n_reads, uint64_t cap, uint32_t k, uint32_t merge_gap, uint32_t min_len,
                    const uint32_t *skip, sw_cal *cals_out, unsigned blocks)
{
    Guarded g_reg(reg, sizeof(sw_region) * n_reg, at_end), g_end(read_end, 8ull * n_reads, at_end);
    Guarded g_cals(nullptr, sizeof(sw_cal) * hpgsw::kCals * n_reads, at_end);
    Guarded g_skip(skip, skip ? 4ull * n_reads : 0, at_end);
    const sw_region *R = g_reg.as<sw_region>();
    const uint64_t *E = g_end.as<uint64_t>();
    const uint32_t *K = skip ? g_skip.as<uint32_t>() : nullptr;
    sw_cal *C = g_cals.as<sw_cal>();
    launch(blocks, 64 * hpgsw::kSeekWaves,
           [&] { hpgsw::k_cal_seek(R, E, n_reads, cap, k, merge_gap, min_len, K, C); });
    memcpy(cals_out, C, sizeof(sw_cal) * hpgsw::kCals * n_reads);
}

void model_stage_b(int at_end, const uint32_t *reads2b, uint64_t reads_len, const uint64_t *read_off,
                   const uint16_t *read_len, uint32_t n_reads, const uint32_t *ref2b,
                   uint64_t ref_len, const sw_region *reg, uint64_t n_reg, const uint64_t *read_end,
                   uint64_t cap, sw_bmap *maps_out, uint32_t *n_maps_out, unsigned blocks)
{
    const uint64_t read_words = (reads_len + 15) / 16, ref_words = (ref_len + 15) / 16;
    Guarded g_reads(reads2b, 4 * read_words, at_end), g_off(read_off, 8ull * n_reads, at_end);
    Guarded g_len(read_len, 2ull * n_reads, at_end), g_ref(ref2b, 4 * ref_words, at_end);
    Guarded g_reg(reg, sizeof(sw_region) * n_reg, at_end), g_end(read_end, 8ull * n_reads, at_end);
    Guarded g_maps(nullptr, sizeof(sw_bmap) * hpgsw::kBMax * n_reads, at_end);
    Guarded g_n(nullptr, 4ull * n_reads, at_end);
    hpgsw::StageBParams P;
    P.reads = g_reads.as<uint32_t>();
    P.read_words = read_words;
    P.read_off = g_off.as<uint64_t>();
    P.read_len = g_len.as<uint16_t>();
    P.n_reads = n_reads;
    P.reads_len = reads_len;
    P.ref = g_ref.as<uint32_t>();
    P.ref_len = ref_len;
    P.reg = g_reg.as<sw_region>();
    P.read_end = g_end.as<uint64_t>();
    P.cap = cap;
    P.maps = g_maps.as<sw_bmap>();
    P.n_maps = g_n.as<uint32_t>();
    launch(blocks, 64 * hpgsw::kBWaves, [&] { hpgsw::k_stage_b(P); });
    memcpy(maps_out, P.maps, sizeof(sw_bmap) * hpgsw::kBMax * n_reads);
    memcpy(n_maps_out, P.n_maps, 4ull * n_reads);
}

}  // extern "C"
