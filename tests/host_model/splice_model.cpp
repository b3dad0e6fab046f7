// Host model of the spliced-read kernels (test infrastructure).
//
// Compiles the unmodified kernel source (paper_1304_0681_amd/csrc/splice.hip)
// as C++ for the CPU, against the stand-in HIP header in hip_stub/, and runs
// its kernels on a caller's inputs.  The kernels use no cross-lane operation
// and no barrier, and every loop over items is grid-strided, so one block of
// 256 lanes run one after the other covers every item; atomics are plain
// read-modify-writes.  Every array lies against an inaccessible guard page
// (after its end, or before its start), so an access outside an array stops
// the process.
#include <stdint.h>
#include <string.h>
#include <sys/mman.h>
#include <unistd.h>

#include <vector>

#include "../../paper_1304_0681_amd/csrc/splice.hip"

thread_local ModelIdx threadIdx, blockIdx, gridDim;

uint32_t atomicAdd(uint32_t *p, uint32_t v)
{
    const uint32_t o = *p;
    *p = o + v;
    return o;
}

unsigned long long atomicCAS(unsigned long long *p, unsigned long long cmp, unsigned long long v)
{
    const unsigned long long o = *p;
    if (o == cmp)
        *p = v;
    return o;
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
        if (bytes && src)
            memcpy(p, src, bytes);
        data = p;
    }
    ~Guarded() { munmap(base, len); }
    template <class T> T *as() { return static_cast<T *>(data); }
};

// One block of 256 lanes, lane after lane.
template <class F> void run_block(F f)
{
    gridDim = ModelIdx{1, 1, 1};
    blockIdx = ModelIdx{0, 0, 0};
    for (unsigned l = 0; l < 256; ++l) {
        threadIdx = ModelIdx{l, 0, 0};
        f();
    }
}

}  // namespace

extern "C" {

void model_seed_cals(int at_end, uint32_t n_seeds, const sw_window *win, uint32_t n_pairs,
                     const uint32_t *best_pair, const sw_aln *aln, const uint32_t *seed_read,
                     int32_t min_score, sw_cal *out)
{
    Guarded g_win(win, sizeof(sw_window) * n_pairs, at_end);
    Guarded g_bp(best_pair, 4ull * n_seeds, at_end), g_aln(aln, sizeof(sw_aln) * n_seeds, at_end);
    Guarded g_sr(seed_read, 4ull * n_seeds, at_end), g_out(nullptr, sizeof(sw_cal) * n_seeds, at_end);
    run_block([&] {
        hpgsw::k_seed_cals(n_seeds, g_win.as<sw_window>(), n_pairs, nullptr, g_bp.as<uint32_t>(),
                           g_aln.as<sw_aln>(), g_sr.as<uint32_t>(), min_score, g_out.as<sw_cal>());
    });
    memcpy(out, g_out.data, sizeof(sw_cal) * n_seeds);
}

// Windows of each run at the run's positions of tmp_out, flags in keep_out.
void model_join(int at_end, uint32_t n, const sw_cal *cals, uint32_t n_reads, uint64_t ref_len,
                uint32_t ext, uint32_t max_gap, sw_window *tmp_out, uint8_t *keep_out)
{
    Guarded g_cals(cals, sizeof(sw_cal) * n, at_end);
    Guarded g_tmp(nullptr, sizeof(sw_window) * n, at_end), g_keep(nullptr, n, at_end);
    run_block([&] { hpgsw::k_fill_u8(n, g_keep.as<uint8_t>()); });
    run_block([&] {
        hpgsw::k_join(n, g_cals.as<sw_cal>(), n_reads, ref_len, ext, max_gap, g_tmp.as<sw_window>(),
                      g_keep.as<uint8_t>());
    });
    memcpy(tmp_out, g_tmp.data, sizeof(sw_window) * n);
    memcpy(keep_out, g_keep.data, n);
}

// Junction search; ops are rewritten in place, the table updated in place.
void model_detect(int at_end, uint32_t n, const uint32_t *pair_ids, const sw_window *win,
                  uint32_t n_pairs, const uint32_t *ref2b, uint64_t ref_len, const sw_aln *aln,
                  uint32_t *ops, uint32_t ops_stride, int32_t min_score, uint32_t min_intron,
                  uint64_t *keys, uint32_t *counts, uint32_t cap, uint32_t *n_junc,
                  uint32_t *dropped)
{
    const uint64_t ref_words = (ref_len + 15) / 16;
    Guarded g_ids(pair_ids, 4ull * n, at_end), g_win(win, sizeof(sw_window) * n_pairs, at_end);
    Guarded g_ref(ref2b, 4 * ref_words, at_end), g_aln(aln, sizeof(sw_aln) * n, at_end);
    Guarded g_ops(ops, 4ull * n * ops_stride, at_end);
    Guarded g_keys(keys, 8ull * cap, at_end), g_counts(counts, 4ull * cap, at_end);
    Guarded g_nj(nullptr, 4ull * n, at_end), g_dr(dropped, 4, at_end);
    hpgsw::DetectParams P;
    P.n = n;
    P.pair_ids = g_ids.as<uint32_t>();
    P.win = g_win.as<sw_window>();
    P.n_pairs = n_pairs;
    P.d_n = nullptr;
    P.ref = g_ref.as<uint32_t>();
    P.ref_len = ref_len;
    P.aln = g_aln.as<sw_aln>();
    P.ops = g_ops.as<uint32_t>();
    P.ops_stride = ops_stride;
    P.min_score = min_score;
    P.min_intron = min_intron;
    P.keys = g_keys.as<unsigned long long>();
    P.counts = g_counts.as<uint32_t>();
    P.cap = cap;
    P.n_junc = g_nj.as<uint32_t>();
    P.dropped = g_dr.as<uint32_t>();
    run_block([&] { hpgsw::k_detect(P); });
    memcpy(ops, g_ops.data, 4ull * n * ops_stride);
    memcpy(keys, g_keys.data, 8ull * cap);
    memcpy(counts, g_counts.data, 4ull * cap);
    memcpy(n_junc, g_nj.data, 4ull * n);
    memcpy(dropped, g_dr.data, 4);
}

uint32_t model_list(int at_end, const uint64_t *keys, const uint32_t *counts, uint32_t cap,
                    sw_junction *out, uint32_t out_cap)
{
    Guarded g_keys(keys, 8ull * cap, at_end), g_counts(counts, 4ull * cap, at_end);
    Guarded g_out(nullptr, sizeof(sw_junction) * out_cap, at_end), g_n(nullptr, 4, at_end);
    run_block([&] { hpgsw::k_zero_one(g_n.as<uint32_t>()); });
    run_block([&] {
        hpgsw::k_list(cap, g_keys.as<unsigned long long>(), g_counts.as<uint32_t>(),
                      g_out.as<sw_junction>(), out_cap, g_n.as<uint32_t>());
    });
    memcpy(out, g_out.data, sizeof(sw_junction) * out_cap);
    return *g_n.as<uint32_t>();
}

}  // extern "C"
