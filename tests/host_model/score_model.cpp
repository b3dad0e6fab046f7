// Host model of the score kernels (test infrastructure).
//
// Compiles the unmodified kernel source (paper_1304_0681_amd/csrc/score.hip)
// as C++ for the CPU, against the stand-in HIP header in hip_stub/, and runs
// any instantiation of the packed int16 kernel or the int32 kernel on a
// caller's batch, on the lockstep wave model of wave_model.h (lanes as
// threads, cross-lane operations and the AMDGPU builtins emulated from their
// definitions, every input array against an inaccessible guard page after its
// end or before its start, so an access outside an array stops the process).
#include <stdint.h>
#include <string.h>

#include "../../paper_1304_0681_amd/csrc/score.hip"

thread_local ModelIdx threadIdx, blockIdx;

#include "wave_model.h"

namespace {

using wave_model::Guarded;

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
    wave_model::run_waves(waves, [&] { fn(P); });
    memcpy(hits_out, g_hits.data, sizeof(sw_hit) * n_pairs);
    return 0;
}

}  // extern "C"
