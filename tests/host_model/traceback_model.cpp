// Host model of the traceback kernel (test infrastructure).
//
// Compiles the unmodified kernel source (paper_1304_0681_amd/csrc/traceback.hip)
// as C++ for the CPU, against the stand-in HIP header in hip_stub/, and runs any
// of its instantiations on the lockstep wave model of wave_model.h.  The DP of a
// task is wave-uniform; the walk after it is not: each lane group walks its own
// pair for as many iterations as the pair needs (idle groups not at all), and
// every cross-lane operation of the walk reads inside the group.  The model
// follows the kernel's block-scope fences to know where the lanes are: in a
// task, each strip's DP starts after a fence and with a DPP shift; the fence
// before the walk is followed by a walk operation (or, for an idle group,
// directly by the fence after the walk).  Between those two fences a lane's
// cross-lane operations meet only its group.  Every input array, the outputs and
// the code scratch lie against an inaccessible guard page (after their end, or
// before their start), so an access outside them stops the process.
#define MODEL_FENCE_HOOK 1
#include <stdint.h>
#include <string.h>

#include "../../paper_1304_0681_amd/csrc/traceback.hip"

thread_local ModelIdx threadIdx, blockIdx;

#include "wave_model.h"

namespace {

thread_local int t_G = 64;            // lanes per group of the running tile
thread_local bool t_pending = false;  // a fence, and no cross-lane operation since
thread_local bool t_walk = false;     // between the fences around the walk

void op_hook(bool dpp)
{
    if (t_pending) {
        t_pending = false;
        if (!dpp)       // the fence before the walk: the group walks alone
            t_walk = true;
    }
    wave_model::t_group = t_walk ? t_G : 64;
}

}  // namespace

void __threadfence_block()
{
    if (t_walk) {           // the fence after the walk: the wave meets again
        t_walk = false;
        wave_model::t_group = 64;
    } else {
        // a strip's DP or the walk starts; an idle group's next fence ends its walk
        t_pending = !t_pending;
    }
}

uint32_t model_bitop3(uint32_t a, uint32_t b, uint32_t c, uint32_t table)
{
    uint32_t r = 0;
    for (int k = 0; k < 32; ++k) {
        const uint32_t idx = (((a >> k) & 1u) << 2) | (((b >> k) & 1u) << 1) | ((c >> k) & 1u);
        r |= ((table >> idx) & 1u) << k;
    }
    return r;
}

namespace {

using wave_model::Guarded;
using KernelFn = void (*)(hpgsw::TBParams);

template <int G, int RPL, bool STRIP>
void tb(hpgsw::TBParams P)
{
    t_G = G;
    t_pending = t_walk = false;
    wave_model::t_group = 64;
    wave_model::t_op_hook = op_hook;
    hpgsw::k_sw_traceback<G, RPL, STRIP>(P);
}

// every shape the library launches (the class table of traceback.hip)
KernelFn pick(int G, int RPL, int strip)
{
    if (strip)
        return G == 64 && RPL == 32 ? tb<64, 32, true> : nullptr;
#define S(g, r) if (G == g && RPL == r) return tb<g, r, false>;
    S(2, 8) S(4, 8) S(8, 8) S(8, 13) S(16, 8) S(8, 20) S(32, 8) S(64, 8) S(64, 12) S(64, 16)
#undef S
    return nullptr;
}

}  // namespace

extern "C" {

// Alignments of the selected pairs sel[ids[0..n_ids)] (one query-length class)
// by the tile of G lanes of RPL rows per pair (strip: the strip-mined tile), on
// `waves` waves sharing the task counter and `codes_words` words of code
// scratch.  maxlen_n / maxlen_m: the class's longest DP window and query.
// hits: the score pass's hits with ends (the band), or null.  aln_out[n_sel],
// ops_out[n_sel * ops_stride] start as given and receive the class's results.
// Returns 0, or -1 for a shape that is not modelled.
int model_traceback(int G, int RPL, int strip, int waves, int at_end, const uint32_t *ref,
                    uint64_t ref_len, const uint32_t *reads, uint64_t read_words,
                    const uint64_t *read_off, const uint16_t *read_len, uint32_t n_reads,
                    const sw_window *win, uint32_t n_pairs, const uint32_t *sel, uint32_t n_sel,
                    const uint32_t *ids, uint32_t n_ids, uint32_t maxlen_n, uint32_t maxlen_m,
                    const int32_t *sc, const sw_hit *hits, uint64_t codes_words, sw_aln *aln_out,
                    uint32_t *ops_out, uint32_t ops_stride)
{
    const KernelFn fn = pick(G, RPL, strip);
    if (!fn || waves < 1 || waves > 4)
        return -1;
    const uint64_t ref_words = (ref_len + 15) / 16;
    Guarded g_ref(ref, 4 * ref_words, at_end), g_reads(reads, 4 * read_words, at_end);
    Guarded g_off(read_off, 8ull * n_reads, at_end), g_len(read_len, 2ull * n_reads, at_end);
    Guarded g_win(win, sizeof(sw_window) * n_pairs, at_end);
    Guarded g_sel(sel, 4ull * n_sel, at_end), g_ids(ids, 4ull * n_ids, at_end);
    Guarded g_hits(hits, hits ? sizeof(sw_hit) * n_pairs : 0, at_end);
    const uint32_t seg_h[2] = {0, n_ids};
    Guarded g_seg(seg_h, sizeof seg_h, at_end);
    uint32_t zero = 0;
    Guarded g_cnt(&zero, 4, at_end);
    uint32_t maxlen_h[2 * hpgsw::kNumClasses] = {};
    maxlen_h[0] = maxlen_n;
    maxlen_h[hpgsw::kNumClasses] = maxlen_m;
    Guarded g_max(maxlen_h, sizeof maxlen_h, at_end);
    Guarded g_aln(aln_out, sizeof(sw_aln) * n_sel, at_end);
    Guarded g_ops(ops_out, 4ull * n_sel * ops_stride, at_end);
    Guarded g_codes(nullptr, 4 * codes_words, at_end);
    hpgsw::TBParams P;
    P.ref = static_cast<const uint32_t *>(g_ref.data);
    P.ref_len = ref_len;
    P.ref_words = ref_words;
    P.reads = static_cast<const uint32_t *>(g_reads.data);
    P.read_off = static_cast<const uint64_t *>(g_off.data);
    P.read_len = static_cast<const uint16_t *>(g_len.data);
    P.n_reads = n_reads;
    P.win = static_cast<const sw_window *>(g_win.data);
    P.sel = static_cast<const uint32_t *>(g_sel.data);
    P.ids = static_cast<const uint32_t *>(g_ids.data);
    P.seg = static_cast<const uint32_t *>(g_seg.data);
    P.counter = static_cast<uint32_t *>(g_cnt.data);
    P.cls = 0;
    P.ma = sc[0];
    P.mi = sc[1];
    P.go = sc[2];
    P.ge = sc[3];
    P.aln = static_cast<sw_aln *>(g_aln.data);
    P.ops = static_cast<uint32_t *>(g_ops.data);
    P.ops_stride = ops_stride;
    P.codes = static_cast<uint32_t *>(g_codes.data);
    P.codes_words = codes_words;
    P.maxlen = static_cast<const uint32_t *>(g_max.data);
    P.band = hpgsw::TbBand{hits ? static_cast<const sw_hit *>(g_hits.data) : nullptr, sc[0], -sc[2],
                           -sc[3]};
    wave_model::run_waves(waves, [&] { fn(P); }, G);
    memcpy(aln_out, g_aln.data, sizeof(sw_aln) * n_sel);
    memcpy(ops_out, g_ops.data, 4ull * n_sel * ops_stride);
    return 0;
}

}  // extern "C"
