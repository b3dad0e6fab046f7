// Internal declarations shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "hpgsw.h"

namespace hpgsw {

// ---------------------------------------------------------------------------
// Length classes.  A pair goes to the class of its read (query) length m; each
// class is served by one instantiation of the wavefront kernel with G lanes per
// pair and RPL query rows per lane (G * RPL >= m), except the last class,
// which strip-mines longer queries in strips of G * RPL rows.
// ---------------------------------------------------------------------------
constexpr int kNumClasses = 11;
// window-length bins per class: 8-base bins below 4096, 128-base bins above
constexpr int kBinsPerClass = 1024;
constexpr int kNumBins = kNumClasses * kBinsPerClass;

struct ClassShape {
    int m_max;  // largest query length served (strip class: 65535)
    int G;      // lanes per pair
    int RPL;    // query rows per lane
};

// Default shapes; the autotuner may replace the shape of a class by another
// instantiated shape with the same or larger capacity.
extern const ClassShape kDefaultClasses[kNumClasses];

// Upper query-length bound of every class, as the bucketing kernel reads it
// (increasing; the last is 65535).  The score path uses the context's edges,
// which the autotuner may move; the traceback always uses the default ones.
struct ClassEdges {
    uint32_t m_max[kNumClasses];
};
ClassEdges default_edges();

// Scratch words used by the bucketing and scheduling kernels.
struct BucketScratch {
    uint32_t *bin;       // [n_pairs] bin of each pair (0xFFFFFFFF: resolved already)
    uint32_t *ids;       // [n_pairs] pair ids sorted by (class, window length desc)
    uint32_t *hist;      // [kNumBins] counts, then cursors
    uint32_t *seg;       // [2 * kNumClasses] begin/end of each class in ids
    uint32_t *counter;   // [kNumClasses] task counters of the persistent kernels
    uint32_t *maxlen;    // [2 * kNumClasses] longest window, then longest read, per class
};

// Traceback band: with a pair's score S and canonical end (i_e, c_e) from the
// score pass, the alignment uses M <= i_e + 1 aligned rows and D deletions with
// S <= match * M - (cost of D deletions); a run of L deletions costs
// go + (L - 1) ge (penalties as positive numbers), so D deletions cost at least
// go + (D - 1) ge when go >= ge and D go otherwise.  The alignment therefore
// lies in window columns [c_e + 1 - (i_e + 1) - D_max, c_e].  The DP over those
// columns gives every cell of the canonical path, and every value compared
// there, the value of the full DP (a band only removes paths, and each path
// cell's best prefix lies inside it), so codes, end and walk are unchanged.
struct TbBand {
    const sw_hit *hits;    // per pair, or null: no band
    int ma, go, ge;        // match score, gap open and extension penalties (> 0)
};

// Width of the pair's DP window (n without a band) and its first column.
__device__ __forceinline__ int tb_band(const TbBand &bd, uint32_t pair, int m, int n, int &c_lo)
{
    c_lo = 0;
    if (!bd.hits || bd.go <= 0 || bd.ge <= 0 || bd.ma <= 0)
        return n;
    const sw_hit h = bd.hits[pair];
    if (h.score <= 0 || h.read_end < 0 || h.read_end >= m || h.ref_end < 0 || h.ref_end >= n)
        return n;
    const int64_t rows = (int64_t)h.read_end + 1;
    const int64_t slack = (int64_t)bd.ma * rows - h.score;
    int64_t dmax = 0;
    if (slack > 0)
        dmax = bd.go >= bd.ge ? (slack < bd.go ? 0 : (slack - bd.go) / bd.ge + 1) : slack / bd.go;
    const int64_t lo = (int64_t)h.ref_end + 1 - (rows + dmax);
    c_lo = lo > 0 ? (int)lo : 0;
    return h.ref_end + 1 - c_lo;
}

struct ScoreParams {
    const uint32_t *ref;
    uint64_t ref_len;
    uint64_t ref_words;
    const uint32_t *reads;
    uint64_t read_words;
    const uint64_t *read_off;
    const uint16_t *read_len;
    const sw_window *win;
    const uint32_t *ids;
    const uint32_t *seg;
    uint32_t *counter;
    int cls;
    int ma, mi, go, ge;
    sw_hit *hits;
    int2 *strip_buf;       // strip class only: [waves][max window] boundary rows
    uint32_t strip_stride; // entries per wave in strip_buf
};

// Launchers (return hipError_t of the launch).
hipError_t launch_pack2b(const uint8_t *ascii, uint64_t n, uint32_t *out, uint32_t *bad,
                         hipStream_t st);
// Traceback pairs (aln != null) are binned by the width of their DP window,
// the band when `band.hits` is given.
hipError_t launch_bucket(const sw_batch &b, const uint32_t *sel, uint32_t n_items,
                         const BucketScratch &s, sw_hit *hits, sw_aln *aln, hipStream_t st,
                         const ClassEdges &edges, const TbBand &band = TbBand{nullptr, 0, 0, 0});
hipError_t launch_score_class(int cls, int G, int RPL, int mode, const ScoreParams &p, int grid,
                              hipStream_t st);
int score_class_m_max(int cls);
hipError_t launch_score16_class(int G, int RPL, const ScoreParams &p, int grid, hipStream_t st);
bool score_shape_available(int G, int RPL);
int score_waves_per_block();
hipError_t launch_best(const sw_batch &b, const sw_hit *hits, uint64_t *keys, int32_t t_map,
                       uint32_t *best_pair, int32_t *best_score, uint8_t *mapped, hipStream_t st);
hipError_t launch_select_windows(const sw_batch &b, const uint32_t *ids, uint32_t n, sw_window *out,
                                 hipStream_t st);
// Per read: its only scoring pair or none (sole), and keep flags for the pairs
// of reads with several; keys: n_reads words of scratch.
hipError_t launch_sole_windows(const sw_batch &b, uint64_t *keys, uint8_t *keep, uint32_t *sole,
                               hipStream_t st);
hipError_t launch_merge_best(uint32_t n_reads, const uint32_t *sole, const uint32_t *sub_best,
                             const uint32_t *ids, uint32_t n_ids, uint32_t *best_pair,
                             hipStream_t st);
int traceback_waves_per_block();
// Query-length class bounds of the traceback (its own above 512 bases).
ClassEdges traceback_edges();
hipError_t launch_traceback_class(int cls, const sw_batch &b, const sw_scoring &sc,
                                  const uint32_t *sel, const uint32_t *ids, const uint32_t *seg,
                                  uint32_t *counter, sw_aln *aln, uint32_t *ops,
                                  uint32_t ops_stride, uint32_t *codes, uint64_t codes_words,
                                  const uint32_t *maxlen, const TbBand &band, int grid,
                                  hipStream_t st);

// Spliced reads (splice.hip).
hipError_t launch_seed_cals(const sw_batch &b, const uint32_t *best_pair, const sw_aln *aln,
                            const uint32_t *seed_read, uint32_t n_seeds, int32_t min_score,
                            sw_cal *out, hipStream_t st);
// Joined windows of each run at the run's own positions of tmp, flagged in keep.
hipError_t launch_join(uint32_t n, const sw_cal *cals, uint32_t n_reads, uint64_t ref_len,
                       uint32_t ext, uint32_t max_gap, sw_window *tmp, uint8_t *keep,
                       hipStream_t st);
hipError_t launch_detect(const sw_batch &b, const uint32_t *pair_ids, uint32_t n, const sw_aln *aln,
                         uint32_t *ops, uint32_t ops_stride, int32_t min_score, uint32_t min_intron,
                         uint64_t *keys, uint32_t *counts, uint32_t cap, uint32_t *n_junc,
                         uint32_t *dropped, hipStream_t st);
hipError_t launch_table_clear(uint64_t *keys, uint32_t *counts, uint32_t cap, hipStream_t st);
hipError_t launch_list(const uint64_t *keys, const uint32_t *counts, uint32_t cap, sw_junction *out,
                       uint32_t out_cap, uint32_t *d_n, hipStream_t st);

// Region and CAL seekers (seeker.hip).
uint64_t kmer_index_codes(uint32_t k);
uint64_t seeker_scan_words(uint64_t n);
hipError_t launch_index_build(const uint32_t *ref, uint64_t ref_len, uint32_t k, uint32_t *starts,
                              uint32_t *pos, uint32_t *tsum, hipStream_t st);
hipError_t launch_regions(const sw_batch &b, const uint32_t *starts, const uint32_t *pos,
                          const sw_seed_params &sp, sw_region *out, uint64_t cap,
                          uint32_t *cnt, uint64_t *read_end, uint64_t *tsum, hipStream_t st);
hipError_t launch_cal_seek(const sw_region *reg, const uint64_t *read_end, uint32_t n_reads,
                           uint64_t cap, uint32_t k, uint32_t merge_gap, uint32_t min_len,
                           const uint32_t *skip, sw_cal *cals, hipStream_t st);
hipError_t launch_stage_b(const sw_batch &b, const sw_region *reg, const uint64_t *read_end,
                          uint64_t cap, sw_bmap *maps, uint32_t *n_maps, hipStream_t st);

}  // namespace hpgsw
