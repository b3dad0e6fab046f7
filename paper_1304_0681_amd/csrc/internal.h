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

// Scratch words used by the bucketing and scheduling kernels.
struct BucketScratch {
    uint32_t *bin;       // [n_pairs] bin of each pair (0xFFFFFFFF: resolved already)
    uint32_t *ids;       // [n_pairs] pair ids sorted by (class, window length desc)
    uint32_t *hist;      // [kNumBins] counts, then cursors
    uint32_t *seg;       // [2 * kNumClasses] begin/end of each class in ids
    uint32_t *counter;   // [kNumClasses] task counters of the persistent kernels
    uint32_t *maxlen;    // [2 * kNumClasses] longest window, then longest read, per class
};

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
hipError_t launch_bucket(const sw_batch &b, const uint32_t *sel, uint32_t n_items,
                         const BucketScratch &s, sw_hit *hits, sw_aln *aln, hipStream_t st);
hipError_t launch_score_class(int cls, int G, int RPL, int mode, const ScoreParams &p, int grid,
                              hipStream_t st);
int score_class_m_max(int cls);
hipError_t launch_score16_class(int G, int RPL, const ScoreParams &p, int grid, hipStream_t st);
bool score_shape_available(int G, int RPL);
int score_waves_per_block();
hipError_t launch_best(const sw_batch &b, const sw_hit *hits, uint64_t *keys, int32_t t_map,
                       uint32_t *best_pair, int32_t *best_score, uint8_t *mapped, hipStream_t st);
int traceback_waves_per_block();
hipError_t launch_traceback_class(int cls, const sw_batch &b, const sw_scoring &sc,
                                  const uint32_t *sel, const uint32_t *ids, const uint32_t *seg,
                                  uint32_t *counter, sw_aln *aln, uint32_t *ops,
                                  uint32_t ops_stride, uint32_t *codes, uint64_t codes_words,
                                  const uint32_t *maxlen, const sw_hit *hits, int grid,
                                  hipStream_t st);

}  // namespace hpgsw
