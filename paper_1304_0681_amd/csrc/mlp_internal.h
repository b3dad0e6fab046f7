// Internal declarations of the candidate filter (features, MLP, decision).
#pragma once

#include "internal.h"

namespace hpgsw {

constexpr int kIn = 64;         // features per candidate
constexpr int kHidden = 128;
constexpr int kParams = kIn * kHidden + kHidden + kHidden * kHidden + kHidden + kHidden + 1;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kIn * kHidden;
constexpr int kOffW2 = kOffB1 + kHidden;
constexpr int kOffB2 = kOffW2 + kHidden * kHidden;
constexpr int kOffW3 = kOffB2 + kHidden;
constexpr int kOffB3 = kOffW3 + kHidden;
constexpr int kMaxCand = 64;    // candidates per read handled by features / decision

// Device view of the network: float32 biases, bfloat16 operand copies.
struct MlpDev {
    uint16_t *w1t;      // [128 out][64 in]
    uint16_t *w2t;      // [128 out][128 in]
    uint16_t *w2;       // [128 in][128 out]
    uint16_t *w3b;      // [128]
    const float *b1, *b2, *b3;
};

hipError_t mlp_cast_params(const float *theta, const MlpDev &W, hipStream_t st);
hipError_t mlp_infer(const MlpDev &W, const uint16_t *X, uint32_t n, const uint32_t *d_n,
                     float *logits, int n_cu, hipStream_t st);
hipError_t mlp_gemm(const uint16_t *A, uint32_t lda, const uint16_t *B, uint32_t ldb, float *C,
                    uint32_t ldc, uint32_t M, uint32_t N, uint32_t K, hipStream_t st);
hipError_t mlp_backprop(const MlpDev &W, const uint16_t *X, const float *y, uint32_t B, float *grad,
                        float *loss, void *ws, hipStream_t st);
size_t mlp_workspace_bytes(uint32_t B);
hipError_t mlp_adam(float *theta, float *m, float *v, const float *g, float lr, int step,
                    hipStream_t st);
hipError_t mlp_labels(uint32_t n_pairs, const sw_window *win, uint32_t n_reads, const sw_hit *hits,
                      const int32_t *best, int32_t margin, int32_t min_best, float *y,
                      hipStream_t st);
hipError_t read_segments(uint32_t n_pairs, const uint32_t *d_n, const sw_window *win,
                         uint32_t n_reads, uint32_t *first, uint32_t *last, uint32_t *count,
                         hipStream_t st);
hipError_t filter_decide(uint32_t n_pairs, const sw_window *win, uint32_t n_reads,
                         const uint32_t *first, const uint32_t *last, const uint32_t *count,
                         const float *logits, float lo, float hi, float drop, uint8_t *keep,
                         uint32_t *n_unsure, hipStream_t st);
size_t compact_scratch_words(uint32_t n);
hipError_t compact_pairs(uint32_t n, const uint8_t *keep, const sw_window *win, sw_window *wout,
                         uint32_t *ids_out, uint32_t *d_n_out, uint32_t *scratch, hipStream_t st);
hipError_t launch_features(const sw_batch &b, const uint32_t *first, const uint32_t *count,
                           uint16_t *feat, int n_cu, hipStream_t st);

}  // namespace hpgsw
