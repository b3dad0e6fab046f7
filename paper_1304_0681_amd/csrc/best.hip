// Best hit per read (stage E, task iv): segmented arg-max over each read's
// windows.  Pairs may come in any order, so the reduction is an atomic max on
// a 64-bit key per read: (score + 1) in the high word, the complement of the
// pair index in the low word, which makes the lowest pair index win ties.
#include "internal.h"

namespace hpgsw {

namespace {

constexpr uint32_t kNoPair = 0xFFFFFFFFu;

__global__ void __launch_bounds__(256) k_best_init(uint32_t n_reads, uint64_t *keys)
{
    for (uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x; r < n_reads;
         r += (uint64_t)gridDim.x * 256)
        keys[r] = 0;
}

__global__ void __launch_bounds__(256) k_best_update(uint32_t n_pairs, const uint32_t *d_n,
                                                     const sw_window *win, const sw_hit *hits,
                                                     uint32_t n_reads, uint64_t *keys)
{
    if (d_n)
        n_pairs = min(n_pairs, *d_n);
    for (uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x; p < n_pairs;
         p += (uint64_t)gridDim.x * 256) {
        const int s = hits[p].score;
        const uint32_t rid = win[p].read_id;
        if (s < 0 || rid >= n_reads)
            continue;
        const uint64_t key = ((uint64_t)(uint32_t)(s + 1) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)p);
        atomicMax(reinterpret_cast<unsigned long long *>(keys + rid), (unsigned long long)key);
    }
}

__global__ void __launch_bounds__(256) k_best_final(uint32_t n_reads, const uint64_t *keys,
                                                    int32_t t_map, uint32_t *best_pair,
                                                    int32_t *best_score, uint8_t *mapped)
{
    for (uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x; r < n_reads;
         r += (uint64_t)gridDim.x * 256) {
        const uint64_t k = keys[r];
        const int score = k ? (int)(k >> 32) - 1 : -1;
        const uint32_t pair = k ? 0xFFFFFFFFu - (uint32_t)k : 0xFFFFFFFFu;
        best_pair[r] = pair;
        best_score[r] = score;
        if (mapped)
            mapped[r] = (k && score >= t_map) ? 1 : 0;
    }
}

// out[k] = win[ids[k]]; an id outside the batch gives a window with an invalid
// read id, which every later call answers as an invalid pair
__global__ void __launch_bounds__(256) k_select_windows(uint32_t n, const uint32_t *ids,
                                                        const sw_window *win, uint32_t n_pairs,
                                                        const uint32_t *d_n, sw_window *out)
{
    if (d_n)
        n_pairs = min(n_pairs, *d_n);
    for (uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (uint64_t)gridDim.x * 256) {
        const uint32_t p = ids[k];
        sw_window w{0xFFFFFFFFu, 0u, 0u, 0u, 0u};
        if (p < n_pairs)
            w = win[p];
        out[k] = w;
    }
}

// Reads with a single scoring pair.  A pair scores when its read id is in
// range and the read lies inside the packed reads (the rule of the bucketing
// pass; empty windows score 0 and count).  Per read, one 64-bit word gathers
// the number of scoring pairs (low half) and the sum of their indices (high
// half), which is the pair itself when the count is one; the count stays far
// below 2^32, so the halves never carry into each other.
__device__ __forceinline__ bool scores(const sw_batch &b, uint32_t p, uint32_t &rid)
{
    rid = b.d_win[p].read_id;
    return rid < b.n_reads && b.d_read_off[rid] + b.d_read_len[rid] <= b.reads_len;
}

__global__ void __launch_bounds__(256) k_sole_count(sw_batch b, uint64_t *keys)
{
    const uint32_t n_pairs = b.d_n_pairs ? min(b.n_pairs, *b.d_n_pairs) : b.n_pairs;
    for (uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x; p < n_pairs;
         p += (uint64_t)gridDim.x * 256) {
        uint32_t rid;
        if (scores(b, (uint32_t)p, rid))
            atomicAdd(reinterpret_cast<unsigned long long *>(keys + rid),
                      (unsigned long long)((p << 32) | 1ull));
    }
}

// keep[p]: a scoring pair of a read with two or more (over all n_pairs
// entries, so that the compaction can run over the host count)
__global__ void __launch_bounds__(256) k_sole_keep(sw_batch b, const uint64_t *keys, uint8_t *keep)
{
    const uint32_t n_valid = b.d_n_pairs ? min(b.n_pairs, *b.d_n_pairs) : b.n_pairs;
    for (uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x; p < b.n_pairs;
         p += (uint64_t)gridDim.x * 256) {
        uint32_t rid;
        keep[p] = (p < n_valid && scores(b, (uint32_t)p, rid) && (uint32_t)keys[rid] >= 2u) ? 1 : 0;
    }
}

__global__ void __launch_bounds__(256) k_sole_final(uint32_t n_reads, const uint64_t *keys,
                                                    uint32_t *sole)
{
    for (uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x; r < n_reads;
         r += (uint64_t)gridDim.x * 256) {
        const uint64_t k = keys[r];
        sole[r] = (uint32_t)k == 1u ? (uint32_t)(k >> 32) : kNoPair;
    }
}

__global__ void __launch_bounds__(256) k_merge_best(uint32_t n_reads, const uint32_t *sole,
                                                    const uint32_t *sub_best, const uint32_t *ids,
                                                    uint32_t n_ids, uint32_t *best_pair)
{
    for (uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x; r < n_reads;
         r += (uint64_t)gridDim.x * 256) {
        const uint32_t s = sole[r];
        const uint32_t q = sub_best[r];
        best_pair[r] = s != kNoPair ? s : (q < n_ids ? ids[q] : kNoPair);
    }
}

unsigned grid_for(uint64_t n)
{
    uint64_t b = (n + 255) / 256;
    if (b > 16384) b = 16384;
    if (b == 0) b = 1;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_best(const sw_batch &b, const sw_hit *hits, uint64_t *keys, int32_t t_map,
                       uint32_t *best_pair, int32_t *best_score, uint8_t *mapped, hipStream_t st)
{
    hipLaunchKernelGGL(k_best_init, dim3(grid_for(b.n_reads)), dim3(256), 0, st, b.n_reads, keys);
    if (b.n_pairs)
        hipLaunchKernelGGL(k_best_update, dim3(grid_for(b.n_pairs)), dim3(256), 0, st, b.n_pairs,
                           b.d_n_pairs, b.d_win, hits, b.n_reads, keys);
    hipLaunchKernelGGL(k_best_final, dim3(grid_for(b.n_reads)), dim3(256), 0, st, b.n_reads, keys,
                       t_map, best_pair, best_score, mapped);
    return hipGetLastError();
}

hipError_t launch_select_windows(const sw_batch &b, const uint32_t *ids, uint32_t n, sw_window *out,
                                 hipStream_t st)
{
    if (n)
        hipLaunchKernelGGL(k_select_windows, dim3(grid_for(n)), dim3(256), 0, st, n, ids, b.d_win,
                           b.n_pairs, b.d_n_pairs, out);
    return hipGetLastError();
}

hipError_t launch_sole_windows(const sw_batch &b, uint64_t *keys, uint8_t *keep, uint32_t *sole,
                               hipStream_t st)
{
    hipLaunchKernelGGL(k_best_init, dim3(grid_for(b.n_reads)), dim3(256), 0, st, b.n_reads, keys);
    if (b.n_pairs) {
        hipLaunchKernelGGL(k_sole_count, dim3(grid_for(b.n_pairs)), dim3(256), 0, st, b, keys);
        hipLaunchKernelGGL(k_sole_keep, dim3(grid_for(b.n_pairs)), dim3(256), 0, st, b, keys, keep);
    }
    hipLaunchKernelGGL(k_sole_final, dim3(grid_for(b.n_reads)), dim3(256), 0, st, b.n_reads, keys,
                       sole);
    return hipGetLastError();
}

hipError_t launch_merge_best(uint32_t n_reads, const uint32_t *sole, const uint32_t *sub_best,
                             const uint32_t *ids, uint32_t n_ids, uint32_t *best_pair,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_merge_best, dim3(grid_for(n_reads)), dim3(256), 0, st, n_reads, sole,
                       sub_best, ids, n_ids, best_pair);
    return hipGetLastError();
}

}  // namespace hpgsw
