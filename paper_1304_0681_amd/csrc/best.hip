// Best hit per read (stage E, task iv): segmented arg-max over each read's
// windows.  Pairs may come in any order, so the reduction is an atomic max on
// a 64-bit key per read: (score + 1) in the high word, the complement of the
// pair index in the low word, which makes the lowest pair index win ties.
#include "internal.h"

namespace hpgsw {

namespace {

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

}  // namespace hpgsw
