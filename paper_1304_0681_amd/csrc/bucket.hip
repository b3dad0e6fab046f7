// Length bucketing of (read, window) pairs.
//
// Every pair is put in a bin keyed by (length class of its query, window length,
// longest first).  A block-level counting sort (LDS histogram, one global
// atomic per block and bin, exclusive scan, scatter) produces the pair order
// the persistent wavefront kernels consume; each class occupies one contiguous
// segment whose bounds stay on the device, so the host never waits for counts.
// Pairs that need no dynamic programming (empty read or window, invalid read
// id) are answered here directly.
#include "internal.h"

namespace hpgsw {

namespace {

constexpr int kBlock = 256;
constexpr int kItems = 16;                 // pairs per thread per block pass
constexpr uint32_t kNone = 0xFFFFFFFFu;

// query-length class of a read: the first class whose upper bound holds it
// (default bounds 16 32 64 100 128 160 256 512 1024 2048 65535)
__device__ __forceinline__ int class_of(uint32_t m, const ClassEdges &e)
{
    int c = 0;
#pragma unroll
    for (int k = 0; k < kNumClasses - 1; ++k)
        c += m > e.m_max[k] ? 1 : 0;
    return c;
}

__device__ __forceinline__ uint32_t len_bin(uint32_t n)
{
    // 8-base bins below 4096, 128-base bins above; longest first
    uint32_t b = n < 4096 ? (n >> 3) : 512u + ((n - 4096u) >> 7);
    return (kBinsPerClass - 1) - b;
}

// Trivial pairs are answered in place: hits[k] (scoring) or aln[k] (traceback).
__device__ __forceinline__ void trivial(uint32_t k, int score, sw_hit *hits, sw_aln *aln)
{
    if (hits)
        hits[k] = sw_hit{score, -1, -1};
    if (aln)
        aln[k] = sw_aln{score, -1, -1, -1, -1, 0u, score < 0 ? 2u : 0u};
}

__device__ __forceinline__ uint32_t pair_bin(const sw_batch &b, const uint32_t *sel, uint32_t k,
                                             sw_hit *hits, sw_aln *aln, const TbBand &band,
                                             const ClassEdges &edges, uint32_t &n_out,
                                             uint32_t &m_out)
{
    const uint32_t p = sel ? sel[k] : k;
    n_out = 0;
    m_out = 0;
    if (p >= b.n_pairs) {
        trivial(k, -1, hits, aln);
        return kNone;
    }
    const sw_window w = b.d_win[p];
    if (w.read_id >= b.n_reads) {
        trivial(k, -1, hits, aln);
        return kNone;
    }
    const uint32_t m = b.d_read_len[w.read_id];
    if (b.d_read_off[w.read_id] + m > b.reads_len) {    // read outside the packed reads
        trivial(k, -1, hits, aln);
        return kNone;
    }
    uint32_t n = 0;
    if ((uint64_t)w.ref_begin < b.ref_len) {
        const uint64_t avail = b.ref_len - w.ref_begin;
        n = w.len < avail ? w.len : (uint32_t)avail;
    }
    if (m == 0 || n == 0) {
        trivial(k, 0, hits, aln);
        return kNone;
    }
    if (aln) {      // traceback: the width its DP covers
        int c_lo;
        n = (uint32_t)tb_band(band, p, (int)m, (int)n, c_lo);
    }
    n_out = n;
    m_out = m;
    return (uint32_t)class_of(m, edges) * kBinsPerClass + len_bin(n);
}

__global__ void __launch_bounds__(kBlock) k_zero(uint32_t *hist, uint32_t *maxlen)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < kNumBins; i += gridDim.x * kBlock)
        hist[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < 2 * kNumClasses)
        maxlen[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(kBlock) k_classify(sw_batch b, const uint32_t *sel, uint32_t n_items,
                                                     uint32_t *bin_out, uint32_t *hist,
                                                     uint32_t *maxlen, sw_hit *hits, sw_aln *aln,
                                                     TbBand band, ClassEdges edges)
{
    __shared__ uint32_t lh[kNumBins];
    __shared__ uint32_t lmax[2 * kNumClasses];
    for (int i = threadIdx.x; i < kNumBins; i += kBlock)
        lh[i] = 0;
    if (threadIdx.x < 2 * kNumClasses)
        lmax[threadIdx.x] = 0;
    __syncthreads();
    if (!sel && b.d_n_pairs)
        n_items = min(n_items, *b.d_n_pairs);
    const uint64_t base = (uint64_t)blockIdx.x * kBlock * kItems;
    for (int k = 0; k < kItems; ++k) {
        const uint64_t p = base + (uint64_t)k * kBlock + threadIdx.x;
        if (p >= n_items)
            break;
        uint32_t n = 0, m = 0;
        const uint32_t bin = pair_bin(b, sel, (uint32_t)p, hits, aln, band, edges, n, m);
        bin_out[p] = bin;
        if (bin != kNone) {
            atomicAdd(&lh[bin], 1u);
            atomicMax(&lmax[bin / kBinsPerClass], n);
            atomicMax(&lmax[kNumClasses + bin / kBinsPerClass], m);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kNumBins; i += kBlock)
        if (lh[i])
            atomicAdd(&hist[i], lh[i]);
    if (threadIdx.x < 2 * kNumClasses && lmax[threadIdx.x])
        atomicMax(&maxlen[threadIdx.x], lmax[threadIdx.x]);
}

// One block: exclusive scan of the bin counts into cursors; class segments.
__global__ void __launch_bounds__(1024) k_scan(uint32_t *hist, uint32_t *seg, uint32_t *counter)
{
    constexpr int T = 1024;
    constexpr int PER = (kNumBins + T - 1) / T;
    __shared__ uint32_t part[T];
    const int t = threadIdx.x;
    uint32_t local[PER];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = t * PER + k;
        local[k] = i < kNumBins ? hist[i] : 0u;
        sum += local[k];
    }
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < T; off <<= 1) {      // Hillis-Steele inclusive scan
        uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = t * PER + k;
        if (i < kNumBins) {
            if (i % kBinsPerClass == 0)
                seg[2 * (i / kBinsPerClass)] = run;
            if (i % kBinsPerClass == kBinsPerClass - 1)
                seg[2 * (i / kBinsPerClass) + 1] = run + local[k];
            hist[i] = run;
        }
        run += local[k];
    }
    if (t < kNumClasses)
        counter[t] = 0;
}

__global__ void __launch_bounds__(kBlock) k_scatter(uint32_t n_pairs, const uint32_t *d_n,
                                                    const uint32_t *bin_in, uint32_t *cursor,
                                                    uint32_t *ids)
{
    if (d_n)
        n_pairs = min(n_pairs, *d_n);
    __shared__ uint32_t lh[kNumBins];
    for (int i = threadIdx.x; i < kNumBins; i += kBlock)
        lh[i] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kBlock * kItems;
    uint32_t rank[kItems];
    uint32_t bins[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint64_t p = base + (uint64_t)k * kBlock + threadIdx.x;
        bins[k] = p < n_pairs ? bin_in[p] : kNone;
        rank[k] = bins[k] != kNone ? atomicAdd(&lh[bins[k]], 1u) : 0u;
    }
    __syncthreads();
    // reserve a contiguous range per (block, bin)
    for (int i = threadIdx.x; i < kNumBins; i += kBlock)
        if (lh[i])
            lh[i] = atomicAdd(&cursor[i], lh[i]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint64_t p = base + (uint64_t)k * kBlock + threadIdx.x;
        if (bins[k] != kNone)
            ids[lh[bins[k]] + rank[k]] = (uint32_t)p;
    }
}

}  // namespace

ClassEdges default_edges()
{
    ClassEdges e;
    for (int c = 0; c < kNumClasses; ++c)
        e.m_max[c] = (uint32_t)kDefaultClasses[c].m_max;
    return e;
}

hipError_t launch_bucket(const sw_batch &b, const uint32_t *sel, uint32_t n_items,
                         const BucketScratch &s, sw_hit *hits, sw_aln *aln, hipStream_t st,
                         const ClassEdges &edges, const TbBand &band)
{
    hipLaunchKernelGGL(k_zero, dim3(64), dim3(kBlock), 0, st, s.hist, s.maxlen);
    const uint64_t per_block = (uint64_t)kBlock * kItems;
    const unsigned blocks = (unsigned)((n_items + per_block - 1) / per_block);
    if (n_items)
        hipLaunchKernelGGL(k_classify, dim3(blocks), dim3(kBlock), 0, st, b, sel, n_items, s.bin,
                           s.hist, s.maxlen, hits, aln, band, edges);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, s.hist, s.seg, s.counter);
    if (n_items)
        hipLaunchKernelGGL(k_scatter, dim3(blocks), dim3(kBlock), 0, st, n_items,
                           sel ? nullptr : b.d_n_pairs, s.bin, s.hist, s.ids);
    return hipGetLastError();
}

}  // namespace hpgsw
