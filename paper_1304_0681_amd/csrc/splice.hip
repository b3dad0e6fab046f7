// Spliced reads (stage E of Sec. 2, tasks i, ii and iv): candidate alignment
// locations (CALs) from seed alignments, their extension and joining into
// windows for whole-read alignment, and splice-junction detection on the
// read alignments, counted in a device hash table (the AVL tree of the paper).
//
// All of this is light next to the dynamic programming it feeds or reads:
// one lane per seed, per read or per alignment, memory-bound on a few bytes
// per item; the hash table is open addressing with linear probing on 64-bit
// keys, updated with atomics, so counts accumulate across calls (chunks).
#include "internal.h"

namespace hpgsw {

namespace {

constexpr int kMaxCals = 16;     // CALs per read taken into the joining

unsigned blocks_for(uint64_t n)
{
    uint64_t b = (n + 255) / 256;
    if (b > 65535) b = 65535;
    return (unsigned)(b ? b : 1);
}

// ---------------------------------------------------------------------------
// CALs from seed alignments: seed s aligned best in window best_pair[s] with
// alignment aln[s]; its CAL is that alignment's reference span.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_seed_cals(uint32_t n_seeds, const sw_window *win,
                                                   uint32_t n_pairs, const uint32_t *d_n,
                                                   const uint32_t *best_pair, const sw_aln *aln,
                                                   const uint32_t *seed_read, int32_t min_score,
                                                   sw_cal *out)
{
    if (d_n)
        n_pairs = min(n_pairs, *d_n);
    for (uint64_t s = (uint64_t)blockIdx.x * 256 + threadIdx.x; s < n_seeds;
         s += (uint64_t)gridDim.x * 256) {
        const uint32_t p = best_pair[s];
        const sw_aln a = aln[s];
        sw_cal c{seed_read[s], 0u, 0u, 0u, 0u, 0u};
        if (p < n_pairs && a.score >= min_score && a.score > 0 && a.ref_begin >= 0) {
            const sw_window w = win[p];
            const uint64_t first = (uint64_t)w.ref_begin + (uint32_t)a.ref_begin;
            const uint64_t last = (uint64_t)w.ref_begin + (uint32_t)a.ref_end;
            if (last < (1ull << 32)) {
                c.first = (uint32_t)first;
                c.last = (uint32_t)last;
                c.strand = w.strand;
                c.valid = 1;
            }
        }
        out[s] = c;
    }
}

// ---------------------------------------------------------------------------
// Joining.  CALs come grouped by read; the first lane of every run of equal
// read ids takes the run's first kMaxCals valid CALs, extends them, sorts them
// by (strand, first, last) and merges neighbours whose gap is below max_gap.
// A run of k CALs yields at most k windows, written to its own positions
// [run start, run start + windows), and flagged for the stable compaction.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_fill_u8(uint64_t n, uint8_t *p)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
        p[i] = 0;
}

__global__ void __launch_bounds__(256) k_join(uint32_t n, const sw_cal *cals, uint32_t n_reads,
                                              uint64_t ref_len, uint32_t ext, uint32_t max_gap,
                                              sw_window *tmp, uint8_t *keep)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        const uint32_t rid = cals[i].read_id;
        if ((i > 0 && cals[i - 1].read_id == rid) || rid >= n_reads)
            continue;
        // extended CALs sorted by (strand, first, last): (strand << 40) | first
        // in kf, last in kl
        uint64_t kf[kMaxCals];
        uint64_t kl[kMaxCals];
        int cnt = 0;
        for (uint64_t j = i; j < n && cnt < kMaxCals; ++j) {
            const sw_cal c = cals[j];
            if (c.read_id != rid)
                break;
            if (!c.valid || c.first > c.last || c.last >= ref_len)
                continue;
            const uint64_t b = c.first >= ext ? (uint64_t)c.first - ext : 0ull;
            const uint64_t e = min((uint64_t)c.last + ext, ref_len - 1);
            // insertion into the sorted prefix
            const uint64_t f = ((uint64_t)(c.strand ? 1 : 0) << 40) | b;
            int k = cnt;
            while (k > 0 && (kf[k - 1] > f || (kf[k - 1] == f && kl[k - 1] > e))) {
                kf[k] = kf[k - 1];
                kl[k] = kl[k - 1];
                --k;
            }
            kf[k] = f;
            kl[k] = e;
            ++cnt;
        }
        uint64_t out = i;
        int k = 0;
        while (k < cnt) {
            const uint64_t st = kf[k] >> 40;
            const uint64_t b = kf[k] & ((1ull << 40) - 1);
            uint64_t e = kl[k];
            ++k;
            // the next CAL joins while it has this strand and fewer than
            // max_gap bases lie strictly between them (overlap joins)
            while (k < cnt && (kf[k] >> 40) == st &&
                   (int64_t)(kf[k] & ((1ull << 40) - 1)) - (int64_t)e - 1 < (int64_t)max_gap) {
                e = max(e, kl[k]);
                ++k;
            }
            const uint64_t len = e - b + 1;
            tmp[out] = sw_window{rid, (uint32_t)b, (uint16_t)(len < 65535 ? len : 65535),
                                 (uint8_t)st, 0u};
            keep[out] = 1;
            ++out;
        }
    }
}

// ---------------------------------------------------------------------------
// Junction detection and counting.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t base_at(const uint32_t *ref, uint64_t p)
{
    return (ref[p >> 4] >> (2u * (uint32_t)(p & 15))) & 3u;
}

// MurmurHash3's 64-bit finaliser (Appleby), as a slot hash.
__device__ __forceinline__ uint64_t fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

__device__ bool table_add(uint64_t key, unsigned long long *keys, uint32_t *counts, uint32_t cap)
{
    const uint32_t mask = cap - 1;
    uint32_t h = (uint32_t)fmix64(key) & mask;
    for (uint32_t t = 0; t < cap; ++t) {
        const unsigned long long prev = atomicCAS(keys + h, 0ull, (unsigned long long)key);
        if (prev == 0ull || prev == key) {
            atomicAdd(counts + h, 1u);
            return true;
        }
        h = (h + 1) & mask;
    }
    return false;
}

struct DetectParams {
    uint32_t n;
    const uint32_t *pair_ids;
    const sw_window *win;
    uint32_t n_pairs;
    const uint32_t *d_n;
    const uint32_t *ref;
    uint64_t ref_len;
    const sw_aln *aln;
    uint32_t *ops;
    uint32_t ops_stride;
    int32_t min_score;
    uint32_t min_intron;
    unsigned long long *keys;
    uint32_t *counts;
    uint32_t cap;
    uint32_t *n_junc;
    uint32_t *dropped;
};

// Motif of the run [x, x + L) of reference positions: 0 GT...AG, 1 CT...AC, -1 none.
__device__ __forceinline__ int motif_at(const uint32_t *ref, uint64_t x, uint32_t L)
{
    const uint32_t h0 = base_at(ref, x), h1 = base_at(ref, x + 1);
    const uint32_t t0 = base_at(ref, x + L - 2), t1 = base_at(ref, x + L - 1);
    if (h0 == 2 && h1 == 3 && t0 == 0 && t1 == 2)
        return 0;
    if (h0 == 1 && h1 == 3 && t0 == 0 && t1 == 1)
        return 1;
    return -1;
}

__global__ void __launch_bounds__(256) k_detect(const DetectParams P)
{
    const uint32_t n_pairs = P.d_n ? min(P.n_pairs, *P.d_n) : P.n_pairs;
    for (uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x; k < P.n; k += (uint64_t)gridDim.x * 256) {
        uint32_t found = 0;
        const uint32_t pair = P.pair_ids[k];
        const sw_aln a = P.aln[k];
        if (pair < n_pairs && (a.status & 7u) == 0 && a.score > 0 && a.score >= P.min_score &&
            a.ref_begin >= 0) {
            const sw_window w = P.win[pair];
            uint32_t *ops = P.ops + k * (uint64_t)P.ops_stride;
            const uint32_t n_ops = min(a.n_ops, P.ops_stride);
            const uint64_t wb = w.ref_begin;       // window column 0
            int64_t r = a.ref_begin;                // window column of the next op
            uint32_t prev = 0, cur = n_ops ? ops[0] : 0u;
            for (uint32_t j = 0; j < n_ops; ++j) {
                uint32_t nxt = j + 1 < n_ops ? ops[j + 1] : 0u;
                const uint32_t L = cur >> 4;
                if ((cur & 15u) == SW_OP_D && L >= P.min_intron && j > 0 && j + 1 < n_ops &&
                    (prev & 15u) == SW_OP_M && (nxt & 15u) == SW_OP_M) {
                    const int64_t ra = prev >> 4, rb = nxt >> 4;
                    const uint64_t x = wb + (uint64_t)r;     // first deleted position
                    // every base read below lies in [x - ra, x + L + rb); ops that
                    // reach outside the reference are not searched
                    if (L <= 0xFFFFu && x >= (uint64_t)ra && x + L + (uint64_t)rb <= P.ref_len) {
                        // neutral shifts: left while the base before the run equals
                        // the run's last base, right while its first equals the base
                        // after it
                        int64_t lo = 0;
                        while (lo < ra - 1 &&
                               base_at(P.ref, x - lo - 1) == base_at(P.ref, x + L - lo - 1))
                            ++lo;
                        int64_t hi = 0;
                        while (hi < rb - 1 && base_at(P.ref, x + hi) == base_at(P.ref, x + L + hi))
                            ++hi;
                        for (int64_t s = -lo; s <= hi; ++s) {
                            const int m = motif_at(P.ref, x + s, L);
                            if (m < 0)
                                continue;
                            prev = (uint32_t)((ra + s) << 4) | SW_OP_M;
                            nxt = (uint32_t)((rb - s) << 4) | SW_OP_M;
                            cur = (L << 4) | SW_OP_N;
                            const uint64_t start = x + s;
                            const uint64_t key = (start << 17) | ((uint64_t)L << 1) | (uint64_t)m;
                            if (!table_add(key, P.keys, P.counts, P.cap) && P.dropped)
                                atomicAdd(P.dropped, 1u);
                            ++found;
                            r += s;
                            break;
                        }
                    }
                }
                if (j > 0)
                    ops[j - 1] = prev;
                const uint32_t c = cur & 15u;
                if (c == SW_OP_M || c == SW_OP_D || c == SW_OP_N)
                    r += cur >> 4;
                prev = cur;
                cur = nxt;
            }
            if (n_ops)
                ops[n_ops - 1] = prev;
        }
        if (P.n_junc)
            P.n_junc[k] = found;
    }
}

__global__ void __launch_bounds__(256) k_table_clear(uint32_t cap, unsigned long long *keys,
                                                     uint32_t *counts)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * 256) {
        keys[i] = 0ull;
        counts[i] = 0u;
    }
}

__global__ void k_zero_one(uint32_t *p)
{
    if (threadIdx.x == 0)
        *p = 0;
}

__global__ void __launch_bounds__(256) k_list(uint32_t cap, const unsigned long long *keys,
                                              const uint32_t *counts, sw_junction *out,
                                              uint32_t out_cap, uint32_t *d_n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * 256) {
        const uint64_t key = keys[i];
        if (!key)
            continue;
        const uint32_t pos = atomicAdd(d_n, 1u);
        if (pos < out_cap) {
            const uint64_t start = key >> 17;
            const uint32_t L = (uint32_t)(key >> 1) & 0xFFFFu;
            out[pos] = sw_junction{start, start + L, counts[i], (uint32_t)(key & 1)};
        }
    }
}

}  // namespace

hipError_t launch_seed_cals(const sw_batch &b, const uint32_t *best_pair, const sw_aln *aln,
                            const uint32_t *seed_read, uint32_t n_seeds, int32_t min_score,
                            sw_cal *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_seed_cals, dim3(blocks_for(n_seeds)), dim3(256), 0, st, n_seeds, b.d_win,
                       b.n_pairs, b.d_n_pairs, best_pair, aln, seed_read, min_score, out);
    return hipGetLastError();
}

hipError_t launch_join(uint32_t n, const sw_cal *cals, uint32_t n_reads, uint64_t ref_len,
                       uint32_t ext, uint32_t max_gap, sw_window *tmp, uint8_t *keep,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u8, dim3(blocks_for(n)), dim3(256), 0, st, (uint64_t)n, keep);
    hipLaunchKernelGGL(k_join, dim3(blocks_for(n)), dim3(256), 0, st, n, cals, n_reads, ref_len,
                       ext, max_gap, tmp, keep);
    return hipGetLastError();
}

hipError_t launch_detect(const sw_batch &b, const uint32_t *pair_ids, uint32_t n, const sw_aln *aln,
                         uint32_t *ops, uint32_t ops_stride, int32_t min_score, uint32_t min_intron,
                         uint64_t *keys, uint32_t *counts, uint32_t cap, uint32_t *n_junc,
                         uint32_t *dropped, hipStream_t st)
{
    DetectParams p;
    p.n = n;
    p.pair_ids = pair_ids;
    p.win = b.d_win;
    p.n_pairs = b.n_pairs;
    p.d_n = b.d_n_pairs;
    p.ref = b.d_ref2b;
    p.ref_len = b.ref_len;
    p.aln = aln;
    p.ops = ops;
    p.ops_stride = ops_stride;
    p.min_score = min_score;
    p.min_intron = min_intron;
    p.keys = reinterpret_cast<unsigned long long *>(keys);
    p.counts = counts;
    p.cap = cap;
    p.n_junc = n_junc;
    p.dropped = dropped;
    hipLaunchKernelGGL(k_detect, dim3(blocks_for(n)), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_table_clear(uint64_t *keys, uint32_t *counts, uint32_t cap, hipStream_t st)
{
    hipLaunchKernelGGL(k_table_clear, dim3(blocks_for(cap)), dim3(256), 0, st, cap,
                       reinterpret_cast<unsigned long long *>(keys), counts);
    return hipGetLastError();
}

hipError_t launch_list(const uint64_t *keys, const uint32_t *counts, uint32_t cap, sw_junction *out,
                       uint32_t out_cap, uint32_t *d_n, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_one, dim3(1), dim3(64), 0, st, d_n);
    hipLaunchKernelGGL(k_list, dim3(blocks_for(cap)), dim3(256), 0, st, cap,
                       reinterpret_cast<const unsigned long long *>(keys), counts, out, out_cap, d_n);
    return hipGetLastError();
}

}  // namespace hpgsw
