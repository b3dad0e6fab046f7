// Region seeker and CAL seeker (stages C and D of Sec. 2): an exact k-mer index
// of the reference, the two-phase seeds of every read looked up in it on both
// strands (regions), and each read's regions merged into candidate alignment
// locations (CALs).
//
// The index is a direct-address table: for k <= 15 the 4^k k-mer codes (at
// most 2^30, 4 GiB of 32-bit offsets) index the start of each k-mer's
// positions, so a seed lookup is two loads, with no hashing or search.  It is
// built by a counting sort on the device (histogram with atomics, inclusive
// scan, scatter with atomic decrements that leaves each code's start).
// Positions within a code come out in no particular order; the region writer
// sorts the few positions of each seed it emits, so regions are deterministic.
#include "internal.h"

namespace hpgsw {

namespace {

constexpr int kTile = 4096;            // entries per tile of the scans
constexpr int kMaxRegions = SW_SEEKER_MAX_REGIONS;
constexpr int kCals = SW_SEEKER_MAX_CALS;

unsigned blocks_for(uint64_t n)
{
    uint64_t b = (n + 255) / 256;
    if (b > 65535) b = 65535;
    return (unsigned)(b ? b : 1);
}

// k bases starting at base p of a packed sequence (base i at bits 2i), k <= 16
__device__ __forceinline__ uint32_t kmer_at(const uint32_t *seq, uint64_t words, uint64_t p,
                                            uint32_t mask)
{
    const uint64_t w = p >> 4;
    const uint32_t lo = seq[w];
    const uint32_t hi = w + 1 < words ? seq[w + 1] : 0u;
    return __builtin_amdgcn_alignbit(hi, lo, (uint32_t)(p & 15) * 2u) & mask;
}

// reverse complement of a k-mer code
__device__ __forceinline__ uint32_t revcomp_k(uint32_t x, uint32_t k)
{
    const uint32_t c = ~x & ((k == 16) ? 0xFFFFFFFFu : ((1u << (2 * k)) - 1u));
    const uint32_t r = __builtin_bitreverse32(c) >> (32 - 2 * k);
    return ((r & 0x55555555u) << 1) | ((r >> 1) & 0x55555555u);
}

// ---------------------------------------------------------------------------
// Inclusive scan of n 32-bit counts into T (uint32 in place, or uint64), in
// tiles of kTile: tile sums, one block over the tile sums, then each tile
// scanned with its offset.  At most 1024 * 256 tiles (2^30 entries).
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) k_tile_sums(const uint32_t *in, uint64_t n, T *tsum)
{
    __shared__ T part[256];
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    T s = 0;
    for (int i = threadIdx.x; i < kTile; i += 256)
        if (base + i < n)
            s += in[base + i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        tsum[blockIdx.x] = part[0];
}

// exclusive scan of the tile sums (one block)
template <class T>
__global__ void __launch_bounds__(1024) k_tile_offsets(uint32_t nt, T *tsum)
{
    __shared__ T part[1024];
    const int t = threadIdx.x;
    const uint32_t per = (nt + 1023) / 1024;
    T s = 0;
    for (uint32_t k = 0; k < per; ++k) {
        const uint64_t i = (uint64_t)t * per + k;
        if (i < nt)
            s += tsum[i];
    }
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const T v = t >= off ? part[t - off] : (T)0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    T run = part[t] - s;
    for (uint32_t k = 0; k < per; ++k) {
        const uint64_t i = (uint64_t)t * per + k;
        if (i < nt) {
            const T c = tsum[i];
            tsum[i] = run;
            run += c;
        }
    }
}

// LDS word of tile entry i: one pad word per 32 keeps a thread's 16
// consecutive entries off a single bank
__device__ __forceinline__ int padded(int i) { return i + (i >> 5); }

template <class T>
__global__ void __launch_bounds__(256) k_tile_scan(const uint32_t *in, uint64_t n, const T *toff,
                                                   T *out)
{
    __shared__ T part[256];
    __shared__ T buf[kTile + kTile / 32];
    constexpr int PER = kTile / 256;   // consecutive entries per thread
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    // coalesced loads through LDS, then each thread takes 16 consecutive entries
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = k * 256 + threadIdx.x;
        buf[padded(i)] = base + i < n ? (T)in[base + i] : (T)0;
    }
    __syncthreads();
    const int my = threadIdx.x * PER;
    T v[PER];
    T s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = buf[padded(my + k)];
        s += v[k];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const T x = threadIdx.x >= off ? part[threadIdx.x - off] : (T)0;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    T run = toff[blockIdx.x] + part[threadIdx.x] - s;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        run += v[k];
        buf[padded(my + k)] = run;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int i = k * 256 + threadIdx.x;
        if (base + i < n)
            out[base + i] = buf[padded(i)];
    }
}

// ---------------------------------------------------------------------------
// Index build.  starts[c] = first slot of k-mer c in pos[]; starts[4^k] = n_pos.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_fill32(uint64_t n, uint32_t *p)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
        p[i] = 0u;
}

__global__ void __launch_bounds__(256) k_kmer_hist(const uint32_t *ref, uint64_t ref_words,
                                                   uint64_t n_pos, uint32_t mask, uint32_t *cnt)
{
    for (uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x; p < n_pos; p += (uint64_t)gridDim.x * 256)
        atomicAdd(cnt + kmer_at(ref, ref_words, p, mask), 1u);
}

// after the inclusive scan cnt[c] is the end of k-mer c; taking one slot per
// position from the top leaves its start
__global__ void __launch_bounds__(256) k_kmer_scatter(const uint32_t *ref, uint64_t ref_words,
                                                      uint64_t n_pos, uint32_t mask, uint32_t *starts,
                                                      uint32_t *pos)
{
    for (uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x; p < n_pos; p += (uint64_t)gridDim.x * 256) {
        const uint32_t slot = atomicSub(starts + kmer_at(ref, ref_words, p, mask), 1u) - 1u;
        pos[slot] = (uint32_t)p;
    }
}

__global__ void k_set_last(uint32_t *starts, uint64_t n_codes, uint32_t n_pos)
{
    if (threadIdx.x == 0)
        starts[n_codes] = n_pos;
}

// ---------------------------------------------------------------------------
// Regions.  One lane per read: its seeds in order (phase one, then phase two),
// strand 0 then strand 1 per seed, each strand's positions ascending.
// ---------------------------------------------------------------------------
struct SeedParams {
    const uint32_t *reads;
    uint64_t read_words;
    const uint64_t *read_off;
    const uint16_t *read_len;
    uint32_t n_reads;
    uint64_t reads_len;
    const uint32_t *starts;
    const uint32_t *pos;
    uint32_t k, step, offset, max_occ, mask;
};

__device__ __forceinline__ uint32_t n_seeds(uint32_t m, const SeedParams &P)
{
    const uint32_t a = m >= P.k ? (m - P.k) / P.step + 1 : 0u;
    const uint32_t b = m >= P.offset + P.k ? (m - P.offset - P.k) / P.step + 1 : 0u;
    return a + b;
}

__device__ __forceinline__ uint32_t seed_start(uint32_t j, uint32_t m, const SeedParams &P)
{
    const uint32_t a = m >= P.k ? (m - P.k) / P.step + 1 : 0u;
    return j < a ? j * P.step : P.offset + (j - a) * P.step;
}

__device__ __forceinline__ bool read_ok(uint32_t r, const SeedParams &P, uint32_t &m, uint64_t &off)
{
    m = P.read_len[r];
    off = P.read_off[r];
    return off + m <= P.reads_len;
}

__global__ void __launch_bounds__(256) k_region_count(const SeedParams P, uint32_t *cnt)
{
    for (uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x; r < P.n_reads; r += (uint64_t)gridDim.x * 256) {
        uint32_t m;
        uint64_t off;
        uint32_t c = 0;
        if (read_ok((uint32_t)r, P, m, off)) {
            const uint32_t ns = n_seeds(m, P);
            for (uint32_t j = 0; j < ns; ++j) {
                const uint32_t s = seed_start(j, m, P);
                const uint32_t fw = kmer_at(P.reads, P.read_words, off + s, P.mask);
                const uint32_t rv = revcomp_k(fw, P.k);
                const uint32_t nf = P.starts[fw + 1] - P.starts[fw];
                const uint32_t nr = P.starts[rv + 1] - P.starts[rv];
                c += (nf <= P.max_occ ? nf : 0u) + (nr <= P.max_occ ? nr : 0u);
            }
        }
        cnt[r] = c;
    }
}

// positions [b, e) of one k-mer (at most max_occ), ascending, as regions
__device__ void emit_sorted(const SeedParams &P, uint32_t b, uint32_t e, uint8_t strand,
                            uint16_t read_pos, sw_region *out, uint64_t &w, uint64_t cap)
{
    uint32_t last = 0;
    bool have = false;
    for (uint32_t t = b; t < e; ++t) {
        // the next position: the smallest one above the last emitted
        uint32_t best = 0xFFFFFFFFu;
        for (uint32_t u = b; u < e; ++u) {
            const uint32_t x = P.pos[u];
            if ((!have || x > last) && x < best)
                best = x;
        }
        if (w < cap)
            out[w] = sw_region{best, read_pos, strand, 0u};
        ++w;
        last = best;
        have = true;
    }
}

__global__ void __launch_bounds__(256) k_region_write(const SeedParams P, const uint64_t *read_end,
                                                      sw_region *out, uint64_t cap)
{
    for (uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x; r < P.n_reads; r += (uint64_t)gridDim.x * 256) {
        uint32_t m;
        uint64_t off;
        if (!read_ok((uint32_t)r, P, m, off))
            continue;
        uint64_t w = r ? read_end[r - 1] : 0ull;
        if (w >= cap)
            continue;
        const uint32_t ns = n_seeds(m, P);
        for (uint32_t j = 0; j < ns; ++j) {
            const uint32_t s = seed_start(j, m, P);
            const uint32_t fw = kmer_at(P.reads, P.read_words, off + s, P.mask);
            const uint32_t rv = revcomp_k(fw, P.k);
            const uint32_t bf = P.starts[fw], ef = P.starts[fw + 1];
            const uint32_t br = P.starts[rv], er = P.starts[rv + 1];
            if (ef - bf <= P.max_occ)
                emit_sorted(P, bf, ef, 0, (uint16_t)s, out, w, cap);
            if (er - br <= P.max_occ)
                emit_sorted(P, br, er, 1, (uint16_t)(m - s - P.k), out, w, cap);
        }
    }
}

// LDS writes of the wave visible to all its lanes
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Bitonic sort of keys[0, P2) (P2 a power of two) by one wave, ascending.
__device__ void sort_keys(uint64_t *keys, uint32_t P2, int lane)
{
    for (uint32_t size = 2; size <= P2; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = lane; i < P2; i += 64) {
                const uint32_t j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const uint64_t x = keys[i], y = keys[j];
                    if ((x > y) == up) {
                        keys[i] = y;
                        keys[j] = x;
                    }
                }
            }
            wave_sync();
        }
    }
}

// ---------------------------------------------------------------------------
// CAL seeker: one wave per read.  Its first kMaxRegions regions are sorted in
// LDS by (strand, first) (bitonic sort), then the first lane merges them and
// writes the read's kCals CAL slots (unused slots invalid).
// ---------------------------------------------------------------------------
constexpr int kSeekWaves = 4;

__global__ void __launch_bounds__(64 * kSeekWaves) k_cal_seek(const sw_region *reg,
                                                              const uint64_t *read_end,
                                                              uint32_t n_reads, uint64_t cap,
                                                              uint32_t k, uint32_t merge_gap,
                                                              uint32_t min_len, const uint32_t *skip,
                                                              sw_cal *cals)
{
    __shared__ uint64_t keys_all[kSeekWaves][kMaxRegions];
    const uint32_t wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    uint64_t *keys = keys_all[wave];
    for (uint64_t r = (uint64_t)blockIdx.x * kSeekWaves + wave; r < n_reads;
         r += (uint64_t)gridDim.x * kSeekWaves) {
        const uint64_t b = r ? read_end[r - 1] : 0ull;
        uint64_t e = read_end[r];
        if (e > cap) e = cap;
        uint32_t n = e > b ? (uint32_t)min(e - b, (uint64_t)kMaxRegions) : 0u;
        if (skip && skip[r])
            n = 0;
        uint32_t P2 = 1;
        while (P2 < n) P2 <<= 1;
        for (uint32_t i = lane; i < P2; i += 64) {
            uint64_t key = ~0ull;       // padding sorts last
            if (i < n) {
                const sw_region g = reg[b + i];
                key = ((uint64_t)(g.strand ? 1 : 0) << 32) | g.first;
            }
            keys[i] = key;
        }
        wave_sync();
        sort_keys(keys, P2, lane);
        if (lane == 0) {
            sw_cal *out = cals + r * (uint64_t)kCals;
            int nc = 0;
            uint64_t cs = 0, cf = 0, cl = 0;
            bool have = false;
            auto close = [&]() {
                if (have && cl - cf + 1 > min_len && nc < kCals)
                    out[nc++] = sw_cal{(uint32_t)r, (uint32_t)cf, (uint32_t)cl, (uint8_t)cs, 1u, 0u};
            };
            for (uint32_t i = 0; i < n; ++i) {
                const uint64_t key = keys[i];
                const uint64_t st = key >> 32, f = key & 0xFFFFFFFFull, l = f + k - 1;
                if (have && st == cs && (int64_t)f - (int64_t)cl - 1 < (int64_t)merge_gap) {
                    cl = max(cl, l);
                } else {
                    close();
                    cs = st;
                    cf = f;
                    cl = l;
                    have = true;
                }
            }
            close();
            for (int j = nc; j < kCals; ++j)
                out[j] = sw_cal{(uint32_t)r, 0u, 0u, 0u, 0u, 0u};
        }
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// Stage B: whole-read mapping with at most one edit.  One wave per read: the
// diagonals of its first kMaxRegions regions are sorted in LDS; walking them in
// (strand, diagonal) order, every candidate start d - 1, d, d + 1 not seen
// before is verified by the whole wave (lane j compares query base j with the
// reference on the candidate's diagonal and its two neighbours, ballots give
// the mismatch positions), and the records of the fewest edits are kept.
// ---------------------------------------------------------------------------
constexpr int kBWaves = 4;
constexpr int kBMax = SW_BMAP_MAX;

struct StageBParams {
    const uint32_t *reads;
    uint64_t read_words;
    const uint64_t *read_off;
    const uint16_t *read_len;
    uint32_t n_reads;
    uint64_t reads_len;
    const uint32_t *ref;
    uint64_t ref_len;
    const sw_region *reg;
    const uint64_t *read_end;
    uint64_t cap;
    sw_bmap *maps;
    uint32_t *n_maps;
};

__device__ __forceinline__ uint32_t base_of(const uint32_t *seq, uint64_t p)
{
    return (seq[p >> 4] >> (2u * (uint32_t)(p & 15))) & 3u;
}

struct Verdict {
    int e;             // 0, 1, or 2 (no mapping at this start)
    int op;
    int pos;
    uint64_t last;
};

// Mismatches of the query (strand s) against the reference on the diagonals
// d - 2 .. d + 2 (index o + 2 for diagonal d + o): their number over the query
// and the first and last mismatching query position (m and -1 if none).  One
// pass of the whole wave: lane j compares query base j with the five
// reference bases it faces, read from one 64-bit window of the packed words;
// positions outside the reference count as mismatches.
struct DiagStats {
    int cnt[5], first[5], last[5];
};

__device__ DiagStats scan_diagonals(const StageBParams &P, uint64_t off, uint32_t m, uint32_t s,
                                    int64_t d, int lane)
{
    DiagStats S;
#pragma unroll
    for (int o = 0; o < 5; ++o) {
        S.cnt[o] = 0;
        S.first[o] = (int)m;
        S.last[o] = -1;
    }
    const int64_t L = (int64_t)P.ref_len;
    const int64_t ref_words = (L + 15) / 16;
    for (uint32_t j0 = 0; j0 < m; j0 += 64) {
        const uint32_t j = j0 + (uint32_t)lane;
        const bool valid = j < m;
        uint32_t qb = 0;
        if (valid)
            qb = s ? 3u - base_of(P.reads, off + (m - 1 - j)) : base_of(P.reads, off + j);
        const int64_t x = d + (int64_t)j - 2;           // reference position of diagonal d - 2
        const int64_t w0 = x >= 0 ? x >> 4 : -1;
        const uint32_t lo = valid && w0 >= 0 && w0 < ref_words ? P.ref[w0] : 0u;
        const uint32_t hi = valid && w0 + 1 >= 0 && w0 + 1 < ref_words ? P.ref[w0 + 1] : 0u;
        const uint64_t v = ((uint64_t)hi << 32) | lo;
#pragma unroll
        for (int o = 0; o < 5; ++o) {
            const int64_t xo = x + o;
            uint32_t rb = 4u;
            if (valid && xo >= 0 && xo < L) {
                if (w0 >= 0)
                    rb = (uint32_t)(v >> (2 * (xo - 16 * w0))) & 3u;
                else   // x < 0: xo lies in word 0, held in `hi`
                    rb = (hi >> (2 * xo)) & 3u;
            }
            const uint64_t mk = __ballot(valid && qb != rb);
            S.cnt[o] += __popcll(mk);
            if (S.first[o] == (int)m && mk)
                S.first[o] = (int)j0 + __ffsll((long long)mk) - 1;
            if (mk)
                S.last[o] = (int)j0 + 63 - __clzll((long long)mk);
        }
    }
    return S;
}

// The verdict at start p = d + t (t in -1..1) from the diagonals' statistics.
__device__ Verdict verdict_at(const DiagStats &S, int t, uint32_t m, int64_t p, uint64_t L)
{
    const int c = t + 2;
    const int cnt0 = S.cnt[c], f0 = S.first[c];
    const int lp = S.last[c + 1] >= 1 ? S.last[c + 1] : -1;   // diagonal p + 1, j >= 1
    const int lm = S.last[c - 1] >= 2 ? S.last[c - 1] : -1;   // diagonal p - 1, j >= 2
    const uint64_t pu = (uint64_t)p;
    if (pu + m <= L) {
        if (cnt0 == 0)
            return Verdict{0, SW_BMAP_EXACT, -1, pu + m - 1};
        if (cnt0 == 1)
            return Verdict{1, SW_BMAP_SUBST, f0, pu + m - 1};
    }
    if (pu + m + 1 <= L && m >= 2) {
        const int i = max(1, lp + 1);
        if (i <= (int)m - 1 && i <= f0)
            return Verdict{1, SW_BMAP_DEL, i, pu + m};
    }
    if (pu + m - 1 <= L && m >= 3) {
        const int i = max(1, lm);
        if (i <= (int)m - 2 && i <= f0)
            return Verdict{1, SW_BMAP_INS, i, pu + m - 2};
    }
    return Verdict{2, 0, 0, 0};
}

__global__ void __launch_bounds__(64 * kBWaves) k_stage_b(const StageBParams P)
{
    __shared__ uint64_t keys_all[kBWaves][kMaxRegions];
    const uint32_t wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    uint64_t *keys = keys_all[wave];
    for (uint64_t r = (uint64_t)blockIdx.x * kBWaves + wave; r < P.n_reads;
         r += (uint64_t)gridDim.x * kBWaves) {
        const uint32_t m = P.read_len[r];
        const uint64_t off = P.read_off[r];
        const uint64_t b = r ? P.read_end[r - 1] : 0ull;
        uint64_t e = P.read_end[r];
        if (e > P.cap) e = P.cap;
        uint32_t n = e > b ? (uint32_t)min(e - b, (uint64_t)kMaxRegions) : 0u;
        if (off + m > P.reads_len)
            n = 0;
        uint32_t P2 = 1;
        while (P2 < n) P2 <<= 1;
        for (uint32_t i = lane; i < P2; i += 64) {
            uint64_t key = ~0ull;
            if (i < n) {
                const sw_region g = P.reg[b + i];
                const int64_t d = (int64_t)g.first - (int64_t)g.read_pos + 65536;
                key = ((uint64_t)(g.strand ? 1 : 0) << 48) | (uint64_t)d;
            }
            keys[i] = key;
        }
        wave_sync();
        sort_keys(keys, P2, lane);
        sw_bmap *out = P.maps + r * (uint64_t)kBMax;
        int best = 2, cnt = 0;
        uint64_t prev = ~0ull;
        uint32_t last_s = 2;
        int64_t last_p = INT64_MIN;
        for (uint32_t i = 0; i < n; ++i) {
            const uint64_t key = keys[i];
            if (key == prev)
                continue;
            prev = key;
            const uint32_t s = (uint32_t)(key >> 48);
            const int64_t d = (int64_t)(key & ((1ull << 48) - 1)) - 65536;
            if (s != last_s) {
                last_s = s;
                last_p = INT64_MIN;
            }
            if (d + 1 <= last_p || d + 1 < 0)
                continue;   // every start of this diagonal is taken or before the reference
            const DiagStats S = scan_diagonals(P, off, m, s, d, lane);
            for (int t = -1; t <= 1; ++t) {
                const int64_t p = d + t;
                if (p <= last_p)
                    continue;
                last_p = p;
                if (p < 0)
                    continue;
                const Verdict v = verdict_at(S, t, m, p, P.ref_len);
                if (v.e > 1)
                    continue;
                if (v.e < best) {
                    best = v.e;
                    cnt = 0;
                }
                if (v.e == best && cnt < kBMax) {
                    if (lane == 0)
                        out[cnt] = sw_bmap{(uint32_t)p, (uint32_t)v.last, (uint8_t)s, (uint8_t)v.e,
                                           (uint8_t)v.op, 0u, v.pos};
                    ++cnt;
                }
            }
        }
        for (int j = lane; j < kBMax; j += 64)
            if (j >= cnt)
                out[j] = sw_bmap{0u, 0u, 0u, 0u, 0u, 0u, 0};
        if (lane == 0)
            P.n_maps[r] = (uint32_t)cnt;
        wave_sync();
    }
}

template <class T>
hipError_t scan_inclusive(const uint32_t *in, uint64_t n, T *out, T *tsum, hipStream_t st)
{
    const uint64_t nt = (n + kTile - 1) / kTile;
    if (nt == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_tile_sums<T>, dim3((unsigned)nt), dim3(256), 0, st, in, n, tsum);
    hipLaunchKernelGGL(k_tile_offsets<T>, dim3(1), dim3(1024), 0, st, (uint32_t)nt, tsum);
    hipLaunchKernelGGL(k_tile_scan<T>, dim3((unsigned)nt), dim3(256), 0, st, in, n, tsum, out);
    return hipGetLastError();
}

}  // namespace

uint64_t kmer_index_codes(uint32_t k) { return 1ull << (2 * k); }

uint64_t seeker_scan_words(uint64_t n) { return (n + kTile - 1) / kTile + 1; }

hipError_t launch_index_build(const uint32_t *ref, uint64_t ref_len, uint32_t k, uint32_t *starts,
                              uint32_t *pos, uint32_t *tsum, hipStream_t st)
{
    const uint64_t n_codes = kmer_index_codes(k);
    const uint64_t n_pos = ref_len >= k ? ref_len - k + 1 : 0;
    const uint64_t ref_words = (ref_len + 15) / 16;
    const uint32_t mask = (k == 16) ? 0xFFFFFFFFu : ((1u << (2 * k)) - 1u);
    hipLaunchKernelGGL(k_fill32, dim3(blocks_for(n_codes)), dim3(256), 0, st, n_codes + 1, starts);
    if (n_pos) {
        hipLaunchKernelGGL(k_kmer_hist, dim3(blocks_for(n_pos)), dim3(256), 0, st, ref, ref_words,
                           n_pos, mask, starts);
        hipError_t e = scan_inclusive<uint32_t>(starts, n_codes, starts, tsum, st);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_kmer_scatter, dim3(blocks_for(n_pos)), dim3(256), 0, st, ref,
                           ref_words, n_pos, mask, starts, pos);
    }
    hipLaunchKernelGGL(k_set_last, dim3(1), dim3(64), 0, st, starts, n_codes, (uint32_t)n_pos);
    return hipGetLastError();
}

hipError_t launch_regions(const sw_batch &b, const uint32_t *starts, const uint32_t *pos,
                          const sw_seed_params &sp, sw_region *out, uint64_t cap,
                          uint32_t *cnt, uint64_t *read_end, uint64_t *tsum, hipStream_t st)
{
    SeedParams P;
    P.reads = b.d_reads2b;
    P.read_words = (b.reads_len + 15) / 16;
    P.read_off = b.d_read_off;
    P.read_len = b.d_read_len;
    P.n_reads = b.n_reads;
    P.reads_len = b.reads_len;
    P.starts = starts;
    P.pos = pos;
    P.k = sp.k;
    P.step = sp.step;
    P.offset = sp.offset;
    P.max_occ = sp.max_occ;
    P.mask = (sp.k == 16) ? 0xFFFFFFFFu : ((1u << (2 * sp.k)) - 1u);
    if (b.n_reads == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_region_count, dim3(blocks_for(b.n_reads)), dim3(256), 0, st, P, cnt);
    hipError_t e = scan_inclusive<uint64_t>(cnt, b.n_reads, read_end, tsum, st);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_region_write, dim3(blocks_for(b.n_reads)), dim3(256), 0, st, P, read_end,
                       out, cap);
    return hipGetLastError();
}

hipError_t launch_cal_seek(const sw_region *reg, const uint64_t *read_end, uint32_t n_reads,
                           uint64_t cap, uint32_t k, uint32_t merge_gap, uint32_t min_len,
                           const uint32_t *skip, sw_cal *cals, hipStream_t st)
{
    if (n_reads == 0)
        return hipSuccess;
    uint64_t blocks = (n_reads + kSeekWaves - 1) / kSeekWaves;
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(k_cal_seek, dim3((unsigned)blocks), dim3(64 * kSeekWaves), 0, st, reg,
                       read_end, n_reads, cap, k, merge_gap, min_len, skip, cals);
    return hipGetLastError();
}

hipError_t launch_stage_b(const sw_batch &b, const sw_region *reg, const uint64_t *read_end,
                          uint64_t cap, sw_bmap *maps, uint32_t *n_maps, hipStream_t st)
{
    if (b.n_reads == 0)
        return hipSuccess;
    StageBParams P;
    P.reads = b.d_reads2b;
    P.read_words = (b.reads_len + 15) / 16;
    P.read_off = b.d_read_off;
    P.read_len = b.d_read_len;
    P.n_reads = b.n_reads;
    P.reads_len = b.reads_len;
    P.ref = b.d_ref2b;
    P.ref_len = b.ref_len;
    P.reg = reg;
    P.read_end = read_end;
    P.cap = cap;
    P.maps = maps;
    P.n_maps = n_maps;
    uint64_t blocks = (b.n_reads + kBWaves - 1) / kBWaves;
    if (blocks > 65535) blocks = 65535;
    hipLaunchKernelGGL(k_stage_b, dim3((unsigned)blocks), dim3(64 * kBWaves), 0, st, P);
    return hipGetLastError();
}

}  // namespace hpgsw
