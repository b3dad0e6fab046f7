// Per-candidate seed-hit features (64 x bf16 per pair) for the learned filter.
//
// The evidence is the one the paper's stage D uses to turn seed matches into
// candidate alignment locations (Sec. 2, "Stage D: CAL Seeker"): where a read's
// short exact seeds (12-mers here) land in a candidate window, and whether they
// line up on one diagonal.
//
// One wave per read.  The read's 12-mers, for both orientations, go into two
// open-addressing hash tables in LDS (at most 245 k-mers in 512 slots each),
// each with an 8192-bit prefilter bitmap indexed by the k-mer's first 6.5
// bases.  The wave takes the read's candidate windows eight at a time and
// treats their reference words (16 bases each) as one flat stream: lane l of
// a 128-word chunk owns words l and l + 64 of the stream, whatever windows
// they belong to.  A
// lane forms the 16 k-mers that start in its word with shifts of the word
// pair and tests them against the bitmap (five VALU operations each).  The
// bitmap hits of the whole chunk (true seed matches plus about 1.5 % false
// positives) are compacted into an LDS list with a wave prefix sum and probed
// 64 at a time, so the dense hits of a true window spread over all lanes
// instead of queueing in the few lanes that own its words.  Every hit (p, j)
// goes into the window's LDS row: diagonal-bin counters (two 16-bit halves
// per word), a bitmap of hit read positions and two 16-bin position
// histograms.  When the group is done, eight lanes per window reduce the row
// to the statistics, and the wave writes one 128-byte feature row per window
// (lane f: feature f).  The next read's descriptors and packed words are
// loaded while the current read is processed.  Features are computed in
// float32 and rounded to bfloat16.
#include "mlp_internal.h"

namespace hpgsw {

namespace {

constexpr int kK = 12;             // seed length
constexpr int kMF = 256;           // query bases used
constexpr int kNF = 1024;          // window bases used
constexpr int kTab = 512;          // hash slots per orientation
constexpr int kBm = 256;           // prefilter bitmap words per orientation (8192 bits)
constexpr int kG = 8;              // windows per group
constexpr int kList = 192;         // bitmap candidates probed per pass
constexpr int kWavesF = 2;         // waves per block
constexpr uint32_t kGold24 = 0x9E3779u;   // odd 24-bit multiplier of the table hash
constexpr uint32_t kEmpty = 0xFFFFFFFFu;

// Row of one window (32-bit words).  Words 0..63 are its feature row: for the
// features divided by max(P, 1) a word holds the integer numerator, for the
// others the finished bfloat16 pattern.  Words 7..38 (the position
// histograms) are accumulated in place.
constexpr int kRowBins = 64;       // 42 words: diagonal-bin counters, 16 bits each
constexpr int kRowPbits = 106;     // 8 words: bitmap of hit read positions
constexpr int kRowGc = 114;        // G+C count of the window
constexpr int kRow = 116;
// features whose value is (integer numerator) / max(P, 1): 0..3, 7..40, 43
constexpr uint64_t kOverP = 0xFull | (((1ull << 34) - 1) << 7) | (1ull << 43);

static_assert((kNF + kMF) / 32 + 2 <= kRowPbits - kRowBins, "diagonal bins do not fit the row");
static_assert(kG <= 16, "window index of a list entry has 4 bits");

struct alignas(16) WaveLds {
    uint32_t tab[2][kTab];         // (k-mer << 8) | read position, kEmpty = empty
    uint32_t acc[kG][kRow];
    uint2 list[kList];             // (k-mer | window << 24 | orientation << 28, j)
    uint16_t lut[256];             // bfloat16 of x / max(P, 1)
    uint32_t rd[kMF / 16 + 2];     // packed words holding the read's first 256 bases
    uint32_t rr[kMF / 16 + 2];     // packed words holding its last 256 bases
    uint32_t wrb[kMaxCand];        // window start
    uint16_t wnf[kMaxCand];        // window bases used
    uint8_t wst[kMaxCand];         // strand
    uint32_t nm3[kMaxCand];
    uint32_t ndp[kMaxCand];
    uint32_t cwo[kG + 1];          // first stream word of each window of the group
    float rj[kG];                  // 16 / max(J, 1)
};

__device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// reverse complement of a 12-mer (base i at bits 2i)
__device__ __forceinline__ uint32_t rc24(uint32_t x)
{
    const uint32_t r = __builtin_bitreverse32(x ^ 0xFFFFFFu) >> 8;
    return ((r & 0x555555u) << 1) | ((r >> 1) & 0x555555u);
}

// (t & 0x3FC) | base in one operation (base has no bits in 0x3FC); the
// compiler turns the or of disjoint fields into an add and splits it up
__device__ __forceinline__ uint32_t and_or_3fc(uint32_t t, uint32_t base)
{
    uint32_t r;
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(t), "s"(0x3FCu), "v"(base));
    return r;
}

__device__ __forceinline__ uint32_t tab_slot(uint32_t km)
{
    return (km * kGold24) >> 23;   // km < 2^24: a 24-bit multiply
}

__device__ __forceinline__ void lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// floor(16 x / d) for 0 <= x < d <= 1013, with r = RN(16 / d):
// (x + 1/32) * 16 / d lies at least 1/(2d) from an integer and the float error
// stays below 2^-18, so the truncation is exact.
__device__ __forceinline__ uint32_t bin16(uint32_t x, float r)
{
    return (uint32_t)__builtin_fmaf((float)x, r, r * 0.03125f);
}

// maximum over the wave: a max-scan inside each 16-lane row, then the row
// results combined with row broadcasts; lane 63 ends with the total
__device__ __forceinline__ uint32_t wave_max(uint32_t v)
{
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true));   // row_shr:1
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true));   // row_shr:2
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true));   // row_shr:4
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true));   // row_shr:8
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__global__ void __launch_bounds__(64 * kWavesF) k_features(const sw_batch b, const uint32_t *first,
                                                           const uint32_t *count, uint16_t *feat)
{
    __shared__ WaveLds lds_all[kWavesF];
    // prefilter bitmaps, [wave][orientation][word]; a flat index keeps the
    // per-position address at two operations
    __shared__ uint32_t bm_all[kWavesF * 2 * kBm];
    const uint32_t wave = threadIdx.x >> 6;
    WaveLds &L = lds_all[wave];
    const uint32_t bm_wave = wave * 2 * kBm;
    const int lane = threadIdx.x & 63;
    const uint64_t ref_words = (b.ref_len + 15) / 16;
    const uint64_t read_words = (b.reads_len + 15) / 16;
    // window rows start at zero; every group clears its rows after use
    for (int i = lane; i < kG * kRow / 4; i += 64)
        reinterpret_cast<uint4 *>(&L.acc[0][0])[i] = make_uint4(0, 0, 0, 0);
    // A read's scalars, window descriptors and packed words are loaded one read
    // ahead, so their latency overlaps the work on the previous read.
    auto load_scalars = [&](uint32_t rx, uint32_t &Kx, uint32_t &ax, int &mx, uint64_t &ox) {
        Kx = 0;
        ax = 0;
        mx = 0;
        ox = 0;
        if (rx < b.n_reads) {
            Kx = count[rx];
            ax = first[rx];
            mx = b.d_read_len[rx];
            ox = b.d_read_off[rx];
        }
    };
    sw_window wd{};
    uint32_t rw = 0;
    auto load_body = [&](uint32_t Kx, uint32_t ax, int mx, uint64_t ox) {
        if ((uint32_t)lane < Kx && Kx <= (uint32_t)kMaxCand)
            wd = b.d_win[ax + lane];
        if (read_words == 0)
            return;
        const int mfx = min(mx, kMF);
        const uint64_t wf = ox >> 4, wr = (ox + (uint64_t)(mx - mfx)) >> 4;
        if (lane < kMF / 16 + 2)
            rw = b.d_reads2b[min(wf + (uint64_t)lane, read_words - 1)];
        else if (lane >= 32 && lane < 32 + kMF / 16 + 2)
            rw = b.d_reads2b[min(wr + (uint64_t)(lane - 32), read_words - 1)];
    };
    const uint32_t stride = gridDim.x * kWavesF;
    uint32_t r = blockIdx.x * kWavesF + wave;
    uint32_t K, a;
    int m_full;
    uint64_t roff;
    load_scalars(r, K, a, m_full, roff);
    load_body(K, a, m_full, roff);
    for (; r < b.n_reads; r += stride) {
        // use up the registers loaded for this read before the next loads are issued
        // (the load counter is in order: a wait for an older load drains newer ones)
        bool go = K != 0 && K <= (uint32_t)kMaxCand;
        if (go) {
            uint32_t ok = 1;
            if ((uint32_t)lane < K) {
                ok = wd.read_id == r;
                int n = 0;
                if ((uint64_t)wd.ref_begin < b.ref_len) {
                    const uint64_t avail = b.ref_len - wd.ref_begin;
                    n = wd.len < avail ? (int)wd.len : (int)avail;
                }
                L.wrb[lane] = wd.ref_begin;
                L.wnf[lane] = (uint16_t)min(n, kNF);
                L.wst[lane] = wd.strand;
            }
            go = __all(ok);   // not contiguous: the decision keeps the whole read
            if (lane < kMF / 16 + 2)
                L.rd[lane] = rw;
            else if (lane >= 32 && lane < 32 + kMF / 16 + 2)
                L.rr[lane - 32] = rw;
        }
        uint32_t Kn, an;
        int mn;
        uint64_t on;
        load_scalars(r + stride, Kn, an, mn, on);
        if (!go) {
            load_body(Kn, an, mn, on);
            K = Kn;
            a = an;
            m_full = mn;
            roff = on;
            continue;
        }
        const int mf = min(m_full, kMF);
        const int P = max(mf - kK + 1, 0);
        const float Pdf = (float)max(P, 1);
        const float rP = 16.f / Pdf;
        // words holding read bases [0, mf) and [m_full - mf, m_full) (for the reverse complement)
        const uint64_t w_f0 = roff >> 4;
        const uint64_t w_r0 = (roff + (uint64_t)(m_full - mf)) >> 4;
        for (int i = lane; i < kTab; i += 64) {
            L.tab[0][i] = kEmpty;
            L.tab[1][i] = kEmpty;
        }
        for (int i = lane; i < 2 * kBm; i += 64)
            bm_all[bm_wave + i] = 0;
        for (int x = lane; x < 256; x += 64)
            L.lut[x] = f2bf((float)x / Pdf);
        // ---- the words of a group of windows as one stream: cwo[k] is the first
        // stream word of window k of the group (cwo[Gn] the total), and cwr[k]
        // holds cwo[k + 1] in a register for the window search of fetch()
        uint32_t cwr[kG];
        uint32_t total = 0, c = 0, gbase = 0;
        auto prep = [&](uint32_t cgx) {
            const int Gx = min((int)(K - cgx), kG);
            uint32_t nw = 0;
            if (lane < Gx) {
                const int nf = L.wnf[cgx + lane];
                const uint64_t rb = L.wrb[cgx + lane];
                nw = nf > 0 ? (uint32_t)(((rb + (uint64_t)nf - 1) >> 4) - (rb >> 4) + 1) : 0u;
                L.rj[lane] = 16.f / (float)max(nf - kK + 1, 1);
            }
#pragma unroll
            for (int off = 1; off < kG; off <<= 1) {
                const uint32_t t = __shfl_up(nw, off, kG);
                if ((lane & (kG - 1)) >= off)
                    nw += t;
            }
            if (lane < kG)
                L.cwo[lane + 1] = nw;
            if (lane == 0)
                L.cwo[0] = 0;
            // lanes at or beyond Gx hold the total, so windows past the group
            // never pass the search's test
#pragma unroll
            for (int k = 0; k < kG; ++k)
                cwr[k] = (uint32_t)__builtin_amdgcn_readlane((int)nw, k);
            total = cwr[kG - 1];
            gbase = cgx;
            c = 0;
        };
        // the window of stream word wn (< total) and its two reference words;
        // c (the window of the lane's latest fetched word) only moves forward
        auto fetch = [&](uint32_t wn, uint32_t &cw, uint32_t &x0, uint32_t &x1) {
            uint32_t cn = 0;
#pragma unroll
            for (int k = 0; k < kG - 1; ++k)
                cn += cwr[k] <= wn ? 1u : 0u;
            c = cn;
            cw = c;
            const uint64_t gw = (uint64_t)(L.wrb[gbase + c] >> 4) + (uint64_t)(wn - L.cwo[c]);
            x0 = b.d_ref2b[min(gw, ref_words - 1)];
            x1 = b.d_ref2b[min(gw + 1, ref_words - 1)];
        };
        uint32_t pca = 0, pa0 = 0, pa1 = 0, pcb = 0, pb0 = 0, pb1 = 0;
        // the first chunk of a group is fetched ahead, here for the first group
        // (its loads overlap the query tables' construction)
        auto first_fetch = [&]() {
            if ((uint32_t)lane < total)
                fetch(lane, pca, pa0, pa1);
            if ((uint32_t)lane + 64 < total)
                fetch(lane + 64, pcb, pb0, pb1);
        };
        prep(0);
        lds_fence();
        first_fetch();
        // ---- query k-mer tables and prefilters (orientation 0: read, 1: reverse complement)
        uint32_t dupf = 0;   // bit o: a k-mer of orientation o occurs twice in the query
        for (int e = lane; e < 2 * P; e += 64) {
            const int o = e >= P;
            const int p = o ? e - P : e;
            uint32_t km;
            if (!o) {
                const uint64_t pos = roff + (uint64_t)p - (w_f0 << 4);
                km = __builtin_amdgcn_alignbit(L.rd[(pos >> 4) + 1], L.rd[pos >> 4],
                                               (uint32_t)(pos & 15) * 2u) & 0xFFFFFFu;
            } else {
                // reverse complement of the read 12-mer at read position m_full - p - 12
                const uint64_t pos = roff + (uint64_t)(m_full - p - kK) - (w_r0 << 4);
                const int wi = (int)(pos >> 4);
                km = rc24(__builtin_amdgcn_alignbit(L.rr[wi + 1], L.rr[wi], (uint32_t)(pos & 15) * 2u) &
                          0xFFFFFFu);
            }
            atomicOr(&bm_all[bm_wave + o * kBm + ((km >> 5) & (kBm - 1))], 1u << (km & 31u));
            const uint32_t entry = (km << 8) | (uint32_t)p;
            uint32_t h = tab_slot(km);
            for (;;) {
                const uint32_t old = atomicCAS(&L.tab[o][h], kEmpty, entry);
                if (old == kEmpty)
                    break;
                if ((old >> 8) == km)
                    dupf |= 1u << o;
                h = (h + 1) & (kTab - 1);
            }
        }
        const bool dup0 = __ballot(dupf & 1u) != 0, dup1 = __ballot(dupf & 2u) != 0;
        lds_fence();
        load_body(Kn, an, mn, on);
        // x / max(P, 1) as bfloat16 for a signed integer numerator
        auto over_p = [&](int32_t x) -> uint16_t {
            const uint32_t ax = (uint32_t)(x < 0 ? -x : x);
            uint16_t v;
            if (ax < 256)
                v = L.lut[ax];
            else
                v = f2bf((float)ax / Pdf);
            return x < 0 ? (uint16_t)(v | 0x8000u) : v;
        };
        for (uint32_t cg = 0; cg < K; cg += kG) {
            const int Gn = min((int)(K - cg), kG);
            // Each lane owns two stream words per step (a 128-word chunk); the
            // first chunk was fetched ahead (prep and first_fetch).
            // bitmap candidates of one word: positions i whose k-mer may occur in the query
            auto scan = [&](uint32_t wc, uint32_t cc, uint32_t a0, uint32_t a1, uint32_t &cand,
                            uint32_t &head, int &j0) {
                const uint32_t ci = cg + cc;
                const uint32_t rb = L.wrb[ci];
                const int nf = L.wnf[ci];
                const int o = L.wst[ci] ? 1 : 0;
                const int J = max(nf - kK + 1, 0);
                j0 = 16 * (int)(wc - L.cwo[cc]) - (int)(rb & 15u);
                // positions i of this word with 0 <= j0 + i < J (k-mers), < nf (bases)
                const int lo = max(-j0, 0);
                const int hiJ = min(J - j0, 16), hiN = min(nf - j0, 16);
                const uint32_t vmask = hiJ > lo ? ((1u << hiJ) - 1u) & ~((1u << lo) - 1u) : 0u;
                const uint32_t gmask =
                    hiN > lo ? (uint32_t)(((1ull << (2 * hiN)) - 1ull) & ~((1ull << (2 * lo)) - 1ull)) : 0u;
                const uint32_t g = __popc((a0 ^ (a0 >> 1)) & 0x55555555u & gmask);   // C = 01, G = 10
                if (g)
                    atomicAdd(&L.acc[cc][kRowGc], g);
                const uint32_t bmo = (bm_wave | (uint32_t)(o * kBm)) * 4u;   // bytes, multiple of 1024
                const uint32_t x16 = __builtin_amdgcn_alignbit(a1, a0, 16);
                uint32_t m = 0;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    // bits 0..12 of the k-mer at position i
                    const uint32_t sh = i < 10 ? (a0 >> (2 * i)) : (x16 >> (2 * i - 16));
                    const uint32_t word = *reinterpret_cast<const uint32_t *>(
                        reinterpret_cast<const char *>(bm_all) + and_or_3fc(sh >> 3, bmo));
                    m |= __builtin_amdgcn_ubfe(word, sh, 1u) << i;
                }
                cand = m & vmask;
                head = (cc | (uint32_t)o << 4) << 24;
            };
            // list entries of one word's candidates with list index in [base, base + kList)
            auto emit = [&](uint32_t cm, uint32_t head, int j0, uint32_t a0, uint32_t a1, uint32_t &o2,
                            uint32_t base) {
                while (cm) {
                    if (o2 >= base + kList)
                        return;
                    const int i = __builtin_ctz(cm);
                    cm &= cm - 1u;
                    if (o2 >= base) {
                        const uint32_t km = __builtin_amdgcn_alignbit(a1, a0, 2u * (uint32_t)i) & 0xFFFFFFu;
                        L.list[o2 - base] = make_uint2(km | head, (uint32_t)(j0 + i));
                    }
                    ++o2;
                }
            };
            const uint32_t g_total = total;
            for (uint32_t W = 0; W < g_total; W += 128) {
                const uint32_t wa = W + lane, wb = W + 64 + lane;
                const uint32_t ca = pca, a0 = pa0, a1 = pa1, cb = pcb, b0 = pb0, b1 = pb1;
                if (wa + 128 < g_total)
                    fetch(wa + 128, pca, pa0, pa1);
                if (wb + 128 < g_total)
                    fetch(wb + 128, pcb, pb0, pb1);
                uint32_t candA = 0, headA = 0, candB = 0, headB = 0;
                int j0A = 0, j0B = 0;
                if (wa < g_total)
                    scan(wa, ca, a0, a1, candA, headA, j0A);
                if (wb < g_total)
                    scan(wb, cb, b0, b1, candB, headB, j0B);
                // offsets of every lane's candidates in the chunk's list (prefix over the wave)
                const uint32_t cnt = __popc(candA) + __popc(candB);
                uint32_t off = 0, tot = 0;
#pragma unroll
                for (int bp = 0; bp < 6; ++bp) {
                    const uint64_t m = __ballot((cnt >> bp) & 1u);
                    off += __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)) << bp;
                    tot += (uint32_t)__popcll(m) << bp;
                }
                for (uint32_t base = 0; base < tot; base += kList) {
                    if (cnt && off < base + kList && off + cnt > base) {
                        uint32_t o2 = off;
                        emit(candA, headA, j0A, a0, a1, o2, base);
                        emit(candB, headB, j0B, b0, b1, o2, base);
                    }
                    lds_fence();
                    // probe the listed k-mers, 64 at a time
                    const uint32_t nq = min(tot - base, (uint32_t)kList);
                    for (uint32_t q = lane; q < nq; q += 64) {
                        const uint2 en = L.list[q];
                        const uint32_t km = en.x & 0xFFFFFFu;
                        const uint32_t cw = (en.x >> 24) & 15u, oo = en.x >> 28;
                        const uint32_t j = en.y;
                        const uint32_t *tabo = L.tab[oo];
                        const bool dup = oo ? dup1 : dup0;
                        uint32_t *A = L.acc[cw];
                        const float rJ = L.rj[cw];
                        uint32_t h = tab_slot(km);
                        for (;;) {
                            const uint32_t t = tabo[h];
                            if (t == kEmpty)
                                break;
                            if ((t >> 8) == km) {
                                const uint32_t p = t & 0xFFu;
                                const uint32_t d = j + (uint32_t)mf - p;   // 16 * bin + offset
                                atomicAdd(&A[kRowBins + (d >> 5)], 1u << (d & 16u));
                                atomicOr(&A[kRowPbits + (p >> 5)], 1u << (p & 31u));
                                atomicAdd(&A[7 + bin16(p, rP)], 1u);
                                atomicAdd(&A[23 + bin16(j, rJ)], 1u);
                                if (!dup)      // a k-mer that occurs once matches once
                                    break;
                            }
                            h = (h + 1) & (kTab - 1);
                        }
                    }
                    lds_fence();
                }
            }
            lds_fence();
            // the next group's stream and first chunk, ahead of this group's
            // statistics (which read neither cwo nor rj)
            if (cg + kG < K) {
                prep(cg + kG);
                lds_fence();
                first_fetch();
            }
            // ---- statistics, eight lanes per window
            {
                const int cw = lane >> 3, q = lane & 7;
                const bool live = cw < Gn;
                const uint32_t ci = cg + (live ? cw : 0);
                const int nf = live ? (int)L.wnf[ci] : 0;
                uint32_t *A = L.acc[cw];
                const int nbw = (((nf + mf) >> 4) + 3) >> 1;   // words of bins 0 .. ((nf + mf) >> 4) + 1
                uint32_t bestc = 0, besti = 0, nz = 0;
                for (int w = q; w < nbw; w += 8) {
                    const uint32_t v = A[kRowBins + w];
                    const uint32_t v0 = v & 0xFFFFu, v1 = v >> 16;
                    nz += (v0 ? 1u : 0u) + (v1 ? 1u : 0u);
                    if (v0 > bestc) {
                        bestc = v0;
                        besti = 2 * w;
                    }
                    if (v1 > bestc) {
                        bestc = v1;
                        besti = 2 * w + 1;
                    }
                }
                uint32_t ndp = __popc(A[kRowPbits + q]);
                uint32_t nh = A[7 + q] + A[15 + q];
#pragma unroll
                for (int off = 1; off < 8; off <<= 1) {
                    const uint32_t oc = __shfl_xor(bestc, off);
                    const uint32_t oi = __shfl_xor(besti, off);
                    if (oc > bestc || (oc == bestc && oi < besti)) {
                        bestc = oc;
                        besti = oi;
                    }
                    nz += __shfl_xor(nz, off);
                    ndp += __shfl_xor(ndp, off);
                    nh += __shfl_xor(nh, off);
                }
                auto bin = [&](uint32_t k) { return (A[kRowBins + (k >> 1)] >> ((k & 1u) * 16u)) & 0xFFFFu; };
                uint32_t nmode = 0, nmode3 = 0, mode = 0, nbins = 0;
                if (nh) {
                    mode = besti;
                    nmode = bestc;
                    nmode3 = bin(mode) + (mode ? bin(mode - 1) : 0u) + bin(mode + 1);
                    nbins = nz;
                }
                if (live) {
                    if (q == 0) {
                        A[0] = ndp;
                        A[1] = min(nh, 4u * (uint32_t)max(P, 1));
                        A[2] = nmode;
                        A[3] = nmode3;
                    } else if (q == 1) {
                        A[4] = f2bf((float)min(nbins, 64u) * 0.0625f);
                        A[5] = nh ? f2bf((float)(16 * (int)mode + 8 - mf) / (float)max(nf, 1)) : 0u;
                        A[6] = nh ? 0x3F80u : 0u;
                    } else if (q == 2) {
                        A[45] = f2bf((float)nf / 1000.f);
                        A[46] = f2bf((float)mf / 1000.f);
                        A[47] = L.wst[ci] ? 0x3F80u : 0u;
                    } else if (q == 3) {
                        A[48] = f2bf((float)A[kRowGc] / (float)max(nf, 1));
                        L.nm3[ci] = nmode3;
                        L.ndp[ci] = ndp;
                    }
                }
            }
            lds_fence();
            // ---- features comparing the read's windows (39..44), when the group is the whole read
            if (K <= (uint32_t)kG) {
                const bool in = (uint32_t)lane < K;
                const uint32_t v3 = in ? L.nm3[lane] : 0u, dp = in ? L.ndp[lane] : 0u;
                const uint32_t mx3 = wave_max(v3), mxd = wave_max(dp);
                const uint64_t at = __ballot(in && v3 == mx3);
                uint32_t second = wave_max(in && v3 != mx3 ? v3 : 0u);
                if (__popcll(at) >= 2)
                    second = mx3;
                uint32_t gt = 0;
                for (uint32_t d = 0; d < K; ++d)
                    gt += L.nm3[d] > v3 ? 1u : 0u;
                if (in) {
                    uint32_t *A = L.acc[lane];
                    A[39] = (uint32_t)((int32_t)v3 - (int32_t)mx3);
                    A[40] = (uint32_t)((int32_t)dp - (int32_t)mxd);
                    A[41] = v3 == mx3 ? 0x3F80u : 0u;
                    A[42] = f2bf((float)gt / (float)K);
                    A[43] = mx3 - second;
                    A[44] = f2bf((float)K * 0.0625f);
                }
                lds_fence();
            }
            // ---- one 128-byte feature row per window: lane f writes feature f
            {
                const bool overp = (kOverP >> lane) & 1u;
                const bool later = K > (uint32_t)kG && lane >= 39 && lane < 45;
                for (int cw = 0; cw < Gn; ++cw) {
                    const int32_t x = (int32_t)L.acc[cw][lane];
                    const uint16_t v = overp ? over_p(x) : (uint16_t)x;
                    if (!later)
                        feat[(uint64_t)(a + cg + cw) * kIn + lane] = v;
                }
            }
            lds_fence();
            for (int i = lane; i < kG * kRow / 4; i += 64)
                reinterpret_cast<uint4 *>(&L.acc[0][0])[i] = make_uint4(0, 0, 0, 0);
            lds_fence();
        }
        // ---- features 39..44 of reads with more windows than a group
        if (K > (uint32_t)kG) {
            const bool in = (uint32_t)lane < K;
            const uint32_t v3 = in ? L.nm3[lane] : 0u, dp = in ? L.ndp[lane] : 0u;
            const uint32_t mx3 = wave_max(v3), mxd = wave_max(dp);
            const uint64_t at = __ballot(in && v3 == mx3);
            uint32_t second = wave_max(in && v3 != mx3 ? v3 : 0u);
            if (__popcll(at) >= 2)
                second = mx3;
            uint32_t gt = 0;
            for (uint32_t d = 0; d < K; ++d)
                gt += L.nm3[d] > v3 ? 1u : 0u;
            if (in) {
                uint16_t *f = feat + (uint64_t)(a + lane) * kIn;
                f[39] = over_p((int32_t)v3 - (int32_t)mx3);
                f[40] = over_p((int32_t)dp - (int32_t)mxd);
                f[41] = v3 == mx3 ? 0x3F80u : 0u;
                f[42] = f2bf((float)gt / (float)K);
                f[43] = over_p((int32_t)(mx3 - second));
                f[44] = f2bf((float)K * 0.0625f);
            }
        }
        lds_fence();
        K = Kn;
        a = an;
        m_full = mn;
        roff = on;
    }
}

}  // namespace

hipError_t launch_features(const sw_batch &b, const uint32_t *first, const uint32_t *count,
                           uint16_t *feat, int n_cu, hipStream_t st)
{
    if (b.n_reads == 0)
        return hipSuccess;
    uint32_t blocks = (b.n_reads + kWavesF - 1) / kWavesF;
    // as many resident blocks as the LDS of a compute unit holds
    const uint32_t per_cu = (uint32_t)(160 * 1024 / (kWavesF * (sizeof(WaveLds) + 2 * kBm * 4)));
    const uint32_t cap = (uint32_t)n_cu * (per_cu > 0 ? per_cu : 1);
    if (blocks > cap)
        blocks = cap;
    hipLaunchKernelGGL(k_features, dim3(blocks), dim3(64 * kWavesF), 0, st, b, first, count, feat);
    return hipGetLastError();
}

}  // namespace hpgsw
