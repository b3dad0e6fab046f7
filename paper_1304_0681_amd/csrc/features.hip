// Per-candidate seed-hit features (64 x bf16 per pair) for the learned filter.
//
// The evidence is the one the paper's stage D uses to turn seed matches into
// candidate alignment locations (Sec. 2, "Stage D: CAL Seeker"): where a read's
// short exact seeds (12-mers here) land in a candidate window, and whether they
// line up on one diagonal.
//
// One wave per read.  The read's 12-mers, for both orientations, go into two
// open-addressing hash tables in LDS (at most 245 k-mers in 512 slots each),
// each with an 8192-bit prefilter bitmap.  The wave then takes the read's
// candidate windows four at a time, 16 lanes per window.  A lane owns whole
// 16-base words of the reference: it loads a word and its successor once and
// forms the 16 k-mers that start in the word with funnel shifts, so the 16
// bitmap reads of a word issue back to back and only bitmap hits (true seed
// matches plus about 3 % false positives) probe the table.  Every hit (p, j)
// goes into LDS accumulators (diagonal bins of width 16, a bitmap of hit read
// positions, two 16-bin position histograms).  When a window is done its 16
// lanes write the per-candidate features (four each); a last pass adds the
// features that compare the read's candidates.  Features are computed in
// float32 and rounded to bfloat16.
#include "mlp_internal.h"

namespace hpgsw {

namespace {

constexpr int kK = 12;             // seed length
constexpr int kMF = 256;           // query bases used
constexpr int kNF = 1024;          // window bases used
constexpr int kTab = 512;          // hash slots per orientation
constexpr int kBm = 256;           // prefilter bitmap words per orientation (8192 bits)
constexpr int kSlots = 4;          // candidates in flight per wave
constexpr int kMaxBins = (kNF + kMF) / 16 + 3;
constexpr int kWavesF = 4;         // waves per block
constexpr uint32_t kGold = 0x9E3779B1u;

struct alignas(16) WaveLds {
    uint32_t key[2][kTab];
    uint32_t bm[2][kBm];
    uint16_t pos[2][kTab];
    uint32_t bins[kSlots][kMaxBins];
    uint32_t pbits[kSlots][kMF / 32];
    uint32_t acc[kSlots][36];      // nh, gc, hist_p[16], hist_j[16], (2 spare)
    uint32_t nm3[kMaxCand];
    uint32_t ndp[kMaxCand];
};

__device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// 12-mer starting at base position `pos` of a packed sequence of `words` words
__device__ __forceinline__ uint32_t kmer_at(const uint32_t *seq, uint64_t words, uint64_t pos)
{
    const uint64_t w0 = pos >> 4;
    const uint64_t w1 = w0 + 1 < words ? w0 + 1 : w0;
    return __builtin_amdgcn_alignbit(seq[w1], seq[w0], (uint32_t)(pos & 15) * 2u) & 0xFFFFFFu;
}

// reverse complement of a 12-mer (base i at bits 2i)
__device__ __forceinline__ uint32_t rc24(uint32_t x)
{
    const uint32_t r = __builtin_bitreverse32(x ^ 0xFFFFFFu) >> 8;
    return ((r & 0x555555u) << 1) | ((r >> 1) & 0x555555u);
}

__device__ __forceinline__ void lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

struct CandStats {
    uint32_t ndp, nh, nmode, nmode3, nbins, mode, gc, nf, strand;
};

// per-candidate feature f (0..63) other than the cross-candidate ones 39..44
__device__ __forceinline__ float cand_feature(int f, const CandStats &S, const uint32_t *acc,
                                              int P, int mf)
{
    const float Pd = (float)max(P, 1);
    const float nfd = (float)max((int)S.nf, 1);
    if (f >= 7 && f < 39)
        return (float)acc[2 + (f - 7)] / Pd;          // hist_p then hist_j are contiguous
    switch (f) {
    case 0: return (float)S.ndp / Pd;
    case 1: return (float)min(S.nh, 4u * (uint32_t)max(P, 1)) / Pd;
    case 2: return (float)S.nmode / Pd;
    case 3: return (float)S.nmode3 / Pd;
    case 4: return (float)min(S.nbins, 64u) / 16.f;
    case 5: return S.nh ? (float)(16 * (int)S.mode + 8 - mf) / nfd : 0.f;
    case 6: return S.nh ? 1.f : 0.f;
    case 45: return (float)S.nf / 1000.f;
    case 46: return (float)mf / 1000.f;
    case 47: return (float)S.strand;
    case 48: return (float)S.gc / nfd;
    default: return 0.f;
    }
}

__global__ void __launch_bounds__(64 * kWavesF) k_features(const sw_batch b, const uint32_t *first,
                                                           const uint32_t *count, uint16_t *feat)
{
    __shared__ WaveLds lds_all[kWavesF];
    WaveLds &L = lds_all[threadIdx.x >> 6];
    const int lane = threadIdx.x & 63;
    const uint64_t ref_words = (b.ref_len + 15) / 16;
    const uint64_t read_words = (b.reads_len + 15) / 16;
    const int slot = lane >> 4, sl = lane & 15;
    for (uint32_t r = blockIdx.x * kWavesF + (threadIdx.x >> 6); r < b.n_reads;
         r += gridDim.x * kWavesF) {
        const uint32_t K = count[r];
        if (K == 0 || K > kMaxCand)
            continue;
        const uint32_t a = first[r];
        uint32_t ok = 1;
        for (uint32_t c = lane; c < K; c += 64)
            ok &= (b.d_win[a + c].read_id == r) ? 1u : 0u;
        if (!__all(ok))       // not contiguous: the decision keeps the whole read
            continue;
        const int m_full = b.d_read_len[r];
        const uint64_t roff = b.d_read_off[r];
        const int mf = min(m_full, kMF);
        const int P = max(mf - kK + 1, 0);
        // ---- query k-mer tables and prefilters (orientation 0: read, 1: reverse complement)
        for (int i = lane; i < kTab; i += 64) {
            L.key[0][i] = 0;
            L.key[1][i] = 0;
        }
        for (int i = lane; i < kBm; i += 64) {
            L.bm[0][i] = 0;
            L.bm[1][i] = 0;
        }
        lds_fence();
        for (int e = lane; e < 2 * P; e += 64) {
            const int o = e >= P;
            const int p = o ? e - P : e;
            const uint32_t km = o ? rc24(kmer_at(b.d_reads2b, read_words, roff + (uint64_t)(m_full - p - kK)))
                                  : kmer_at(b.d_reads2b, read_words, roff + (uint64_t)p);
            const uint32_t H = km * kGold;
            atomicOr(&L.bm[o][H >> 24], 1u << ((H >> 19) & 31u));
            uint32_t h = H >> 23;
            for (;;) {
                const uint32_t old = atomicCAS(&L.key[o][h], 0u, km + 1u);
                if (old == 0) {
                    L.pos[o][h] = (uint16_t)p;
                    break;
                }
                h = (h + 1) & (kTab - 1);
            }
        }
        lds_fence();
        // ---- candidate windows, four at a time
        for (uint32_t c0 = 0; c0 < K; c0 += kSlots) {
            const uint32_t c = c0 + slot;
            const bool act = c < K;
            const sw_window w = b.d_win[a + (act ? c : 0)];
            int n = 0;
            if (act && (uint64_t)w.ref_begin < b.ref_len) {
                const uint64_t avail = b.ref_len - w.ref_begin;
                n = w.len < avail ? (int)w.len : (int)avail;
            }
            const int nf = min(n, kNF);
            const int J = max(nf - kK + 1, 0);
            const int nb = ((nf + mf) >> 4) + 2;
            for (int i = sl; i < nb; i += 16)
                L.bins[slot][i] = 0;
            if (sl < kMF / 32)
                L.pbits[slot][sl] = 0;
            for (int i = sl; i < 36; i += 16)
                L.acc[slot][i] = 0;
            lds_fence();
            const int o = w.strand ? 1 : 0;
            const int Pd = max(P, 1), Jd = max(J, 1);
            const uint64_t rb = w.ref_begin;
            uint32_t gc = 0;
            if (nf > 0) {
                const uint64_t wfirst = rb >> 4, wlast = (rb + (uint64_t)nf - 1) >> 4;
                for (uint64_t wd = wfirst + (uint64_t)sl; wd <= wlast; wd += 16) {
                    const uint32_t u0 = b.d_ref2b[wd];
                    const uint32_t u1 = b.d_ref2b[wd + 1 < ref_words ? wd + 1 : wd];
                    const int j0 = (int)((int64_t)(wd * 16) - (int64_t)rb);   // window position of base 0
                    uint32_t cand = 0;
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int j = j0 + i;
                        const uint32_t km = __builtin_amdgcn_alignbit(u1, u0, 2u * i) & 0xFFFFFFu;
                        const uint32_t base = km & 3u;
                        gc += ((unsigned)j < (unsigned)nf && (base == 1u || base == 2u)) ? 1u : 0u;
                        const uint32_t H = km * kGold;
                        const uint32_t bit = (L.bm[o][H >> 24] >> ((H >> 19) & 31u)) & 1u;
                        cand |= ((unsigned)j < (unsigned)J && bit) ? (1u << i) : 0u;
                    }
                    while (cand) {
                        const int i = __builtin_ctz(cand);
                        cand &= cand - 1;
                        const int j = j0 + i;
                        const uint32_t km = __builtin_amdgcn_alignbit(u1, u0, 2u * i) & 0xFFFFFFu;
                        uint32_t h = (km * kGold) >> 23;
                        for (;;) {
                            const uint32_t key = L.key[o][h];
                            if (key == 0)
                                break;
                            if (key == km + 1u) {
                                const int p = L.pos[o][h];
                                atomicAdd(&L.bins[slot][(j - p + mf) >> 4], 1u);
                                atomicOr(&L.pbits[slot][p >> 5], 1u << (p & 31));
                                atomicAdd(&L.acc[slot][0], 1u);
                                atomicAdd(&L.acc[slot][2 + (16 * p) / Pd], 1u);
                                atomicAdd(&L.acc[slot][18 + (16 * j) / Jd], 1u);
                            }
                            h = (h + 1) & (kTab - 1);
                        }
                    }
                }
            }
#pragma unroll
            for (int off = 1; off < 16; off <<= 1)
                gc += __shfl_xor(gc, off);
            lds_fence();
            // modal bin (most hits, smallest index on ties) and occupied bins
            uint32_t bestc = 0, besti = 0x7FFFFFFF, nz = 0;
            for (int i = sl; i < nb; i += 16) {
                const uint32_t v = L.bins[slot][i];
                nz += v ? 1u : 0u;
                if (v > bestc) {
                    bestc = v;
                    besti = i;
                }
            }
            uint32_t ndp = sl < kMF / 32 ? __popc(L.pbits[slot][sl]) : 0u;
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                const uint32_t oc = __shfl_xor(bestc, off);
                const uint32_t oi = __shfl_xor(besti, off);
                if (oc > bestc || (oc == bestc && oi < besti)) {
                    bestc = oc;
                    besti = oi;
                }
                nz += __shfl_xor(nz, off);
                ndp += __shfl_xor(ndp, off);
            }
            if (act) {
                CandStats S;
                S.nh = L.acc[slot][0];
                S.ndp = ndp;
                S.mode = S.nh ? besti : 0u;
                S.nmode = S.nh ? bestc : 0u;
                S.nmode3 = S.nh ? L.bins[slot][S.mode] + (S.mode ? L.bins[slot][S.mode - 1] : 0u) +
                                      L.bins[slot][S.mode + 1]
                                : 0u;
                S.nbins = nz;
                S.gc = gc;
                S.nf = (uint32_t)nf;
                S.strand = w.strand;
                uint16_t v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    v[q] = f2bf(cand_feature(4 * sl + q, S, L.acc[slot], P, mf));
                uint2 pk;
                pk.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
                pk.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
                *reinterpret_cast<uint2 *>(feat + (uint64_t)(a + c) * kIn + 4 * sl) = pk;
                if (sl == 0) {
                    L.nm3[c] = S.nmode3;
                    L.ndp[c] = S.ndp;
                }
            }
            lds_fence();
        }
        // ---- features comparing the read's candidates (39..44)
        uint32_t mx3 = 0, mxd = 0;
        for (uint32_t c = lane; c < K; c += 64) {
            mx3 = max(mx3, L.nm3[c]);
            mxd = max(mxd, L.ndp[c]);
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            mx3 = max(mx3, (uint32_t)__shfl_xor((int)mx3, off));
            mxd = max(mxd, (uint32_t)__shfl_xor((int)mxd, off));
        }
        uint32_t at_max = 0, second = 0;
        for (uint32_t c = lane; c < K; c += 64) {
            const uint32_t v = L.nm3[c];
            at_max += v == mx3 ? 1u : 0u;
            if (v != mx3)
                second = max(second, v);
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            at_max += __shfl_xor(at_max, off);
            second = max(second, (uint32_t)__shfl_xor((int)second, off));
        }
        if (at_max >= 2)
            second = mx3;
        const float Pd = (float)max(P, 1);
        for (uint32_t idx = lane; idx < 6 * K; idx += 64) {
            const uint32_t c = idx / 6;
            const int f = 39 + (int)(idx % 6);
            const uint32_t v3 = L.nm3[c];
            float v;
            if (f == 39) v = (float)((int)v3 - (int)mx3) / Pd;
            else if (f == 40) v = (float)((int)L.ndp[c] - (int)mxd) / Pd;
            else if (f == 41) v = v3 == mx3 ? 1.f : 0.f;
            else if (f == 42) {
                uint32_t gt = 0;
                for (uint32_t d = 0; d < K; ++d)
                    gt += L.nm3[d] > v3 ? 1u : 0u;
                v = (float)gt / (float)K;
            } else if (f == 43) v = (float)(mx3 - second) / Pd;
            else v = (float)K / 16.f;
            feat[(uint64_t)(a + c) * kIn + f] = f2bf(v);
        }
        lds_fence();
    }
}

}  // namespace

hipError_t launch_features(const sw_batch &b, const uint32_t *first, const uint32_t *count,
                           uint16_t *feat, int n_cu, hipStream_t st)
{
    if (b.n_reads == 0)
        return hipSuccess;
    uint32_t blocks = (b.n_reads + kWavesF - 1) / kWavesF;
    const uint32_t cap = (uint32_t)n_cu * 8;
    if (blocks > cap)
        blocks = cap;
    hipLaunchKernelGGL(k_features, dim3(blocks), dim3(64 * kWavesF), 0, st, b, first, count, feat);
    return hipGetLastError();
}

}  // namespace hpgsw
