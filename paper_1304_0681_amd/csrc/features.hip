// Per-candidate seed-hit features (64 x bf16 per pair) for the learned filter.
//
// The evidence is the one the paper's stage D uses to turn seed matches into
// candidate alignment locations (Sec. 2, "Stage D: CAL Seeker"): where a read's
// short exact seeds (12-mers here) land in a candidate window, and whether they
// line up on one diagonal.
//
// One wave per read.  The read's 12-mers, for both orientations, go into two
// open-addressing hash tables in LDS (at most 245 k-mers in 512 slots each).
// The wave then takes the read's candidate windows four at a time, 16 lanes per
// window: each lane rolls over window positions j, builds the 12-mer from the
// 2-bit reference words, probes the table of the window's strand and records
// every hit (p, j) in LDS accumulators (diagonal bins of width 16, a bitmap of
// hit read positions, two 16-bin position histograms).  Per-candidate
// statistics are kept in LDS and a last pass writes the 64 features, one lane
// per feature.  Features are computed in float32 and rounded to bfloat16.
#include "mlp_internal.h"

namespace hpgsw {

namespace {

constexpr int kK = 12;             // seed length
constexpr int kMF = 256;           // query bases used
constexpr int kNF = 4096;          // window bases used
constexpr int kTab = 512;          // hash slots per orientation
constexpr int kSlots = 4;          // candidates in flight per wave
constexpr int kMaxBins = (kNF + kMF) / 16 + 3;
constexpr int kWavesF = 2;         // waves per block
constexpr int kStat = 41;          // statistics words per candidate
// statistic indices
enum { S_NDP, S_NH, S_NMODE, S_NMODE3, S_NBINS, S_MODE, S_GC, S_N, S_STRAND, S_HP = 9, S_HJ = 25 };

struct alignas(16) WaveLds {
    uint32_t key[2][kTab];
    uint16_t pos[2][kTab];
    uint32_t bins[kSlots][kMaxBins];
    uint32_t pbits[kSlots][kMF / 32];
    uint32_t acc[kSlots][36];      // nh, gc, hist_p[16], hist_j[16]
    uint32_t stat[kMaxCand][kStat];
};

__device__ __forceinline__ uint32_t hash24(uint32_t k)
{
    return (k * 0x9E3779B1u) >> 23;   // 9 bits
}

__device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint32_t base_at(const uint32_t *seq, uint64_t pos)
{
    return (seq[pos >> 4] >> (2 * (uint32_t)(pos & 15))) & 3u;
}

// 12-mer of the reference starting at absolute position s (2 bits per base,
// base i of the k-mer at bits 2i)
__device__ __forceinline__ uint32_t ref_kmer(const uint32_t *ref, uint64_t words, uint64_t s)
{
    const uint64_t w0 = s >> 4;
    const uint64_t w1 = w0 + 1 < words ? w0 + 1 : w0;
    const uint32_t v = __builtin_amdgcn_alignbit(ref[w1], ref[w0], (uint32_t)(s & 15) * 2u);
    return v & 0xFFFFFFu;
}

__device__ __forceinline__ void lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__global__ void __launch_bounds__(64 * kWavesF) k_features(const sw_batch b, const uint32_t *first,
                                                           const uint32_t *count, uint16_t *feat)
{
    __shared__ WaveLds lds_all[kWavesF];
    WaveLds &L = lds_all[threadIdx.x >> 6];
    const int lane = threadIdx.x & 63;
    const uint64_t ref_words = (b.ref_len + 15) / 16;
    for (uint32_t r = blockIdx.x * kWavesF + (threadIdx.x >> 6); r < b.n_reads;
         r += gridDim.x * kWavesF) {
        const uint32_t K = count[r];
        if (K == 0 || K > kMaxCand)
            continue;
        const uint32_t a = first[r];
        // the decision treats non-contiguous reads as unsure; skip them here
        bool contiguous = true;
        {
            uint32_t ok = 1;
            for (uint32_t c = lane; c < K; c += 64)
                ok &= (b.d_win[a + c].read_id == r) ? 1u : 0u;
            contiguous = __all(ok);
        }
        if (!contiguous)
            continue;
        const int m_full = b.d_read_len[r];
        const uint64_t roff = b.d_read_off[r];
        const int mf = min(m_full, kMF);
        const int P = max(mf - kK + 1, 0);
        // ---- hash tables of the query k-mers (orientation 0: read, 1: reverse complement)
        for (int i = lane; i < kTab; i += 64) {
            L.key[0][i] = 0;
            L.key[1][i] = 0;
        }
        lds_fence();
        for (int e = lane; e < 2 * P; e += 64) {
            const int o = e >= P;
            const int p = o ? e - P : e;
            uint32_t km = 0;
            for (int i = 0; i < kK; ++i) {
                const int qi = p + i;   // query position
                const uint32_t q = o ? 3u - base_at(b.d_reads2b, roff + (uint64_t)(m_full - 1 - qi))
                                     : base_at(b.d_reads2b, roff + (uint64_t)qi);
                km |= q << (2 * i);
            }
            uint32_t h = hash24(km);
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
        const int slot = lane >> 4, sl = lane & 15;
        // ---- candidates, four at a time
        for (uint32_t c0 = 0; c0 < K; c0 += kSlots) {
            const uint32_t c = c0 + slot;
            const bool act = c < K;
            sw_window w = b.d_win[a + (act ? c : 0)];
            int n = 0;
            if (act && (uint64_t)w.ref_begin < b.ref_len) {
                const uint64_t avail = b.ref_len - w.ref_begin;
                n = w.len < avail ? (int)w.len : (int)avail;
            }
            const int nf = min(n, kNF);
            const int J = max(nf - kK + 1, 0);
            const int nb = ((nf + mf) >> 4) + 2;
            for (int i = sl; i < kMaxBins; i += 16)
                L.bins[slot][i] = 0;
            if (sl < kMF / 32)
                L.pbits[slot][sl] = 0;
            for (int i = sl; i < 36; i += 16)
                L.acc[slot][i] = 0;
            lds_fence();
            const int o = w.strand ? 1 : 0;
            const int Pd = max(P, 1), Jd = max(J, 1);
            uint32_t gc = 0;
            for (int j = sl; j < nf; j += 16) {
                const uint64_t s = (uint64_t)w.ref_begin + (uint64_t)j;
                const uint32_t km = ref_kmer(b.d_ref2b, ref_words, s);
                const uint32_t b0 = km & 3u;
                gc += (b0 == 1u || b0 == 2u) ? 1u : 0u;
                if (j >= J || P == 0)
                    continue;
                uint32_t h = hash24(km);
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
            if (act && gc)
                atomicAdd(&L.acc[slot][1], gc);
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
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                const uint32_t oc = __shfl_xor(bestc, off);
                const uint32_t oi = __shfl_xor(besti, off);
                if (oc > bestc || (oc == bestc && oi < besti)) {
                    bestc = oc;
                    besti = oi;
                }
                nz += __shfl_xor(nz, off);
            }
            uint32_t ndp = sl < kMF / 32 ? __popc(L.pbits[slot][sl]) : 0u;
#pragma unroll
            for (int off = 1; off < 16; off <<= 1)
                ndp += __shfl_xor(ndp, off);
            if (act) {
                uint32_t *S = L.stat[c];
                const uint32_t nh = L.acc[slot][0];
                if (sl == 0) {
                    const uint32_t mode = nh ? besti : 0u;
                    S[S_NDP] = ndp;
                    S[S_NH] = nh;
                    S[S_NMODE] = nh ? bestc : 0u;
                    S[S_NMODE3] = nh ? (L.bins[slot][mode] + (mode ? L.bins[slot][mode - 1] : 0u) +
                                        L.bins[slot][mode + 1])
                                     : 0u;
                    S[S_NBINS] = nz;
                    S[S_MODE] = mode;
                    S[S_GC] = L.acc[slot][1];
                    S[S_N] = (uint32_t)nf;
                    S[S_STRAND] = w.strand;
                }
                S[S_HP + sl] = L.acc[slot][2 + sl];
                S[S_HJ + sl] = L.acc[slot][18 + sl];
            }
            lds_fence();
        }
        // ---- features, one lane per feature
        uint32_t mx3 = 0, mxd = 0;
        for (uint32_t c = 0; c < K; ++c) {
            mx3 = max(mx3, L.stat[c][S_NMODE3]);
            mxd = max(mxd, L.stat[c][S_NDP]);
        }
        uint32_t n_at_max = 0, second = 0;
        for (uint32_t c = 0; c < K; ++c) {
            const uint32_t v = L.stat[c][S_NMODE3];
            if (v == mx3)
                ++n_at_max;
            else
                second = max(second, v);
        }
        if (n_at_max >= 2)
            second = mx3;
        const float Pd = (float)max(P, 1);
        for (uint32_t c = 0; c < K; ++c) {
            const uint32_t *S = L.stat[c];
            const int f = lane;
            float v = 0.f;
            const float nf_ = (float)max((int)S[S_N], 1);
            if (f == 0) v = (float)S[S_NDP] / Pd;
            else if (f == 1) v = (float)min(S[S_NH], 4u * (uint32_t)max(P, 1)) / Pd;
            else if (f == 2) v = (float)S[S_NMODE] / Pd;
            else if (f == 3) v = (float)S[S_NMODE3] / Pd;
            else if (f == 4) v = (float)min(S[S_NBINS], 64u) / 16.f;
            else if (f == 5) v = S[S_NH] ? (float)(16 * (int)S[S_MODE] + 8 - mf) / nf_ : 0.f;
            else if (f == 6) v = S[S_NH] ? 1.f : 0.f;
            else if (f < 23) v = (float)S[S_HP + f - 7] / Pd;
            else if (f < 39) v = (float)S[S_HJ + f - 23] / Pd;
            else if (f == 39) v = (float)((int)S[S_NMODE3] - (int)mx3) / Pd;
            else if (f == 40) v = (float)((int)S[S_NDP] - (int)mxd) / Pd;
            else if (f == 41) v = S[S_NMODE3] == mx3 ? 1.f : 0.f;
            else if (f == 42) {
                uint32_t gt = 0;
                for (uint32_t d = 0; d < K; ++d)
                    gt += L.stat[d][S_NMODE3] > S[S_NMODE3] ? 1u : 0u;
                v = (float)gt / (float)K;
            } else if (f == 43) v = (float)(mx3 - second) / Pd;
            else if (f == 44) v = (float)K / 16.f;
            else if (f == 45) v = (float)S[S_N] / 1000.f;
            else if (f == 46) v = (float)mf / 1000.f;
            else if (f == 47) v = (float)S[S_STRAND];
            else if (f == 48) v = (float)S[S_GC] / nf_;
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
