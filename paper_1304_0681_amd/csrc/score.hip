// Batched Smith-Waterman / Gotoh scoring: the hot loop.
//
// Layout.  A pair is processed by a group of G lanes of one wave (64/G pairs
// per wave).  Lane l of the group owns query rows [l*RPL, (l+1)*RPL) and walks
// the window columns with a skew of one step per lane: at step t it computes
// column c = t - l for all its rows, top to bottom.  The row above a lane's
// first row lives in lane l-1, which finished that column one step earlier, so
// the only cross-lane traffic per step is two DPP row/wave shifts (H of the
// last row and the vertical-gap value entering the next row).  Nothing goes
// through LDS or memory in the inner loop; the window's 2-bit bases arrive in
// one 32-bit word per 16 steps.
//
// Recurrences per cell (exact integers, int32):
//   s  = bfe_i32(profile_row, 8*r_c, w)         w = 8, or 0 outside the window
//   h  = max3(diag + s, E, Gv)                  Gv = max(F, 0)
//   hg = h + gap_open
//   E' = max(E + gap_extend, hg)                deletion value of the next column
//   Gv'= max3(Gv + gap_extend, hg, 0)           vertical value of the next row
// Clamping the vertical value at zero folds the local-alignment zero of
// max(0, ...) into Gv without changing any H (H >= 0 and every F < 0 only
// ever feeds max(...) together with 0).  The profile holds the four scores of
// the row's query base, one signed byte per window base; a field width of
// zero gives s = 0 for columns before the window (fill) and after it (drain),
// which keeps the fill lanes at the boundary state H = 0 and makes drain
// cells harmless: they can only repeat values of cells to their left.
//
// Query rows past the read length use the profile -128 (never better than
// the row above).  The result per pair is the maximum H; with ends, the key
// (H << 16) + (0xFFFF - c) per row picks the smallest window column among
// equal scores, and the row reduction picks the smallest read row.
#include "internal.h"

namespace hpgsw {

namespace {

constexpr int kWaves = 4;  // waves per block

template <int G>
__device__ __forceinline__ int shift_up(int x, bool first, int boundary)
{
    // value of lane l-1 within the G-lane group; `boundary` for the first lane
    if constexpr (G == 1) {
        return boundary;
    } else if constexpr (G == 16) {
        return __builtin_amdgcn_update_dpp(boundary, x, 0x111, 0xF, 0xF, false);  // row_shr:1
    } else if constexpr (G == 64) {
        return __builtin_amdgcn_update_dpp(boundary, x, 0x138, 0xF, 0xF, false);  // wave_shr:1
    } else if constexpr (G == 32) {
        int y = __builtin_amdgcn_update_dpp(boundary, x, 0x138, 0xF, 0xF, false);
        return first ? boundary : y;
    } else {
        int y = __builtin_amdgcn_update_dpp(boundary, x, 0x111, 0xF, 0xF, false);
        return first ? boundary : y;
    }
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = max(v, __shfl_xor(v, off));
    return v;
}

__device__ __forceinline__ uint32_t read_base(const ScoreParams &P, uint64_t pos)
{
    return (P.reads[pos >> 4] >> (2 * (uint32_t)(pos & 15))) & 3u;
}

// 16 window bases for the columns [c0, c0+16) of a window starting at `rb`
// (absolute reference position of column 0), base c0+k at bits 2k..2k+1.
// Columns outside the reference are masked by the zero field width, so their
// bits are don't-care, but the in-range ones must keep their positions.
__device__ __forceinline__ uint32_t load_window_word(const ScoreParams &P, int64_t rb, int64_t c0)
{
    const int64_t s = rb + c0;   // reference position of column c0
    if (s < 0) {
        // columns before the reference start are masked; the rest begin at base 0
        if (s <= -16)
            return 0u;
        return P.ref[0] << (2u * (uint32_t)(-s));
    }
    uint64_t w0 = (uint64_t)s >> 4;
    uint64_t w1 = w0 + 1;
    const uint64_t last = P.ref_words - 1;
    if (w0 > last) w0 = last;   // only columns past the reference end read these
    if (w1 > last) w1 = last;
    return __builtin_amdgcn_alignbit(P.ref[w1], P.ref[w0], (uint32_t)(s & 15) * 2u);
}

// MODE 0: score only.  MODE 1: score + ends (16-bit score key).  MODE 2: ends,
// scores that may exceed 16 bits.  STRIP: queries longer than G*RPL, processed
// in strips whose boundary row goes through `strip_buf` (requires G == 64).
template <int G, int RPL, int MODE, bool STRIP>
__global__ void __launch_bounds__(64 * kWaves) k_sw_score(const ScoreParams P)
{
    static_assert(64 % G == 0, "G must divide the wave");
    static_assert(!STRIP || G == 64, "strips use whole waves");
    constexpr int PPW = 64 / G;  // pairs per wave
    constexpr int SR = G * RPL;  // rows per strip
    const int lane = threadIdx.x & 63;
    const int grp = lane / G;
    const int l = lane % G;
    const bool first = l == 0;
    const uint32_t seg_begin = P.seg[2 * P.cls];
    const uint32_t seg_end = P.seg[2 * P.cls + 1];
    if (seg_end == seg_begin)
        return;
    const uint32_t n_tasks = (seg_end - seg_begin + PPW - 1) / PPW;
    const int go = P.go, ge = P.ge;
    const uint32_t wave_global = blockIdx.x * kWaves + (threadIdx.x >> 6);
    int2 *bnd = STRIP ? P.strip_buf + (uint64_t)wave_global * P.strip_stride : nullptr;

    for (;;) {
        uint32_t task = 0;
        if (lane == 0)
            task = atomicAdd(&P.counter[P.cls], 1u);
        task = __shfl(task, 0);
        if (task >= n_tasks)
            break;
        const uint32_t slot = seg_begin + task * PPW + grp;
        const bool active = slot < seg_end;
        const uint32_t pair = active ? P.ids[slot] : 0u;
        const sw_window w = P.win[pair];
        int m = 0, n = 0;
        uint64_t roff = 0;
        if (active) {
            m = P.read_len[w.read_id];
            roff = P.read_off[w.read_id];
            const uint64_t avail = P.ref_len - w.ref_begin;
            n = w.len < avail ? (int)w.len : (int)avail;
        }
        const int n_wave = wave_max(n);
        const int T = n_wave + G - 1;  // steps until the last lane leaves the window
        const int m_wave = STRIP ? wave_max(m) : SR;
        const int n_strips = STRIP ? (m_wave + SR - 1) / SR : 1;
        const int64_t rb = (int64_t)w.ref_begin;

        // running best of the lane: MODE 0 score, MODE 1 key + row, MODE 2 score + col + row
        int best = 0;
        uint32_t kbest = 0;
        int rbest = 0x7FFFFFFF, cbest = 0x7FFFFFFF;

        for (int strip = 0; strip < n_strips; ++strip) {
            const int row0 = strip * SR + l * RPL;
            int prof[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = row0 + r;
                if (i < m) {
                    uint32_t q = w.strand ? 3u - read_base(P, roff + (uint64_t)(m - 1 - i))
                                          : read_base(P, roff + (uint64_t)i);
                    uint32_t v = 0;
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        v |= ((uint32_t)(b == (int)q ? P.ma : P.mi) & 0xFFu) << (8 * b);
                    prof[r] = (int)v;
                } else {
                    prof[r] = (int)0x80808080u;
                }
            }
            int H[RPL], E[RPL];
            uint32_t key[MODE == 1 ? RPL : 1];
            int bh[MODE == 2 ? RPL : 1], bj[MODE == 2 ? RPL : 1];
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                H[r] = 0;
                E[r] = go;
                if constexpr (MODE == 1) key[r] = 0;
                if constexpr (MODE == 2) { bh[r] = 0; bj[r] = 0x7FFFFFFF; }
            }
            int hup_prev = 0, gout = 0;
            const bool read_bnd = STRIP && strip > 0;
            const bool write_bnd = STRIP && strip + 1 < n_strips;
            if constexpr (STRIP) {
                if (strip > 0)
                    __threadfence_block();
            }
            // one step of the wavefront: column t - l of this lane's rows; `k` is the
            // position of the step inside its 16-column window word
            auto step = [&](const int t, const int k, const uint32_t word, const int2 bnd_in) {
                const int c = t - l;
                const bool valid = (unsigned)c < (unsigned)n;
                const int wd = valid ? 8 : 0;
                const int rc8 = (int)((word >> (2 * k)) & 3u) << 3;
                const int hup = shift_up<G>(H[RPL - 1], first, bnd_in.x);
                const int gin = shift_up<G>(gout, first, bnd_in.y);
                int diag = hup_prev;
                hup_prev = hup;
                int g = gin;
                const uint32_t cj = valid ? 0xFFFFu - (uint32_t)c : 0u;
                int hprev_row = 0;
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    const int s = __builtin_amdgcn_sbfe(prof[r], rc8, wd);
                    const int dd = diag + s;
                    diag = H[r];
                    const int h = max(max(dd, E[r]), g);
                    H[r] = h;
                    const int hg = h + go;
                    E[r] = max(E[r] + ge, hg);
                    g = max(max(g + ge, hg), 0);
                    if constexpr (MODE == 0) {
                        if (r & 1)
                            best = max(max(best, hprev_row), h);
                        else if (r == RPL - 1)
                            best = max(best, h);
                        else
                            hprev_row = h;
                    } else if constexpr (MODE == 1) {
                        key[r] = max(key[r], ((uint32_t)h << 16) + cj);
                    } else {
                        const bool better = valid && h > bh[r];
                        bh[r] = better ? h : bh[r];
                        bj[r] = better ? c : bj[r];
                    }
                }
                gout = g;
                if constexpr (STRIP) {
                    if (write_bnd && l == G - 1 && valid)
                        bnd[c] = make_int2(H[RPL - 1], g);
                }
            };
            auto bnd_at = [&](int t) -> int2 {
                return (read_bnd && (unsigned)t < (unsigned)n_wave) ? bnd[t] : make_int2(0, 0);
            };

            uint32_t cur = load_window_word(P, rb, -l);
            int2 bcur[STRIP ? 16 : 1];
            if constexpr (STRIP) {
#pragma unroll
                for (int k = 0; k < 16; ++k)
                    bcur[k] = bnd_at(k);
            }
            int t0 = 0;
            for (; t0 + 16 <= T; t0 += 16) {
                const uint32_t nxt = load_window_word(P, rb, t0 + 16 - l);
                int2 bnxt[STRIP ? 16 : 1];
                if constexpr (STRIP) {
#pragma unroll
                    for (int k = 0; k < 16; ++k)
                        bnxt[k] = bnd_at(t0 + 16 + k);
                }
#pragma unroll
                for (int k = 0; k < 16; ++k)
                    step(t0 + k, k, cur, STRIP ? bcur[STRIP ? k : 0] : make_int2(0, 0));
                cur = nxt;
                if constexpr (STRIP) {
#pragma unroll
                    for (int k = 0; k < 16; ++k)
                        bcur[k] = bnxt[k];
                }
            }
            // tail: fewer than 16 steps left
#pragma nounroll
            for (int k = 0; t0 + k < T; ++k)
                step(t0 + k, k, cur, STRIP ? bnd_at(t0 + k) : make_int2(0, 0));
            // fold this strip's per-row bests into the lane's running best
            if constexpr (MODE == 1) {
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    const int row = row0 + r;
                    if (key[r] > kbest || (key[r] == kbest && row < rbest)) {
                        kbest = key[r];
                        rbest = row;
                    }
                }
            } else if constexpr (MODE == 2) {
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    const int row = row0 + r;
                    const bool better = bh[r] > best ||
                                        (bh[r] == best && bh[r] > 0 &&
                                         (bj[r] < cbest || (bj[r] == cbest && row < rbest)));
                    if (better) {
                        best = bh[r];
                        cbest = bj[r];
                        rbest = row;
                    }
                }
            }
        }

        // reduce over the G lanes of the group and write the hit
        sw_hit hit;
        if constexpr (MODE == 0) {
#pragma unroll
            for (int off = 1; off < G; off <<= 1)
                best = max(best, __shfl_xor(best, off));
            hit = sw_hit{best, -1, -1};
        } else if constexpr (MODE == 1) {
            // larger key first, then smaller row
            uint64_t v = ((uint64_t)kbest << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)rbest);
#pragma unroll
            for (int off = 1; off < G; off <<= 1) {
                const uint64_t o = __shfl_xor(v, off);
                v = o > v ? o : v;
            }
            const uint32_t kb = (uint32_t)(v >> 32);
            const int score = (int)(kb >> 16);
            const int row = (int)(0xFFFFFFFFu - (uint32_t)v);
            hit = score > 0 ? sw_hit{score, row, (int)(0xFFFFu - (kb & 0xFFFFu))}
                            : sw_hit{0, -1, -1};
        } else {
#pragma unroll
            for (int off = 1; off < G; off <<= 1) {
                const int ob = __shfl_xor(best, off);
                const int oc = __shfl_xor(cbest, off);
                const int orow = __shfl_xor(rbest, off);
                const bool take = ob > best ||
                                  (ob == best && (oc < cbest || (oc == cbest && orow < rbest)));
                best = take ? ob : best;
                cbest = take ? oc : cbest;
                rbest = take ? orow : rbest;
            }
            hit = best > 0 ? sw_hit{best, rbest, cbest} : sw_hit{0, -1, -1};
        }
        if (active && first)
            P.hits[pair] = hit;
    }
}

// ---------------------------------------------------------------------------
// Packed int16 scoring: two pairs per lane group, one in each 16-bit half of
// every register (v_pk_* arithmetic), score only.
//
// Exact when match * min(m, n) <= 32767 and mismatch <= 0 (checked by the
// host per query-length class).  Differences from the int32 kernel:
//   - The deletion and vertical values are kept clamped at zero with the
//     unsigned-saturating subtract (v_pk_sub_u16 clamp), which folds the
//     local-alignment zero into them: E' = max(sat(E - |ge|), sat(H - |go|)).
//   - The substitution score of both halves comes from one v_perm_b32 over a
//     constant 8-byte table of four 16-bit entries {match, mismatch x3}: the
//     selector bytes are Q ^ R with Q = (2q, 2q) per half and row and
//     R = (2r, 2r+1) per half and column, so entry q XOR r is picked and
//     entry 0 is the match.  Padded rows use Q = (12, 12) and columns outside
//     the window R = (8, 9); every such selector lands on sign, zero or 0xFF
//     bytes or a mismatch entry, i.e. a score <= 0, which keeps fill lanes at
//     the zero boundary and makes drain and padding cells harmless.
// ---------------------------------------------------------------------------
typedef short v2i16 __attribute__((ext_vector_type(2)));
typedef unsigned short v2u16 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_max_i16(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(v2i16, a),
                                                                   __builtin_bit_cast(v2i16, b)));
}

__device__ __forceinline__ uint32_t pk_add_u16(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(v2u16, a) + __builtin_bit_cast(v2u16, b));
}

__device__ __forceinline__ uint32_t pk_sub_sat_u16(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(v2u16, a),
                                                                      __builtin_bit_cast(v2u16, b)));
}

template <int G, int RPL>
__global__ void __launch_bounds__(64 * kWaves) k_sw_score16(const ScoreParams P)
{
    static_assert(64 % G == 0, "G must divide the wave");
    constexpr int GPW = 64 / G;      // lane groups per wave
    constexpr int PPW = 2 * GPW;     // pairs per wave
    const int lane = threadIdx.x & 63;
    const int grp = lane / G;
    const int l = lane % G;
    const bool first = l == 0;
    const uint32_t seg_begin = P.seg[2 * P.cls];
    const uint32_t seg_end = P.seg[2 * P.cls + 1];
    if (seg_end == seg_begin)
        return;
    const uint32_t n_tasks = (seg_end - seg_begin + PPW - 1) / PPW;
    const uint32_t tbl_lo = ((uint32_t)P.ma & 0xFFFFu) | ((uint32_t)P.mi << 16);
    const uint32_t tbl_hi = ((uint32_t)P.mi & 0xFFFFu) | ((uint32_t)P.mi << 16);
    const uint32_t ugo = (uint32_t)(-P.go) * 0x10001u;
    const uint32_t uge = (uint32_t)(-P.ge) * 0x10001u;

    for (;;) {
        uint32_t task = 0;
        if (lane == 0)
            task = atomicAdd(&P.counter[P.cls], 1u);
        task = __shfl(task, 0);
        if (task >= n_tasks)
            break;
        const uint32_t slot_a = seg_begin + task * PPW + 2 * grp;
        const bool act_a = slot_a < seg_end;
        const bool act_b = slot_a + 1 < seg_end;
        const uint32_t pair_a = act_a ? P.ids[slot_a] : 0u;
        const uint32_t pair_b = act_b ? P.ids[slot_a + 1] : pair_a;
        const sw_window wa = P.win[pair_a];
        const sw_window wb = P.win[pair_b];
        int ma_ = 0, na = 0, mb = 0, nb = 0;
        uint64_t roa = 0, rob = 0;
        if (act_a) {
            ma_ = P.read_len[wa.read_id];
            roa = P.read_off[wa.read_id];
            const uint64_t avail = P.ref_len - wa.ref_begin;
            na = wa.len < avail ? (int)wa.len : (int)avail;
        }
        if (act_b) {
            mb = P.read_len[wb.read_id];
            rob = P.read_off[wb.read_id];
            const uint64_t avail = P.ref_len - wb.ref_begin;
            nb = wb.len < avail ? (int)wb.len : (int)avail;
        }
        const int n_wave = wave_max(max(na, nb));
        const int T = n_wave + G - 1;

        uint32_t Q[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = l * RPL + r;
            uint32_t qa = 0x0C0Cu, qb = 0x0C0Cu;
            if (i < ma_) {
                uint32_t q = wa.strand ? 3u - read_base(P, roa + (uint64_t)(ma_ - 1 - i))
                                       : read_base(P, roa + (uint64_t)i);
                qa = 2u * q * 0x0101u;
            }
            if (i < mb) {
                uint32_t q = wb.strand ? 3u - read_base(P, rob + (uint64_t)(mb - 1 - i))
                                       : read_base(P, rob + (uint64_t)i);
                qb = 2u * q * 0x0101u;
            }
            Q[r] = qa | (qb << 16);
        }
        uint32_t H[RPL], E[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            H[r] = 0;
            E[r] = 0;
        }
        uint32_t hup_prev = 0, gout = 0, best = 0;
        const int64_t rba = (int64_t)wa.ref_begin, rbb = (int64_t)wb.ref_begin;

        auto step = [&](const int t, const int k, const uint32_t wa_word, const uint32_t wb_word) {
            const int c = t - l;
            const uint32_t ra = (wa_word >> (2 * k)) & 3u;
            const uint32_t rb = (wb_word >> (2 * k)) & 3u;
            const uint32_t sa = (unsigned)c < (unsigned)na ? ra * 0x0202u + 0x0100u : 0x0908u;
            const uint32_t sb = (unsigned)c < (unsigned)nb ? rb * 0x0202u + 0x0100u : 0x0908u;
            const uint32_t R = sa | (sb << 16);
            const uint32_t hup = (uint32_t)shift_up<G>((int)H[RPL - 1], first, 0);
            const uint32_t gin = (uint32_t)shift_up<G>((int)gout, first, 0);
            uint32_t diag = hup_prev;
            hup_prev = hup;
            uint32_t g = gin;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const uint32_t s = __builtin_amdgcn_perm(tbl_hi, tbl_lo, Q[r] ^ R);
                const uint32_t d = pk_add_u16(diag, s);
                diag = H[r];
                const uint32_t h = pk_max_i16(pk_max_i16(d, E[r]), g);
                H[r] = h;
                const uint32_t hgz = pk_sub_sat_u16(h, ugo);
                E[r] = pk_max_i16(pk_sub_sat_u16(E[r], uge), hgz);
                g = pk_max_i16(pk_sub_sat_u16(g, uge), hgz);
                best = pk_max_i16(best, h);
            }
            gout = g;
        };

        uint32_t cur_a = load_window_word(P, rba, -l);
        uint32_t cur_b = load_window_word(P, rbb, -l);
        int t0 = 0;
        for (; t0 + 16 <= T; t0 += 16) {
            const uint32_t nxt_a = load_window_word(P, rba, t0 + 16 - l);
            const uint32_t nxt_b = load_window_word(P, rbb, t0 + 16 - l);
#pragma unroll
            for (int k = 0; k < 16; ++k)
                step(t0 + k, k, cur_a, cur_b);
            cur_a = nxt_a;
            cur_b = nxt_b;
        }
#pragma nounroll
        for (int k = 0; t0 + k < T; ++k)
            step(t0 + k, k, cur_a, cur_b);

#pragma unroll
        for (int off = 1; off < G; off <<= 1)
            best = pk_max_i16(best, (uint32_t)__shfl_xor((int)best, off));
        if (first) {
            if (act_a)
                P.hits[pair_a] = sw_hit{(int)(int16_t)(best & 0xFFFFu), -1, -1};
            if (act_b)
                P.hits[pair_b] = sw_hit{(int)(int16_t)(best >> 16), -1, -1};
        }
    }
}

template <int G, int RPL>
hipError_t launch_packed(const ScoreParams &p, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_sw_score16<G, RPL>), dim3(grid), dim3(64 * kWaves), 0, st, p);
    return hipGetLastError();
}

template <int G, int RPL, int MODE, bool STRIP>
hipError_t launch_one(const ScoreParams &p, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_sw_score<G, RPL, MODE, STRIP>), dim3(grid), dim3(64 * kWaves), 0, st, p);
    return hipGetLastError();
}

template <int G, int RPL, bool STRIP = false>
hipError_t launch_modes(int mode, const ScoreParams &p, int grid, hipStream_t st)
{
    switch (mode) {
    case 0: return launch_one<G, RPL, 0, STRIP>(p, grid, st);
    case 1: return launch_one<G, RPL, 1, STRIP>(p, grid, st);
    default: return launch_one<G, RPL, 2, STRIP>(p, grid, st);
    }
}

}  // namespace

int score_waves_per_block() { return kWaves; }

#define HPGSW_SHAPES(X) \
    X(1, 16) X(1, 32) X(2, 32) X(4, 16) X(4, 25) X(4, 32) X(8, 13) X(8, 20) X(8, 32) X(16, 32) \
    X(32, 32) X(64, 32)

bool score_shape_available(int G, int RPL)
{
#define X(g, r) if (G == g && RPL == r) return true;
    HPGSW_SHAPES(X)
#undef X
    return false;
}

hipError_t launch_score16_class(int G, int RPL, const ScoreParams &p, int grid, hipStream_t st)
{
#define X(g, r) if (G == g && RPL == r) return launch_packed<g, r>(p, grid, st);
    HPGSW_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_score_class(int cls, int G, int RPL, int mode, const ScoreParams &p, int grid,
                              hipStream_t st)
{
    if (cls == kNumClasses - 1)
        return launch_modes<64, 32, true>(mode, p, grid, st);
#define X(g, r) if (G == g && RPL == r) return launch_modes<g, r>(mode, p, grid, st);
    HPGSW_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace hpgsw
