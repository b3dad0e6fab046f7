// Packed int16 scoring, the body of one wave of the persistent kernel.
//
// Two pairs per lane group, one in each 16-bit half of every register
// (v_pk_* arithmetic), score only.  Exact when match * min(m, n) <= 32767
// and mismatch <= 0 (checked by the host per query-length class).  The layout
// is the int32 kernel's (G lanes per pair group, RPL query rows per lane, one
// skewed window column per step); the differences:
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
//
// The wave's cross-lane and special instructions come from the policy W
// (static member functions): lane(), dpp_row_shr1(old, x) and
// dpp_wave_shr1(old, x) (DPP row_shr:1 / wave_shr:1 of x, `old` in lanes
// without a source), shfl(v, src), shfl_xor(v, mask), atomic_add(p, v),
// perm(hi, lo, sel) (v_perm_b32) and alignbit(hi, lo, shift).  The kernel
// instantiates it with the hardware instructions; a host model of the wave
// instantiates it with emulated lanes, so both run this one source.  PT is the
// parameter struct (ScoreParams on the device).
#pragma once

#include <stdint.h>

#include "hpgsw.h"

#if defined(__HIPCC__)
#define SW16_INLINE __device__ __forceinline__
#else
#define SW16_INLINE inline __attribute__((always_inline))
#endif

namespace hpgsw {
namespace sw16 {

constexpr int kWaves = 4;   // waves per block of the kernel

typedef short v2i16 __attribute__((ext_vector_type(2)));
typedef unsigned short v2u16 __attribute__((ext_vector_type(2)));

SW16_INLINE uint32_t pk_max_i16(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(v2i16, a),
                                                                   __builtin_bit_cast(v2i16, b)));
}

SW16_INLINE uint32_t pk_add_u16(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(v2u16, a) + __builtin_bit_cast(v2u16, b));
}

SW16_INLINE uint32_t pk_sub_sat_u16(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(v2u16, a),
                                                                      __builtin_bit_cast(v2u16, b)));
}

// value of lane l-1 within the G-lane group; `boundary` for the first lane
template <int G, class W>
SW16_INLINE int shift_up(int x, bool first, int boundary)
{
    if constexpr (G == 1) {
        return boundary;
    } else if constexpr (G == 16) {
        return W::dpp_row_shr1(boundary, x);
    } else if constexpr (G == 64) {
        return W::dpp_wave_shr1(boundary, x);
    } else if constexpr (G == 32) {
        const int y = W::dpp_wave_shr1(boundary, x);
        return first ? boundary : y;
    } else {
        const int y = W::dpp_row_shr1(boundary, x);
        return first ? boundary : y;
    }
}

template <class W>
SW16_INLINE int wave_max(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int o = W::shfl_xor(v, off);
        v = v > o ? v : o;
    }
    return v;
}

template <class PT>
SW16_INLINE uint32_t read_base(const PT &P, uint64_t pos)
{
    return (P.reads[pos >> 4] >> (2 * (uint32_t)(pos & 15))) & 3u;
}

// 16 window bases for the columns [c0, c0+16) of a window starting at `rb`
// (absolute reference position of column 0), base c0+k at bits 2k..2k+1.
// Columns outside the reference are masked, so their bits are don't-care,
// but the in-range ones must keep their positions.
template <class W, class PT>
SW16_INLINE uint32_t window_word(const PT &P, int64_t rb, int64_t c0)
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
    return W::alignbit(P.ref[w1], P.ref[w0], (uint32_t)(s & 15) * 2u);
}

template <int G, int RPL, class W, class PT>
SW16_INLINE void wave_body(const PT &P)
{
    static_assert(64 % G == 0, "G must divide the wave");
    constexpr int GPW = 64 / G;      // lane groups per wave
    constexpr int PPW = 2 * GPW;     // pairs per wave
    const int lane = W::lane();
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
            task = W::atomic_add(&P.counter[P.cls], 1u);
        task = (uint32_t)W::shfl((int)task, 0);
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
        const int n_wave = wave_max<W>(na > nb ? na : nb);
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
            const uint32_t hup = (uint32_t)shift_up<G, W>((int)H[RPL - 1], first, 0);
            const uint32_t gin = (uint32_t)shift_up<G, W>((int)gout, first, 0);
            uint32_t diag = hup_prev;
            hup_prev = hup;
            uint32_t g = gin;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const uint32_t s = W::perm(tbl_hi, tbl_lo, Q[r] ^ R);
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

        uint32_t cur_a = window_word<W>(P, rba, -l);
        uint32_t cur_b = window_word<W>(P, rbb, -l);
        int t0 = 0;
        for (; t0 + 16 <= T; t0 += 16) {
            const uint32_t nxt_a = window_word<W>(P, rba, t0 + 16 - l);
            const uint32_t nxt_b = window_word<W>(P, rbb, t0 + 16 - l);
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
            best = pk_max_i16(best, (uint32_t)W::shfl_xor((int)best, off));
        if (first) {
            if (act_a)
                P.hits[pair_a] = sw_hit{(int)(int16_t)(best & 0xFFFFu), -1, -1};
            if (act_b)
                P.hits[pair_b] = sw_hit{(int)(int16_t)(best >> 16), -1, -1};
        }
    }
}

}  // namespace sw16
}  // namespace hpgsw
