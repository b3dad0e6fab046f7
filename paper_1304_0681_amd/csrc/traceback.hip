// Traceback: full alignments with CIGAR for selected pairs.
//
// The DP of the score kernel is recomputed with the same lane layout (G lanes
// per pair, RPL rows per lane).  Every cell stores a 4-bit direction code in a
// per-pair slot of device scratch, four comparison bits:
//   bit 3  H(i,c) is not the diagonal value H(i-1,c-1) + s(i,c)
//   bit 2  H(i,c) is not the deletion value E(i,c)
//   bit 1  the deletion value of the NEXT column extends rather than opens
//          (E(i,c) + gap_extend > H(i,c) + gap_open; an open wins ties)
//   bit 0  the insertion value of the NEXT row extends rather than opens
// Each bit is the sign of a difference; three bit selects gather a cell's four
// and one funnel shift moves them into the lane's code word, so a cell costs
// no compare/select pairs.  The stop
// condition (H == 0) needs no bit: every step of the walk fixes the value of
// the cell it moves to (a diagonal step subtracts s(i,c), a gap step the
// extension or opening penalty), so the walk knows H along the path and stops
// where it reaches 0, which is the canonical rule (stop first, then diagonal,
// deletion, insertion).
// Codes are stored by step: at step t lane l computes column t - l, and its
// RPL rows fill ceil(RPL/8) 32-bit words (8 codes each, the lane's first row in
// the highest nibble used) at word (t * G + l) * ceil(RPL/8) of the slot, so the
// lanes of a group store one contiguous run per step and a tile needs no
// multiple of 8 rows per lane (104 rows cover 100-nt queries, 160 rows 150-nt
// ones).  The
// lanes of each group then walk back together from the end cell (smallest window
// column, then smallest read row among the maxima), G cells per step, and the
// first lane run-length encodes the ops.  Given the score pass's hits (score
// and end cell), a pair's DP covers only the window columns an alignment of
// that score ending there can reach (tb_band), which changes no code the walk
// reads.
#include "internal.h"

namespace hpgsw {

namespace {

constexpr int kWaves = 4;

struct TBParams {
    const uint32_t *ref;
    uint64_t ref_len, ref_words;
    const uint32_t *reads;
    const uint64_t *read_off;
    const uint16_t *read_len;
    uint32_t n_reads;
    const sw_window *win;
    const uint32_t *sel;       // caller's selected pair ids
    const uint32_t *ids;       // indices into sel, bucketed
    const uint32_t *seg;
    uint32_t *counter;
    int cls;
    int ma, mi, go, ge;
    sw_aln *aln;
    uint32_t *ops;
    uint32_t ops_stride;
    uint32_t *codes;           // scratch holding one slot per pair in flight
    uint64_t codes_words;      // size of the scratch in 32-bit words
    const uint32_t *maxlen;    // per class: longest window, then longest read
    TbBand band;               // score-pass hits for the DP band (hits may be null)
};

template <bool B>
struct Flag {
    static constexpr bool value = B;
};

template <int G>
__device__ __forceinline__ int tb_shift_up(int x, bool first, int boundary)
{
    if constexpr (G == 16) {
        return __builtin_amdgcn_update_dpp(boundary, x, 0x111, 0xF, 0xF, false);
    } else if constexpr (G == 64) {
        return __builtin_amdgcn_update_dpp(boundary, x, 0x138, 0xF, 0xF, false);
    } else if constexpr (G == 32) {
        int y = __builtin_amdgcn_update_dpp(boundary, x, 0x138, 0xF, 0xF, false);
        return first ? boundary : y;
    } else {
        int y = __builtin_amdgcn_update_dpp(boundary, x, 0x111, 0xF, 0xF, false);
        return first ? boundary : y;
    }
}

__device__ __forceinline__ int tb_wave_max(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = max(v, __shfl_xor(v, off));
    return v;
}

// (w << 4) | the sign bits of a, b, c and d, a's the highest.  Every argument
// lies in (-2^27, 2^27) (scores and penalties are at most 127 in magnitude and
// H stays below 2^24), so its bits 31..28 all equal its sign bit: three bit
// selects (v_bitop3_b32, table 0xE4: the third operand's set bits take the
// first operand, its clear bits the second) gather bit 31 of a, 30 of b, 29 of
// c and 28 of d, and one funnel shift moves the four in.  The selects issue at
// the rate of an add, twice that of the funnel shift they replace three of.
__device__ __forceinline__ uint32_t ins_signs4(uint32_t w, int a, int b, int c, int d)
{
    const uint32_t ab = __builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, 0x80000000u, 0xE4);
    const uint32_t cd = __builtin_amdgcn_bitop3_b32((uint32_t)c, (uint32_t)d, 0x20000000u, 0xE4);
    const uint32_t y = __builtin_amdgcn_bitop3_b32(ab, cd, 0xC0000000u, 0xE4);
    return __builtin_amdgcn_alignbit(w, y, 28u);
}

// Keeps x in a register at this point: the code bits of a cell are computed
// right after its values instead of being sunk into the column's store branch,
// which would keep every row's differences live until the column ends.
__device__ __forceinline__ void keep_here(uint32_t &x)
{
    asm volatile("" : "+v"(x));
}

__device__ __forceinline__ uint32_t tb_window_word(const TBParams &P, int64_t rb, int64_t c0)
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

// STRIP: queries longer than one strip of G*RPL rows (G == 64); the boundary
// row between strips goes through the tail of the pair's slot.
// Waves per SIMD: the 12- and 13-row tiles are held to 128 VGPRs for four (a few
// registers spill outside the cell loop; measured faster than three), the 16-
// and 20-row tiles to 168 for three, the 32-row strip tile to 256 for two; the
// 8-row tiles fit four as they are.
template <int RPL>
constexpr int tb_min_waves()
{
    return RPL >= 24 ? 2 : (RPL == 12 || RPL == 13) ? 4 : (RPL == 16 || RPL == 20) ? 3 : 1;
}

template <int G, int RPL, bool STRIP>
__global__ void __launch_bounds__(64 * kWaves, tb_min_waves<RPL>()) k_sw_traceback(const TBParams P)
{
    constexpr int PPW = 64 / G;
    constexpr int SR = G * RPL;
    constexpr int WPL = (RPL + 7) / 8;   // code words per lane per column
    const int lane = threadIdx.x & 63;
    const int grp = lane / G;
    const int l = lane % G;
    const bool first = l == 0;
    const uint32_t seg_begin = P.seg[2 * P.cls];
    const uint32_t seg_end = P.seg[2 * P.cls + 1];
    // an empty class ends at once, before every wave takes a turn at the task counter
    if (seg_end <= seg_begin)
        return;
    const uint32_t n_tasks = (seg_end - seg_begin + PPW - 1) / PPW;
    const int go = P.go, ge = P.ge;
    const uint32_t wave_global = blockIdx.x * kWaves + (threadIdx.x >> 6);
    // Slot size from the class maxima (read on the device, so no host round
    // trip): codes of every column, the strip boundary row, and the op runs.
    // Waves whose slots do not fit the scratch take no work; with no room for
    // even one wave every pair of the class is marked and skipped.
    const uint64_t nmax = P.maxlen[P.cls], mmax = P.maxlen[kNumClasses + P.cls];
    const uint64_t strips_max = STRIP ? (mmax + SR - 1) / SR : 1;
    const uint64_t slot_words =
        strips_max * G * WPL * (nmax + G - 1) + (STRIP ? 2 * nmax : 0) + mmax + nmax + 8;
    const uint64_t fit = P.codes_words / ((uint64_t)PPW * slot_words);
    // (a slot is addressed with 32-bit word offsets)
    const bool no_room = fit == 0 || slot_words > 0xFFFFFFFFull;
    if (!no_room && wave_global >= fit)
        return;
    uint32_t *slot_codes = P.codes + (no_room ? 0 : (uint64_t)(wave_global * PPW + grp) * slot_words);

    for (;;) {
        uint32_t task = 0;
        if (lane == 0)
            task = atomicAdd(&P.counter[P.cls], 1u);
        task = __shfl(task, 0);
        if (task >= n_tasks)
            break;
        const uint32_t slot = seg_begin + task * PPW + grp;
        const bool active = slot < seg_end;
        const uint32_t k_sel = active ? P.ids[slot] : 0u;
        if (no_room) {        // wave-uniform
            if (active && first)
                P.aln[k_sel] = sw_aln{-1, -1, -1, -1, -1, 0u, 4u};
            continue;
        }
        // an idle group reads window 0 (the batch has pairs): the caller's ids may
        // name no pair (e.g. 0xFFFFFFFF for a read without a hit), the first one too
        const uint32_t pair = active ? P.sel[k_sel] : 0u;
        const sw_window w = P.win[pair];
        int m = 0, n = 0, c_lo = 0;
        uint64_t roff = 0;
        if (active) {
            m = P.read_len[w.read_id];
            roff = P.read_off[w.read_id];
            const uint64_t avail = P.ref_len - w.ref_begin;
            n = w.len < avail ? (int)w.len : (int)avail;
            // the band the bucketing kernel binned the pair by (same function)
            n = tb_band(P.band, pair, m, n, c_lo);
        }
        const int n_wave = tb_wave_max(n);
        const int T = n_wave + G - 1;
        const int m_wave = STRIP ? tb_wave_max(m) : SR;
        const int n_strips = STRIP ? (m_wave + SR - 1) / SR : 1;
        const uint32_t col_words = (uint32_t)(n_strips * G * WPL);   // code words per step
        const uint64_t code_words = (uint64_t)col_words * (uint64_t)T;
        int2 *bnd = reinterpret_cast<int2 *>(slot_codes + code_words);  // strip boundary row
        uint32_t *runs = slot_codes + code_words + (STRIP ? 2 * (uint64_t)n_wave : 0);
        const int64_t rb = (int64_t)w.ref_begin + c_lo;   // window column 0 of the DP

        // The end cell, when the caller's hit gives it (scored with ends): the DP
        // then only has to store codes.  A wave tracks the best cell unless every
        // pair of it has a known end.
        int best = 0, cbest = 0x7FFFFFFF, rbest = 0x7FFFFFFF;
        bool known = false;
        int kbest = 0, kcol = 0, krow = 0;
        if (active && P.band.hits) {
            const sw_hit hh = P.band.hits[pair];
            if (hh.score == 0) {
                known = true;
            } else if (hh.score > 0 && hh.read_end >= 0 && hh.read_end < m && hh.ref_end >= c_lo &&
                       hh.ref_end - c_lo < n) {
                known = true;
                kbest = hh.score;
                kcol = hh.ref_end - c_lo;
                krow = hh.read_end;
            }
        }
        const bool track = __ballot(active && !known) != 0;

        auto dp = [&](auto track_tag) {
        constexpr bool TRACK = decltype(track_tag)::value;
        for (int strip = 0; strip < n_strips; ++strip) {
            const int row0 = strip * SR + l * RPL;
            int prof[RPL];
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = row0 + r;
                if (i < m) {
                    const uint64_t pos = w.strand ? roff + (uint64_t)(m - 1 - i) : roff + (uint64_t)i;
                    uint32_t q = (P.reads[pos >> 4] >> (2 * (uint32_t)(pos & 15))) & 3u;
                    if (w.strand)
                        q = 3u - q;
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
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                H[r] = 0;
                E[r] = go;
            }
            // this lane's best cell of the strip: columns arrive in increasing order, so
            // a strictly larger column maximum keeps the smallest column, and the smallest
            // row holding that maximum in the column is taken
            int lbest = 0, lcol = 0x7FFFFFFF, lrow = 0x7FFFFFFF;
            int hup_prev = 0, gout = 0;
            const bool read_bnd = STRIP && strip > 0;
            const bool write_bnd = STRIP && strip + 1 < n_strips;
            __threadfence_block();
            uint32_t cur = tb_window_word(P, rb, -l);
            for (int t0 = 0; t0 < T; t0 += 16) {
                const uint32_t nxt = tb_window_word(P, rb, t0 + 16 - l);
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const int t = t0 + k;
                    if (t >= T)
                        break;
                    const int c = t - l;
                    const bool valid = (unsigned)c < (unsigned)n;
                    const int wd = valid ? 8 : 0;
                    const int rc8 = (int)((cur >> (2 * k)) & 3u) << 3;
                    int bh_in = 0, bg_in = 0;
                    if (read_bnd && first && (unsigned)t < (unsigned)n_wave) {
                        const int2 v = bnd[t];
                        bh_in = v.x;
                        bg_in = v.y;
                    }
                    const int hup = tb_shift_up<G>(H[RPL - 1], first, bh_in);
                    const int gin = tb_shift_up<G>(gout, first, bg_in);
                    int diag = hup_prev;
                    hup_prev = hup;
                    int g = gin;
                    uint32_t cw[WPL];
#pragma unroll
                    for (int q = 0; q < WPL; ++q)
                        cw[q] = 0;
                    int cmax = 0;
#pragma unroll
                    for (int r = 0; r < RPL; ++r) {
                        const int s = __builtin_amdgcn_sbfe(prof[r], rc8, wd);
                        const int dd = diag + s;
                        diag = H[r];
                        const int e = E[r];
                        const int h = max(max(dd, e), g);
                        H[r] = h;
                        const int hg = h + go;
                        const int ege = e + ge, gge = g + ge;
                        const int en = max(ege, hg);
                        const int gn = max(max(gge, hg), 0);
                        // code bits, most significant first (h >= dd and h >= e, so the
                        // first two differences are negative exactly when h differs);
                        // a clamped insertion value (0) is never the source of a
                        // positive H, so its bit ignores the clamp
                        uint32_t &cq = cw[r >> 3];
                        cq = ins_signs4(cq, dd - h, e - h, hg - ege, hg - gge);
                        keep_here(cq);
                        E[r] = en;
                        g = gn;
                        if constexpr (TRACK)
                            cmax = max(cmax, h);
                    }
                    gout = g;
                    if (TRACK && valid && cmax > lbest) {
                        int row = RPL;
#pragma unroll
                        for (int r = RPL - 1; r >= 0; --r)
                            row = H[r] == cmax ? r : row;
                        lbest = cmax;
                        lcol = c;
                        lrow = row0 + row;
                    }
                    if (valid) {
                        // codes are stored by step, so a group's lanes write one
                        // contiguous run
                        uint32_t *dst = slot_codes + (uint64_t)t * col_words + (uint32_t)((strip * G + l) * WPL);
#pragma unroll
                        for (int q = 0; q < WPL; ++q)
                            dst[q] = cw[q];
                        if (write_bnd && l == G - 1)
                            bnd[c] = make_int2(H[RPL - 1], g);
                    }
                }
                cur = nxt;
            }
            if constexpr (TRACK) {
                const bool better = lbest > best ||
                                    (lbest == best && lbest > 0 &&
                                     (lcol < cbest || (lcol == cbest && lrow < rbest)));
                if (better) {
                    best = lbest;
                    cbest = lcol;
                    rbest = lrow;
                }
            }
        }
        };
        if (track)
            dp(Flag<true>{});
        else
            dp(Flag<false>{});
#pragma unroll
        for (int off = 1; off < G; off <<= 1) {
            const int ob = __shfl_xor(best, off);
            const int oc = __shfl_xor(cbest, off);
            const int orow = __shfl_xor(rbest, off);
            const bool take = ob > best || (ob == best && (oc < cbest || (oc == cbest && orow < rbest)));
            best = take ? ob : best;
            cbest = take ? oc : cbest;
            rbest = take ? orow : rbest;
        }
        if (known) {   // the same cell a tracking DP finds for a hit of this batch
            best = kbest;
            cbest = kcol;
            rbest = krow;
        }
        __threadfence_block();   // code stores of the whole wave before the walk

        if (active) {
            // Walk back.  The G lanes of the group hold the same walk state and look
            // at G cells at once along the current direction: in H state the cells
            // of the diagonal (i - q, c - q), whose H values follow from v and the
            // substitution scores of the cells before them (a prefix sum over the
            // group), so a whole run of diagonal steps advances in one iteration; in
            // a gap the extension bits of the next G cells, so a gap of any length
            // closes in one or a few iterations.  Runs are collected last-to-first
            // in `runs` by the first lane.
            const int q = l;
            const int gbase = grp * G;
            const uint64_t gmask = G == 64 ? ~0ull : (((1ull << G) - 1ull) << gbase);
            int i = rbest, c = cbest, state = 0, bi = rbest, bc = cbest, v = best;
            uint32_t nruns = 0, cur_op = 0xFFu, cur_len = 0;
            const uint32_t max_runs = (uint32_t)(m + n + 2);
            // code of an in-bounds cell: lane-layout position of its row (strip,
            // lane, row in the lane), then its nibble in the lane's word
            auto code_of = [&](int ii, int cc) -> uint32_t {
                const int sp = STRIP ? (int)((uint32_t)ii / (uint32_t)SR) : 0;
                const int rs = ii - sp * SR;
                const int ln = (int)((uint32_t)rs / (uint32_t)RPL), r = rs - ln * RPL;
                const uint32_t wv = slot_codes[(uint32_t)(cc + ln) * col_words + (uint32_t)((sp * G + ln) * WPL + (r >> 3))];
                const int nq = min(8, RPL - (r & ~7));   // rows in the row's word
                return (wv >> (4u * (uint32_t)(nq - 1 - (r & 7)))) & 15u;
            };
            // substitution score of an in-bounds cell; positions are 32-bit offsets
            // from the 16-base words holding the pair's first read and window bases
            const uint32_t *rdw = P.reads + (roff >> 4);
            const uint32_t *fww = P.ref + ((uint64_t)rb >> 4);
            const uint32_t r0 = (uint32_t)(roff & 15), f0 = (uint32_t)((uint64_t)rb & 15);
            auto subst_of = [&](int ii, int cc) -> int {
                const uint32_t pos = r0 + (uint32_t)(w.strand ? m - 1 - ii : ii);
                const uint32_t fpos = f0 + (uint32_t)cc;
                uint32_t qb = (rdw[pos >> 4] >> (2u * (pos & 15u))) & 3u;
                if (w.strand)
                    qb = 3u - qb;
                const uint32_t fb = (fww[fpos >> 4] >> (2u * (fpos & 15u))) & 3u;
                return qb == fb ? P.ma : P.mi;
            };
            auto emit = [&](uint32_t op, uint32_t cnt) {
                if (op == cur_op) {
                    cur_len += cnt;
                } else {
                    if (cur_len && nruns < max_runs) {
                        if (first)
                            runs[nruns] = (cur_len << 4) | cur_op;
                        ++nruns;
                    }
                    cur_op = op;
                    cur_len = cnt;
                }
            };
            if (best > 0) {
                for (;;) {
                    if (state == 0) {
                        if (i < 0 || c < 0 || v == 0)
                            break;
                        const int ii = i - q, cc = c - q;
                        const bool inb = ii >= 0 && cc >= 0;
                        uint32_t code = 8u;
                        int sq = 0;
                        if (inb) {
                            code = code_of(ii, cc);
                            sq = subst_of(ii, cc);
                        }
                        int incl = sq;   // inclusive prefix sum of the scores over the group
#pragma unroll
                        for (int off = 1; off < G; off <<= 1) {
                            const int t = __shfl_up(incl, off, G);
                            if (q >= off)
                                incl += t;
                        }
                        // this cell continues the diagonal run when it is inside the
                        // matrix, its H (v minus the scores of the cells before it)
                        // is not 0 and its H comes from the diagonal
                        const bool ok = inb && v - (incl - sq) != 0 && !(code & 8u);
                        const uint64_t bad = __ballot(!ok) & gmask;
                        const int r = bad ? (int)__builtin_ctzll(bad) - gbase : G;
                        if (r > 0) {
                            emit(SW_OP_M, (uint32_t)r);
                            v -= __shfl(incl, gbase + r - 1);
                            bi = i - (r - 1);
                            bc = c - (r - 1);
                            i -= r;
                            c -= r;
                        }
                        if (r < G) {
                            // the cell that ended the run is (i, c) now: a stop (the
                            // loop's test) or the start of a gap
                            const uint32_t code_r = __shfl(code, gbase + r);
                            if (i >= 0 && c >= 0 && v != 0)
                                state = (code_r & 4u) ? 2 : 1;   // 1: deletion run, 2: insertion run
                        }
                    } else {
                        // extension bits of the cells before (i, c) in the gap's
                        // direction; a gap reaching the matrix edge opens there
                        const int ii = state == 2 ? i - 1 - q : i;
                        const int cc = state == 1 ? c - 1 - q : c;
                        bool ext = false;
                        if (ii >= 0 && cc >= 0) {
                            const uint32_t code = code_of(ii, cc);
                            ext = state == 1 ? (code & 2u) != 0 : (code & 1u) != 0;
                        }
                        const uint64_t opens = __ballot(!ext) & gmask;
                        const int e = opens ? (int)__builtin_ctzll(opens) - gbase : G;
                        const int steps = e < G ? e + 1 : G;   // e extensions, then the opening
                        emit(state == 1 ? SW_OP_D : SW_OP_I, (uint32_t)steps);
                        if (state == 1)
                            c -= steps;
                        else
                            i -= steps;
                        v -= e * ge + (e < G ? go : 0);
                        if (e < G)
                            state = 0;
                    }
                }
                if (cur_len && nruns < max_runs) {
                    if (first)
                        runs[nruns] = (cur_len << 4) | cur_op;
                    ++nruns;
                }
            }
            if (first) {
                sw_aln a;
                a.status = 0;
                uint32_t *out = P.ops + (uint64_t)k_sel * P.ops_stride;
                if (best <= 0) {
                    a.score = 0;
                    a.read_begin = a.read_end = a.ref_begin = a.ref_end = -1;
                    a.n_ops = 0;
                } else {
                    a.score = best;
                    a.read_begin = bi;
                    a.read_end = rbest;
                    a.ref_begin = bc + c_lo;
                    a.ref_end = cbest + c_lo;
                    uint32_t k = 0;
                    bool trunc = false;
                    auto put = [&](uint32_t val) {
                        if (k < P.ops_stride)
                            out[k] = val;
                        else
                            trunc = true;
                        ++k;
                    };
                    if (bi > 0)
                        put(((uint32_t)bi << 4) | SW_OP_S);
                    for (int qq = (int)nruns - 1; qq >= 0; --qq)
                        put(runs[qq]);
                    if (m - 1 - rbest > 0)
                        put(((uint32_t)(m - 1 - rbest) << 4) | SW_OP_S);
                    a.n_ops = trunc ? P.ops_stride : k;
                    if (trunc)
                        a.status |= 1u;
                }
                P.aln[k_sel] = a;
            }
        }
        __threadfence_block();   // the walk's reads finish before the slot is reused
    }
}

template <int G, int RPL, bool STRIP>
hipError_t tb_launch(const TBParams &p, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_sw_traceback<G, RPL, STRIP>), dim3(grid), dim3(64 * kWaves), 0, st, p);
    return hipGetLastError();
}

}  // namespace

// Traceback shapes per query-length class (G lanes x RPL rows >= the class
// bound).  Above 512 bases the classes differ from the score path's: a
// 768-row tile for 513-768-base queries (a 1,024-row tile leaves a third of
// its rows empty on them), a 1,024-row tile for 769-1,024, and strips of
// 2,048 rows for everything longer.  From 257 bases on, a pair takes the whole
// wave: 8, 12 or 16 rows per lane keep three or four waves per SIMD (32 lanes
// with 16, 24 or 32 rows held two or three).
static const ClassShape kTBShapes[kNumClasses] = {
    {16, 2, 8},   {32, 4, 8},   {64, 8, 8},    {100, 8, 13},   {128, 16, 8},  {160, 8, 20},
    {256, 32, 8}, {512, 64, 8}, {768, 64, 12}, {1024, 64, 16}, {65535, 64, 32}};

ClassEdges traceback_edges()
{
    ClassEdges e;
    for (int c = 0; c < kNumClasses; ++c)
        e.m_max[c] = (uint32_t)kTBShapes[c].m_max;
    return e;
}

int traceback_waves_per_block() { return kWaves; }

hipError_t launch_traceback_class(int cls, const sw_batch &b, const sw_scoring &sc,
                                  const uint32_t *sel, const uint32_t *ids, const uint32_t *seg,
                                  uint32_t *counter, sw_aln *aln, uint32_t *ops,
                                  uint32_t ops_stride, uint32_t *codes, uint64_t codes_words,
                                  const uint32_t *maxlen, const TbBand &band, int grid,
                                  hipStream_t st)
{
    TBParams p;
    p.ref = b.d_ref2b;
    p.ref_len = b.ref_len;
    p.ref_words = (b.ref_len + 15) / 16;
    p.reads = b.d_reads2b;
    p.read_off = b.d_read_off;
    p.read_len = b.d_read_len;
    p.n_reads = b.n_reads;
    p.win = b.d_win;
    p.sel = sel;
    p.ids = ids;
    p.seg = seg;
    p.counter = counter;
    p.cls = cls;
    p.ma = sc.match;
    p.mi = sc.mismatch;
    p.go = sc.gap_open;
    p.ge = sc.gap_extend;
    p.aln = aln;
    p.ops = ops;
    p.ops_stride = ops_stride;
    p.codes = codes;
    p.codes_words = codes_words;
    p.maxlen = maxlen;
    p.band = band;
    switch (cls) {
    case 0: return tb_launch<2, 8, false>(p, grid, st);
    case 1: return tb_launch<4, 8, false>(p, grid, st);
    case 2: return tb_launch<8, 8, false>(p, grid, st);
    case 3: return tb_launch<8, 13, false>(p, grid, st);
    case 4: return tb_launch<16, 8, false>(p, grid, st);
    case 5: return tb_launch<8, 20, false>(p, grid, st);
    case 6: return tb_launch<32, 8, false>(p, grid, st);
    case 7: return tb_launch<64, 8, false>(p, grid, st);
    case 8: return tb_launch<64, 12, false>(p, grid, st);
    case 9: return tb_launch<64, 16, false>(p, grid, st);
    default: return tb_launch<64, 32, true>(p, grid, st);
    }
}

}  // namespace hpgsw
