/*
 * hpgsw.h -- batched Smith-Waterman (affine gaps) for RNA-seq read alignment
 * on AMD Instinct MI355X (gfx950).
 *
 * The operation is the alignment task of the paper's stage E (Sec. 2,
 * "Stage E: SWA + Splice Junctions", task iii): every read is aligned with
 * the Smith-Waterman local alignment algorithm against each of its extended
 * candidate alignment locations (windows), and the alignment, its score and
 * its start position are returned; task iv keeps the alignments whose score
 * reaches a threshold.  Windows come from the CAL seeker (Sec. 2, "Stage D:
 * CAL Seeker"), extended on both sides (stage E, task i).
 *
 * Scoring model (the paper leaves it open; this library fixes Gotoh's affine
 * gaps with signed integer scores):
 *   E(i,j) = max(H(i,j-1) + gap_open, E(i,j-1) + gap_extend)   deletion (consumes window)
 *   F(i,j) = max(H(i-1,j) + gap_open, F(i-1,j) + gap_extend)   insertion (consumes read)
 *   H(i,j) = max(0, H(i-1,j-1) + s(q_i, r_j), E(i,j), F(i,j)),  H = 0 on row/column 0
 * so a gap of k bases costs gap_open + (k-1)*gap_extend.  The best score S is
 * the maximum of H.  End cell: among cells with H == S, the smallest window
 * position, then the smallest read position.  Traceback from the end cell:
 * diagonal before deletion before insertion, a gap opens as soon as opening
 * reaches the value, and the path stops at the first H == 0.  All results are
 * exact integers; the library never approximates.
 *
 * Conventions for every call:
 *   - Returns sw_status (0 = SW_OK, < 0 = error) and never throws or aborts;
 *     sw_last_error() holds a message for the last failing call on a context.
 *   - Pointers named d_* are DEVICE pointers owned by the caller; the library
 *     never frees them.  Other pointers are host pointers, read during the call.
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL = the
 *     default stream) and is asynchronous: outputs are valid once the stream
 *     has synchronised.  Scratch that the library allocates belongs to the
 *     context; calls on one context must not overlap (one context per host
 *     thread and stream).
 *   - Sequences are 2-bit packed: base p of a sequence buffer sits in 32-bit
 *     word p >> 4, bits 2*(p & 15) .. 2*(p & 15)+1, codes A=0 C=1 G=2 T=3.  A
 *     packed buffer of L bases holds ceil(L/16) words (sw_pack2b writes this).
 *   - Window coordinates are 0-based and inclusive; ref_* coordinates are
 *     relative to the window start, read_* coordinates to the query.  For a
 *     window with strand 1 the query is the reverse complement of the read.
 *
 * Limits: read and window lengths up to 65,535; scores with
 * 0 < match <= 127, -127 <= mismatch < match, -127 <= gap_open < 0 and
 * gap_open <= gap_extend <= 0 (otherwise SW_E_INVALID).
 */
#ifndef HPGSW_H
#define HPGSW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SW_OK = 0,
    SW_E_INVALID = -1,  /* bad argument (NULL pointer, bad scoring, bad flags) */
    SW_E_RANGE = -2,    /* a size is out of the supported range */
    SW_E_NOMEM = -3,    /* device allocation of scratch failed */
    SW_E_DEVICE = -4,   /* a HIP runtime call failed */
    SW_E_NODEVICE = -5, /* no usable gfx950 device */
    SW_E_STATE = -6     /* object used in the wrong state */
} sw_status;

typedef struct sw_ctx sw_ctx;

/* Integer scoring scheme; e.g. {+5, -4, -10, -1}. */
typedef struct {
    int32_t match, mismatch, gap_open, gap_extend;
} sw_scoring;

/* One candidate window (an extended CAL) of one read: 12 bytes, packed.
 * The window is reference bases [ref_begin, ref_begin + len), clipped to the
 * reference.  strand 1: align the reverse complement of the read.  flags are
 * carried for the caller and ignored by the library. */
typedef struct {
    uint32_t read_id;
    uint32_t ref_begin;
    uint16_t len;
    uint8_t strand;
    uint8_t flags;
} sw_window;

/* A batch: one packed reference, packed reads, and (read, window) pairs. */
typedef struct {
    const uint32_t *d_ref2b;      /* packed reference, ceil(ref_len/16) words */
    uint64_t ref_len;             /* bases */
    const uint32_t *d_reads2b;    /* packed reads, concatenated */
    uint64_t reads_len;           /* bases in d_reads2b */
    const uint64_t *d_read_off;   /* [n_reads] base offset of each read in d_reads2b */
    const uint16_t *d_read_len;   /* [n_reads] read lengths */
    uint32_t n_reads;
    const sw_window *d_win;       /* [n_pairs] windows, any order */
    uint32_t n_pairs;
    /* optional device count of valid pairs: when not NULL, only the first
     * min(n_pairs, *d_n_pairs) windows are used and n_pairs is the capacity
     * (lets a compacted work list be scored without a host round trip) */
    const uint32_t *d_n_pairs;
} sw_batch;

/* Score result of one pair.  score -1 marks an invalid pair (read_id out of
 * range); score 0 means no alignment (ends -1).  Ends are filled only with
 * SW_WANT_ENDS, else -1. */
typedef struct {
    int32_t score, read_end, ref_end;
} sw_hit;

/* Full alignment of one pair (sw_batch_traceback). */
typedef struct {
    int32_t score, read_begin, read_end, ref_begin, ref_end;
    uint32_t n_ops;   /* CIGAR ops written for this pair */
    uint32_t status;  /* bit0: ops truncated to ops_stride; bit1: invalid pair
                         (id >= n_pairs or read_id out of range); bit2: not
                         aligned, traceback scratch too small (see
                         SW_OPT_TB_SCRATCH_MB) */
} sw_aln;

#define SW_WANT_ENDS 1u

/* CIGAR op codes, as in SAM/BAM; an op is (len << 4) | code. */
#define SW_OP_M 0u
#define SW_OP_I 1u
#define SW_OP_D 2u
#define SW_OP_N 3u
#define SW_OP_S 4u

/* Create a context on HIP device `hip_device` (must be gfx950).  *out receives
 * the context; destroy it with sw_ctx_destroy.  SW_E_NODEVICE if the device
 * does not exist or is not gfx950. */
sw_status sw_ctx_create(int hip_device, sw_ctx **out);
sw_status sw_ctx_destroy(sw_ctx *ctx);
const char *sw_last_error(const sw_ctx *ctx);

/* Encode step: pack n ASCII bases (d_ascii, bytes 'A','C','G','T') into
 * d_out (ceil(n/16) 32-bit words, unused high bits zero).  Any other byte is
 * encoded as A and counted into *d_bad (device uint32, may be NULL; it is
 * incremented, not cleared).  The read and reference encoding of Sec. 2,
 * stage A (reads are held with their sequence), in the 2-bit form the
 * aligner reads.
 * Invalid input is reported through *d_bad, not through the return value: the
 * call is asynchronous, so the count is known only once the stream has
 * synchronised.  A nonzero count means d_out is not the input sequence, and
 * every result computed from it is invalid: the caller must clear the counter
 * before the call and check it afterwards (pass d_bad whenever the input may
 * hold other bytes, e.g. the N of a sequencer). */
sw_status sw_pack2b(sw_ctx *ctx, const uint8_t *d_ascii, uint64_t n, uint32_t *d_out,
                    uint32_t *d_bad, void *stream);

/* Best local alignment score of every (read, window) pair of `batch` (Sec. 2,
 * stage E task iii).  d_hits[n_pairs] receives scores, and end coordinates if
 * flags has SW_WANT_ENDS.  Pairs are bucketed by length and scheduled onto
 * persistent kernels; results do not depend on pair order or bucketing. */
sw_status sw_batch_score(sw_ctx *ctx, const sw_batch *batch, const sw_scoring *sc,
                         uint32_t flags, sw_hit *d_hits, void *stream);

/* Allocation-free variant of sw_batch_score, for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as sw_batch_score,
 * and the same kernels; the scratch is a fixed array in the library's device
 * memory (about 36 MiB on every GPU the library runs on, held until the
 * process ends) instead of context scratch, and the call allocates nothing.
 * Limits: n_pairs <= SW_NOALLOC_MAX_PAIRS (otherwise SW_E_RANGE); queries
 * longer than 2,048 bases are scored by 8 waves (same results, slower).
 * Every call on one GPU shares that array, which keeps the last call's
 * contents (each call rebuilds everything it reads): calls that overlap on
 * one GPU (two streams, contexts or threads) race and give undefined results,
 * so the caller must serialise them. */
#define SW_NOALLOC_MAX_PAIRS (1u << 22)
sw_status sw_batch_score_noalloc(sw_ctx *ctx, const sw_batch *batch, const sw_scoring *sc,
                                 uint32_t flags, sw_hit *d_hits, void *stream);

/* Best hit per read (Sec. 2, stage E task iv): for every read, the pair with
 * the highest score among its windows (lowest pair index on ties) and that
 * score.  Reads without windows get best_pair 0xFFFFFFFF and score -1.
 * d_mapped (may be NULL) receives 1 where best_score >= t_map (a successful
 * mapping), else 0. */
sw_status sw_best_per_read(sw_ctx *ctx, const sw_batch *batch, const sw_hit *d_hits,
                           int32_t t_map, uint32_t *d_best_pair, int32_t *d_best_score,
                           uint8_t *d_mapped, void *stream);

/* d_win_out[k] = the window of pair d_pair_ids[k] of `batch`, for k < n (ids
 * at or beyond the batch's pairs give a window with read id 0xFFFFFFFF, which
 * every call answers as an invalid pair).  With the ids from
 * sw_best_per_read this builds a batch of each read's best window, which can
 * be scored with SW_WANT_ENDS and traced back with those hits (the traceback's
 * band) at the cost of one pass over the best windows only. */
sw_status sw_select_windows(sw_ctx *ctx, const sw_batch *batch, const uint32_t *d_pair_ids,
                            uint32_t n, sw_window *d_win_out, void *stream);

/* Reads with a single candidate (Sec. 2, stage E tasks iii-iv: a read's best
 * window is the best-scoring of its candidates, so a read with one candidate
 * needs no score pass to pick it; its alignment gives its score).
 * A pair "scores" when sw_batch_score would align it or answer it with 0:
 * read id below n_reads and the read inside the packed reads (an empty or
 * clipped window counts; pairs at or beyond batch->d_n_pairs do not).  For
 * every read r < n_reads: d_sole[r] = the index of r's scoring pair when the
 * batch holds exactly one, else 0xFFFFFFFF.  The scoring pairs of the reads
 * with two or more are compacted in pair order into d_win_out and d_ids_out
 * (their index in `batch`), *d_n_out = their number; both arrays must hold
 * n_pairs entries.  Scoring that list (sw_batch.d_n_pairs = d_n_out), taking
 * its best pair per read (sw_best_per_read) and merging (sw_merge_best) gives
 * the best pairs sw_best_per_read gives over the whole batch (ties keep the
 * lowest pair index in both).  Device arrays; d_sole[n_reads].  Uses context
 * scratch (8 bytes per read and about 1 per pair; growing it fails with
 * SW_E_STATE during capture or while a captured graph of the context lives). */
sw_status sw_sole_windows(sw_ctx *ctx, const sw_batch *batch, uint32_t *d_sole,
                          sw_window *d_win_out, uint32_t *d_ids_out, uint32_t *d_n_out,
                          void *stream);

/* For r < n_reads: d_best_pair[r] = d_sole[r] when it is not 0xFFFFFFFF, else
 * d_ids[d_sub_best[r]] when d_sub_best[r] < n_ids, else 0xFFFFFFFF.  d_sole and
 * d_ids as written by sw_sole_windows, d_sub_best by sw_best_per_read over its
 * compacted list; n_ids = that list's capacity.  Device arrays. */
sw_status sw_merge_best(sw_ctx *ctx, uint32_t n_reads, const uint32_t *d_sole,
                        const uint32_t *d_sub_best, const uint32_t *d_ids, uint32_t n_ids,
                        uint32_t *d_best_pair, void *stream);

/* Full alignments with CIGAR for the pairs listed in d_pair_ids[n_sel]
 * (Sec. 2, stage E task iii: the alignment and its start position, which the
 * junction search of task iv reads).  d_aln[n_sel] receives coordinates;
 * d_ops[n_sel * ops_stride] receives each pair's ops, soft clips included.
 * A pair whose CIGAR needs more than ops_stride ops gets the first
 * ops_stride ops and status bit0.  m + n + 2 ops always suffice.
 * d_hits (may be NULL): d_hits[n_pairs] as written by sw_batch_score with
 * SW_WANT_ENDS for the same batch and scoring (indexed by pair, like
 * d_pair_ids).  With it, each pair's DP covers only the window columns an
 * alignment of that score ending at that cell can reach, which gives the same
 * alignments and CIGARs in less time; pairs whose hit has no end, and every
 * pair when a gap penalty is 0, use the whole window; the walk starts at the
 * hit's end cell.  Hits that do not come from that call give undefined
 * alignments (never out-of-bounds accesses).  Pairs are bucketed by query
 * length as in sw_batch_score up to 512 bases, and above into 513-768,
 * 769-1,024 and longer queries (the last in strips of 2,048 rows). */
sw_status sw_batch_traceback(sw_ctx *ctx, const sw_batch *batch, const sw_scoring *sc,
                             const uint32_t *d_pair_ids, uint32_t n_sel, sw_aln *d_aln,
                             uint32_t *d_ops, uint32_t ops_stride, const sw_hit *d_hits,
                             void *stream);

/* ---------------------------------------------------------------------------
 * Spliced reads (Sec. 2, "Stage E: SWA + Splice Junctions", tasks i, ii, iv).
 *
 * A long read is cut into seeds; every seed is aligned against its candidate
 * windows (sw_batch_score, sw_best_per_read, sw_batch_traceback).  The
 * reference span of a seed's best alignment is a candidate alignment location
 * (CAL) of the read.  Each CAL is extended on both sides (task i, 30 bases by
 * default) and the extended CALs of a read that lie closer than the longest
 * intron are joined into one window (task ii); the whole read is aligned
 * against its joined windows (task iii, the calls above, with a scoring whose
 * gap extension is 0 so that an intron costs one gap open), and a long run of
 * deletions whose ends carry an intron motif becomes a splice junction
 * (task iv), counted in a table that lives across batches (the paper's AVL
 * tree; here a device hash table).
 * ------------------------------------------------------------------------- */

/* One CAL: reference bases [first, last] (absolute, inclusive) of read read_id
 * on strand `strand` (1: the read's reverse complement aligns there); valid 0
 * marks a seed without a CAL.  16 bytes. */
typedef struct {
    uint32_t read_id;
    uint32_t first, last;
    uint8_t strand;
    uint8_t valid;
    uint16_t reserved;   /* written as 0 */
} sw_cal;

/* One splice junction: intron [start, end) in absolute reference positions;
 * strand 0: the intron reads GT...AG on the reference (a gene on the forward
 * strand), 1: CT...AC (a gene on the reverse strand); count: the alignments
 * that reported it.  24 bytes. */
typedef struct {
    uint64_t start, end;
    uint32_t count;
    uint32_t strand;
} sw_junction;

/* CALs of n_seeds seeds: seed s belongs to long read d_seed_read[s], its best
 * window is d_best_pair[s] (a pair of `seeds`, from sw_best_per_read) and
 * d_aln[s] its alignment there (sw_batch_traceback with those pair ids).
 * d_cals[s] = {d_seed_read[s], window start + aln.ref_begin, window start +
 * aln.ref_end, window strand, 1} when the pair exists, the alignment scores at
 * least max(min_score, 1) and its last base lies below 2^32; otherwise
 * {d_seed_read[s], 0, 0, 0, 0}.  All arrays are device arrays of n_seeds. */
sw_status sw_seed_cals(sw_ctx *ctx, const sw_batch *seeds, const uint32_t *d_best_pair,
                       const sw_aln *d_aln, const uint32_t *d_seed_read, uint32_t n_seeds,
                       int32_t min_score, sw_cal *d_cals, void *stream);

/* Joined windows from n_cals CALs, which must be grouped by read (non-decreasing
 * read ids: a read whose CALs form several separate runs has each run joined
 * on its own; the call cannot check the order without a host round trip).
 * Per read, the first 16 valid CALs with first <= last < ref_len count; CALs
 * of reads >= n_reads are ignored.  Each becomes [max(first - ext, 0),
 * min(last + ext, ref_len - 1)]; sorted by (strand, first, last), a CAL joins
 * the current window when it has the window's strand and fewer than max_gap
 * bases lie strictly between the window's end and its first base (overlap
 * joins); the window's end becomes the larger of the two.  Windows are
 * written to d_win_out (capacity n_cals, never exceeded) read by read in that
 * order, as {read, first, min(length, 65535), strand, flags 0}, and their
 * number to *d_n_out (device), ready for a batch with d_n_pairs = d_n_out.
 * Uses context scratch (about 17 bytes per CAL; growing it fails with
 * SW_E_STATE under capture or while a captured graph is alive). */
sw_status sw_join_cals(sw_ctx *ctx, const sw_cal *d_cals, uint32_t n_cals, uint32_t n_reads,
                       uint64_t ref_len, uint32_t ext, uint32_t max_gap, sw_window *d_win_out,
                       uint32_t *d_n_out, void *stream);

/* ---------------------------------------------------------------------------
 * Region seeker and CAL seeker (Sec. 2, "Stage C: Region Seeker" and
 * "Stage D: CAL Seeker").
 *
 * Every read is cut into seeds of k bases in two phases (starts 0, step,
 * 2 step, ... and offset, offset + step, ...; k = 15, step = 12, offset = 7 give
 * a 100-nt read the paper's 8 + 7 seeds); each seed is mapped exactly onto
 * the reference through a k-mer index, on both strands, and every match is a
 * region; a read's regions closer than merge_gap bases are merged, and a
 * merged region longer than min_len bases is a CAL.  The CALs feed
 * sw_join_cals (stage E tasks i, ii), whose windows feed sw_batch_score.
 * ------------------------------------------------------------------------- */

/* Exact k-mer index of a packed reference, for k in [4, 15], in one
 * caller-owned device buffer of sw_kmer_index_bytes bytes: a 32-bit start
 * offset for every one of the 4^k codes plus one (code c's positions are
 * pos[start[c] .. start[c + 1])), then the positions (one 32-bit word per
 * k-mer of the reference, L - k + 1 of them, in no particular order within a
 * code).  A k-mer's code holds base i at bits 2i.  For k = 15 the offsets take
 * 4 GiB.  SW_E_RANGE if k is out of range or the reference holds 2^32 or more
 * k-mers. */
sw_status sw_kmer_index_bytes(uint64_t ref_len, uint32_t k, uint64_t *bytes);
/* Build the index (counting sort on the device; context scratch of about
 * 4^k / 1024 bytes).  index_bytes must be at least sw_kmer_index_bytes. */
sw_status sw_kmer_index_build(sw_ctx *ctx, const uint32_t *d_ref2b, uint64_t ref_len, uint32_t k,
                              void *d_index, uint64_t index_bytes, void *stream);

typedef struct {
    uint32_t k;         /* seed length, the index's k */
    uint32_t step;      /* distance between the seeds of one phase, >= 1 */
    uint32_t offset;    /* first base of the second phase */
    uint32_t max_occ;   /* a seed matching more places than this on a strand gives
                           no region there */
} sw_seed_params;

/* One region: reference bases [first, first + k) match a seed exactly; strand 1:
 * the seed's reverse complement matches there, and read_pos is the seed's
 * position in the read's reverse complement (so first - read_pos is the read's
 * diagonal on either strand).  8 bytes; the read is the segment it lies in. */
typedef struct {
    uint32_t first;
    uint16_t read_pos;
    uint8_t strand;
    uint8_t reserved;   /* written as 0 */
} sw_region;

/* Regions of every read of `reads` (its reads, and its reference length for
 * the index size check: the windows and reference bases are not used) against
 * the index d_index of index_bytes bytes, built by sw_kmer_index_build with
 * sp->k from the batch's reference.  An index_bytes below
 * sw_kmer_index_bytes(reads->ref_len, sp->k) is refused (SW_E_RANGE), so a k
 * larger than the index's cannot read past it; an index of another reference
 * or a smaller k gives undefined regions (never out-of-bounds accesses).  Read r's
 * regions are d_regions[read_end[r - 1] .. read_end[r]) (read_end[-1] = 0;
 * d_read_end: device uint64 array of n_reads), in seed order (first phase
 * first), strand 0 before strand 1 for each seed, reference positions
 * ascending.  Regions at or beyond cap are counted in read_end but not written.
 * Reads outside the packed reads get none.  Context scratch: about 4 bytes per
 * read. */
sw_status sw_seed_regions(sw_ctx *ctx, const sw_batch *reads, const void *d_index,
                          uint64_t index_bytes, const sw_seed_params *sp, sw_region *d_regions,
                          uint64_t cap, uint64_t *d_read_end, void *stream);

/* CALs of every read from its regions (the first SW_SEEKER_MAX_REGIONS of
 * them that lie below cap): per strand, regions sorted by first base merge
 * while fewer than merge_gap bases lie strictly between the next region and
 * the merged region's end (overlap merges); a merged region [first, last] is
 * a CAL when last - first + 1 > min_len.  Read r's CALs go to
 * d_cals[r * SW_SEEKER_MAX_CALS ...], ordered by (strand, first), at most
 * SW_SEEKER_MAX_CALS of them (the first in that order), and the remaining
 * slots get invalid CALs {r, 0, 0, 0, 0}: the array is grouped by read, as
 * sw_join_cals takes it.  k is the regions' length.  d_skip (device, n_reads,
 * may be NULL): reads with a nonzero entry get invalid CALs only (pass
 * sw_stage_b's d_n_maps so that the reads stage B mapped skip stages C-E, as
 * in the paper). */
#define SW_SEEKER_MAX_CALS 16
#define SW_SEEKER_MAX_REGIONS 1024
sw_status sw_cal_seeker(sw_ctx *ctx, const sw_region *d_regions, const uint64_t *d_read_end,
                        uint32_t n_reads, uint64_t cap, uint32_t k, uint32_t merge_gap,
                        uint32_t min_len, const uint32_t *d_skip, sw_cal *d_cals, void *stream);

/* Stage B (Sec. 2, "Stage B: BWT"): whole-read mapping with at most one error,
 * insertion or deletion.  The paper searches a BWT; here the candidate starts
 * come from the read's exact seed regions (sw_seed_regions; the first
 * SW_SEEKER_MAX_REGIONS below cap): every region diagonal d = first - read_pos
 * gives the starts d - 1, d and d + 1 on its strand.  The query (the read, or
 * its reverse complement on strand 1; m bases) is verified at each start p, in
 * this order: exact (ref[p, p + m)), one substitution, one deletion (the
 * reference holds one base the read lacks after query base i - 1, smallest i
 * in [1, m - 1]), one insertion (query base i is extra, smallest i in
 * [1, m - 2]); spans leaving the reference do not apply, nor do indels at the
 * query's ends.  A read is mapped when a start verifies; only the starts with
 * the fewest edits are reported, by (strand, start), at most SW_BMAP_MAX:
 * d_maps[r * SW_BMAP_MAX + j] for j < d_n_maps[r] (the rest zero), 0 records =
 * unmapped here (the read goes on to the seekers).  `batch` gives the
 * reference and the reads (the regions' reads); its windows are not used. */
#define SW_BMAP_MAX 16
#define SW_BMAP_EXACT 0u
#define SW_BMAP_SUBST 1u
#define SW_BMAP_DEL 2u
#define SW_BMAP_INS 3u
typedef struct {
    uint32_t first, last;   /* reference bases of the mapping, inclusive */
    uint8_t strand;
    uint8_t edits;          /* 0 or 1 */
    uint8_t op;             /* SW_BMAP_* */
    uint8_t reserved;       /* written as 0 */
    int32_t edit_pos;       /* query position of the edit (i for indels), -1 if exact */
} sw_bmap;
sw_status sw_stage_b(sw_ctx *ctx, const sw_batch *batch, const sw_region *d_regions,
                     const uint64_t *d_read_end, uint64_t cap, sw_bmap *d_maps,
                     uint32_t *d_n_maps, void *stream);

/* Junction table: caller-owned device arrays d_keys[capacity] (uint64) and
 * d_counts[capacity] (uint32), capacity a power of two in [1, 2^31].  Zero
 * them with sw_junctions_clear before first use; sw_detect_junctions adds to
 * them, so a table accumulates over any number of batches.  An entry is key
 * (start << 17 | length << 1 | strand, 0 = empty) and its count. */
sw_status sw_junctions_clear(sw_ctx *ctx, uint64_t *d_keys, uint32_t *d_counts,
                             uint32_t capacity, void *stream);

/* Junction search on n alignments of `batch`: alignment k is d_aln[k] with ops
 * d_ops[k * ops_stride ...] for pair d_pair_ids[k] (the arguments of the
 * sw_batch_traceback call that produced them).  Alignments with status bits
 * set, score < max(min_score, 1), or a pair outside the batch are left alone.
 * In the others, every deletion run of L >= min_intron bases (min_intron >= 4)
 * whose neighbours are match runs of a and b bases may move by s,
 * -(a-1) <= s <= b-1, where each step keeps the score (a step left needs the
 * reference base before the run to equal the run's last base, a step right the
 * run's first base to equal the base after it); the leftmost reachable
 * placement whose run starts with GT and ends with AG (strand 0) or starts with
 * CT and ends with AC (strand 1) is a junction: the run is rewritten in place
 * as an N op (its neighbours as a + s and b - s matches, so the score is
 * unchanged) and the junction's count in the table goes up by one.  Runs
 * without such a placement stay deletions.  d_n_junc (device, may be NULL)
 * receives the junctions found per alignment; *d_dropped (device, may be
 * NULL) is incremented once per junction the full table could not take. */
sw_status sw_detect_junctions(sw_ctx *ctx, const sw_batch *batch, const uint32_t *d_pair_ids,
                              uint32_t n, const sw_aln *d_aln, uint32_t *d_ops,
                              uint32_t ops_stride, int32_t min_score, uint32_t min_intron,
                              uint64_t *d_keys, uint32_t *d_counts, uint32_t capacity,
                              uint32_t *d_n_junc, uint32_t *d_dropped, void *stream);

/* The table's junctions, in no particular order: the first out_cap go to
 * d_out, and their total number to *d_n (device; may exceed out_cap). */
sw_status sw_list_junctions(sw_ctx *ctx, const uint64_t *d_keys, const uint32_t *d_counts,
                            uint32_t capacity, sw_junction *d_out, uint32_t out_cap,
                            uint32_t *d_n, void *stream);

/* Graph capture (the orchestration of a batch without per-call launch cost).
 * Every library call issued on `stream` between sw_graph_begin and
 * sw_graph_end is recorded, not run; sw_graph_launch replays the recording on
 * any stream, reading and writing the same device buffers.  The calls of the
 * score / best-hit / traceback path (and sw_pack2b, sw_filter_candidates with
 * a host pair count) need no host round trip, so they can be captured.  A call
 * that would have to grow a scratch buffer during capture fails with
 * SW_E_STATE: make the same calls once, uncaptured, before capturing.  The
 * stream must be a created stream (not the null stream); phase timing must be
 * off.  If a captured call fails, end the capture with sw_graph_end (which
 * then returns an error too) before using the context again.
 * A graph's kernels use the context's scratch buffers as they were at capture
 * time.  While any graph ended on a context is alive (until sw_graph_destroy),
 * a call on that context that would have to grow a scratch buffer (a larger
 * batch, a larger SW_OPT_TB_SCRATCH_MB) fails with SW_E_STATE and changes
 * nothing; destroy the graphs first.  sw_autotune, sw_mlp_grad and
 * sw_mlp_train_step cannot be captured (SW_E_STATE). */
typedef struct sw_graph sw_graph;
sw_status sw_graph_begin(sw_ctx *ctx, void *stream);
sw_status sw_graph_end(sw_ctx *ctx, void *stream, sw_graph **out);
sw_status sw_graph_launch(sw_ctx *ctx, const sw_graph *g, void *stream);
sw_status sw_graph_destroy(sw_ctx *ctx, sw_graph *g);

/* ---------------------------------------------------------------------------
 * Learned candidate filter.
 *
 * The paper's stage D keeps a merged seed region as a candidate alignment
 * location only when enough seed matches support it (Sec. 2, "Stage D: CAL
 * Seeker"); stage E then runs Smith-Waterman on every candidate.  Here a
 * small network scores each candidate window from its seed-hit features and
 * Smith-Waterman runs only on the likely winners, with every candidate of a
 * read kept whenever the network is unsure.
 *
 * Features: 64 bfloat16 values per pair (uint16_t storage), from the exact
 * 12-mer matches of the read (first 256 query bases) in the window (first 1024
 * bases): hit counts, diagonal concentration, position histograms, the same
 * quantities relative to the read's other candidates, window length, GC and
 * strand.  The pairs of one read must be contiguous in d_win and a read may
 * have at most 64 candidates; other reads get no features and are always
 * kept whole by sw_filter_candidates.
 *
 * Network: 64 -> 128 (ReLU) -> 128 (ReLU) -> 1 logit; bfloat16 operands on
 * the matrix cores with float32 accumulation; float32 master parameters
 * (SW_MLP_PARAMS values: W1[64][128], b1[128], W2[128][128], b2[128], w3[128],
 * b3) trained with the mean binary cross-entropy on logits and Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8).
 * ------------------------------------------------------------------------- */
#define SW_FEATURES 64
#define SW_MLP_PARAMS 24961

typedef struct sw_mlp sw_mlp;

typedef struct {
    float logit_lo, logit_hi;   /* unsure band [lo, hi); keep logits >= hi */
    float logit_drop;           /* reads whose best logit is below this keep no
                                   candidate (-INFINITY: never); <= logit_lo */
} sw_filter_params;

sw_status sw_mlp_create(sw_ctx *ctx, sw_mlp **out);
sw_status sw_mlp_destroy(sw_ctx *ctx, sw_mlp *mlp);
/* Copy SW_MLP_PARAMS host floats into the network; resets the Adam state
 * (moments and step count; sw_mlp_load restores them). */
sw_status sw_mlp_set_params(sw_ctx *ctx, sw_mlp *mlp, const float *h_params);
/* Copy the float32 master parameters to host memory (synchronous). */
sw_status sw_mlp_get_params(sw_ctx *ctx, const sw_mlp *mlp, float *h_params);

/* Checkpoint of the network with its optimiser state, so that training can stop
 * and resume with bit-identical results: SW_MLP_STATE_BYTES bytes in a
 * caller-owned HOST buffer, little-endian: 8 bytes "HPGSWMLP", uint32 format
 * version (1), uint32 parameter count (SW_MLP_PARAMS), uint32 Adam step count,
 * uint32 zero, then float32 parameters, first moments and second moments
 * (SW_MLP_PARAMS each, parameter layout).  Both calls wait for the device and
 * copy synchronously; they cannot be captured (SW_E_STATE).
 * sw_mlp_save: SW_E_RANGE if cap < SW_MLP_STATE_BYTES.
 * sw_mlp_load: SW_E_INVALID if len differs from SW_MLP_STATE_BYTES or the
 * header is not this format (the network is then left unchanged); after a
 * load, sw_mlp_train_step continues from the saved step. */
#define SW_MLP_STATE_BYTES (24u + 12u * SW_MLP_PARAMS)
sw_status sw_mlp_save(sw_ctx *ctx, const sw_mlp *mlp, void *h_buf, uint64_t cap);
sw_status sw_mlp_load(sw_ctx *ctx, sw_mlp *mlp, const void *h_buf, uint64_t len);

/* Features of every pair: d_feat[n_pairs * SW_FEATURES] (bfloat16 bits). */
sw_status sw_features(sw_ctx *ctx, const sw_batch *batch, uint16_t *d_feat, void *stream);

/* Logits of n feature rows (d_x[n * 64]) into d_logits[n]. */
sw_status sw_mlp_forward(sw_ctx *ctx, const sw_mlp *mlp, const uint16_t *d_x, uint32_t n,
                         float *d_logits, void *stream);

/* Mean binary cross-entropy of n rows with labels d_y[n] (0 or 1) and its
 * gradient (SW_MLP_PARAMS floats, parameter layout) without updating. */
sw_status sw_mlp_grad(sw_ctx *ctx, const sw_mlp *mlp, const uint16_t *d_x, const float *d_y,
                      uint32_t n, float *d_grad, float *d_loss, void *stream);

/* One Adam step on the minibatch (d_x, d_y) with learning rate lr; d_loss
 * (device float, may be NULL) receives the minibatch loss before the step. */
sw_status sw_mlp_train_step(sw_ctx *ctx, sw_mlp *mlp, const uint16_t *d_x, const float *d_y,
                            uint32_t n, float lr, float *d_loss, void *stream);

/* Training labels from plain scores: d_y[p] = 1 if score(p) >= best score of
 * its read - margin and that best score is >= min_best (d_best_score from
 * sw_best_per_read), else 0 (also for a pair whose read id is out of range).  min_best = INT32_MIN gives the plain margin label;
 * min_best = the mapping threshold labels only candidates that can become the
 * record of a mapped read (stage E task iv), which is what a rule that may skip
 * predicted-unmapped reads needs. */
sw_status sw_mlp_labels(sw_ctx *ctx, const sw_batch *batch, const sw_hit *d_hits,
                        const int32_t *d_best_score, int32_t margin, int32_t min_best, float *d_y,
                        void *stream);

/* Filter step: features (into d_feat[n_pairs * 64]), logits (d_logits[n_pairs]),
 * per-read decision (d_keep[n_pairs]: a read whose best logit is below
 * logit_drop keeps no candidate, so sw_best_per_read reports it without a hit,
 * i.e. unmapped (stage E task iv records only alignments above the mapping
 * threshold); otherwise a read is unsure when its best logit is below
 * logit_hi or any logit lies in [logit_lo, logit_hi); unsure reads keep every
 * candidate, others keep the candidates with logit >= logit_hi; reads whose
 * pairs are not contiguous or number more than 64 keep every candidate) and
 * stable compaction of the kept pairs into d_win_out / d_sel_ids (original
 * pair index), with their number in *d_n_sel.  *d_n_unsure (device, may be
 * NULL) is incremented by the number of unsure reads.  The kept list is ready
 * for sw_batch_score through sw_batch.d_n_pairs. */
sw_status sw_filter_candidates(sw_ctx *ctx, const sw_batch *batch, const sw_mlp *mlp,
                               const sw_filter_params *fp, uint16_t *d_feat, float *d_logits,
                               uint8_t *d_keep, sw_window *d_win_out, uint32_t *d_sel_ids,
                               uint32_t *d_n_sel, uint32_t *d_n_unsure, void *stream);

/* Context options (sw_ctx_set_option).
 * SW_OPT_INT16: 1 (default) lets score-only calls use the packed int16
 *   datapath for the query-length classes where it is exact (match * longest
 *   query of the class <= 32767 and mismatch <= 0); 0 forces int32.  Results
 *   are identical either way.
 * SW_OPT_BLOCKS_PER_CU: workgroups (4 waves each) per compute unit of the
 *   persistent scoring kernels, 1..64 (default 2).
 * SW_OPT_TB_SCRATCH_MB: device scratch of sw_batch_traceback in MiB, 1..65536
 *   (default 2048).  Each query-length class runs as many pairs at once as
 *   their direction codes fit; a class whose single largest slot does not fit
 *   marks its pairs with status bit 2 (score -1) instead of aligning them. */
#define SW_OPT_INT16 1
#define SW_OPT_BLOCKS_PER_CU 2
#define SW_OPT_TB_SCRATCH_MB 3

/* Autotuning of the score path (the batching pattern's buckets and tiles).
 * Pairs are bucketed by query length into SW_NUM_CLASSES classes (default
 * upper bounds 16, 32, 64, 100, 128, 160, 256, 512, 1024, 2048 and 65535
 * bases); each class runs a persistent kernel whose tile is G lanes per pair x
 * RPL query rows per lane (G * RPL >= the class bound; the last class walks
 * the query in strips of 64 x 32 rows).  sw_autotune times the caller's sample
 * batch (`repeats` calls per candidate, HIP events around each class's kernel)
 * in two passes and keeps the result in ctx for later sw_batch_score calls:
 *   1. class bounds: for each bound between two classes (the last two bounds
 *      stay fixed), the candidates are the capacities of the default tiles
 *      and the sample's query-length quantiles (10, 25, 50, 75, 90 %) between
 *      its neighbours; a class whose bound exceeds its tile gets the smallest
 *      default tile that holds it; a bound moves when the two classes it
 *      separates get faster;
 *   2. tiles: for every populated class, the three smallest tiles that hold
 *      its bound, at 1, 2 or 4 workgroups per compute unit;
 *   3. the whole choice and the defaults are timed again side by side
 *      (2 x repeats calls each); unless the choice is at least 1 % faster over
 *      all classes, the defaults are kept.
 * Tune on a sample of the size the calls will have: how many pairs a class
 * holds decides how well a tile fills the GPU.  The tiles searched are the classes' default tiles.  Results are identical
 * for every candidate: only time changes.  Packed int16 runs on the 4 x 25
 * tile of the 65-100-base class with its default bounds.  out[SW_NUM_CLASSES]
 * (host, may be NULL) receives the choice (m_max: the tuned class bound).
 * Synchronises the stream; not capturable; allocates a temporary hit buffer;
 * the sample must have a host pair count.  The traceback keeps the default
 * classes. */
#define SW_NUM_CLASSES 11
typedef struct {
    int32_t m_max;          /* query-length bound of the class (tuned) */
    int32_t G, RPL;         /* chosen tile: lanes per pair, rows per lane */
    int32_t blocks_per_cu;  /* chosen workgroups (4 waves) per compute unit */
    int32_t path;           /* 0 class not run, 1 int32, 2 int32 with ends, 3 packed int16 */
    int32_t candidates;     /* candidates timed */
    float ms;               /* time of the class per call under the choice, from the
                               final side-by-side timing (0: empty) */
    float ms_default;       /* time of the class under the default bounds and tiles in
                               that timing (0: empty there); when a bound moved the
                               classes hold other pairs, so compare the sums */
} sw_tune_entry;
sw_status sw_autotune(sw_ctx *ctx, const sw_batch *sample, const sw_scoring *sc, uint32_t flags,
                      int repeats, sw_tune_entry *out, void *stream);

/* sw_autotune with a persisted cache: a JSON-lines file at cache_path (host
 * path) holding one object per tuning: {"key": ..., "edges": [...], "G": [...],
 * "RPL": [...], "blocks_per_cu": [...], "path": [...], "candidates": [...],
 * "ms": [...], "ms_default": [...]} (11 values each, by class).  The key names
 * the device (architecture and compute units), the scoring, the flags and the
 * sample's length profile (share of pairs per 8-base query-length bin and per
 * 64-base window-length bin, in thousandths, and the order of magnitude of the
 * pair count).  If the file holds a valid entry with this key (the last one
 * wins), its choice is applied without timing and *cache_hit (may be NULL) is
 * 1; otherwise the sample is tuned, the entry appended (the file is created if
 * needed) and *cache_hit is 0.  SW_E_INVALID if the file cannot be written. */
sw_status sw_autotune_cached(sw_ctx *ctx, const sw_batch *sample, const sw_scoring *sc,
                             uint32_t flags, int repeats, const char *cache_path, int *cache_hit,
                             sw_tune_entry *out, void *stream);
sw_status sw_ctx_set_option(sw_ctx *ctx, int option, int value);

/* Phase timing of sw_batch_score, from HIP events recorded on the call's
 * stream.  bucket_ms covers the length bucketing; class_ms[c] the wavefront
 * kernel of query-length class c (classes: m <= 16, 32, 64, 100, 128, 160,
 * 256, 512, 1024, 2048, longer); score_ms their sum. */
typedef struct {
    float bucket_ms;
    float score_ms;
    float class_ms[16];
    int32_t class_path[16];   /* 0 not launched, 1 int32, 2 int32 with ends, 3 packed int16 */
} sw_timing;

/* Turn event recording on (on != 0) or off for later sw_batch_score calls. */
sw_status sw_timing_enable(sw_ctx *ctx, int on);

/* Times of the last timed sw_batch_score call; waits for its events.
 * SW_E_STATE if timing is off or no call was timed. */
sw_status sw_timing_get(sw_ctx *ctx, sw_timing *out);

/* Format ops as CIGAR text into buf (host memory); returns the length
 * written, or -1 if cap is too small. */
int sw_cigar_string(const uint32_t *ops, uint32_t n_ops, char *buf, uint32_t cap);

#ifdef __cplusplus
}
#endif

#endif /* HPGSW_H */
