"""Reference of the spliced-read steps (test infrastructure only: imported by
tests, never by the product path).

Stage E of the paper (Sec. 2, "Stage E: SWA + Splice Junctions") extends every
candidate alignment location (CAL) of a read on both sides (30 nt by default,
task i), joins extended CALs that are closer than the longest intron into one
"joined extended CAL" (task ii), aligns the read against each window (task
iii), and reads a splice junction off an alignment that holds a long run of
consecutive deletions whose borders carry the canonical intron motif: GT...AG,
or CT...AC for a gene on the other strand (task iv).  Junctions are counted
over all reads (the paper keeps the counts in an AVL tree).  This module is
the plain definition of those steps:

CALs.  A CAL is (read, first reference base, last reference base, strand,
valid), absolute inclusive coordinates.  Here a read's CALs are the reference
spans of its seeds' best local alignments scoring at least a threshold
(positions are 32-bit, like a window's start: a span reaching 2^32 is not a
CAL).

Joining (per read, at most MAX_CALS CALs: the first valid ones in input order
with first <= last < ref_len).
Each CAL [b, e] becomes [max(b - ext, 0), min(e + ext, ref_len - 1)].  The
extended CALs are sorted by (strand, first base, last base); walking that
order, a CAL joins the current window when it has the window's strand and the
bases strictly between them number fewer than max_gap (gap = b - end - 1,
overlap counts as joining); the window then ends at the larger last base.  Each
window is written as (read, first base, length, strand) with the length capped
at 65,535.  Windows are listed read by read, in that sorted order.

Junctions.  In an alignment (CIGAR over query q against window t, both 2-bit
codes), a deletion run of L >= min_intron bases whose neighbours are match
runs of a and b bases (M ops) may be placed at any shift s with
-(a - 1) <= s <= b - 1 that leaves the score unchanged: a shift left by one
moves the query base aligned to t[r - 1] onto t[r + L - 1], which keeps the
score when those two reference bases are equal (r = first deleted column); a
shift right by one likewise needs t[r] == t[r + L].  Among the placements
reachable this way (contiguous around s = 0), the leftmost whose deleted
bases start with GT and end with AG (plus-strand motif) or start with CT and
end with AC (minus-strand motif) makes the run a junction: the run becomes an
N op, its neighbours a + s and b - s bases long, and the junction is
(window start + r + s, window start + r + s + L, motif strand) with the end
exclusive.  Runs without such a placement stay deletions.
"""
from __future__ import annotations

from collections import Counter

import numpy as np

EXT = 30
MAX_CALS = 16
OP_M, OP_I, OP_D, OP_N, OP_S = 0, 1, 2, 3, 4
PLUS = ((2, 3), (0, 2))     # GT ... AG
MINUS = ((1, 3), (0, 1))    # CT ... AC


def seed_cals(windows, best_pair, aln, seed_read, min_score):
    """One CAL per seed: (read, first, last, strand, valid) from the seed's best
    window and its alignment (valid when the score reaches min_score)."""
    out = []
    for s in range(len(best_pair)):
        p = int(best_pair[s])
        a = aln[s]
        ok = p < len(windows) and int(a["score"]) >= min_score and int(a["score"]) > 0
        if ok:
            w = windows[p]
            b = int(w["ref_begin"]) + int(a["ref_begin"])
            e = int(w["ref_begin"]) + int(a["ref_end"])
            ok = e < 2 ** 32
        if ok:
            out.append((int(seed_read[s]), b, e, int(w["strand"]), 1))
        else:
            out.append((int(seed_read[s]), 0, 0, 0, 0))
    return out


def join_cals(cals, n_reads, ref_len, ext=EXT, max_gap=5000):
    """Joined windows, read by read: list of (read, first base, length, strand)."""
    by_read = [[] for _ in range(n_reads)]
    for c in cals:
        r = c[0]
        if r < n_reads and c[4] and c[1] <= c[2] < ref_len and len(by_read[r]) < MAX_CALS:
            by_read[r].append(c)
    out = []
    for r in range(n_reads):
        ext_cals = sorted((c[3], max(c[1] - ext, 0), min(c[2] + ext, ref_len - 1))
                          for c in by_read[r])
        cur = None
        for st, b, e in ext_cals:
            if cur is not None and st == cur[0] and b - cur[2] - 1 < max_gap:
                cur[2] = max(cur[2], e)
            else:
                if cur is not None:
                    out.append((r, cur[1], min(cur[2] - cur[1] + 1, 65535), cur[0]))
                cur = [st, b, e]
        if cur is not None:
            out.append((r, cur[1], min(cur[2] - cur[1] + 1, 65535), cur[0]))
    return out


def _motif(t, start, L):
    head = (int(t[start]), int(t[start + 1]))
    tail = (int(t[start + L - 2]), int(t[start + L - 1]))
    if (head, tail) == PLUS:
        return 0
    if (head, tail) == MINUS:
        return 1
    return -1


def detect(t, ops, ref_begin, min_intron, window_start):
    """Junctions of one alignment.  t: window codes; ops: CIGAR ops
    ((len << 4) | code); ref_begin: first window column of the alignment.
    Returns (new ops, [(start, end, motif strand)])."""
    ops = [int(o) for o in ops]
    lens = [o >> 4 for o in ops]
    codes = [o & 15 for o in ops]
    junctions = []
    r = ref_begin
    for k in range(len(ops)):
        c, L = codes[k], lens[k]
        if (c == OP_D and L >= min_intron and 0 < k < len(ops) - 1
                and codes[k - 1] == OP_M and codes[k + 1] == OP_M):
            a, b = lens[k - 1], lens[k + 1]
            lo = 0
            while lo < a - 1 and t[r - lo - 1] == t[r + L - lo - 1]:
                lo += 1
            hi = 0
            while hi < b - 1 and t[r + hi] == t[r + L + hi]:
                hi += 1
            for s in range(-lo, hi + 1):
                m = _motif(t, r + s, L)
                if m >= 0:
                    lens[k - 1], lens[k + 1] = a + s, b - s
                    codes[k] = OP_N
                    junctions.append((window_start + r + s, window_start + r + s + L, m))
                    r += s          # the run now starts s columns later
                    break
        if codes[k] in (OP_M, OP_D, OP_N):
            r += lens[k]
    return [(ln << 4) | cd for ln, cd in zip(lens, codes)], junctions


def count(junction_lists):
    """Counts of distinct junctions over many alignments (the AVL tree of the
    paper as a plain dictionary)."""
    c = Counter()
    for js in junction_lists:
        for j in js:
            c[j] += 1
    return c


def codes_of(ascii_bytes) -> np.ndarray:
    lut = np.full(256, 255, dtype=np.uint8)
    for k, ch in enumerate(b"ACGT"):
        lut[ch] = k
    return lut[np.frombuffer(bytes(ascii_bytes), dtype=np.uint8)]
