"""Reference of the region seeker and the CAL seeker (test infrastructure only:
imported by tests, never by the product path).

Stage C of the paper (Sec. 2, "Stage C: Region Seeker") cuts a read into short
overlapping seeds (15 nt, as a provisional choice), in two phases: one series of seeds
from the read's first base and a second series from its eighth, so that a
100-nt read gives 8 + 7 seeds.  Every seed is mapped exactly (no errors) onto
the reference; each place it matches is a region.  Stage D ("Stage D: CAL
Seeker") merges a read's regions that lie less than a given number of bases
apart and keeps a merged region as a candidate alignment location (CAL) when
it spans more than a given number of bases.

This module is the plain definition of those steps:

Seeds.  For a read of m bases, seeds of k bases start at 0, step, 2 step, ...
(phase one) and at offset, offset + step, ... (phase two), every start s with
s + k <= m; phase one first, starts ascending.  With k = 15, step = 12 and
offset = 7 a 100-nt read gets the paper's 8 + 7 seeds.

Index.  The exact occurrences of every k-mer of the reference (positions p,
0 <= p <= L - k, whose k bases spell it).

Regions.  Seed q at read position s matches forward at every occurrence p of
q (region: strand 0, reference bases [p, p + k - 1], read position s) and
reverse at every occurrence p of the reverse complement of q (strand 1: the
read's reverse complement aligns there; that complement holds the seed at
position m - s - k).  A seed with more than max_occ occurrences on a strand
gives no region on that strand (a repeat says nothing about where the read
lies).

CALs.  Of a read's regions (in the order above) the first MAX_REGIONS count.
Per read and strand, regions sorted by (first base, last base) are
merged while the next one starts fewer than merge_gap bases after the end of
the current merged region (bases strictly between them; overlap merges); a
merged region [first, last] is a CAL when last - first + 1 > min_len.  CALs
are listed by (strand, first), at most MAX_CALS per read (the first ones in
that order), as (read, first, last, strand, 1), in the CAL format of
junction_ref.
"""
from __future__ import annotations

import numpy as np

K = 15
STEP = 12
OFFSET = 7
MAX_OCC = 64
MAX_CALS = 16
MAX_REGIONS = 1024


def seed_starts(m: int, k: int = K, step: int = STEP, offset: int = OFFSET) -> list[int]:
    a = list(range(0, m - k + 1, step)) if m >= k else []
    b = list(range(offset, m - k + 1, step)) if m >= offset + k else []
    return a + b


def kmer_code(codes) -> int:
    """Base i of the k-mer at bits 2i (A0 C1 G2 T3)."""
    c = 0
    for i, x in enumerate(codes):
        c |= int(x) << (2 * i)
    return c


def revcomp(codes) -> np.ndarray:
    return (3 - np.asarray(codes, dtype=np.uint8)[::-1]).astype(np.uint8)


def build_index(ref_codes: np.ndarray, k: int = K) -> dict:
    """k-mer code -> sorted list of its positions (plain scan of the reference)."""
    idx: dict[int, list[int]] = {}
    ref = np.asarray(ref_codes, dtype=np.uint8)
    for p in range(len(ref) - k + 1):
        idx.setdefault(kmer_code(ref[p:p + k]), []).append(p)
    return idx


def position_codes(ref_codes: np.ndarray, k: int = K) -> np.ndarray:
    """Code of the k-mer at every position 0 .. L - k (numpy)."""
    ref = np.asarray(ref_codes, dtype=np.int64)
    n = max(len(ref) - k + 1, 0)
    codes = np.zeros(n, dtype=np.int64)
    for i in range(k):
        codes |= ref[i:i + n] << (2 * i)
    return codes


def build_index_fast(ref_codes: np.ndarray, k: int = K) -> dict:
    """The same index with numpy: every position's code as a weighted sum of
    its k bases, positions grouped by code with a stable sort."""
    codes = position_codes(ref_codes, k)
    n = len(codes)
    if n <= 0:
        return {}
    order = np.argsort(codes, kind="stable")
    sc = codes[order]
    cut = np.nonzero(np.diff(sc))[0] + 1
    starts = np.concatenate([[0], cut])
    ends = np.concatenate([cut, [n]])
    return {int(sc[a]): order[a:b].tolist() for a, b in zip(starts, ends)}


def regions(read_codes, index: dict, k: int = K, step: int = STEP, offset: int = OFFSET,
            max_occ: int = MAX_OCC) -> list[tuple]:
    """Regions of one read: (strand, first, last, read position) in seed order,
    strand 0 before strand 1 for each seed, positions ascending."""
    q = np.asarray(read_codes, dtype=np.uint8)
    m = len(q)
    out = []
    for s in seed_starts(m, k, step, offset):
        seed = q[s:s + k]
        fw = index.get(kmer_code(seed), [])
        if len(fw) <= max_occ:
            out += [(0, p, p + k - 1, s) for p in fw]
        rv = index.get(kmer_code(revcomp(seed)), [])
        if len(rv) <= max_occ:
            out += [(1, p, p + k - 1, m - s - k) for p in rv]
    return out


def cals(read: int, regs, merge_gap: int, min_len: int, max_cals: int = MAX_CALS,
         max_regions: int = MAX_REGIONS) -> list[tuple]:
    """CALs of one read from its regions."""
    regs = list(regs)[:max_regions]
    out = []
    for st in (0, 1):
        rs = sorted((f, l) for (s, f, l, _) in regs if s == st)
        cur = None
        for f, l in rs:
            if cur is not None and f - cur[1] - 1 < merge_gap:
                cur[1] = max(cur[1], l)
            else:
                if cur is not None and cur[1] - cur[0] + 1 > min_len:
                    out.append((read, cur[0], cur[1], st, 1))
                cur = [f, l]
        if cur is not None and cur[1] - cur[0] + 1 > min_len:
            out.append((read, cur[0], cur[1], st, 1))
    return out[:max_cals]
