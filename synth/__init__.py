"""Seeded synthetic inputs shaped like the paper's RNA-seq workloads.

This module only *generates data*: a reference genome, reads sampled from it
with substitutions and short indels, and the candidate windows (extended CALs,
Sec. 2 "Stage E", tasks i-ii) each read is later aligned against.  It holds
none of the alignment arithmetic; both the GPU library and the CPU oracle take
its output as plain input arrays.

The paper's own benchmark reads were simulated with dwgsim (Sec. 4.1,
"Benchmarks": 100 and 250 nt reads, error rate 0.1 % or 1 %, 30 % of the errors
indels).  Those datasets are not available, so these generators stand in for
them with the same shapes: uniform or GC-biased references, per-base
substitution and indel events, reads on both strands, and several candidate
windows per read of which at most one contains the read's true origin.

Everything is ASCII (``A C G T``) so that the encode step of the hot path is
exercised on the device.  Every generator takes an explicit seed and uses
``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

ASCII = np.frombuffer(b"ACGT", dtype=np.uint8)
# complement of a code is 3 - code (A<->T, C<->G)
WINDOW_DTYPE = np.dtype([("read_id", "<u4"), ("ref_begin", "<u4"), ("len", "<u2"),
                         ("strand", "u1"), ("flags", "u1")])
assert WINDOW_DTYPE.itemsize == 12

# window flag bits (metadata only; the aligner ignores them)
FLAG_TRUE_ORIGIN = 1

BASE_SEED = 20130301


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Batch:
    """A batch of reads and candidate windows, host side, ASCII sequences."""
    ref: np.ndarray            # uint8 ASCII, reference genome
    reads: np.ndarray          # uint8 ASCII, all reads concatenated
    read_off: np.ndarray       # uint64, offset (in bases) of each read in `reads`
    read_len: np.ndarray       # uint16, length of each read
    windows: np.ndarray        # WINDOW_DTYPE, one row per (read, window) pair
    truth: dict = field(default_factory=dict)   # origins/strands, for reporting only

    @property
    def n_reads(self) -> int:
        return int(self.read_len.shape[0])

    @property
    def n_pairs(self) -> int:
        return int(self.windows.shape[0])

    def read(self, k: int) -> bytes:
        o = int(self.read_off[k])
        return self.reads[o:o + int(self.read_len[k])].tobytes()

    def cells(self) -> int:
        """Sum of m*n over all pairs (windows clipped to the reference)."""
        m = self.read_len[self.windows["read_id"]].astype(np.int64)
        b = self.windows["ref_begin"].astype(np.int64)
        n = np.minimum(self.windows["len"].astype(np.int64),
                       np.maximum(len(self.ref) - b, 0))
        return int((m * n).sum())


def make_reference(g: np.random.Generator, length: int, gc: float = 0.5) -> np.ndarray:
    """iid reference codes with P(C)=P(G)=gc/2, P(A)=P(T)=(1-gc)/2."""
    p = np.array([(1 - gc) / 2, gc / 2, gc / 2, (1 - gc) / 2])
    return g.choice(4, size=length, p=p).astype(np.uint8)


def plant_repeats(g: np.random.Generator, ref: np.ndarray, frac: float,
                  fam_len=(300, 3000), copies=(3, 12), div=(0.02, 0.10)) -> None:
    """Overwrite ~`frac` of `ref` with diverged copies of repeat families (in place)."""
    L = len(ref)
    target = int(frac * L)
    done = 0
    while done < target:
        flen = int(g.integers(fam_len[0], fam_len[1] + 1))
        src = int(g.integers(0, L - flen))
        fam = ref[src:src + flen].copy()
        for _ in range(int(g.integers(copies[0], copies[1] + 1))):
            dst = int(g.integers(0, L - flen))
            d = g.uniform(*div)
            cp = fam.copy()
            mut = g.random(flen) < d
            cp[mut] = (cp[mut] + g.integers(1, 4, size=int(mut.sum()))) % 4
            ref[dst:dst + flen] = cp
            done += flen


def _mutate(g, ref, origins, m, p_sub, p_indel):
    """Emit reads of length m from ref starting at origins.

    Per emitted base: with p_sub a substitution (uniform over the 3 other bases),
    with p_indel an indel event (insertion or deletion 50/50, length U{1,2,3}),
    otherwise a copy.  Returns (codes[n, m], span[n]) where span is the number of
    reference bases consumed.
    """
    n = len(origins)
    u = g.random((n, m))
    kind = g.random((n, m)) < 0.5           # True = insertion
    ilen = g.integers(1, 4, size=(n, m))
    subs = g.integers(1, 4, size=(n, m)).astype(np.uint8)
    rnd = g.integers(0, 4, size=(n, m), dtype=np.uint8)
    is_sub = u < p_sub
    is_indel = (u >= p_sub) & (u < p_sub + p_indel)
    has_indel = is_indel.any(axis=1)

    out = np.empty((n, m), dtype=np.uint8)
    span = np.full(n, m, dtype=np.int64)
    plain = np.nonzero(~has_indel)[0]
    if len(plain):
        idx = origins[plain, None] + np.arange(m)[None, :]
        seq = ref[idx]
        s = is_sub[plain]
        seq[s] = (seq[s] + subs[plain][s]) % 4
        out[plain] = seq
    for r in np.nonzero(has_indel)[0]:
        o = int(origins[r])
        buf = []
        k = 0          # emitted bases
        p = o          # next reference position
        ev = np.nonzero(is_sub[r] | is_indel[r])[0]
        ei = 0
        while k < m:
            nxt = int(ev[ei]) if ei < len(ev) else m
            if nxt < k:
                ei += 1
                continue
            if nxt > k:                       # copy a run
                run = nxt - k
                buf.append(ref[p:p + run])
                p += run
                k += run
                continue
            ei += 1
            if is_sub[r, k]:
                buf.append(np.array([(ref[p] + subs[r, k]) % 4], dtype=np.uint8))
                p += 1
                k += 1
            elif kind[r, k]:                   # insertion: bases not in the reference
                ln = min(int(ilen[r, k]), m - k)
                buf.append(rnd[r, k:k + ln])
                k += ln
            else:                              # deletion: skip reference bases
                p += int(ilen[r, k])
                buf.append(ref[p:p + 1])
                p += 1
                k += 1
        seq = np.concatenate(buf)[:m]
        out[r] = seq
        span[r] = p - o
    return out, span


def _revcomp_rows(codes: np.ndarray) -> np.ndarray:
    return (3 - codes[..., ::-1]).astype(np.uint8)


def _true_window(g, L, origin, span, wlen):
    lo = max(0, origin + span - wlen)
    hi = min(origin, L - wlen)
    if hi < lo:                                # read span longer than window
        lo = hi = max(0, min(origin, L - wlen))
    return int(g.integers(lo, hi + 1))


def sample_reads(g, ref, n_reads, m, p_sub, p_indel, random_frac=0.0):
    """Reads of fixed length m; returns codes[n, m] plus truth arrays."""
    L = len(ref)
    origins = g.integers(0, L - 2 * m - 16, size=n_reads)
    strand = (g.random(n_reads) < 0.5).astype(np.uint8)
    codes, span = _mutate(g, ref, origins, m, p_sub, p_indel)
    rev = strand == 1
    codes[rev] = _revcomp_rows(codes[rev])
    is_random = g.random(n_reads) < random_frac
    nr = int(is_random.sum())
    if nr:
        codes[is_random] = g.integers(0, 4, size=(nr, m), dtype=np.uint8)
    return codes, dict(origin=origins, span=span, strand=strand, is_random=is_random)


def assemble(ref_codes, read_codes_list, windows, truth) -> Batch:
    lens = np.array([len(c) for c in read_codes_list], dtype=np.uint16)
    off = np.zeros(len(lens), dtype=np.uint64)
    if len(lens) > 1:
        off[1:] = np.cumsum(lens[:-1], dtype=np.uint64)
    reads = ASCII[np.concatenate(read_codes_list)] if len(lens) else np.zeros(0, np.uint8)
    return Batch(ref=ASCII[ref_codes], reads=reads, read_off=off, read_len=lens,
                 windows=windows, truth=truth)


def _assemble_fixed(ref_codes, codes, windows, truth) -> Batch:
    n, m = codes.shape
    lens = np.full(n, m, dtype=np.uint16)
    off = (np.arange(n, dtype=np.uint64) * np.uint64(m))
    return Batch(ref=ASCII[ref_codes], reads=ASCII[codes.reshape(-1)], read_off=off,
                 read_len=lens, windows=windows, truth=truth)


def candidate_windows(g, L, truth, k_per_read, wlen_lo, wlen_hi, true_frac):
    """Windows for each read: k_per_read[r] of them, lengths U[wlen_lo, wlen_hi].

    For a fraction `true_frac` of the non-random reads exactly one window (at a
    uniform slot) contains the read's origin span on the read's strand; all
    other windows are decoys at uniform positions and strands.
    """
    n = len(k_per_read)
    P = int(k_per_read.sum())
    win = np.zeros(P, dtype=WINDOW_DTYPE)
    rid = np.repeat(np.arange(n, dtype=np.uint32), k_per_read)
    win["read_id"] = rid
    wl = g.integers(wlen_lo, wlen_hi + 1, size=P)
    win["len"] = wl
    win["ref_begin"] = g.integers(0, L - wl + 1)
    win["strand"] = (g.random(P) < 0.5)
    first = np.zeros(n, dtype=np.int64)
    if n > 1:
        first[1:] = np.cumsum(k_per_read[:-1])
    has_true = (g.random(n) < true_frac) & ~truth["is_random"]
    slot = (g.random(n) * k_per_read).astype(np.int64)
    for r in np.nonzero(has_true)[0]:
        p = int(first[r] + slot[r])
        w = int(wl[p])
        win["ref_begin"][p] = _true_window(g, L, int(truth["origin"][r]),
                                           int(truth["span"][r]), w)
        win["strand"][p] = truth["strand"][r]
        win["flags"][p] = FLAG_TRUE_ORIGIN
    return win


def config1(seed: int = BASE_SEED + 1, n_reads: int = 1000) -> Batch:
    """1,000 x 100-nt reads from a uniform 1 Mb reference (1 % subs, 0.1 % indels),
    each against one 300-nt window containing its origin."""
    g = rng(seed)
    ref = make_reference(g, 1_000_000)
    codes, truth = sample_reads(g, ref, n_reads, 100, 0.01, 0.001)
    k = np.ones(n_reads, dtype=np.int64)
    win = candidate_windows(g, len(ref), truth, k, 300, 300, 1.0)
    return _assemble_fixed(ref, codes, win, truth)


def config2(seed: int = BASE_SEED + 2, n_reads: int = 1_000_000, k_max: int = 8,
            k_fixed: int | None = None, ref_len: int = 4_000_000,
            repeat_frac: float = 0.0) -> Batch:
    """100-nt reads from a GC-40 % 4 Mb reference: 95 % mutated (1 % subs, 0.1 %
    indels), 5 % fully random; K ~ U{1..k_max} windows of U[200, 600] nt per read,
    for 80 % of the reads exactly one of them containing the origin."""
    g = rng(seed)
    ref = make_reference(g, ref_len, gc=0.40)
    if repeat_frac > 0:
        plant_repeats(g, ref, repeat_frac)
    codes, truth = sample_reads(g, ref, n_reads, 100, 0.01, 0.001, random_frac=0.05)
    if k_fixed is not None:
        k = np.full(n_reads, k_fixed, dtype=np.int64)
    else:
        k = g.integers(1, k_max + 1, size=n_reads)
    win = candidate_windows(g, len(ref), truth, k, 200, 600, 0.8)
    return _assemble_fixed(ref, codes, win, truth)


def config4(seed: int = BASE_SEED + 4, n_reads: int = 1_000_000, **kw) -> Batch:
    """Learned-filter workload: as config2 but exactly 16 candidates per read."""
    return config2(seed=seed, n_reads=n_reads, k_fixed=16, **kw)


def seeded_decoys(g, ref: np.ndarray, codes: np.ndarray, win: np.ndarray, truth: dict,
                  k: int = 15, chunk: int = 1 << 20) -> None:
    """Move decoy windows (in place) to where one of their read's k-mers occurs.

    For each decoy a k-mer of the query (the read, or its reverse complement for
    a strand-1 window) is drawn at a uniform position p; if it occurs in the
    reference away from the read's origin, the window is placed around the
    alignment that occurrence implies (query start = occurrence - p), as true
    windows are placed around the origin.  Decoys whose k-mer does not occur
    elsewhere stay where they were."""
    L = len(ref)
    m = codes.shape[1]
    n = L - k + 1
    v = np.zeros(n, dtype=np.int64)
    for t in range(k):
        v |= ref[t:t + n].astype(np.int64) << (2 * t)
    order = np.argsort(v, kind="stable")
    sv = v[order]
    dec_all = np.nonzero((win["flags"] & FLAG_TRUE_ORIGIN) == 0)[0]
    for a in range(0, len(dec_all), chunk):
        dec = dec_all[a:a + chunk]
        rid = win["read_id"][dec].astype(np.int64)
        strand = win["strand"][dec].astype(bool)
        p = g.integers(0, m - k + 1, size=len(dec))
        # query base t of the k-mer: read[p + t], or 3 - read[m - 1 - (p + t)] on strand 1
        t = np.arange(k)
        fwd = codes[rid[:, None], p[:, None] + t[None, :]]
        rev = 3 - codes[rid[:, None], (m - 1 - p)[:, None] - t[None, :]]
        kq = np.where(strand[:, None], rev, fwd).astype(np.int64)
        val = (kq << (2 * t[None, :])).sum(axis=1)
        lo = np.searchsorted(sv, val, "left")
        hi = np.searchsorted(sv, val, "right")
        pick = lo + (g.random(len(dec)) * np.maximum(hi - lo, 1)).astype(np.int64)
        pos = order[np.minimum(pick, n - 1)]
        o = pos - p
        w = win["len"][dec].astype(np.int64)
        ok = (hi > lo) & (np.abs(o - truth["origin"][rid]) >= m) & (o >= 0) & (o + m <= L)
        lo_s = np.maximum(0, o + m - w)
        hi_s = np.minimum(o, L - w)
        hi_s = np.maximum(hi_s, lo_s)
        start = lo_s + (g.random(len(dec)) * (hi_s - lo_s + 1)).astype(np.int64)
        win["ref_begin"][dec[ok]] = start[ok].astype(np.uint32)


def config4_hard(seed: int = BASE_SEED + 40, n_reads: int = 1_000_000,
                 repeat_frac: float = 0.2, ref_len: int = 4_000_000) -> Batch:
    """Hard variant of the learned-filter workload: the config-4 reads and
    windows on a reference of which `repeat_frac` is made of repeat families
    (copies at 2-10 % divergence), with decoy windows placed where one of the
    read's 15-mers occurs (uniform where none does)."""
    g = rng(seed)
    ref = make_reference(g, ref_len, gc=0.40)
    plant_repeats(g, ref, repeat_frac)
    codes, truth = sample_reads(g, ref, n_reads, 100, 0.01, 0.001, random_frac=0.05)
    k = np.full(n_reads, 16, dtype=np.int64)
    win = candidate_windows(g, len(ref), truth, k, 200, 600, 0.8)
    seeded_decoys(g, ref, codes, win, truth, 15)
    return _assemble_fixed(ref, codes, win, truth)


def spliced(seed: int = BASE_SEED + 3, n_reads: int = 200_000, ref_len: int = 16_000_000,
            seed_len: int = 100, p_sub: float = 0.01, p_indel: float = 0.001) -> Batch:
    """Spliced long reads split into seeds.

    Each read is 2-4 exons of U[50, 300] nt separated by introns of U[50, 5000] nt,
    rejection-sampled to a total of 400-800 nt; every intron starts with GT and
    ends with AG in the reference.  The read is cut into ceil(L/seed_len) seeds of
    seed_len nt (the last one right-aligned); each seed is an independent query
    (a "read" of this batch) with K ~ U{4..12} windows of U[200, 1000] nt, one of
    which covers the seed's largest exonic part.
    """
    g = rng(seed)
    ref = make_reference(g, ref_len)
    L = len(ref)
    seeds = []
    seed_parent = []
    seed_true = []      # (ref position of the seed's largest exonic part, its length)
    for r in range(n_reads):
        while True:
            ne = int(g.integers(2, 5))
            ex = g.integers(50, 301, size=ne)
            if 400 <= ex.sum() <= 800:
                break
        intr = g.integers(50, 5001, size=ne - 1)
        total_span = int(ex.sum() + intr.sum())
        o = int(g.integers(0, L - total_span - 8))
        pos = o
        exon_starts = []
        for e in range(ne):
            exon_starts.append(pos)
            pos += int(ex[e])
            if e < ne - 1:
                ref[pos:pos + 2] = (2, 3)                       # GT
                ref[pos + int(intr[e]) - 2:pos + int(intr[e])] = (0, 2)   # AG
                pos += int(intr[e])
        parts = [ref[s:s + int(l)] for s, l in zip(exon_starts, ex)]
        seq_pos = np.concatenate([np.arange(s, s + int(l)) for s, l in zip(exon_starts, ex)])
        seq = np.concatenate(parts).copy()
        mut = g.random(len(seq)) < p_sub
        seq[mut] = (seq[mut] + g.integers(1, 4, size=int(mut.sum()))) % 4
        Lr = len(seq)
        ns = -(-Lr // seed_len)
        for s in range(ns):
            b = min(s * seed_len, Lr - seed_len)
            seeds.append(seq[b:b + seed_len])
            seed_parent.append(r)
            p = seq_pos[b:b + seed_len]
            # largest run of consecutive reference positions inside this seed
            brk = np.nonzero(np.diff(p) != 1)[0]
            starts = np.concatenate([[0], brk + 1])
            ends = np.concatenate([brk + 1, [len(p)]])
            best = int(np.argmax(ends - starts))
            seed_true.append((int(p[starts[best]]), int(ends[best] - starts[best]),
                              int(p[0]), int(p[-1])))
    ns_total = len(seeds)
    strand = (g.random(ns_total) < 0.5).astype(np.uint8)
    codes = np.stack(seeds).astype(np.uint8)
    codes[strand == 1] = _revcomp_rows(codes[strand == 1])
    k = g.integers(4, 13, size=ns_total)
    P = int(k.sum())
    win = np.zeros(P, dtype=WINDOW_DTYPE)
    win["read_id"] = np.repeat(np.arange(ns_total, dtype=np.uint32), k)
    wl = g.integers(200, 1001, size=P)
    win["len"] = wl
    win["ref_begin"] = g.integers(0, L - wl + 1)
    win["strand"] = g.random(P) < 0.5
    first = np.concatenate([[0], np.cumsum(k[:-1])])
    slot = (g.random(ns_total) * k).astype(np.int64)
    for s in range(ns_total):
        p = int(first[s] + slot[s])
        w = int(wl[p])
        lo_pos, span_len, p0, p1 = seed_true[s]
        # cover the whole seed span when it fits (short introns), else its main part
        if p1 - p0 + 1 <= w:
            lo, ln = p0, p1 - p0 + 1
        else:
            lo, ln = lo_pos, span_len
        a = max(0, lo + ln - w)
        bmax = min(lo, L - w)
        win["ref_begin"][p] = int(g.integers(a, max(a, bmax) + 1))
        win["strand"][p] = strand[s]
        win["flags"][p] = FLAG_TRUE_ORIGIN
    truth = dict(parent=np.array(seed_parent), strand=strand, n_long_reads=n_reads)
    return _assemble_fixed(ref, codes, win, truth)


def paired_chunk(seed: int, n_frags: int, ref_codes: np.ndarray, read_len: int = 150,
                 k: int = 16, p_sub: float = 0.01, p_indel: float = 0.001) -> Batch:
    """Paired-end fragments (insert U[200, 500]); mate 1 = first read_len nt,
    mate 2 = reverse complement of the last read_len nt.  Each mate is one query
    with k windows of U[200, 1000] nt, 80 % of mates with one true window."""
    g = rng(seed)
    L = len(ref_codes)
    ins = g.integers(200, 501, size=n_frags)
    o = g.integers(0, L - 520, size=n_frags)
    fwd = g.random(n_frags) < 0.5
    m1, sp1 = _mutate(g, ref_codes, o, read_len, p_sub, p_indel)
    o2 = o + ins - read_len
    m2, sp2 = _mutate(g, ref_codes, o2, read_len, p_sub, p_indel)
    m2 = _revcomp_rows(m2)
    codes = np.empty((2 * n_frags, read_len), dtype=np.uint8)
    codes[0::2] = m1
    codes[1::2] = m2
    origin = np.empty(2 * n_frags, dtype=np.int64)
    origin[0::2] = o
    origin[1::2] = o2
    span = np.empty(2 * n_frags, dtype=np.int64)
    span[0::2] = sp1
    span[1::2] = sp2
    strand = np.empty(2 * n_frags, dtype=np.uint8)
    strand[0::2] = 0
    strand[1::2] = 1
    # fragments from the reverse strand: swap mate roles
    rv = np.repeat(~fwd, 2)
    codes_rv = codes.copy()
    codes_rv[0::2], codes_rv[1::2] = codes[1::2], codes[0::2]
    codes = np.where(rv[:, None], codes_rv, codes)
    strand_rv = strand.copy()
    strand_rv[0::2], strand_rv[1::2] = strand[1::2], strand[0::2]
    strand = np.where(rv, strand_rv, strand)
    origin_rv = origin.copy()
    origin_rv[0::2], origin_rv[1::2] = origin[1::2], origin[0::2]
    origin = np.where(rv, origin_rv, origin)
    span_rv = span.copy()
    span_rv[0::2], span_rv[1::2] = span[1::2], span[0::2]
    span = np.where(rv, span_rv, span)
    truth = dict(origin=origin, span=span, strand=strand,
                 is_random=np.zeros(2 * n_frags, dtype=bool))
    kk = np.full(2 * n_frags, k, dtype=np.int64)
    win = candidate_windows(g, L, truth, kk, 200, 1000, 0.8)
    return _assemble_fixed(ref_codes, codes, win, truth)


def subset(b: Batch, pair_idx: np.ndarray) -> Batch:
    """A batch holding only the given pairs (reads re-indexed, sequences shared)."""
    pair_idx = np.asarray(pair_idx)
    win = b.windows[pair_idx].copy()
    rids, inv = np.unique(win["read_id"], return_inverse=True)
    win["read_id"] = inv.astype(np.uint32)
    parts = [b.reads[int(b.read_off[r]):int(b.read_off[r]) + int(b.read_len[r])] for r in rids]
    lens = b.read_len[rids].copy()
    off = np.zeros(len(rids), dtype=np.uint64)
    if len(rids) > 1:
        off[1:] = np.cumsum(lens[:-1].astype(np.uint64))
    reads = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    return Batch(ref=b.ref, reads=reads, read_off=off, read_len=lens, windows=win,
                 truth={"orig_pairs": pair_idx, "orig_reads": rids})


def custom(ref: bytes, reads: list[bytes], windows: list[tuple]) -> Batch:
    """Small hand-made batch: windows are (read_id, ref_begin, len, strand)."""
    win = np.zeros(len(windows), dtype=WINDOW_DTYPE)
    for i, (rid, b, ln, st) in enumerate(windows):
        win[i] = (rid, b, ln, st, 0)
    lens = np.array([len(r) for r in reads], dtype=np.uint16)
    off = np.zeros(len(reads), dtype=np.uint64)
    if len(reads) > 1:
        off[1:] = np.cumsum(lens[:-1].astype(np.uint64))
    rd = np.frombuffer(b"".join(reads), dtype=np.uint8).copy()
    return Batch(ref=np.frombuffer(ref, dtype=np.uint8).copy(), reads=rd, read_off=off,
                 read_len=lens, windows=win, truth={})


def spliced_long(seed: int = BASE_SEED + 6, n_reads: int = 20_000, ref_len: int = 16_000_000,
                 seed_len: int = 100, p_sub: float = 0.01) -> tuple:
    """Spliced long reads with their seeds, for whole-read alignment over joined
    windows and junction detection.

    Each read is 2-4 exons of U[50, 300] nt with introns of U[50, 5000] nt,
    rejection-sampled to 400-800 nt, from a gene on either reference strand: a
    plus-strand gene's introns read GT...AG on the reference, a minus-strand
    gene's CT...AC (the reverse complement of GT...AG).  The read is the exons'
    reference sequence or, for half the reads, its reverse complement
    (read strand 1), with substitutions at p_sub.  Seeds as in `spliced`: the
    read cut into ceil(L/seed_len) seeds (last one right-aligned), each with
    K ~ U{4..12} windows of U[200, 1000] nt on the read's strand, one covering
    the seed's largest exonic part.

    Returns (reads, seeds, truth): `reads` holds the long reads (no windows),
    `seeds` the seed batch, and truth["seed_read"] the long read of every seed
    (seeds of a read are contiguous), truth["junctions"] the planted introns as
    rows (reference start, reference end exclusive, gene strand), and
    truth["read_strand"], truth["exons"] (per read, list of (start, length))."""
    g = rng(seed)
    ref = make_reference(g, ref_len)
    L = len(ref)
    plans = []
    for r in range(n_reads):
        while True:
            ne = int(g.integers(2, 5))
            ex = g.integers(50, 301, size=ne)
            if 400 <= ex.sum() <= 800:
                break
        intr = g.integers(50, 5001, size=ne - 1)
        span = int(ex.sum() + intr.sum())
        o = int(g.integers(8, L - span - 8))
        gene_minus = bool(g.random() < 0.5)
        starts = [o + int(ex[:e].sum() + intr[:e].sum()) for e in range(ne)]
        plans.append((starts, ex, intr, gene_minus))
    # motifs first, reads second: a later gene's motif may land in an earlier
    # gene's exon (the read then carries it) or overwrite an earlier motif (that
    # junction is then left out of the truth)
    motif = {False: ((2, 3), (0, 2)), True: ((1, 3), (0, 1))}      # GT..AG / CT..AC
    for starts, ex, intr, gm in plans:
        for e in range(len(ex) - 1):
            a = starts[e] + int(ex[e])
            ref[a:a + 2] = motif[gm][0]
            ref[a + int(intr[e]) - 2:a + int(intr[e])] = motif[gm][1]
    reads, read_strand, exons_all, junctions = [], [], [], []
    seeds, seed_read, seed_true = [], [], []
    for r, (starts, ex, intr, gm) in enumerate(plans):
        for e in range(len(ex) - 1):
            a, b = starts[e] + int(ex[e]), starts[e] + int(ex[e]) + int(intr[e])
            if (tuple(ref[a:a + 2]), tuple(ref[b - 2:b])) == motif[gm]:
                junctions.append((a, b, 1 if gm else 0))
        exons_all.append([(s, int(l)) for s, l in zip(starts, ex)])
        seq = np.concatenate([ref[s:s + int(l)] for s, l in zip(starts, ex)]).copy()
        seq_pos = np.concatenate([np.arange(s, s + int(l)) for s, l in zip(starts, ex)])
        mut = g.random(len(seq)) < p_sub
        seq[mut] = (seq[mut] + g.integers(1, 4, size=int(mut.sum()))) % 4
        st = int(g.random() < 0.5)
        read_strand.append(st)
        reads.append((3 - seq[::-1]).astype(np.uint8) if st else seq)
        Lr = len(seq)
        for s in range(-(-Lr // seed_len)):
            b = min(s * seed_len, Lr - seed_len)
            part = seq[b:b + seed_len]
            seeds.append((3 - part[::-1]).astype(np.uint8) if st else part.copy())
            seed_read.append(r)
            p = seq_pos[b:b + seed_len]
            brk = np.nonzero(np.diff(p) != 1)[0]
            bs = np.concatenate([[0], brk + 1])
            be = np.concatenate([brk + 1, [len(p)]])
            best = int(np.argmax(be - bs))
            seed_true.append((int(p[bs[best]]), int(be[best] - bs[best]), int(p[0]), int(p[-1]), st))
    ns = len(seeds)
    k = g.integers(4, 13, size=ns)
    P = int(k.sum())
    win = np.zeros(P, dtype=WINDOW_DTYPE)
    win["read_id"] = np.repeat(np.arange(ns, dtype=np.uint32), k)
    wl = g.integers(200, 1001, size=P)
    win["len"] = wl
    win["ref_begin"] = g.integers(0, L - wl + 1)
    st_seed = np.array([t[4] for t in seed_true], dtype=np.uint8)
    win["strand"] = np.repeat(st_seed, k)
    first = np.concatenate([[0], np.cumsum(k[:-1])])
    slot = (g.random(ns) * k).astype(np.int64)
    for s in range(ns):
        p = int(first[s] + slot[s])
        w = int(wl[p])
        lo_pos, span_len, p0, p1, _ = seed_true[s]
        if p1 - p0 + 1 <= w:
            lo, ln = p0, p1 - p0 + 1
        else:
            lo, ln = lo_pos, span_len
        a = max(0, lo + ln - w)
        bmax = min(lo, L - w)
        win["ref_begin"][p] = int(g.integers(a, max(a, bmax) + 1))
        win["flags"][p] = FLAG_TRUE_ORIGIN
    rs = np.array(read_strand, dtype=np.uint8)
    seed_b = _assemble_fixed(ref, np.stack(seeds).astype(np.uint8), win,
                             dict(seed_read=np.array(seed_read, dtype=np.uint32)))
    long_b = assemble(ref, reads, np.zeros(0, dtype=WINDOW_DTYPE), {})
    truth = dict(seed_read=np.array(seed_read, dtype=np.uint32), read_strand=rs,
                 junctions=np.array(junctions, dtype=np.int64).reshape(-1, 3), exons=exons_all)
    return long_b, seed_b, truth
