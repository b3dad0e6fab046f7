"""Seeded inputs of the spliced-read steps, shared by the host-model tests, the
GPU parity tests and the oracle side of both (input construction only: no step
of the method is computed here).

random_cals: CAL lists grouped by read, with clustered and scattered CALs,
  both strands, invalid entries, geometry the joining must ignore (first >
  last, last past the reference), reads with more than 16 CALs, reads at or
  beyond n_reads, and pairs of CALs whose extended gap is exactly max_gap - 1,
  max_gap or max_gap + 1.
planted_alignments: alignments (window, alignment record, CIGAR ops) over a
  reference with deletion runs whose ends carry an intron motif at a planted
  shift, with the bases between the run's start and that shift made equal
  (reachable) or not, plus short runs, insertion neighbours, soft clips, runs
  without a motif, a two-letter stretch where many shifts are neutral, and
  records the search must leave alone (status bits, low scores).
"""
from __future__ import annotations

import numpy as np

CAL_DTYPE = np.dtype([("read_id", "<u4"), ("first", "<u4"), ("last", "<u4"), ("strand", "u1"),
                      ("valid", "u1"), ("reserved", "<u2")])
ALN_DTYPE = np.dtype([("score", "<i4"), ("read_begin", "<i4"), ("read_end", "<i4"),
                      ("ref_begin", "<i4"), ("ref_end", "<i4"), ("n_ops", "<u4"),
                      ("status", "<u4")])
WINDOW_DTYPE = np.dtype([("read_id", "<u4"), ("ref_begin", "<u4"), ("len", "<u2"),
                         ("strand", "u1"), ("flags", "u1")])
M, I, D, N, S = 0, 1, 2, 3, 4
MOTIFS = (((2, 3), (0, 2)), ((1, 3), (0, 1)))     # GT..AG, CT..AC


def random_cals(seed: int, n_reads: int, ref_len: int, ext: int, max_gap: int) -> np.ndarray:
    g = np.random.default_rng(seed)
    rows = []

    def add(r, first, last, strand, valid=1):
        rows.append((r, first, last, strand, valid, 0))

    for r in range(n_reads):
        kind = g.random()
        if kind < 0.08:                      # exact gap boundaries
            b = int(g.integers(ext, ref_len - 4 * max_gap - 500))
            d = int(g.integers(-1, 2))
            st = int(g.integers(0, 2))
            add(r, b, b + 99, st)
            f2 = b + 99 + 2 * ext + 1 + (max_gap + d)
            add(r, f2, f2 + 50, st)
            continue
        k = int(g.integers(0, 22))
        center = int(g.integers(0, ref_len))
        spread = 3 * max(max_gap, 200)
        for _ in range(k):
            u = g.random()
            if u < 0.7:
                first = center + int(g.integers(-spread, spread))
            elif u < 0.8:                    # near either end of the reference
                first = int(g.integers(0, 40)) if g.random() < 0.5 else ref_len - int(g.integers(1, 80))
            else:
                first = int(g.integers(0, ref_len))
            first = min(max(first, 0), ref_len - 1)
            last = first + int(g.integers(0, 300))
            if g.random() < 0.04:
                first, last = last + 3, first    # first > last
            if g.random() < 0.03:
                last = ref_len + int(g.integers(0, 50))
            last = min(last, 2**32 - 1)
            add(r, first, last, int(g.random() < 0.4), int(g.random() > 0.1))
    for _ in range(5):                       # reads beyond the batch
        add(n_reads + int(g.integers(0, 3)), 100, 200, 0)
    out = np.array(rows, dtype=CAL_DTYPE)
    return out[np.argsort(out["read_id"], kind="stable")]


def planted_alignments(seed: int, n_aln: int, min_intron: int, ops_stride: int = 48,
                       min_score: int = 30):
    """Returns (ref codes, windows, aln records, ops[n_aln, ops_stride]); every
    alignment owns a disjoint reference region."""
    g = np.random.default_rng(seed)
    regions, wins, alns, opss = [], [], [], []
    pos = 0
    for k in range(n_aln):
        ops = []
        if g.random() < 0.3:
            ops.append((int(g.integers(1, 6)), S))
        n_runs = int(g.integers(1, 4))
        ops.append((int(g.integers(1, 40)), M))
        plan = []                            # op indices of the deletion runs
        for _ in range(n_runs):
            u = g.random()
            if u < 0.6:
                L = int(g.integers(min_intron, min_intron + 400))
            elif u < 0.75:
                L = int(g.integers(1, min_intron))
            else:
                L = int(g.integers(min_intron, min_intron + 60))
            if g.random() < 0.1:
                ops.append((int(g.integers(1, 4)), I))
            ops.append((L, D))
            plan.append(len(ops) - 1)
            if g.random() < 0.1:
                ops.append((int(g.integers(1, 4)), I))
            ops.append((int(g.integers(1, 40)), M))
        if g.random() < 0.3:
            ops.append((int(g.integers(1, 6)), S))
        span = sum(n for n, c in ops if c in (M, D))
        lead = int(g.integers(0, 30))
        tail = int(g.integers(0, 30))
        wlen = lead + span + tail
        two_letter = g.random() < 0.2
        t = (g.integers(0, 2, wlen) * 2 if two_letter else g.integers(0, 4, wlen)).astype(np.uint8)
        # plant motifs
        col = lead
        for j, (n, c) in enumerate(ops):
            if j in plan and c == D and j > 0 and j + 1 < len(ops) and \
                    ops[j - 1][1] == M and ops[j + 1][1] == M and g.random() < 0.85:
                a, b = ops[j - 1][0], ops[j + 1][0]
                s0 = int(g.integers(-(a - 1), b))
                mh, mt = MOTIFS[int(g.integers(0, 2))]
                x = col + s0
                if n >= 4:
                    t[x:x + 2] = mh
                    t[x + n - 2:x + n] = mt
                if g.random() < 0.7:
                    # make every step from the run's place to s0 neutral, copying
                    # away from the motif so that it stays
                    if s0 > 0:
                        for i in range(s0):
                            t[col + i] = t[col + n + i]
                    else:
                        for i in range(-s0):
                            t[col + n - i - 1] = t[col - i - 1]
            if c in (M, D):
                col += n
        gap = int(g.integers(0, 50))
        regions.append(g.integers(0, 4, gap).astype(np.uint8))
        pos += gap
        wins.append((k, pos, wlen, int(g.integers(0, 2)), 0))
        regions.append(t)
        pos += wlen
        u = g.random()
        status = 0
        score = int(g.integers(min_score, 400))
        if u < 0.05:
            status = int(g.choice([1, 2, 4]))
        elif u < 0.1:
            score = int(g.integers(1, min_score))
        q_len = sum(n for n, c in ops if c in (M, I, S))
        alns.append((score, 0, q_len - 1, lead, lead + span - 1, len(ops), status))
        row = np.zeros(ops_stride, np.uint32)
        row[:len(ops)] = [(n << 4) | c for n, c in ops]
        opss.append(row)
    ref = np.concatenate(regions) if regions else np.zeros(0, np.uint8)
    win = np.array(wins, dtype=WINDOW_DTYPE)
    return ref, win, np.array(alns, dtype=ALN_DTYPE), np.stack(opss)
