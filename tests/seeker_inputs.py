"""Seeded inputs of the region / CAL seeker tests (input construction only: no
step of the method is computed here).

reference_with_repeats: iid bases with a few families of exact repeats, so
  that some seeds match many places (the max_occ cut-off) and some a few.
reads_from: reads copied from the reference at uniform origins on either
  strand with substitutions and the odd indel, plus random reads, reads
  shorter than a seed, exactly one seed long, and long reads.
"""
from __future__ import annotations

import numpy as np


def reference_with_repeats(seed: int, length: int, families: int = 6,
                           copies=(3, 120), fam_len=(40, 400)) -> np.ndarray:
    g = np.random.default_rng(seed)
    ref = g.integers(0, 4, length).astype(np.uint8)
    for _ in range(families):
        n = int(g.integers(*fam_len))
        src = ref[int(g.integers(0, length - n)):][:n].copy()
        for _ in range(int(g.integers(*copies))):
            d = int(g.integers(0, length - n))
            ref[d:d + n] = src
    return ref


def reads_from(seed: int, ref: np.ndarray, n_reads: int, p_sub: float = 0.02):
    """Returns (list of code arrays, origins, strands); random reads have origin -1."""
    g = np.random.default_rng(seed)
    reads, origins, strands = [], [], []
    for r in range(n_reads):
        u = g.random()
        m = int(g.choice([100, 100, 100, 150, 60, 15, 10, 300, 37]))
        if u < 0.1:
            q = g.integers(0, 4, m).astype(np.uint8)
            o, st = -1, 0
        else:
            o = int(g.integers(0, len(ref) - m - 4))
            q = ref[o:o + m + 4].copy()
            if g.random() < 0.15:              # a short indel
                k = int(g.integers(10, max(11, m - 10)))
                q = np.delete(q, k) if g.random() < 0.5 else np.insert(q, k, int(g.integers(0, 4)))
            q = q[:m]
            mut = g.random(m) < p_sub
            q[mut] = (q[mut] + g.integers(1, 4, int(mut.sum()))) % 4
            st = int(g.random() < 0.5)
            if st:
                q = (3 - q[::-1]).astype(np.uint8)
        reads.append(q.astype(np.uint8))
        origins.append(o)
        strands.append(st)
    return reads, np.array(origins), np.array(strands)


def one_edit_reads(seed: int, ref: np.ndarray, n_reads: int, m: int = 100):
    """Reads at most one edit away from the reference: exact copies, one
    substitution, one deleted or one inserted base at an interior position,
    on either strand, some at the very start or end of the reference."""
    g = np.random.default_rng(seed)
    L = len(ref)
    reads = []
    for r in range(n_reads):
        kind = r % 4
        u = g.random()
        o = 0 if u < 0.05 else (L - m - 1 if u < 0.1 else int(g.integers(0, L - m - 2)))
        if kind == 0:
            q = ref[o:o + m].copy()
        elif kind == 1:
            q = ref[o:o + m].copy()
            j = int(g.integers(0, m))
            q[j] = (q[j] + int(g.integers(1, 4))) % 4
        elif kind == 2:
            q = np.delete(ref[o:o + m + 1], int(g.integers(1, m)))
        else:
            q = np.insert(ref[o:o + m - 1], int(g.integers(1, m - 1)), int(g.integers(0, 4)))
        if g.random() < 0.5:
            q = (3 - q[::-1]).astype(np.uint8)
        reads.append(q.astype(np.uint8))
    return reads
