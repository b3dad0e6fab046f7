"""Pins of the region / CAL seeker reference (oracle/seeker_ref.py): the paper's
seed count for a 100-nt read, two independent index builds that must agree and
spell their k-mers, regions of planted reads on both strands worked out by
hand, the repeat cut-off, the merge and length boundaries, and the property
that a read's own origin becomes a CAL."""
import numpy as np

from oracle import seeker_ref as sr


def test_seed_starts_two_phases():
    s = sr.seed_starts(100)
    assert len(s) == 15                      # 8 + 7 seeds for a 100-nt read
    assert s[:8] == [0, 12, 24, 36, 48, 60, 72, 84] and s[8:] == [7, 19, 31, 43, 55, 67, 79]
    assert sr.seed_starts(14) == [] and sr.seed_starts(15) == [0]
    assert sr.seed_starts(22) == [0, 7] and sr.seed_starts(27) == [0, 12, 7]


def test_index_builds_agree_and_spell_their_kmers():
    g = np.random.default_rng(3)
    for L, k in ((2000, 6), (5000, 8), (300, 15)):
        ref = g.integers(0, 4, L).astype(np.uint8)
        a, b = sr.build_index(ref, k), sr.build_index_fast(ref, k)
        assert a == b
        assert sum(len(v) for v in a.values()) == L - k + 1
        for code, pos in list(a.items())[:200]:
            for p in pos:
                assert sr.kmer_code(ref[p:p + k]) == code


def test_regions_of_planted_reads_both_strands():
    g = np.random.default_rng(4)
    ref = g.integers(0, 4, 50_000).astype(np.uint8)
    idx = sr.build_index_fast(ref)
    p, m = 12_345, 100
    fw = ref[p:p + m].copy()
    r = sr.regions(fw, idx)
    want = {(0, p + s, p + s + 14, s) for s in sr.seed_starts(m)}
    assert want <= set(r)
    rv = sr.revcomp(ref[p:p + m])
    r = sr.regions(rv, idx)
    # the seed at s of the reversed read is the reference at p + m - s - 15
    want = {(1, p + m - s - 15, p + m - s - 1, m - s - 15) for s in sr.seed_starts(m)}
    assert want <= set(r)
    # reference minus read position is the origin on both strands
    assert all(f - rp == p for st, f, l, rp in r if (st, f, l, rp) in want)


def test_repeat_cut_off():
    g = np.random.default_rng(5)
    ref = g.integers(0, 4, 20_000).astype(np.uint8)
    rep = g.integers(0, 4, 15).astype(np.uint8)
    read = np.concatenate([rep, g.integers(0, 4, 10).astype(np.uint8)])
    for copies, kept in ((5, True), (6, False)):
        r2 = ref.copy()
        for c in range(copies):
            r2[1000 + 700 * c:1015 + 700 * c] = rep
        idx = sr.build_index_fast(r2)
        n = len(idx.get(sr.kmer_code(rep), []))
        assert n >= copies
        regs = [x for x in sr.regions(read, idx, max_occ=5) if x[3] == 0 and x[0] == 0]
        assert (len(regs) == n) == kept and (len(regs) == 0) != kept


def test_merge_and_length_boundaries():
    regs = [(0, 100, 114, 0), (0, 130, 144, 12)]          # 15 bases strictly between
    assert sr.cals(7, regs, merge_gap=16, min_len=20) == [(7, 100, 144, 0, 1)]
    assert sr.cals(7, regs, merge_gap=15, min_len=20) == []          # two 15-nt regions
    assert sr.cals(7, regs, merge_gap=15, min_len=14) == [(7, 100, 114, 0, 1), (7, 130, 144, 0, 1)]
    assert sr.cals(7, [(0, 5, 19, 0)], 10, 15) == []                  # 15 bases, not > 15
    # strands never merge; order is (strand, first); the cap keeps the first ones
    regs = [(1, 50, 80, 0), (0, 60, 90, 0), (0, 10, 40, 3)]
    assert sr.cals(1, regs, 5, 20) == [(1, 10, 40, 0, 1), (1, 60, 90, 0, 1), (1, 50, 80, 1, 1)]
    assert sr.cals(1, regs, 5, 20, max_cals=2) == [(1, 10, 40, 0, 1), (1, 60, 90, 0, 1)]
    # overlapping and contained regions
    regs = [(0, 10, 24, 0), (0, 12, 20, 2), (0, 22, 36, 12)]
    assert sr.cals(2, regs, 0, 10) == [(2, 10, 36, 0, 1)]


def test_origin_becomes_a_cal():
    """Reads copied from the reference with 2 % substitutions: the merged
    regions of the read's own strand cover its origin."""
    g = np.random.default_rng(6)
    ref = g.integers(0, 4, 200_000).astype(np.uint8)
    idx = sr.build_index_fast(ref)
    hit = 0
    for t in range(200):
        p = int(g.integers(0, len(ref) - 100))
        q = ref[p:p + 100].copy()
        mut = g.random(100) < 0.02
        q[mut] = (q[mut] + 1) % 4
        st = t % 2
        if st:
            q = sr.revcomp(q)
        cs = sr.cals(t, sr.regions(q, idx), merge_gap=50, min_len=20)
        hit += any(c[3] == st and c[1] <= p + 90 and c[2] >= p + 10 for c in cs)
    assert hit >= 196
