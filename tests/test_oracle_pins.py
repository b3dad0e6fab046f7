"""Pins of the CPU oracle against things other than itself: hand-worked
examples, brute-force enumeration, closed forms, textbook reductions and
invariants.  A dropped term, a wrong sign or index, a transposed operand or a
wrong tie rule in the oracle fails at least one of these."""
import itertools
import os

import numpy as np
import pytest

from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.txt")
DEF = (5, -4, -10, -1)
SCHEMES = [DEF, (2, -3, -4, -4), (3, -1, -5, -2), (1, 0, -2, -1), (4, -6, -7, -3),
           (5, -4, -20, 0), (2, -3, -4, 0)]    # the last two: length-free gaps


def _cig(orc, ops):
    return orc.cigar_string(ops) or "*"


def _check_vs_brute(orc, q, r, sc, check_ops=True):
    res, ops = orc.align_codes(np.array(q, np.uint8), np.array(r, np.uint8), sc)
    b = brute.brute_align(list(q), list(r), sc)
    got = (int(res["score"]), int(res["read_begin"]), int(res["read_end"]),
           int(res["ref_begin"]), int(res["ref_end"]))
    exp = (b["score"], b["read_begin"], b["read_end"], b["ref_begin"], b["ref_end"])
    assert got == exp, (q, r, sc, got, exp)
    if check_ops:
        bc = brute.cigar_of(b["ops"], b["read_begin"], b["read_end"], len(q)) or "*"
        assert _cig(orc, ops) == bc, (q, r, sc, _cig(orc, ops), bc)
    lin = orc.score_codes(np.array(q, np.uint8), np.array(r, np.uint8), sc)
    assert (int(lin["score"]), int(lin["read_end"]), int(lin["ref_end"])) == (got[0], got[2], got[4])


def test_hand_examples(orc):
    n = 0
    for line in open(GOLDEN):
        if not line.strip() or line.startswith("#"):
            continue
        f = line.split("#")[0].split()
        q, r = orc.codes(f[0]), orc.codes(f[1])
        res, ops = orc.align_codes(q, r, DEF)
        got = [int(res[k]) for k in ("score", "read_begin", "read_end", "ref_begin", "ref_end")]
        assert got == [int(x) for x in f[2:7]], (f, got)
        assert _cig(orc, ops) == f[7]
        n += 1
    assert n == 9


@pytest.mark.parametrize("sc", SCHEMES)
def test_exhaustive_binary_alphabet(orc, sc):
    """Every pair over {A, C} with 1 <= m, n and m + n <= 9 (many ties)."""
    for total in range(2, 10):
        for m in range(1, total):
            n = total - m
            for q in itertools.product((0, 1), repeat=m):
                for r in itertools.product((0, 1), repeat=n):
                    _check_vs_brute(orc, q, r, sc)


def test_exhaustive_four_letters(orc):
    for total in range(2, 8):
        for m in range(1, total):
            n = total - m
            for q in itertools.product(range(4), repeat=m):
                for r in itertools.product(range(4), repeat=n):
                    _check_vs_brute(orc, q, r, DEF)


def test_random_small_vs_brute(orc):
    g = np.random.default_rng(7)
    for k in range(1500):
        m, n = int(g.integers(1, 8)), int(g.integers(1, 9))
        alpha = 2 if k % 2 else 4
        q = g.integers(0, alpha, m).tolist()
        r = g.integers(0, alpha, n).tolist()
        if k % 5 == 0 and m >= 3:            # plant a shared segment with an indel
            r = q[:2] + [int(g.integers(0, 4))] + q[2:]
            r = r[:8]
        _check_vs_brute(orc, q, r, SCHEMES[k % len(SCHEMES)])


def test_empty_inputs(orc):
    for q, r in [([], [0, 1]), ([2], []), ([], [])]:
        res, ops = orc.align_codes(np.array(q, np.uint8), np.array(r, np.uint8), DEF)
        assert int(res["score"]) == 0 and int(res["read_end"]) == -1 and len(ops) == 0


# ---- closed forms -----------------------------------------------------------

def test_identity_and_substring(orc):
    g = np.random.default_rng(1)
    for L in (1, 2, 17, 100, 257):
        q = g.integers(0, 4, L).astype(np.uint8)
        res, ops = orc.align_codes(q, q, DEF)
        assert int(res["score"]) == 5 * L
        assert orc.cigar_string(ops) == f"{L}M"
        assert (int(res["read_end"]), int(res["ref_end"])) == (L - 1, L - 1)
    for _ in range(20):
        m = int(g.integers(20, 60))
        q = g.integers(0, 4, m).astype(np.uint8)
        o = int(g.integers(0, 200))
        r = np.concatenate([g.integers(0, 4, o), q, g.integers(0, 4, 50)]).astype(np.uint8)
        res, ops = orc.align_codes(q, r, DEF)
        assert int(res["score"]) == 5 * m
        # the first occurrence of q in r ends at the smallest window column
        first = min(k for k in range(len(r) - m + 1) if (r[k:k + m] == q).all())
        assert int(res["ref_begin"]) == first and int(res["ref_end"]) == first + m - 1
        assert orc.cigar_string(ops) == f"{m}M"


@pytest.mark.parametrize("m,n", [(1, 1), (3, 7), (7, 3), (40, 40), (64, 65), (100, 300), (300, 100)])
def test_homopolymer(orc, m, n):
    q = np.zeros(m, np.uint8)
    r = np.zeros(n, np.uint8)
    res, ops = orc.align_codes(q, r, DEF)
    k = min(m, n)
    assert int(res["score"]) == 5 * k
    assert (int(res["read_end"]), int(res["ref_end"])) == (k - 1, k - 1)
    assert (int(res["read_begin"]), int(res["ref_begin"])) == (0, 0)


def test_disjoint_alphabets(orc):
    g = np.random.default_rng(3)
    for _ in range(20):
        q = g.integers(0, 2, int(g.integers(1, 80))).astype(np.uint8)
        r = g.integers(2, 4, int(g.integers(1, 80))).astype(np.uint8)
        assert int(orc.score_codes(q, r, DEF)["score"]) == 0


# ---- textbook reductions ------------------------------------------------------

def _kadane_diagonals(q, r, ma, mi):
    """No gaps: best max-subarray sum of s(q_i, r_{i+d}) over all diagonals d."""
    best = 0
    m, n = len(q), len(r)
    for d in range(-(m - 1), n):
        cur = 0
        for i in range(m):
            j = i + d
            if 0 <= j < n:
                cur = max(0, cur) + (ma if q[i] == r[j] else mi)
                best = max(best, cur)
    return best


def _linear_gap_sw(q, r, ma, mi, g):
    """Textbook single-matrix Smith-Waterman with a linear gap cost g per base."""
    m, n = len(q), len(r)
    H = [[0] * (n + 1) for _ in range(m + 1)]
    best = 0
    for i in range(1, m + 1):
        for j in range(1, n + 1):
            s = ma if q[i - 1] == r[j - 1] else mi
            H[i][j] = max(0, H[i - 1][j - 1] + s, H[i - 1][j] + g, H[i][j - 1] + g)
            best = max(best, H[i][j])
    return best


def test_gapless_reduction_is_kadane(orc):
    g = np.random.default_rng(11)
    for _ in range(60):
        q = g.integers(0, 4, int(g.integers(1, 40))).astype(np.uint8)
        r = g.integers(0, 4, int(g.integers(1, 40))).astype(np.uint8)
        big = -(5 * min(len(q), len(r)) + 1)     # no gap can ever pay for itself
        sc = (5, -4, big, big)
        assert int(orc.score_codes(q, r, sc)["score"]) == _kadane_diagonals(q, r, 5, -4)


def test_linear_gap_reduction(orc):
    g = np.random.default_rng(12)
    for k in range(60):
        q = g.integers(0, 4, int(g.integers(1, 35))).astype(np.uint8)
        r = g.integers(0, 4, int(g.integers(1, 35))).astype(np.uint8)
        gap = int(g.integers(-6, 0))
        sc = (3, -2, gap, gap)
        assert int(orc.score_codes(q, r, sc)["score"]) == _linear_gap_sw(q, r, 3, -2, gap)


# ---- invariants ---------------------------------------------------------------

def _mutated(g, m, n):
    q = g.integers(0, 4, m).astype(np.uint8)
    r = g.integers(0, 4, n).astype(np.uint8)
    if m <= n and g.random() < 0.7:                  # plant a noisy copy
        o = int(g.integers(0, n - m + 1))
        seg = q.copy()
        flip = g.random(m) < 0.1
        seg[flip] = (seg[flip] + 1) % 4
        r[o:o + m] = seg
        if m > 10:
            r = np.delete(r, o + m // 2)
    return q, r


def test_invariants(orc):
    g = np.random.default_rng(5)
    comp = lambda x: (3 - x).astype(np.uint8)
    for _ in range(150):
        m, n = int(g.integers(1, 70)), int(g.integers(1, 140))
        q, r = _mutated(g, m, n)
        sc = SCHEMES[int(g.integers(0, len(SCHEMES)))]
        res, ops = orc.align_codes(q, r, sc)
        S = int(res["score"])
        assert 0 <= S <= sc[0] * min(len(q), len(r))
        assert (S > 0) == bool(set(q.tolist()) & set(r.tolist()))
        assert int(orc.score_codes(r, q, sc)["score"]) == S
        assert int(orc.score_codes(q[::-1].copy(), r[::-1].copy(), sc)["score"]) == S
        assert int(orc.score_codes(comp(q), comp(r), sc)["score"]) == S
        ext = np.concatenate([r, g.integers(0, 4, 5).astype(np.uint8)])
        assert int(orc.score_codes(q, ext, sc)["score"]) >= S
        if S == 0:
            assert len(ops) == 0
            continue
        names = [int(o) & 15 for o in ops]
        lens = [int(o) >> 4 for o in ops]
        core = [(o, L) for o, L in zip(names, lens) if o != 4]
        assert core[0][0] == 0 and core[-1][0] == 0            # starts and ends with M
        for (a, _), (b, _) in zip(core, core[1:]):
            assert a != b                                        # runs are maximal
        n_m = sum(L for o, L in core if o == 0)
        n_i = sum(L for o, L in core if o == 1)
        n_d = sum(L for o, L in core if o == 2)
        n_s = sum(L for o, L in zip(names, lens) if o == 4)
        assert n_m + n_i + n_s == len(q)
        assert n_m + n_d == int(res["ref_end"]) - int(res["ref_begin"]) + 1
        assert n_m + n_i == int(res["read_end"]) - int(res["read_begin"]) + 1
        flat = [o for o, L in core for _ in range(L)]
        assert brute.rescore(flat, q, r, int(res["read_begin"]), int(res["ref_begin"]), sc) == S
        lin = orc.score_codes(q, r, sc)
        assert (int(lin["score"]), int(lin["read_end"]), int(lin["ref_end"])) == \
            (S, int(res["read_end"]), int(res["ref_end"]))
