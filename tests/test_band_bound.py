"""The column bound behind the traceback band, checked on the oracle's alignments.

An alignment with score S that ends at read row i_e uses at most M <= i_e + 1
aligned rows, and S <= match * M - (cost of its deletions), where a run of L
deletions costs gap_open + (L - 1) * gap_extend.  Hence its window span is at
most (i_e + 1) + D_max, with D_max the most deletions the slack
match * (i_e + 1) - S can pay for.  The traceback kernel restricts its DP to that
span; these tests pin the bound on alignments the oracle computes, independently
of any GPU code."""
import numpy as np
import pytest


def d_max(slack, go, ge):
    """Most deletions a slack can pay for (go, ge: penalties as positive numbers)."""
    if slack <= 0:
        return 0
    if go >= ge:
        return 0 if slack < go else (slack - go) // ge + 1
    return slack // go


def _mutate(g, seq, n_events):
    s = list(seq)
    for _ in range(n_events):
        if len(s) < 3:
            break
        p = int(g.integers(1, len(s) - 1))
        kind = g.random()
        if kind < 0.4:
            s[p] = int(g.integers(0, 4))
        elif kind < 0.7:
            del s[p:p + int(g.integers(1, 12))]
        else:
            s[p:p] = list(g.integers(0, 4, int(g.integers(1, 12))))
    return np.array(s, dtype=np.uint8)


@pytest.mark.parametrize("sc", [(5, -4, -10, -1), (2, -3, -4, -4), (3, -1, -5, -2), (4, -2, -3, -6)])
def test_alignment_span_within_band(orc, sc):
    ma, _, go, ge = sc
    g = np.random.default_rng(2024 + ma)
    tight = 0
    for _ in range(400):
        m = int(g.integers(20, 160))
        ref = g.integers(0, 4, 900).astype(np.uint8)
        o = int(g.integers(0, 900 - m - 40))
        q = _mutate(g, ref[o:o + m], int(g.integers(0, 6)))
        if len(q) < 5:
            continue
        res, _ = orc.align_codes(q, ref, sc)
        s = int(res["score"])
        if s <= 0:
            continue
        rows = int(res["read_end"]) + 1
        span = int(res["ref_end"]) - int(res["ref_begin"]) + 1
        bound = rows + d_max(ma * rows - s, -go, -ge)
        assert span <= bound, (sc, m, s, rows, span, bound)
        tight += span == bound
    assert tight > 0      # the bound is reached, so it is not looser than it needs to be


def test_d_max_cases():
    assert d_max(0, 10, 1) == 0
    assert d_max(9, 10, 1) == 0          # cannot pay for an opening
    assert d_max(10, 10, 1) == 1
    assert d_max(15, 10, 1) == 6
    assert d_max(12, 3, 6) == 4          # opening cheaper than extending: runs of one
    assert d_max(7, 4, 4) == 1
