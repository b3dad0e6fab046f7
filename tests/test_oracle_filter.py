"""Pins of the filter decision reference (oracle/filter_ref.py) on hand-built
cases whose outcome follows from the rule by inspection."""
import numpy as np

from oracle import filter_ref as fr

INF = float("inf")


def test_sure_read_keeps_logits_at_or_above_hi():
    keep, un = fr.decide([3.0, -1.0, 2.0, 1.0], [0, 0, 0, 0], 1, lo=0.0, hi=1.0)
    assert keep.tolist() == [True, False, True, True] and un == 0     # z == hi is kept


def test_logit_in_band_makes_read_unsure():
    keep, un = fr.decide([3.0, -1.0, 0.5], [0, 0, 0], 1, lo=0.0, hi=1.0)
    assert keep.tolist() == [True, True, True] and un == 1
    # lo itself is inside the band, hi is not
    keep, un = fr.decide([3.0, 0.0], [0, 0], 1, lo=0.0, hi=1.0)
    assert keep.tolist() == [True, True] and un == 1
    keep, un = fr.decide([3.0, -0.01], [0, 0], 1, lo=0.0, hi=1.0)
    assert keep.tolist() == [True, False] and un == 0


def test_best_logit_below_hi_makes_read_unsure():
    keep, un = fr.decide([0.2, -4.0], [0, 0], 1, lo=0.5, hi=1.0)
    assert keep.tolist() == [True, True] and un == 1


def test_drop_keeps_nothing_and_is_not_unsure():
    keep, un = fr.decide([-3.0, -5.0, 4.0, -9.0], [0, 0, 1, 1], 2, lo=0.0, hi=1.0, drop=-2.0)
    assert keep.tolist() == [False, False, True, False] and un == 0
    # a best logit equal to drop is not dropped (and is unsure: below hi)
    keep, un = fr.decide([-2.0], [0], 1, lo=0.0, hi=1.0, drop=-2.0)
    assert keep.tolist() == [True] and un == 1


def test_reads_are_independent():
    z = [5.0, -5.0, 0.5, 5.0, 5.0, -5.0]
    rid = [0, 0, 1, 1, 2, 2]
    keep, un = fr.decide(z, rid, 3, lo=0.0, hi=1.0)
    assert keep.tolist() == [True, False, True, True, True, False] and un == 1


def test_non_contiguous_and_oversized_reads_keep_everything():
    # read 0 is split by read 1: all of read 0 kept and unsure; read 1 is sure
    keep, un = fr.decide([9.0, 9.0, -9.0], [0, 1, 0], 2, lo=0.0, hi=1.0, drop=0.5)
    assert keep.tolist() == [True, True, True] and un == 1
    # 65 candidates: every one kept (even below drop), 64 candidates: the rule
    z = np.full(65, -9.0, np.float32)
    z[0] = 9.0
    keep, un = fr.decide(z, np.zeros(65, int), 1, lo=0.0, hi=1.0, drop=-20.0)
    assert keep.all() and un == 1
    keep, un = fr.decide(z[:64], np.zeros(64, int), 1, lo=0.0, hi=1.0, drop=-20.0)
    assert keep.tolist() == [True] + [False] * 63 and un == 0


def test_invalid_read_ids_are_never_kept():
    keep, un = fr.decide([5.0, 5.0], [0, 7], 1, lo=0.0, hi=1.0)
    assert keep.tolist() == [True, False] and un == 0


def test_compaction_is_stable():
    w = np.array([(0, 10, 5, 0, 0), (0, 20, 5, 0, 0), (1, 30, 5, 1, 0), (2, 40, 5, 0, 0)],
                 dtype=[("read_id", "<u4"), ("ref_begin", "<u4"), ("len", "<u2"),
                        ("strand", "u1"), ("flags", "u1")])
    ids, wk = fr.compact([True, False, True, True], w)
    assert ids.tolist() == [0, 2, 3]
    assert wk["ref_begin"].tolist() == [10, 30, 40]


def test_a_planted_rule_mistake_is_caught():
    """The cases above fail a rule that forgets the band (a plausible mistake)."""
    def no_band(z, rid, n, lo, hi, drop=-INF):
        z = np.asarray(z, np.float32)
        keep = np.zeros(len(z), bool)
        for r in range(n):
            idx = np.nonzero(np.asarray(rid) == r)[0]
            if len(idx) and z[idx].max() >= drop:
                keep[idx] = z[idx] >= hi if z[idx].max() >= hi else True
        return keep
    assert no_band([3.0, -1.0, 0.5], [0, 0, 0], 1, 0.0, 1.0).tolist() != \
        fr.decide([3.0, -1.0, 0.5], [0, 0, 0], 1, 0.0, 1.0)[0].tolist()
