"""Host logic of the filter: the decision rule and threshold calibration."""
import numpy as np

from paper_1304_0681_amd import train as tr


def test_decision_rule_and_recall():
    rid = np.array([0, 0, 0, 1, 1, 2, 2, 2])
    z = np.array([5.0, -3.0, -4.0, 0.5, -2.0, 4.0, 1.0, -5.0])
    scores = np.array([90, 10, 20, 30, 40, 70, 70, 5])
    best = np.array([90, 40, 70])
    keep, hit, unsure = tr.filter_outcome(z, scores, best, rid, lo=0.0, hi=2.0)
    # read 0: sure (max 5 >= 2, nothing in [0, 2)) -> keeps only pair 0, the best
    # read 1: max 0.5 < 2 -> unsure -> keeps both
    # read 2: z = 1.0 in [0, 2) -> unsure -> keeps all three
    assert keep.tolist() == [True, False, False, True, True, True, True, True]
    assert unsure.tolist() == [False, True, True]
    assert hit.all()
    keep, hit, _ = tr.filter_outcome(z, scores, best, rid, lo=1.5, hi=1.5)
    assert keep.tolist() == [True, False, False, True, True, True, False, False]
    assert hit.tolist() == [True, True, True]      # pair 5 (score 70) is a best pair


def test_calibration_meets_target():
    g = np.random.default_rng(0)
    n_reads, K = 3000, 16
    rid = np.repeat(np.arange(n_reads), K)
    scores = g.integers(20, 60, n_reads * K)
    true = g.integers(0, K, n_reads)
    has = g.random(n_reads) < 0.8
    idx = np.arange(n_reads) * K + true
    scores[idx[has]] = 480
    best = np.maximum.reduceat(scores, np.arange(n_reads) * K)
    z = g.normal(-4, 1, n_reads * K)
    z[idx[has]] = g.normal(4, 1, has.sum())
    lo, hi, rec = tr.calibrate(z, scores, best, rid, target=0.999)
    keep, hit, _ = tr.filter_outcome(z, scores, best, rid, lo, hi)
    assert hit.mean() >= 0.999 and rec == hit.mean()
    assert keep.mean() < 0.5


def test_drop_rule():
    rid = np.array([0, 0, 1, 1, 2, 2])
    z = np.array([5.0, -3.0, -6.0, -7.0, 0.5, -1.0])
    scores = np.array([90, 10, 30, 20, 60, 70])
    best = np.array([90, 30, 70])
    keep, hit, unsure = tr.filter_outcome(z, scores, best, rid, lo=1.0, hi=2.0, drop=-5.0)
    # read 1: best logit -6 < drop -> keeps nothing, is not unsure, has no hit
    # read 2: best logit 0.5 >= drop but < hi -> unsure -> keeps both
    assert keep.tolist() == [True, False, False, False, True, True]
    assert unsure.tolist() == [False, False, True]
    assert hit.tolist() == [True, False, True]


def test_output_calibration_meets_target():
    g = np.random.default_rng(1)
    n_reads, K = 4000, 16
    rid = np.repeat(np.arange(n_reads), K)
    scores = g.integers(20, 60, n_reads * K)
    true = g.integers(0, K, n_reads)
    has = g.random(n_reads) < 0.75
    idx = np.arange(n_reads) * K + true
    scores[idx[has]] = 480
    best = np.maximum.reduceat(scores, np.arange(n_reads) * K)
    z = g.normal(-4, 1, n_reads * K)
    z[idx[has]] = g.normal(4, 1, has.sum())
    t_map = 100
    drop, lo, hi, rec = tr.calibrate_output(z, scores, best, rid, t_map, target=0.999)
    assert drop <= lo <= hi
    keep, hit, _ = tr.filter_outcome(z, scores, best, rid, lo, hi, drop)
    mapped = best >= t_map
    assert (hit & mapped).sum() / mapped.sum() >= 0.999
    assert abs(rec - (hit & mapped).sum() / mapped.sum()) < 1e-12
    # unmapped reads are dropped, so far fewer pairs than the strict rule keeps
    lo_s, hi_s, _ = tr.calibrate(z, scores, best, rid, target=0.999)
    keep_s, _, _ = tr.filter_outcome(z, scores, best, rid, lo_s, hi_s)
    assert keep.sum() < 0.5 * keep_s.sum()


def test_calibration_rule_equals_reference_decision():
    """The rule the calibration evaluates (train.filter_outcome, host logic of
    the product) keeps exactly the pairs the reference decision keeps, on
    random logits with contiguous reads of 1-16 candidates."""
    from oracle import filter_ref as flt
    g = np.random.default_rng(11)
    counts = g.integers(1, 17, 500)
    rid = np.repeat(np.arange(len(counts)), counts)
    z = g.normal(0, 2, len(rid)).astype(np.float32)
    scores = g.integers(0, 100, len(rid))
    best = np.zeros(len(counts), np.int64)
    np.maximum.at(best, rid, scores)
    for lo, hi, drop in ((0.0, 1.0, float("-inf")), (0.5, 0.5, -1.0), (-1.0, 2.5, -3.0)):
        keep, _, unsure = tr.filter_outcome(z, scores, best, rid, lo, hi, drop)
        exp_keep, n_unsure = flt.decide(z, rid, len(counts), lo, hi, drop)
        assert (keep == exp_keep).all()
        assert int(unsure.sum()) == n_unsure
