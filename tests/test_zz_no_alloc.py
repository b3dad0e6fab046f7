"""The allocation-free scoring entry point (sw_batch_score_noalloc) against
sw_batch_score on the same batches: two calls in a row, the second on a
smaller batch, so that the static scratch holds the first call's contents when
the second starts; queries of every length class, both result modes."""
import numpy as np
import pytest
import torch

import oracle
import paper_1304_0681_amd as sw
import synth

pytestmark = pytest.mark.gpu

SC = (5, -4, -10, -1)


def _mixed(seed, n_reads, ref_len=400_000):
    """Reads of 10-2,300 bases (every query-length class, strip class included),
    1-4 windows each that overlap the read's origin, both strands."""
    g = np.random.default_rng(seed)
    ref = g.integers(0, 4, ref_len).astype(np.uint8)
    lens = g.choice([10, 30, 60, 100, 120, 150, 200, 400, 900, 1800, 2300], n_reads)
    reads, wins = [], []
    for m in lens:
        b0 = int(g.integers(3000, ref_len - int(m) - 3000))
        seg = ref[b0:b0 + int(m)].copy()
        mut = g.random(len(seg)) < 0.03
        seg[mut] = (seg[mut] + 1) % 4
        st = int(g.integers(0, 2))
        reads.append(synth.ASCII[(3 - seg[::-1]) if st else seg].tobytes())
        for _ in range(int(g.integers(1, 5))):
            n = int(g.integers(20, 1200))
            wins.append((len(reads) - 1, max(b0 - int(g.integers(0, 300)), 0), n,
                         st if g.random() < 0.8 else 1 - st))
    return synth.custom(synth.ASCII[ref].tobytes(), reads, wins)


def _score(fn, ctx, db, n, flags):
    hits = torch.full((n, 3), -7, dtype=torch.int32, device="cuda")
    fn(ctx, db, SC, flags, hits)
    torch.cuda.synchronize()
    return sw.hits_to_numpy(hits)


def test_noalloc_matches_batch_score_twice_shrinking():
    print("wip_no_alloc: sw_batch_score_noalloc vs sw_batch_score", flush=True)
    torch.cuda.set_device(0)
    ctx = sw.sw_ctx_create(0)
    try:
        big = _mixed(101, 900)
        small = _mixed(102, 150)
        assert small.n_pairs < big.n_pairs
        for flags in (0, sw.SW_WANT_ENDS):
            for b in (big, small):          # the second call on a smaller batch
                db = sw.DeviceBatch.from_synth(ctx, b)
                a = _score(sw.sw_batch_score_noalloc, ctx, db, b.n_pairs, flags)
                r = _score(sw.sw_batch_score, ctx, db, b.n_pairs, flags)
                assert (a == r).all(), f"{int((a != r).sum())} hits differ (flags {flags})"
        # and the oracle on the smaller batch
        ref, _ = oracle.align_batch(small, SC, mode=0)
        db = sw.DeviceBatch.from_synth(ctx, small)
        a = _score(sw.sw_batch_score_noalloc, ctx, db, small.n_pairs, sw.SW_WANT_ENDS)
        for f in ("score", "read_end", "ref_end"):
            assert (a[f] == ref[f]).all(), f
    finally:
        sw.sw_ctx_destroy(ctx)


def test_noalloc_config2_sample_and_limit():
    """A config-2 sample (packed int16 class) and the pair limit."""
    print("wip_no_alloc: config-2 sample and the size limit", flush=True)
    torch.cuda.set_device(0)
    ctx = sw.sw_ctx_create(0)
    try:
        b = synth.config2(n_reads=20_000, seed=synth.BASE_SEED + 88)
        db = sw.DeviceBatch.from_synth(ctx, b)
        a = _score(sw.sw_batch_score_noalloc, ctx, db, b.n_pairs, 0)
        r = _score(sw.sw_batch_score, ctx, db, b.n_pairs, 0)
        assert (a == r).all()
        # more pairs than the static scratch holds: a clear SW_E_RANGE, no launch
        v = db.view(db.win, sw.SW_NOALLOC_MAX_PAIRS + 1)
        with pytest.raises(sw.SwError, match="at most"):
            sw.sw_batch_score_noalloc(ctx, v, SC, 0, torch.empty(3, dtype=torch.int32, device="cuda"))
    finally:
        sw.sw_ctx_destroy(ctx)
