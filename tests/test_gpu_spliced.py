"""Spliced long-read seeds (100-nt seeds of 400-800-nt reads made of 2-4 exons,
4-12 windows of 200-1000 nt each): every pair scored, the best window of every
seed traced back to a CIGAR, eagerly and as a replayed graph; all bit-exact
against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_1304_0681_amd as sw
import synth
from paper_1304_0681_amd.pipeline import AlignPass

pytestmark = pytest.mark.gpu

SC = (5, -4, -10, -1)


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = sw.sw_ctx_create(0)
    yield c
    sw.sw_ctx_destroy(c)


@pytest.fixture(scope="module")
def spliced():
    b = synth.spliced(n_reads=600, ref_len=2_000_000, seed=synth.BASE_SEED + 33)
    ref, _ = oracle.align_batch(b, SC, mode=0)
    rid = b.windows["read_id"].astype(np.int64)
    # best pair per seed: highest score, lowest pair index on ties
    best = np.full(b.n_reads, -1, np.int64)
    np.maximum.at(best, rid, ref["score"].astype(np.int64))
    is_best = ref["score"] == best[rid]
    bp = np.full(b.n_reads, -1, np.int64)
    idx = np.nonzero(is_best)[0][::-1]
    bp[rid[idx]] = idx                     # lowest index wins (written last)
    ra, rops = oracle.align_batch(b, SC, mode=1, sel=bp.astype(np.uint32))
    return b, ref, best, bp, ra, rops


def check(b, out, best, bp, ra, rops):
    gp, gs, ga, go = out
    assert (gs == best).all()
    assert (gp == bp.astype(np.uint32)).all()
    for f in ("score", "read_begin", "read_end", "ref_begin", "ref_end", "n_ops", "status"):
        bad = np.nonzero(ga[f] != ra[f])[0]
        assert len(bad) == 0, f"{len(bad)} {f} mismatches, first {bad[:5]}"
    for k in range(b.n_reads):
        n = int(ra[k]["n_ops"])
        assert (go[k, :n] == rops[k, :n]).all(), \
            f"seed {k}: {oracle.cigar_string(go[k, :n])} vs {oracle.cigar_string(rops[k, :n])}"


@pytest.mark.parametrize("band", [False, True])
def test_spliced_seeds_eager(ctx, spliced, band):
    b, ref, best, bp, ra, rops = spliced
    assert b.n_reads > 2000 and b.windows["len"].max() > 900
    db = sw.DeviceBatch.from_synth(ctx, b)
    ap = AlignPass(ctx, db, SC, band=band)
    ap.run()
    torch.cuda.synchronize()
    h = sw.hits_to_numpy(ap.hits)
    assert (h["score"] == ref["score"]).all()
    check(b, ap.results(), best, bp, ra, rops)


@pytest.mark.parametrize("band", [False, True])
def test_spliced_seeds_graph_replays(ctx, spliced, band):
    """The captured pass replays correctly several times, with unrelated eager
    work and synchronisations between replays, and its outputs (and, with the
    band, the best windows and their hits) cleared before each replay."""
    b, ref, best, bp, ra, rops = spliced
    db = sw.DeviceBatch.from_synth(ctx, b)
    ap = AlignPass(ctx, db, SC, band=band)
    s = torch.cuda.Stream()
    ap.capture(s)
    try:
        for rep in range(3):
            bufs = [ap.hits, ap.best_pair, ap.best_score, ap.aln, ap.ops]
            if band:
                bufs += [ap.bbt.win, ap.bbt.hits]
            for t in bufs:
                t.fill_(-3)
            junk = torch.arange(1 << 20, device="cuda", dtype=torch.float32).sum()
            torch.cuda.synchronize()
            ap.replay(s)
            s.synchronize()
            assert float(junk.item()) > 0
            check(b, ap.results(), best, bp, ra, rops)
    finally:
        ap.close()


def test_graph_capture_refuses_growth(ctx):
    """A call that would have to grow scratch while capturing fails cleanly and
    the context stays usable."""
    b = synth.config1(seed=synth.BASE_SEED + 71, n_reads=50)
    db = sw.DeviceBatch.from_synth(ctx, b)
    big = synth.config2(n_reads=30_000, seed=synth.BASE_SEED + 72)
    dbig = sw.DeviceBatch.from_synth(ctx, big)
    s = torch.cuda.Stream()
    ctx2 = sw.sw_ctx_create(0)       # fresh context: no scratch yet
    try:
        hits = torch.empty((big.n_pairs, 3), dtype=torch.int32, device="cuda")
        sw.sw_graph_begin(ctx2, s)
        with pytest.raises(sw.SwError, match="graph capture"):
            sw.sw_batch_score(ctx2, dbig, SC, 0, hits, s)
        try:                              # nothing was recorded; close the capture
            sw.sw_graph_destroy(ctx2, sw.sw_graph_end(ctx2, s))
        except sw.SwError:
            pass
        torch.cuda.synchronize()
        # usable afterwards, eagerly
        h1 = torch.empty((b.n_pairs, 3), dtype=torch.int32, device="cuda")
        sw.sw_batch_score(ctx2, db, SC, 0, h1)
        torch.cuda.synchronize()
        ref, _ = oracle.align_batch(b, SC, mode=0)
        assert (sw.hits_to_numpy(h1)["score"] == ref["score"]).all()
    finally:
        sw.sw_ctx_destroy(ctx2)


def test_sole_first_pass_equals_oracle(ctx, spliced):
    """AlignPass with sole_first on seeds of which every third keeps one window,
    every third all of them and a few none: best pairs, best scores, alignments
    and CIGARs equal the oracle's, eagerly and over graph replays."""
    b0 = spliced[0]
    rid = b0.windows["read_id"].astype(np.int64)
    first = np.ones(len(rid), bool)
    first[1:] = rid[1:] != rid[:-1]
    keep = (rid % 3 == 1) | ((rid % 3 == 0) & first) | ((rid % 3 == 2) & (rid % 7 != 0))
    b = synth.Batch(ref=b0.ref, reads=b0.reads, read_off=b0.read_off, read_len=b0.read_len,
                    windows=b0.windows[keep], truth={})
    per = np.bincount(b.windows["read_id"].astype(np.int64), minlength=b.n_reads)
    assert (per == 0).sum() > 20 and (per == 1).sum() > 500 and (per > 1).sum() > 500
    ref, _ = oracle.align_batch(b, SC, mode=0)
    ep, es = oracle.best_per_read(ref["score"], b.windows["read_id"].astype(np.int64), b.n_reads)
    has = ep != 0xFFFFFFFF
    ra, rops = oracle.align_batch(b, SC, mode=1, sel=ep[has])
    db = sw.DeviceBatch.from_synth(ctx, b)
    ap = AlignPass(ctx, db, SC, band=True, sole_first=True)

    def check_sole(out):
        gp, gs, ga, go = out
        assert (gp == ep).all()
        assert (gs[has] == es[has]).all() and (gs[~has] == -1).all()
        for f in ("score", "read_begin", "read_end", "ref_begin", "ref_end", "n_ops", "status"):
            assert (ga[f][has] == ra[f]).all(), f
        for k, r in enumerate(np.nonzero(has)[0]):
            n = int(ra[k]["n_ops"])
            assert (go[r, :n] == rops[k, :n]).all(), r

    ap.run()
    torch.cuda.synchronize()
    check_sole(ap.results())
    s = torch.cuda.Stream()
    ap.capture(s)
    try:
        for rep in range(3):
            for t in (ap.best_pair, ap.best_score, ap.aln, ap.ops, ap.sole, ap.multi_best,
                      ap.bbt.hits):
                t.fill_(-3)
            torch.cuda.synchronize()
            ap.replay(s)
            s.synchronize()
            check_sole(ap.results())
    finally:
        ap.close()
