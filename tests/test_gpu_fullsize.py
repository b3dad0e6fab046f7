"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times: the whole batch goes through the device in one call, and the
oracle checks large seeded samples of it (pair by pair, and the CIGAR of every
sampled read's best window).

  * 1M-read batch of 100-nt reads vs 1-8 windows of 200-600 nt (4.5M pairs):
    scores and end cells of every pair of 250,000 sampled reads (about 1.1M
    pairs) and their best hits.
  * Spliced long reads (200,000 reads split into 1.26M 100-nt seeds, 10M
    pairs): the captured-size pass (score every pair, best window per seed,
    banded traceback); 100,000 sampled seeds: every window's score, the best
    window and its alignment and CIGAR.
  * Paired 150-nt mates vs 16 windows of 200-1,000 nt (100,000 mates, 1.6M
    pairs): every score, the best window of every mate and its CIGAR.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1304_0681_amd as sw
import synth
from paper_1304_0681_amd.pipeline import AlignPass

pytestmark = pytest.mark.gpu

SC = (5, -4, -10, -1)
NTHREADS = min(len(os.sched_getaffinity(0)), 16)


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = sw.sw_ctx_create(0)
    yield c
    sw.sw_ctx_destroy(c)


def _pairs_of_reads(rid, reads):
    return np.nonzero(np.isin(rid, reads))[0].astype(np.uint32)


def _check_alignments(a, o, ra, rops):
    for f in ("score", "read_begin", "read_end", "ref_begin", "ref_end", "n_ops", "status"):
        bad = np.nonzero(a[f] != ra[f])[0]
        assert len(bad) == 0, f"{len(bad)} {f} mismatches, first {bad[:5]}"
    for k in range(len(ra)):
        n = int(ra[k]["n_ops"])
        assert (o[k, :n] == rops[k, :n]).all(), \
            f"row {k}: {oracle.cigar_string(o[k, :n])} vs {oracle.cigar_string(rops[k, :n])}"


def test_config2_full_batch_million_pairs(ctx):
    print("fullsize: 1M reads x 1-8 windows, one call", flush=True)
    b = synth.config2()
    db = sw.DeviceBatch.from_synth(ctx, b)
    rid = b.windows["read_id"].astype(np.int64)
    reads = np.sort(np.random.default_rng(2).choice(b.n_reads, 250_000, replace=False))
    sel = _pairs_of_reads(rid, reads)
    assert len(sel) >= 1_000_000
    ref, _ = oracle.align_batch(b, SC, mode=0, sel=sel, nthreads=NTHREADS)
    for flags in (0, sw.SW_WANT_ENDS):           # packed int16, then int32 with ends
        hits = torch.full((b.n_pairs, 3), -7, dtype=torch.int32, device="cuda")
        sw.sw_batch_score(ctx, db, SC, flags, hits)
        torch.cuda.synchronize()
        h = sw.hits_to_numpy(hits)[sel]
        assert (h["score"] == ref["score"]).all()
        if flags:
            assert (h["read_end"] == ref["read_end"]).all() and (h["ref_end"] == ref["ref_end"]).all()
    bp = torch.empty(b.n_reads, dtype=torch.int32, device="cuda")
    bs = torch.empty(b.n_reads, dtype=torch.int32, device="cuda")
    sw.sw_best_per_read(ctx, db, hits, 0, bp, bs)
    torch.cuda.synchronize()
    full = np.full(b.n_pairs, -2, np.int32)
    full[sel] = ref["score"]
    ep, es = oracle.best_per_read(full, rid, b.n_reads)
    assert (bp.cpu().numpy().view(np.uint32)[reads] == ep[reads]).all()
    assert (bs.cpu().numpy()[reads] == es[reads]).all()


def test_config3_full_pass_hundred_thousand_seeds(ctx):
    print("fullsize: spliced reads, 1.26M seeds, 10M pairs", flush=True)
    b = synth.spliced()
    assert b.n_reads > 1_200_000 and b.n_pairs > 9_000_000
    db = sw.DeviceBatch.from_synth(ctx, b)
    ap = AlignPass(ctx, db, SC, band=True)
    ap.run()
    torch.cuda.synchronize()
    gbp, gbs, ga, go = ap.results()
    h = sw.hits_to_numpy(ap.hits)
    rid = b.windows["read_id"].astype(np.int64)
    seeds = np.sort(np.random.default_rng(3).choice(b.n_reads, 100_000, replace=False))
    sel = _pairs_of_reads(rid, seeds)
    ref, _ = oracle.align_batch(b, SC, mode=0, sel=sel, nthreads=NTHREADS)
    assert (h["score"][sel] == ref["score"]).all()
    full = np.full(b.n_pairs, -2, np.int32)
    full[sel] = ref["score"]
    ep, es = oracle.best_per_read(full, rid, b.n_reads)
    assert (gbp[seeds] == ep[seeds]).all() and (gbs[seeds] == es[seeds]).all()
    ra, rops = oracle.align_batch(b, SC, mode=1, sel=ep[seeds], nthreads=NTHREADS,
                                  ops_stride=ap.ops_stride)
    _check_alignments(ga[seeds], go[seeds], ra, rops)
    ap.close()


def test_paired_mates_hundred_thousand(ctx):
    print("fullsize: 100k paired 150-nt mates x 16 windows", flush=True)
    refc = synth.make_reference(synth.rng(synth.BASE_SEED + 5), 64_000_000)
    b = synth.paired_chunk(synth.BASE_SEED + 500, 50_000, refc)
    assert b.n_reads == 100_000 and b.n_pairs == 1_600_000
    db = sw.DeviceBatch.from_synth(ctx, b)
    ap = AlignPass(ctx, db, SC, band=True)
    ap.run()
    torch.cuda.synchronize()
    gbp, gbs, ga, go = ap.results()
    ref, _ = oracle.align_batch(b, SC, mode=0, nthreads=NTHREADS)
    assert (sw.hits_to_numpy(ap.hits)["score"] == ref["score"]).all()
    rid = b.windows["read_id"].astype(np.int64)
    ep, es = oracle.best_per_read(ref["score"], rid, b.n_reads)
    assert (gbp == ep).all() and (gbs == es).all()
    ra, rops = oracle.align_batch(b, SC, mode=1, sel=ep, nthreads=NTHREADS, ops_stride=ap.ops_stride)
    _check_alignments(ga, go, ra, rops)
    ap.close()
