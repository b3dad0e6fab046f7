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
  * The splice-junction pass on 200,000 spliced long reads (1.25M seeds, 10M
    seed pairs, 207k joined windows): for 300 sampled reads, every seed's best
    window and CAL, the read's joined windows, its best window, alignment and
    CIGAR with the junctions rewritten, and its junctions in the table; once
    with the generator's seed windows, once with the device seeker's.
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



@pytest.fixture(scope="module")
def spliced_200k():
    return synth.spliced_long(n_reads=200_000)


def _run_junction_pass(long_b, seed_b, truth, seeker: bool):
    """The pass at the benchmark's settings in a context of its own (64 GiB of
    traceback scratch); returns its outputs as host arrays."""
    from paper_1304_0681_amd.seeker import KmerIndex
    from paper_1304_0681_amd.splice import SeekerSplicedPass, SplicedPass
    c2 = sw.sw_ctx_create(0)
    try:
        seed_db = sw.DeviceBatch(c2, seed_b.ref, seed_b.reads, seed_b.read_off, seed_b.read_len,
                                 np.zeros(0, sw.WINDOW_DTYPE) if seeker else seed_b.windows)
        long_db = sw.DeviceBatch(c2, None, long_b.reads, long_b.read_off, long_b.read_len,
                                 np.zeros(0, sw.WINDOW_DTYPE), ref2b=(seed_db.ref2b, seed_db.ref_len))
        if seeker:
            idx = KmerIndex(c2, seed_db.ref2b, seed_db.ref_len, k=15)
            sp = SeekerSplicedPass(c2, seed_db, idx, truth["seed_read"], long_db,
                                   table_capacity=1 << 21, tb_scratch_mb=65536)
        else:
            sp = SplicedPass(c2, seed_db, truth["seed_read"], long_db, table_capacity=1 << 21,
                             tb_scratch_mb=65536)
        sp.run()
        torch.cuda.synchronize()
        sw_win = sp.seeker.windows() if seeker else seed_b.windows
        out = dict(seed_windows=sw_win, ops_stride=sp.ops_stride,
                   seed_bp=sp.seeds.best_pair.cpu().numpy().view(np.uint32),
                   cals=sp.cals.cpu().numpy().view(sw.CAL_DTYPE), windows=sp.windows())
        out["bp"], out["bs"], out["aln"], out["ops"], out["nj"] = sp.results()
        out["table"] = {(int(j["start"]), int(j["end"]), int(j["strand"])): int(j["count"])
                        for j in sp.junctions()}
        return out
    finally:
        sw.sw_ctx_destroy(c2)


def _wtuple(w):
    return (int(w["read_id"]), int(w["ref_begin"]), int(w["len"]), int(w["strand"]))


def _check_junction_sample(long_b, seed_b, truth, g, seed_windows_of):
    """The oracle's chain on every seed of 300 sampled long reads against the
    pass's outputs `g`; seed_windows_of(seeds) gives the oracle's candidate
    windows of those seeds (read id = seed index)."""
    from oracle import junction_ref as jr
    from paper_1304_0681_amd.splice import LONG_SCORING
    seed_read = np.asarray(truth["seed_read"], dtype=np.int64)
    longs = np.sort(np.random.default_rng(7).choice(long_b.n_reads, 300, replace=False))
    seeds = np.nonzero(np.isin(seed_read, longs))[0]
    # seeds: every window's score, the best window, its alignment, the CAL
    swin = seed_windows_of(seeds)
    sb = synth.Batch(ref=seed_b.ref, reads=seed_b.reads, read_off=seed_b.read_off,
                     read_len=seed_b.read_len, windows=swin, truth={})
    res, _ = oracle.align_batch(sb, SC, mode=0, nthreads=NTHREADS)
    ep, _ = oracle.best_per_read(res["score"], swin["read_id"].astype(np.int64), seed_b.n_reads)
    for s in seeds:
        if ep[s] == 0xFFFFFFFF:
            assert g["seed_bp"][s] == 0xFFFFFFFF, s
        else:
            assert _wtuple(g["seed_windows"][g["seed_bp"][s]]) == _wtuple(swin[ep[s]]), s
    has_s = ep[seeds] != 0xFFFFFFFF
    sa = np.zeros(len(seeds), oracle.RESULT_DTYPE)
    sa["score"] = -1
    sa["ref_begin"] = sa["ref_end"] = -1
    sa[has_s] = oracle.align_batch(sb, SC, mode=1, sel=ep[seeds][has_s], nthreads=NTHREADS)[0]
    ocals = jr.seed_cals(swin, ep[seeds], sa, seed_read[seeds].astype(np.uint32), 100)
    assert [(int(c["read_id"]), int(c["first"]), int(c["last"]), int(c["strand"]), int(c["valid"]))
            for c in g["cals"][seeds]] == ocals
    # joined windows of each sampled read
    ref_len = len(long_b.ref)
    gw = g["windows"]
    win = []
    for r in longs:
        mine = [(0,) + c[1:] for c in ocals if c[0] == r]
        jw = jr.join_cals(mine, 1, ref_len, ext=30, max_gap=5000)
        gwr = gw[gw["read_id"] == r]
        assert [(int(x["ref_begin"]), int(x["len"]), int(x["strand"])) for x in gwr] == \
            [(b, n, st) for _, b, n, st in jw], r
        win += [(int(r), b, n, st, 0) for _, b, n, st in jw]
    win = np.array(win, dtype=synth.WINDOW_DTYPE)
    # whole-read alignment: best window, alignment, CIGAR, detection
    lb = synth.Batch(ref=long_b.ref, reads=long_b.reads, read_off=long_b.read_off,
                     read_len=long_b.read_len, windows=win, truth={})
    lres, _ = oracle.align_batch(lb, LONG_SCORING, mode=0, nthreads=NTHREADS)
    lbp, lbs = oracle.best_per_read(lres["score"], win["read_id"].astype(np.int64), long_b.n_reads)
    has = lbp[longs] != 0xFFFFFFFF
    assert has.mean() > 0.98
    for r in longs[~has]:
        assert g["bp"][r] == 0xFFFFFFFF, r
    la, lops = oracle.align_batch(lb, LONG_SCORING, mode=1, sel=lbp[longs][has],
                                  nthreads=NTHREADS, ops_stride=g["ops_stride"])
    ref_codes = jr.codes_of(long_b.ref.tobytes())
    ga, gops = g["aln"], g["ops"]
    n_found = 0
    for k, r in enumerate(longs[has]):
        w = win[lbp[r]]
        assert _wtuple(gw[g["bp"][r]]) == _wtuple(w), r
        assert int(g["bs"][r]) == int(lbs[r])
        a = la[k]
        for f in ("score", "read_begin", "read_end", "ref_begin", "ref_end", "n_ops", "status"):
            assert int(ga[f][r]) == int(a[f]), (r, f)
        n = int(a["n_ops"])
        if a["score"] >= 100 and not a["status"]:
            t = ref_codes[int(w["ref_begin"]):int(w["ref_begin"]) + int(w["len"])]
            new, js = jr.detect(t, lops[k, :n], int(a["ref_begin"]), 40, int(w["ref_begin"]))
            assert list(gops[r, :n]) == list(new), r
            assert int(g["nj"][r]) == len(js)
            for j in js:
                assert g["table"].get(tuple(int(x) for x in j), 0) >= 1, (r, j)
            n_found += len(js)
        else:
            assert (gops[r, :n] == lops[k, :n]).all(), r
    assert n_found > 300


def test_junction_pass_two_hundred_thousand_reads(spliced_200k):
    """The junction pass at the benchmark's size (the generator's seed windows),
    checked read by read for a sample of 300 long reads and all their seeds."""
    print("fullsize: junction pass, 200k spliced long reads", flush=True)
    long_b, seed_b, truth = spliced_200k
    g = _run_junction_pass(long_b, seed_b, truth, seeker=False)
    rid = seed_b.windows["read_id"].astype(np.int64)
    _check_junction_sample(long_b, seed_b, truth, g,
                           lambda seeds: seed_b.windows[_pairs_of_reads(rid, seeds)])


def test_junction_pass_from_seeker_two_hundred_thousand_reads(spliced_200k):
    """The same with the seeds' windows found by the device seeker; the oracle
    seeker gives the sampled seeds' windows."""
    from oracle import junction_ref as jr
    from oracle import seeker_ref as sr
    print("fullsize: seeker-fed junction pass, 200k spliced long reads", flush=True)
    long_b, seed_b, truth = spliced_200k
    g = _run_junction_pass(long_b, seed_b, truth, seeker=True)
    ref = jr.codes_of(long_b.ref.tobytes())
    oidx = sr.build_index_fast(ref, 15)

    def seeker_windows(seeds):
        out = []
        for s in seeds:
            c = sr.cals(0, sr.regions(jr.codes_of(seed_b.read(int(s))), oidx), 50, 20)
            out += [(int(s), b, n, st, 0) for _, b, n, st in
                    jr.join_cals(c, 1, len(ref), ext=30, max_gap=5000)]
        return np.array(out, dtype=synth.WINDOW_DTYPE)

    _check_junction_sample(long_b, seed_b, truth, g, seeker_windows)
