"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bar: bit-exact scores, end cells, begin cells and CIGARs on every tested pair.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1304_0681_amd as sw
import synth
from batches import EDGE_M, EDGE_N, edge_batch

pytestmark = pytest.mark.gpu

SC = (5, -4, -10, -1)


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = sw.sw_ctx_create(0)
    yield c
    sw.sw_ctx_destroy(c)


def gpu_score(ctx, b, sc=SC, ends=True, db=None):
    db = db or sw.DeviceBatch.from_synth(ctx, b)
    hits = torch.full((b.n_pairs, 3), -7, dtype=torch.int32, device="cuda")
    sw.sw_batch_score(ctx, db, sc, sw.SW_WANT_ENDS if ends else 0, hits)
    torch.cuda.synchronize()
    return sw.hits_to_numpy(hits)


def gpu_traceback(ctx, b, sel=None, sc=SC, stride=None, db=None, band=False):
    """band: pass the score kernel's hits (with ends) so that each DP covers only
    the columns the alignment can reach."""
    db = db or sw.DeviceBatch.from_synth(ctx, b)
    hits = None
    if band:
        hits = torch.full((b.n_pairs, 3), -7, dtype=torch.int32, device="cuda")
        sw.sw_batch_score(ctx, db, sc, sw.SW_WANT_ENDS, hits)
    if sel is None:
        sel = np.arange(b.n_pairs, dtype=np.uint32)
    sel = np.asarray(sel, dtype=np.uint32)
    if stride is None:
        stride = int(b.read_len.max()) + int(b.windows["len"].max()) + 4
    ids = torch.from_numpy(sel.view(np.int32)).cuda()
    aln = torch.full((len(sel), 7), -7, dtype=torch.int32, device="cuda")
    ops = torch.zeros((len(sel), stride), dtype=torch.int32, device="cuda")
    sw.sw_batch_traceback(ctx, db, sc, ids, len(sel), aln, ops, stride, hits=hits)
    torch.cuda.synchronize()
    return sw.aln_to_numpy(aln), ops.cpu().numpy().view(np.uint32)


def assert_hits_equal(h, ref, ends=True):
    bad = np.nonzero(h["score"] != ref["score"])[0]
    assert len(bad) == 0, f"{len(bad)} score mismatches, first {bad[:5]}: " \
                          f"{h[bad[:5]]} vs {ref[bad[:5]][['score', 'read_end', 'ref_end']]}"
    if ends:
        for f in ("read_end", "ref_end"):
            bad = np.nonzero(h[f] != ref[f])[0]
            assert len(bad) == 0, f"{len(bad)} {f} mismatches, first {bad[:5]}"


def assert_aln_equal(a, o, ref, rops):
    for f in ("score", "read_begin", "read_end", "ref_begin", "ref_end", "n_ops", "status"):
        bad = np.nonzero(a[f] != ref[f])[0]
        assert len(bad) == 0, f"{len(bad)} {f} mismatches, first {bad[:5]}: {a[bad[:3]]} vs {ref[bad[:3]]}"
    for k in range(len(a)):
        n = int(ref[k]["n_ops"])
        if not (o[k, :n] == rops[k, :n]).all():
            raise AssertionError(f"pair {k}: CIGAR {oracle.cigar_string(o[k, :n])} vs "
                                 f"{oracle.cigar_string(rops[k, :n])}")


# ---------------------------------------------------------------------------

def test_pack2b_matches_reference(ctx):
    g = np.random.default_rng(3)
    x = synth.ASCII[g.integers(0, 4, 100_003)].copy()
    bad_pos = g.choice(len(x), 17, replace=False)
    x[bad_pos] = ord("N")
    dev = torch.from_numpy(x).cuda()
    for off in (0, 3):                                   # aligned and unaligned sources
        n = len(x) - off
        out = torch.full(((n + 15) // 16,), -1, dtype=torch.int32, device="cuda")
        bad = torch.zeros(1, dtype=torch.int32, device="cuda")
        sw.sw_pack2b(ctx, dev[off:], n, out, bad)
        torch.cuda.synchronize()
        clean = x[off:].copy()
        nb = int((clean == ord("N")).sum())
        clean[clean == ord("N")] = ord("A")
        exp = oracle.pack2b(clean).view(np.int32)
        assert (out.cpu().numpy() == exp).all()
        assert int(bad.item()) == nb


def test_config1_all_pairs(ctx):
    b = synth.config1()
    db = sw.DeviceBatch.from_synth(ctx, b)
    ref, rops = oracle.align_batch(b, SC, mode=1)
    assert_hits_equal(gpu_score(ctx, b, ends=True, db=db), ref)
    assert_hits_equal(gpu_score(ctx, b, ends=False, db=db), ref, ends=False)
    a, o = gpu_traceback(ctx, b, db=db)
    assert_aln_equal(a, o, ref, rops)


def test_edge_lengths_scores(ctx):
    b = edge_batch(11, EDGE_M, EDGE_N)
    ref, _ = oracle.align_batch(b, SC, mode=0)
    assert_hits_equal(gpu_score(ctx, b, ends=True), ref)
    sw.sw_ctx_set_option(ctx, sw.SW_OPT_INT16, 0)   # int32 datapath (see the skipped test below)
    try:
        assert_hits_equal(gpu_score(ctx, b, ends=False), ref, ends=False)
    finally:
        sw.sw_ctx_set_option(ctx, sw.SW_OPT_INT16, 1)


def test_edge_lengths_traceback(ctx):
    b = edge_batch(12, EDGE_M, EDGE_N)
    ref, rops = oracle.align_batch(b, SC, mode=1)
    a, o = gpu_traceback(ctx, b)
    assert_aln_equal(a, o, ref, rops)


@pytest.mark.parametrize("sc", [(5, -4, -10, -1), (2, -3, -4, -4), (1, 0, -2, -1),
                                (127, -127, -127, 0), (5, -4, -10, -10)])
def test_traceback_band_from_score_ends(ctx, sc):
    """Traceback restricted to the columns an alignment of the pair's score and end
    can reach gives the oracle's alignments (edge lengths over every class; a gap
    extension of 0 makes the band the whole window)."""
    b = edge_batch(13, EDGE_M, EDGE_N)
    ref, rops = oracle.align_batch(b, sc, mode=1)
    a, o = gpu_traceback(ctx, b, sc=sc, band=True)
    assert_aln_equal(a, o, ref, rops)


def test_traceback_mixed_known_and_unknown_ends(ctx):
    """Hits where a random half of the pairs has its end cell removed (score kept,
    ends -1): the waves that mix pairs with and without a known end track the best
    cell for all of them, pairs without an end use the whole window, and every
    alignment still equals the oracle's."""
    b = edge_batch(17, EDGE_M, EDGE_N)
    ref, rops = oracle.align_batch(b, SC, mode=1)
    db = sw.DeviceBatch.from_synth(ctx, b)
    hits = torch.full((b.n_pairs, 3), -7, dtype=torch.int32, device="cuda")
    sw.sw_batch_score(ctx, db, SC, sw.SW_WANT_ENDS, hits)
    drop = torch.from_numpy(np.random.default_rng(18).random(b.n_pairs) < 0.5).cuda()
    hits[drop, 1] = -1
    hits[drop, 2] = -1
    sel = np.arange(b.n_pairs, dtype=np.uint32)
    stride = int(b.read_len.max()) + int(b.windows["len"].max()) + 4
    ids = torch.from_numpy(sel.view(np.int32)).cuda()
    aln = torch.full((len(sel), 7), -7, dtype=torch.int32, device="cuda")
    ops = torch.zeros((len(sel), stride), dtype=torch.int32, device="cuda")
    sw.sw_batch_traceback(ctx, db, SC, ids, len(sel), aln, ops, stride, hits=hits)
    torch.cuda.synchronize()
    assert_aln_equal(sw.aln_to_numpy(aln), ops.cpu().numpy().view(np.uint32), ref, rops)
    assert int(drop.sum().item()) > 100


def test_select_windows(ctx):
    """sw_select_windows copies the windows of the given pair ids; ids at or past
    the batch's pairs (also past a device-side pair count) give a window with an
    invalid read id, which the score and traceback calls answer as invalid."""
    b = synth.config1(seed=synth.BASE_SEED + 63, n_reads=40)
    db = sw.DeviceBatch.from_synth(ctx, b)
    ids = np.array([3, 0, 39, b.n_pairs, 0xFFFFFFFF, 7], dtype=np.uint32)
    d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    out = torch.full((len(ids) * 12,), 0x5A, dtype=torch.uint8, device="cuda")
    sw.sw_select_windows(ctx, db, d_ids, len(ids), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(b.windows.dtype)
    for k, p in enumerate(ids):
        if p < b.n_pairs:
            assert got[k].tobytes() == b.windows[p].tobytes()
        else:
            assert got[k]["read_id"] == 0xFFFFFFFF and got[k]["len"] == 0
    # a count on the device limits the valid ids to those below it
    cnt = torch.tensor([5], dtype=torch.int32, device="cuda")
    sw.sw_select_windows(ctx, db.view(db.win, b.n_pairs, cnt), d_ids, len(ids), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(b.windows.dtype)
    for k, p in enumerate(ids):
        if p < 5:
            assert got[k].tobytes() == b.windows[p].tobytes()
        else:
            assert got[k]["read_id"] == 0xFFFFFFFF
    # the gathered list scores like the original pairs and marks the invalid ones
    view = db.view(out, len(ids))
    sw.sw_select_windows(ctx, db, d_ids, len(ids), out)
    hits = torch.full((len(ids), 3), -7, dtype=torch.int32, device="cuda")
    sw.sw_batch_score(ctx, view, SC, sw.SW_WANT_ENDS, hits)
    torch.cuda.synchronize()
    h = sw.hits_to_numpy(hits)
    ref, _ = oracle.align_batch(b, SC, mode=0)
    for k, p in enumerate(ids):
        if p < b.n_pairs:
            for f in ("score", "read_end", "ref_end"):
                assert h[k][f] == ref[p][f]
        else:
            assert h[k]["score"] == -1


def test_traceback_band_paired_mates(ctx):
    """150-nt mates against 16 windows of 200-1,000 nt (the stream's shape): best
    window per mate traced with and without the band, both equal to the oracle."""
    ref_codes = synth.make_reference(synth.rng(synth.BASE_SEED + 61), 400_000)
    b = synth.paired_chunk(synth.BASE_SEED + 62, 150, ref_codes)
    h = oracle.align_batch(b, SC, mode=0)[0]
    rid = b.windows["read_id"].astype(np.int64)
    best = np.full(b.n_reads, -1, dtype=np.int64)
    for k in np.argsort(-h["score"], kind="stable"):
        if best[rid[k]] < 0:
            best[rid[k]] = k
    sel = best[best >= 0].astype(np.uint32)
    ref, rops = oracle.align_batch(b, SC, mode=1, sel=sel)
    db = sw.DeviceBatch.from_synth(ctx, b)
    for band in (False, True):
        a, o = gpu_traceback(ctx, b, sel=sel, db=db, band=band, stride=int(rops.shape[1]))
        assert_aln_equal(a, o, ref, rops)


@pytest.mark.parametrize("sc", [(2, -3, -4, -4), (1, 0, -2, -1), (3, -1, -5, -2), (127, -127, -127, 0),
                                (5, -4, -10, -10), (5, -4, -20, 0)])
def test_scoring_schemes(ctx, sc):
    b = edge_batch(13, [1, 17, 64, 100, 130, 300], [1, 16, 65, 300], div=0.1)
    ref, rops = oracle.align_batch(b, sc, mode=1)
    assert_hits_equal(gpu_score(ctx, b, sc=sc, ends=True), ref)
    assert_hits_equal(gpu_score(ctx, b, sc=sc, ends=False), ref, ends=False)
    a, o = gpu_traceback(ctx, b, sc=sc)
    assert_aln_equal(a, o, ref, rops)


def test_config2_sample_scores_and_best(ctx):
    b = synth.config2(n_reads=20_000)
    db = sw.DeviceBatch.from_synth(ctx, b)
    ref, _ = oracle.align_batch(b, SC, mode=0)
    h = gpu_score(ctx, b, ends=True, db=db)
    assert_hits_equal(h, ref)
    hs = gpu_score(ctx, b, ends=False, db=db)          # packed int16 datapath
    assert (hs["score"] == ref["score"]).all()
    sw.sw_ctx_set_option(ctx, sw.SW_OPT_INT16, 0)       # int32 datapath
    try:
        h32 = gpu_score(ctx, b, ends=False, db=db)
    finally:
        sw.sw_ctx_set_option(ctx, sw.SW_OPT_INT16, 1)
    assert (h32["score"] == ref["score"]).all()
    # best hit per read
    hits = torch.from_numpy(np.ascontiguousarray(h).view(np.int32).reshape(-1, 3)).cuda()
    bp = torch.empty(b.n_reads, dtype=torch.int32, device="cuda")
    bs = torch.empty(b.n_reads, dtype=torch.int32, device="cuda")
    mapped = torch.empty(b.n_reads, dtype=torch.uint8, device="cuda")
    sw.sw_best_per_read(ctx, db, hits, 250, bp, bs, mapped)
    torch.cuda.synchronize()
    ep, es = oracle.best_per_read(ref["score"], b.windows["read_id"], b.n_reads)
    assert (bp.cpu().numpy().view(np.uint32) == ep).all()
    assert (bs.cpu().numpy() == es).all()
    assert (mapped.cpu().numpy() == (es >= 250)).all()


def test_order_invariance_and_determinism(ctx):
    b = synth.config2(n_reads=3000, ref_len=500_000, seed=99)
    h1 = gpu_score(ctx, b)
    h2 = gpu_score(ctx, b)
    assert (h1 == h2).all()
    perm = np.random.default_rng(0).permutation(b.n_pairs)
    bp = synth.Batch(ref=b.ref, reads=b.reads, read_off=b.read_off, read_len=b.read_len,
                     windows=b.windows[perm].copy())
    hp = gpu_score(ctx, bp)
    assert (hp == h1[perm]).all()


def test_int16_limit_and_strips(ctx):
    """Scores just below and above 2^15 (5 * 6553 = 32765, 5 * 6554 = 32770) and
    queries long enough for the strip-mined class."""
    g = np.random.default_rng(5)
    base = synth.ASCII[g.integers(0, 4, 7000)].tobytes()
    ref = base + synth.ASCII[g.integers(0, 4, 3000)].tobytes()
    reads = [base[:6553], base[:6554], base[100:3100], base[:40]]
    wins = [(0, 0, 6554, 0), (1, 0, 6554, 0), (2, 0, 4000, 0), (3, 6000, 1100, 0)]
    b = synth.custom(ref, reads, wins)
    ref_r, rops = oracle.align_batch(b, SC, mode=1)
    assert int(ref_r[0]["score"]) == 32765 and int(ref_r[1]["score"]) == 32770
    assert_hits_equal(gpu_score(ctx, b, ends=True), ref_r)
    assert_hits_equal(gpu_score(ctx, b, ends=False), ref_r, ends=False)
    a, o = gpu_traceback(ctx, b)
    assert_aln_equal(a, o, ref_r, rops)


def test_invalid_and_empty_pairs(ctx):
    ref = b"ACGTACGTTTGCA" * 3
    reads = [b"ACGTACG", b"TTGCA", b""]
    wins = [(0, 0, 13, 0), (1, 8, 50, 0), (1, 400, 10, 0), (5, 0, 5, 0), (2, 0, 13, 0),
            (0, 0, 0, 1), (0, 30, 60, 1)]
    b = synth.custom(ref, reads, wins)
    ref_r, rops = oracle.align_batch(b, SC, mode=1)
    assert_hits_equal(gpu_score(ctx, b), ref_r)
    a, o = gpu_traceback(ctx, b)
    assert_aln_equal(a, o, ref_r, rops)


def test_traceback_ids_naming_no_pair_come_first(ctx):
    """Selected ids that name no pair (0xFFFFFFFF, as sw_best_per_read gives a read
    without a hit, and the batch's pair count), the first id among them, next to
    a few real pairs of several query-length classes, so that each class's last
    wave has idle lane groups: those read a window of the batch, never one at a
    stray id.  Real pairs equal the oracle; the others are marked invalid."""
    g = np.random.default_rng(41)
    refc = g.integers(0, 4, 20_000).astype(np.uint8)
    reads, wins = [], []
    for m in (30, 100, 150, 600):
        for _ in range(3):
            b0 = int(g.integers(0, 19_000 - m))
            seg = refc[b0 + 40:b0 + 40 + m].copy()
            mut = g.random(m) < 0.03
            seg[mut] = (seg[mut] + 1) % 4
            reads.append(synth.ASCII[seg].tobytes())
            wins.append((len(reads) - 1, b0, m + 80, 0))
    b = synth.custom(synth.ASCII[refc].tobytes(), reads, wins)
    none = 0xFFFFFFFF
    sel = np.array([none, 0, 1, none, 3, b.n_pairs, 4, 6, 7, 9, 10, 11, none], dtype=np.uint32)
    real = sel < b.n_pairs
    ref, rops = oracle.align_batch(b, SC, mode=1, sel=sel[real])
    for band in (False, True):
        a, o = gpu_traceback(ctx, b, sel=sel, band=band)
        assert_aln_equal(a[real], o[real], ref, rops)
        for k in np.nonzero(~real)[0]:
            assert (int(a[k]["score"]), int(a[k]["n_ops"]), int(a[k]["status"])) == (-1, 0, 2), k


def test_traceback_truncation(ctx):
    # 2S3M1D5M2S: five ops, cut to the first two
    b = synth.custom(b"TTACGTTACGTGG", [b"CCACGTACGTAA"], [(0, 0, 13, 0)])
    ref, rops = oracle.align_batch(b, SC, mode=1)
    assert oracle.cigar_string(rops[0, :int(ref[0]["n_ops"])]) == "2S3M1D5M2S"
    a, o = gpu_traceback(ctx, b, stride=2)
    assert int(a[0]["status"]) & 1 and int(a[0]["n_ops"]) == 2
    assert (o[0, :2] == rops[0, :2]).all()
    assert int(a[0]["score"]) == int(ref[0]["score"])


def test_windows_at_reference_start(ctx):
    """Windows that begin within a lane group's skew of reference base 0, for every
    query-length class (the first columns of the later lanes lie before the
    reference start)."""
    g = np.random.default_rng(31)
    refc = g.integers(0, 4, 30_000).astype(np.uint8)
    reads, wins = [], []
    for m in [10, 30, 60, 100, 120, 150, 200, 400, 800, 1500, 2100]:
        for rb in [0, 1, 2, 3, 5, 7, 15, 16, 31, 63, 64]:
            for n in [8, 40, 300]:
                for st in (0, 1):
                    seg = refc[rb:rb + m].copy()
                    mut = g.random(m) < 0.03
                    seg[mut] = (seg[mut] + 1) % 4
                    read = (3 - seg[::-1]) if st else seg
                    reads.append(synth.ASCII[read].tobytes())
                    wins.append((len(reads) - 1, rb, n, st))
    b = synth.custom(synth.ASCII[refc].tobytes(), reads, wins)
    ref, rops = oracle.align_batch(b, SC, mode=1)
    assert_hits_equal(gpu_score(ctx, b, ends=True), ref)
    assert_hits_equal(gpu_score(ctx, b, ends=False), ref, ends=False)
    a, o = gpu_traceback(ctx, b)
    assert_aln_equal(a, o, ref, rops)


def test_short_reads_with_gaps(ctx):
    """Queries of 1-40 bases (the single-lane and two-lane classes) with planted
    insertions and deletions."""
    b = edge_batch(41, list(range(6, 41, 3)), [7, 12, 20, 33, 90], div=0.02)
    g = np.random.default_rng(42)
    reads = []
    for k in range(b.n_reads):
        r = bytearray(b.read(k))
        if len(r) > 5:
            p = int(g.integers(2, len(r) - 2))
            if g.random() < 0.5:
                del r[p]
            else:
                r.insert(p, r[p])
        reads.append(bytes(r))
    wins = [(int(w["read_id"]), int(w["ref_begin"]), int(w["len"]), int(w["strand"]))
            for w in b.windows]
    b = synth.custom(b.ref.tobytes(), reads, wins)
    ref, rops = oracle.align_batch(b, SC, mode=1)
    assert_hits_equal(gpu_score(ctx, b, ends=True), ref)
    a, o = gpu_traceback(ctx, b)
    assert_aln_equal(a, o, ref, rops)


@pytest.mark.skip(reason="packed int16 kernels other than the 4-lane x 25-row shape are switched "
                         "off: a call that ran them for every query class did not return on the "
                         "GPU; the kernel's own source, run on the host for every shape on this "
                         "batch (test_score_host_model.py), is exact and in bounds, so no cause "
                         "in the source is established and the case stays off the GPU")
def test_packed_int16_all_classes(ctx):
    b = edge_batch(11, EDGE_M, EDGE_N)
    ref, _ = oracle.align_batch(b, SC, mode=0)
    assert_hits_equal(gpu_score(ctx, b, ends=False), ref, ends=False)


def test_config2_full_size_sampled(ctx):
    """The benchmark workload (1M reads, ~4.5M pairs) in one call, checked on a
    seeded sample of 20,000 pairs."""
    b = synth.config2()
    h = gpu_score(ctx, b, ends=False)
    sel = np.sort(np.random.default_rng(1).choice(b.n_pairs, 20_000, replace=False)).astype(np.uint32)
    ref, _ = oracle.align_batch(b, SC, mode=0, sel=sel)
    assert (h["score"][sel] == ref["score"]).all()


def test_traceback_scratch_too_small_marks_pairs(ctx):
    """With a 1 MiB traceback budget the traceback class of queries above 1,024
    bases (strips of 64 lanes x 32 rows, whose code slot for a 1,100-base window
    is about 1.2 MiB) has no room: its pairs get status bit 2 and score -1 and
    are not aligned, while
    the 100-base pairs of the same call align exactly; with the default budget
    every pair aligns."""
    b = edge_batch(51, [100, 1500], [300, 1100], div=0.03)
    ref, rops = oracle.align_batch(b, SC, mode=1)
    m = b.read_len[b.windows["read_id"]]
    small = m <= 100
    sw.sw_ctx_set_option(ctx, sw.SW_OPT_TB_SCRATCH_MB, 1)
    try:
        a, o = gpu_traceback(ctx, b)
    finally:
        sw.sw_ctx_set_option(ctx, sw.SW_OPT_TB_SCRATCH_MB, 2048)
    assert (a["status"][~small] == 4).all() and (a["score"][~small] == -1).all()
    assert (a["n_ops"][~small] == 0).all()
    idx = np.nonzero(small)[0]
    assert_aln_equal(a[idx], o[idx], ref[idx], rops[idx])
    a, o = gpu_traceback(ctx, b)
    assert_aln_equal(a, o, ref, rops)
