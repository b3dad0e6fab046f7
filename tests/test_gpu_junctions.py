"""Spliced reads on the GPU: CALs from seed alignments, joined windows, junction
detection and counting, each bit-exact against the oracle
(oracle/junction_ref.py) on the seeded inputs of tests/splice_inputs.py, and
the whole spliced pass (seeds -> CALs -> joined windows -> whole-read
alignment -> junctions) on spliced long reads against the oracle's chain."""
import numpy as np
import pytest
import torch

import oracle
import paper_1304_0681_amd as sw
import synth
from oracle import junction_ref as jr
from paper_1304_0681_amd.splice import LONG_SCORING, SEED_SCORING, SplicedPass
from splice_inputs import ALN_DTYPE, CAL_DTYPE, WINDOW_DTYPE, planted_alignments, random_cals

pytestmark = pytest.mark.gpu

MIN_INTRON = 40


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = sw.sw_ctx_create(0)
    yield c
    sw.sw_ctx_destroy(c)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.uint8).copy()).cuda()


def _cal_tuples(c):
    return [(int(x["read_id"]), int(x["first"]), int(x["last"]), int(x["strand"]), int(x["valid"]))
            for x in c]


def _batch_for(ctx, ref_codes, windows, n_reads):
    """A device batch over `ref_codes` with `windows` and n_reads one-base reads
    (the calls tested here read the windows and the reference only)."""
    reads = [b"A"] * n_reads
    b = synth.custom(synth.ASCII[ref_codes].tobytes(), reads, [])
    return sw.DeviceBatch(ctx, b.ref, b.reads, b.read_off, b.read_len, windows)


def test_seed_cals(ctx):
    g = np.random.default_rng(31)
    n_pairs, n_seeds = 900, 700
    ref = g.integers(0, 4, 200_000).astype(np.uint8)
    win = np.zeros(n_pairs, WINDOW_DTYPE)
    win["read_id"] = g.integers(0, n_seeds, n_pairs)
    win["ref_begin"] = g.integers(0, 199_000, n_pairs)
    win["len"] = g.integers(1, 1000, n_pairs)
    win["strand"] = g.integers(0, 2, n_pairs)
    best = g.integers(0, n_pairs + 50, n_seeds).astype(np.uint32)
    best[:5] = 0xFFFFFFFF
    aln = np.zeros(n_seeds, ALN_DTYPE)
    aln["score"] = g.integers(-1, 300, n_seeds)
    aln["ref_begin"] = g.integers(0, 500, n_seeds)
    aln["ref_end"] = aln["ref_begin"] + g.integers(0, 400, n_seeds)
    neg = aln["score"] <= 0
    aln["ref_begin"][neg] = -1
    aln["ref_end"][neg] = -1
    seed_read = np.sort(g.integers(0, 150, n_seeds)).astype(np.uint32)
    db = _batch_for(ctx, ref, win, n_seeds)
    out = torch.empty(n_seeds * 16, dtype=torch.uint8, device="cuda")
    sw.sw_seed_cals(ctx, db, _dev(best), _dev(aln), _dev(seed_read), n_seeds, 60, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(CAL_DTYPE)
    assert _cal_tuples(got) == jr.seed_cals(win, best, aln, seed_read, 60)
    assert 100 < int(got["valid"].sum()) < n_seeds


@pytest.mark.parametrize("ext,max_gap", [(30, 5000), (0, 1), (100, 0)])
def test_join(ctx, ext, max_gap):
    ref_len, n_reads = 3_000_000, 3000
    cals = random_cals(40 + ext, n_reads, ref_len, ext, max_gap)
    n = len(cals)
    out = torch.empty(n * 12, dtype=torch.uint8, device="cuda")
    n_out = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    sw.sw_join_cals(ctx, _dev(cals), n, n_reads, ref_len, ext, max_gap, out, n_out)
    torch.cuda.synchronize()
    k = int(n_out.item())
    w = out.cpu().numpy().view(WINDOW_DTYPE)[:k]
    got = [(int(x["read_id"]), int(x["ref_begin"]), int(x["len"]), int(x["strand"])) for x in w]
    ref = jr.join_cals(_cal_tuples(cals), n_reads, ref_len, ext=ext, max_gap=max_gap)
    assert got == ref
    assert (w["flags"] == 0).all() and k > 1500


def test_join_edge_cases(ctx):
    n_out = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    out = torch.empty(64 * 12, dtype=torch.uint8, device="cuda")
    # no CALs at all
    sw.sw_join_cals(ctx, None, 0, 10, 1000, 30, 100, None, n_out)
    torch.cuda.synchronize()
    assert int(n_out.item()) == 0
    # only invalid CALs, and one read with a single CAL at both reference ends
    c = np.zeros(6, CAL_DTYPE)
    c["read_id"] = [0, 0, 1, 2, 2, 5]
    c["first"] = [10, 50, 0, 990, 995, 3]
    c["last"] = [20, 40, 5, 999, 999, 4]
    c["valid"] = [0, 1, 1, 1, 1, 1]         # (0, 50..40) has first > last; read 5 >= n_reads
    n_out.fill_(-1)
    sw.sw_join_cals(ctx, _dev(c), 6, 3, 1000, 30, 100, out, n_out)
    torch.cuda.synchronize()
    k = int(n_out.item())
    w = out.cpu().numpy().view(WINDOW_DTYPE)[:k]
    got = [(int(x["read_id"]), int(x["ref_begin"]), int(x["len"]), int(x["strand"])) for x in w]
    assert got == jr.join_cals(_cal_tuples(c), 3, 1000, ext=30, max_gap=100) == \
        [(1, 0, 36, 0), (2, 960, 40, 0)]


def _oracle_detect(ref, win, aln, ops, min_score, ids=None):
    want_ops, want_nj, lists = ops.copy(), [], []
    for k in range(len(aln)):
        a = aln[k]
        p = k if ids is None else int(ids[k])
        if a["status"] or a["score"] < max(min_score, 1) or p >= len(win):
            want_nj.append(0)
            continue
        w = win[p]
        t = ref[int(w["ref_begin"]):int(w["ref_begin"]) + int(w["len"])]
        n = int(a["n_ops"])
        new, js = jr.detect(t, ops[k, :n], int(a["ref_begin"]), MIN_INTRON, int(w["ref_begin"]))
        want_ops[k, :n] = new
        want_nj.append(len(js))
        lists.append(js)
    return want_ops, np.array(want_nj), jr.count(lists)


def _listed(ctx, keys, counts, cap):
    out = torch.empty(cap * 24, dtype=torch.uint8, device="cuda")
    n = torch.zeros(1, dtype=torch.int32, device="cuda")
    sw.sw_list_junctions(ctx, keys, counts, cap, out, cap, n)
    torch.cuda.synchronize()
    j = sw.junctions_to_numpy(out)[:int(n.item())]
    return {(int(r["start"]), int(r["end"]), int(r["strand"])): int(r["count"]) for r in j}


def test_detect_count_accumulate(ctx):
    n_aln, stride, cap = 4000, 48, 1 << 14
    ref, win, aln, ops = planted_alignments(51, n_aln, MIN_INTRON, stride, 30)
    db = _batch_for(ctx, ref, win, n_aln)
    d_ops = _dev(ops)
    keys = torch.empty(cap, dtype=torch.int64, device="cuda")
    counts = torch.empty(cap, dtype=torch.int32, device="cuda")
    nj = torch.empty(n_aln, dtype=torch.int32, device="cuda")
    dropped = torch.zeros(1, dtype=torch.int32, device="cuda")
    ids = _dev(np.arange(n_aln, dtype=np.uint32))
    sw.sw_junctions_clear(ctx, keys, counts, cap)
    sw.sw_detect_junctions(ctx, db, ids, n_aln, _dev(aln), d_ops, stride, 30, MIN_INTRON, keys,
                           counts, cap, nj, dropped)
    torch.cuda.synchronize()
    want_ops, want_nj, want = _oracle_detect(ref, win, aln, ops, 30)
    assert (d_ops.cpu().numpy().view(np.uint32).reshape(n_aln, stride) == want_ops).all()
    assert (nj.cpu().numpy() == want_nj).all()
    assert int(dropped.item()) == 0
    assert _listed(ctx, keys, counts, cap) == dict(want)
    assert sum(want.values()) > 2000 and {s for _, _, s in want} == {0, 1}
    # the same alignments again (from their original ops) double every count
    sw.sw_detect_junctions(ctx, db, ids, n_aln, _dev(aln), _dev(ops), stride, 30, MIN_INTRON,
                           keys, counts, cap, None, None)
    torch.cuda.synchronize()
    assert _listed(ctx, keys, counts, cap) == {k: 2 * v for k, v in want.items()}
    # a table too small: what fits is exact, the rest is counted as dropped
    small = 64
    ks = torch.empty(small, dtype=torch.int64, device="cuda")
    cs = torch.empty(small, dtype=torch.int32, device="cuda")
    sw.sw_junctions_clear(ctx, ks, cs, small)
    dropped.zero_()
    sw.sw_detect_junctions(ctx, db, ids, n_aln, _dev(aln), _dev(ops), stride, 30, MIN_INTRON, ks,
                           cs, small, None, dropped)
    torch.cuda.synchronize()
    tab = _listed(ctx, ks, cs, small)
    assert len(tab) == small and all(want[k] == v for k, v in tab.items())
    assert int(dropped.item()) == sum(want.values()) - sum(tab.values())


def test_detect_argument_errors(ctx):
    ref, win, aln, ops = planted_alignments(52, 4, MIN_INTRON)
    db = _batch_for(ctx, ref, win, 4)
    keys = torch.zeros(8, dtype=torch.int64, device="cuda")
    counts = torch.zeros(8, dtype=torch.int32, device="cuda")
    ids = _dev(np.arange(4, dtype=np.uint32))
    with pytest.raises(sw.SwError):      # capacity not a power of two
        sw.sw_junctions_clear(ctx, keys, counts, 6)
    with pytest.raises(sw.SwError):      # min_intron below 4
        sw.sw_detect_junctions(ctx, db, ids, 4, _dev(aln), _dev(ops), 48, 30, 3, keys, counts, 8)


@pytest.fixture(scope="module")
def spliced_long():
    long_b, seed_b, truth = synth.spliced_long(n_reads=240, ref_len=1_500_000,
                                               seed=synth.BASE_SEED + 61)
    return long_b, seed_b, truth


def _oracle_chain(long_b, seed_b, truth, p, every_seed_has_windows=True):
    """The spliced pass computed by the oracle alone."""
    ns = seed_b.n_reads
    res, _ = oracle.align_batch(seed_b, SEED_SCORING, mode=0)
    rid = seed_b.windows["read_id"].astype(np.int64)
    best = np.full(ns, -1, np.int64)
    np.maximum.at(best, rid, res["score"].astype(np.int64))
    bp = np.full(ns, 0xFFFFFFFF, np.int64)
    idx = np.nonzero(res["score"] == best[rid])[0][::-1]
    bp[rid[idx]] = idx
    bp = bp.astype(np.uint32)
    if every_seed_has_windows:
        assert (bp != 0xFFFFFFFF).all()
    sa = np.zeros(ns, oracle.RESULT_DTYPE)
    sa["score"] = -1
    sa["ref_begin"] = sa["ref_end"] = -1
    with_win = bp != 0xFFFFFFFF
    if with_win.any():
        sa[with_win] = oracle.align_batch(seed_b, SEED_SCORING, mode=1, sel=bp[with_win])[0]
    cals = jr.seed_cals(seed_b.windows, bp, sa, truth["seed_read"], p["min_seed_score"])
    joined = jr.join_cals(cals, long_b.n_reads, len(long_b.ref), ext=p["ext"],
                          max_gap=p["max_gap"])
    win = np.array([(r, b, n, s, 0) for r, b, n, s in joined], dtype=synth.WINDOW_DTYPE)
    lb = synth.Batch(ref=long_b.ref, reads=long_b.reads, read_off=long_b.read_off,
                     read_len=long_b.read_len, windows=win, truth={})
    lres, _ = oracle.align_batch(lb, LONG_SCORING, mode=0)
    nl = long_b.n_reads
    lrid = win["read_id"].astype(np.int64)
    lbest = np.full(nl, -1, np.int64)
    np.maximum.at(lbest, lrid, lres["score"].astype(np.int64))
    lbp = np.full(nl, 0xFFFFFFFF, np.int64)
    lidx = np.nonzero(lres["score"] == lbest[lrid])[0][::-1]
    lbp[lrid[lidx]] = lidx
    lbp = lbp.astype(np.uint32)
    has = lbp != 0xFFFFFFFF
    la = np.zeros(nl, oracle.RESULT_DTYPE)
    la["score"] = -1
    lops = np.zeros((nl, p["ops_stride"]), np.uint32)
    if has.any():
        a, o = oracle.align_batch(lb, LONG_SCORING, mode=1, sel=lbp[has],
                                  ops_stride=p["ops_stride"])
        la[has] = a
        lops[has] = o
    ref_codes = jr.codes_of(long_b.ref.tobytes())
    lists, det_ops = [], lops.copy()
    for r in np.nonzero(has)[0]:
        a = la[r]
        if a["score"] < p["min_score"] or a["status"]:
            continue
        w = win[lbp[r]]
        t = ref_codes[int(w["ref_begin"]):int(w["ref_begin"]) + int(w["len"])]
        n = int(a["n_ops"])
        new, js = jr.detect(t, lops[r, :n], int(a["ref_begin"]), p["min_intron"],
                            int(w["ref_begin"]))
        det_ops[r, :n] = new
        lists.append(js)
    return dict(bp=bp, cals=cals, joined=joined, lbp=lbp, lbest=lbest, la=la, lops=det_ops,
                table=dict(jr.count(lists)))


def test_spliced_pass_vs_oracle(ctx, spliced_long):
    long_b, seed_b, truth = spliced_long
    p = dict(min_seed_score=100, ext=30, max_gap=5000, min_score=100, min_intron=MIN_INTRON,
             ops_stride=256)
    want = _oracle_chain(long_b, seed_b, truth, p)
    seed_db = sw.DeviceBatch.from_synth(ctx, seed_b)
    long_db = sw.DeviceBatch(ctx, None, long_b.reads, long_b.read_off, long_b.read_len,
                             np.zeros(0, sw.WINDOW_DTYPE), ref2b=(seed_db.ref2b, seed_db.ref_len))
    sp = SplicedPass(ctx, seed_db, truth["seed_read"], long_db, min_seed_score=100, ext=30,
                     max_gap=5000, min_score=100, min_intron=MIN_INTRON, table_capacity=1 << 16,
                     ops_stride=256, tb_scratch_mb=4096)
    sp.run()
    torch.cuda.synchronize()
    # seeds and their CALs
    assert (sp.seeds.best_pair.cpu().numpy().view(np.uint32) == want["bp"]).all()
    got_cals = sp.cals.cpu().numpy().view(CAL_DTYPE)
    assert _cal_tuples(got_cals) == want["cals"]
    # joined windows
    w = sp.windows()
    assert [(int(x["read_id"]), int(x["ref_begin"]), int(x["len"]), int(x["strand"]))
            for x in w] == want["joined"]
    assert len(w) >= long_b.n_reads and int(w["len"].max()) > 2000
    # whole-read alignments
    bp, bs, aln, ops, nj = sp.results()
    assert (bp == want["lbp"]).all()
    assert (bs == want["lbest"]).all()
    has = want["lbp"] != 0xFFFFFFFF
    for f in ("score", "read_begin", "read_end", "ref_begin", "ref_end", "n_ops", "status"):
        assert (aln[f][has] == want["la"][f][has]).all(), f
    for r in np.nonzero(has)[0]:
        n = int(aln["n_ops"][r])
        assert (ops[r, :n] == want["lops"][r, :n]).all(), r
    # junctions
    got = {(int(j["start"]), int(j["end"]), int(j["strand"])): int(j["count"])
           for j in sp.junctions()}
    assert got == want["table"]
    truth_j = {(int(a), int(b), int(s)) for a, b, s in truth["junctions"]}
    found = set(got) & truth_j
    assert len(found) >= 0.8 * len(truth_j), (len(found), len(truth_j))
    assert len(set(got) - truth_j) <= 0.05 * len(got)


def test_spliced_pass_from_seeker_vs_oracle(ctx, spliced_long):
    """The same spliced reads with the seeds' windows found on the device (k = 15
    index, regions, CALs and joining of the seeds) instead of the generator's:
    the seeds' windows equal the oracle seeker's, and every later step equals
    the oracle's chain run on those windows."""
    from oracle import seeker_ref as sr
    from paper_1304_0681_amd.seeker import KmerIndex
    from paper_1304_0681_amd.splice import SeekerSplicedPass
    long_b, seed_b, truth = spliced_long
    p = dict(min_seed_score=100, ext=30, max_gap=5000, min_score=100, min_intron=MIN_INTRON,
             ops_stride=256)
    ref = jr.codes_of(long_b.ref.tobytes())
    oidx = sr.build_index_fast(ref, 15)
    ns = seed_b.n_reads
    ocals = []
    for s in range(ns):
        c = sr.cals(s, sr.regions(jr.codes_of(seed_b.read(s)), oidx, 15, 12, 7, 64), 50, 20)
        ocals += c + [(s, 0, 0, 0, 0)] * (sw.SW_SEEKER_MAX_CALS - len(c))
    jw = jr.join_cals(ocals, ns, len(ref), ext=30, max_gap=5000)
    swin = np.array([(r, b, n, st, 0) for r, b, n, st in jw], dtype=synth.WINDOW_DTYPE)
    seed_w = synth.Batch(ref=seed_b.ref, reads=seed_b.reads, read_off=seed_b.read_off,
                         read_len=seed_b.read_len, windows=swin, truth={})
    want = _oracle_chain(long_b, seed_w, truth, p, every_seed_has_windows=False)

    seed_db = sw.DeviceBatch(ctx, seed_b.ref, seed_b.reads, seed_b.read_off, seed_b.read_len,
                             np.zeros(0, sw.WINDOW_DTYPE))
    idx = KmerIndex(ctx, seed_db.ref2b, seed_db.ref_len, k=15)
    long_db = sw.DeviceBatch(ctx, None, long_b.reads, long_b.read_off, long_b.read_len,
                             np.zeros(0, sw.WINDOW_DTYPE), ref2b=(seed_db.ref2b, seed_db.ref_len))
    sp = SeekerSplicedPass(ctx, seed_db, idx, truth["seed_read"], long_db, max_occ=64,
                           merge_gap=50, min_len=20, seed_ext=30, seed_max_gap=5000,
                           min_seed_score=100, ext=30, max_gap=5000, min_score=100,
                           min_intron=MIN_INTRON, table_capacity=1 << 16, ops_stride=256,
                           tb_scratch_mb=4096)
    sp.run()
    torch.cuda.synchronize()
    gw = sp.seeker.windows()
    assert [(int(x["read_id"]), int(x["ref_begin"]), int(x["len"]), int(x["strand"]))
            for x in gw] == jw
    assert len(jw) >= 0.9 * ns
    assert (sp.seeds.best_pair.cpu().numpy().view(np.uint32) == want["bp"]).all()
    assert _cal_tuples(sp.cals.cpu().numpy().view(CAL_DTYPE)) == want["cals"]
    w = sp.windows()
    assert [(int(x["read_id"]), int(x["ref_begin"]), int(x["len"]), int(x["strand"]))
            for x in w] == want["joined"]
    bp, bs, aln, ops, nj = sp.results()
    assert (bp == want["lbp"]).all() and (bs == want["lbest"]).all()
    has = want["lbp"] != 0xFFFFFFFF
    for f in ("score", "read_begin", "read_end", "ref_begin", "ref_end", "n_ops", "status"):
        assert (aln[f][has] == want["la"][f][has]).all(), f
    for r in np.nonzero(has)[0]:
        n = int(aln["n_ops"][r])
        assert (ops[r, :n] == want["lops"][r, :n]).all(), r
    got = {(int(j["start"]), int(j["end"]), int(j["strand"])): int(j["count"])
           for j in sp.junctions()}
    assert got == want["table"]
    truth_j = {(int(a), int(b), int(s)) for a, b, s in truth["junctions"]}
    assert len(set(got) & truth_j) >= 0.8 * len(truth_j), (len(set(got) & truth_j), len(truth_j))


def _sole_expected(win, n_valid, read_off, read_len, reads_len):
    """sw_sole_windows by its definition: a pair scores when it lies below the
    device count, its read id is in range and the read lies inside the packed
    reads; a read with exactly one scoring pair has it as sole pair, the
    scoring pairs of the other reads form the list, in pair order."""
    n_reads = len(read_len)
    scoring = [p < n_valid and int(w["read_id"]) < n_reads and
               int(read_off[int(w["read_id"])]) + int(read_len[int(w["read_id"])]) <= reads_len
               for p, w in enumerate(win)]
    per = {}
    for p, ok in enumerate(scoring):
        if ok:
            per.setdefault(int(win[p]["read_id"]), []).append(p)
    sole = np.full(n_reads, 0xFFFFFFFF, np.uint32)
    for r, ps in per.items():
        if len(ps) == 1:
            sole[r] = ps[0]
    ids = [p for p, ok in enumerate(scoring) if ok and len(per[int(win[p]["read_id"])]) >= 2]
    return sole, np.array(ids, np.uint32)


def test_sole_windows_and_merge_equal_best_over_all_pairs(ctx):
    """Edge cases of the single-window split: reads with no, one and several
    windows (interleaved with other reads' windows), empty and clipped windows,
    an empty read, read ids out of range, a read outside the packed reads, and
    a device count that cuts the list; then score -> best -> merge over the
    compacted list against sw_best_per_read over the whole batch and against
    the oracle's best pairs."""
    rng = np.random.default_rng(91)
    ref = rng.integers(0, 4, 6000).astype(np.uint8)
    lens = [60, 80, 70, 50, 90, 0, 75, 40, 65, 30]
    planted = {1: 1250, 6: 4550}     # reads copied from inside their second window
    reads, off = [], []
    o = 0
    for r, n in enumerate(lens):
        q = ref[planted[r]:planted[r] + n] if r in planted else rng.integers(0, 4, n).astype(np.uint8)
        reads.append(synth.ASCII[q].tobytes())
        off.append(o)
        o += n
    read_off = np.array(off, np.uint64)
    read_len = np.array(lens, np.uint16)
    read_off[9] = o - 10           # read 9 (30 bases) lies partly outside the packed reads
    W = [  # (read, ref_begin, len, strand)
        (0, 100, 300, 1),                          # read 0: one window
        (1, 500, 250, 0), (3, 900, 0, 0),          # read 3: one empty window
        (1, 1200, 300, 0), (99, 10, 100, 0),       # read id out of range
        (4, 5900, 300, 1), (4, 2000, 200, 0),      # read 4: one window clipped at the end
        (5, 3000, 200, 0),                         # read 5: empty read, one window
        (1, 3500, 280, 1), (6, 4000, 300, 0),      # read 1: three windows, interleaved
        (6, 4500, 250, 0), (9, 100, 200, 0),       # read 9: outside the packed reads
        (8, 6500, 100, 0),                         # read 8: starts past the reference
        (7, 200, 300, 0), (7, 700, 300, 1),        # read 7: its second window is cut by the count
    ]
    win = np.zeros(len(W), sw.WINDOW_DTYPE)
    for k, w in enumerate(W):
        win[k] = w + (0,)
    ascii_reads = np.frombuffer(b"".join(reads), np.uint8)
    ref_ascii = synth.ASCII[ref]
    db = sw.DeviceBatch(ctx, ref_ascii, ascii_reads, read_off, read_len, win)
    n_valid = len(W) - 1
    d_n = torch.tensor([n_valid], dtype=torch.int32, device="cuda")
    full = db.view(db.win, len(W), d_n)
    nr = len(lens)
    sole = torch.full((nr,), -7, dtype=torch.int32, device="cuda")
    mwin = torch.zeros(len(W) * 12, dtype=torch.uint8, device="cuda")
    mids = torch.full((len(W),), -7, dtype=torch.int32, device="cuda")
    n_out = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    sw.sw_sole_windows(ctx, full, sole, mwin, mids, n_out)
    torch.cuda.synchronize()
    want_sole, want_ids = _sole_expected(win, n_valid, read_off, read_len, len(ascii_reads))
    assert (sole.cpu().numpy().view(np.uint32) == want_sole).all()
    k = int(n_out.item())
    assert k == len(want_ids) == 7
    assert (mids.cpu().numpy().view(np.uint32)[:k] == want_ids).all()
    assert (mwin.cpu().numpy().view(sw.WINDOW_DTYPE)[:k] == win[want_ids]).all()
    assert list(want_sole[[0, 3, 5, 7, 8]]) == [0, 2, 7, 13, 12]
    assert (want_sole[[1, 2, 4, 6, 9]] == 0xFFFFFFFF).all()
    # score -> best over the list -> merge, against best over all pairs
    hits_all = torch.empty((len(W), 3), dtype=torch.int32, device="cuda")
    bp_all = torch.empty(nr, dtype=torch.int32, device="cuda")
    bs_all = torch.empty(nr, dtype=torch.int32, device="cuda")
    sw.sw_batch_score(ctx, full, SEED_SCORING, 0, hits_all)
    sw.sw_best_per_read(ctx, full, hits_all, 0, bp_all, bs_all)
    mv = db.view(mwin, len(W), n_out)
    hits = torch.empty((len(W), 3), dtype=torch.int32, device="cuda")
    sub = torch.empty(nr, dtype=torch.int32, device="cuda")
    sub_s = torch.empty(nr, dtype=torch.int32, device="cuda")
    sw.sw_batch_score(ctx, mv, SEED_SCORING, 0, hits)
    sw.sw_best_per_read(ctx, mv, hits, 0, sub, sub_s)
    best = torch.full((nr,), -7, dtype=torch.int32, device="cuda")
    sw.sw_merge_best(ctx, nr, sole, sub, mids, len(W), best)
    torch.cuda.synchronize()
    got = best.cpu().numpy().view(np.uint32)
    assert (got == bp_all.cpu().numpy().view(np.uint32)).all()
    # the oracle's best pairs over the scoring pairs below the count
    ok = np.array([p for p in range(n_valid) if int(win[p]["read_id"]) < nr and p != 11])
    ob = synth.Batch(ref=ref_ascii, reads=ascii_reads, read_off=read_off, read_len=read_len,
                     windows=win[ok], truth={})
    res, _ = oracle.align_batch(ob, SEED_SCORING, mode=0)
    ep, _ = oracle.best_per_read(res["score"], win["read_id"][ok].astype(np.int64), nr)
    ep = np.where(ep != 0xFFFFFFFF, ok[np.minimum(ep, len(ok) - 1)], 0xFFFFFFFF).astype(np.uint32)
    assert (got == ep).all()
    assert got[1] == 3 and got[6] == 10          # the planted windows win
    # empty batches: no pairs, and no reads
    sw.sw_sole_windows(ctx, db.view(mwin, 0), sole, mwin, mids, n_out)
    torch.cuda.synchronize()
    assert int(n_out.item()) == 0 and (sole.cpu().numpy() == -1).all()
    nb = db.view(db.win, len(W))
    nb.c.n_reads = 0
    n_out.fill_(-7)
    sw.sw_sole_windows(ctx, nb, sole, mwin, mids, n_out)
    torch.cuda.synchronize()
    assert int(n_out.item()) == 0
