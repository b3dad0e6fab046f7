"""Region and CAL seekers on the GPU: the k-mer index (k = 10 in full, k = 15
by counts, bucket membership and a permutation check), the regions of every
read in exact order, the CALs, and the joined windows, against the oracle
(oracle/seeker_ref.py, oracle/junction_ref.py); then the windows found this
way scored and the best window checked against the reads' origins."""
import numpy as np
import pytest
import torch

import oracle
import paper_1304_0681_amd as sw
import synth
from oracle import junction_ref as jr
from oracle import seeker_ref as sr
from paper_1304_0681_amd.seeker import CandidateSeeker, KmerIndex
from seeker_inputs import reads_from, reference_with_repeats

pytestmark = pytest.mark.gpu

SC = (5, -4, -10, -1)


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = sw.sw_ctx_create(0)
    yield c
    sw.sw_ctx_destroy(c)


def _db(ctx, ref, reads):
    b = synth.custom(synth.ASCII[ref].tobytes(), [synth.ASCII[q].tobytes() for q in reads], [])
    return sw.DeviceBatch(ctx, b.ref, b.reads, b.read_off, b.read_len, b.windows)


def test_index_k10_exact(ctx):
    ref = reference_with_repeats(61, 300_000)
    db = _db(ctx, ref, [ref[:20]])
    idx = KmerIndex(ctx, db.ref2b, db.ref_len, k=10)
    starts, pos = idx.arrays()
    torch.cuda.synchronize()
    st = starts.cpu().numpy().view(np.uint32).astype(np.int64)
    p = pos.cpu().numpy().view(np.uint32)
    want = sr.build_index_fast(ref, 10)
    assert st[-1] == len(ref) - 9 and (np.diff(st) >= 0).all()
    got = {c: sorted(p[st[c]:st[c + 1]].tolist()) for c in np.nonzero(np.diff(st))[0]}
    assert got == want


def test_index_k15_counts_and_membership(ctx):
    ref = reference_with_repeats(62, 2_000_000, families=20)
    db = _db(ctx, ref, [ref[:20]])
    idx = KmerIndex(ctx, db.ref2b, db.ref_len, k=15)
    starts, pos = idx.arrays()
    torch.cuda.synchronize()
    n_pos = len(ref) - 14
    assert int(starts[-1].item()) == n_pos
    assert bool((starts[1:] >= starts[:-1]).all().item())
    codes = sr.position_codes(ref, 15)
    uniq, cnt = np.unique(codes, return_counts=True)
    u = torch.from_numpy(uniq).cuda()
    got_cnt = (starts[u + 1].long() - starts[u].long()).cpu().numpy()
    assert (got_cnt == cnt).all() and int(cnt.sum()) == n_pos
    # every slot's position spells its bucket's code, and positions are a permutation
    pl = pos.long()
    assert bool((torch.sort(pl).values == torch.arange(n_pos, device="cuda")).all().item())
    bucket = torch.repeat_interleave(u, torch.from_numpy(cnt).cuda())
    assert bool((torch.from_numpy(codes).cuda()[pl] == bucket).all().item())


@pytest.fixture(scope="module")
def seeded(ctx):
    ref = reference_with_repeats(63, 1_000_000, families=10, copies=(2, 8))
    reads, origins, strands = reads_from(64, ref, 6000)
    db = _db(ctx, ref, reads)
    idx = KmerIndex(ctx, db.ref2b, db.ref_len, k=15)
    cs = CandidateSeeker(ctx, db, idx, max_occ=40, merge_gap=50, min_len=20, ext=30,
                         max_gap=5000)
    cs.run()
    torch.cuda.synchronize()
    oidx = sr.build_index_fast(ref, 15)
    return ref, reads, origins, strands, db, cs, oidx


def test_regions_exact(seeded):
    ref, reads, origins, strands, db, cs, oidx = seeded
    regs, end = cs.region_list()
    b = 0
    for r, q in enumerate(reads):
        want = sr.regions(q, oidx, 15, 12, 7, 40)
        e = int(end[r])
        got = [(int(x["strand"]), int(x["first"]), int(x["first"]) + 14, int(x["read_pos"]))
               for x in regs[b:e]]
        assert got == want, r
        b = e
    assert b > 50_000


def _oracle_cals(reads, oidx):
    out = []
    for r, q in enumerate(reads):
        c = sr.cals(r, sr.regions(q, oidx, 15, 12, 7, 40), 50, 20)
        out += c + [(r, 0, 0, 0, 0)] * (sw.SW_SEEKER_MAX_CALS - len(c))
    return out


def test_cals_and_windows_exact(seeded):
    ref, reads, origins, strands, db, cs, oidx = seeded
    got = cs.cals.cpu().numpy().view(jr_dtype())
    want = _oracle_cals(reads, oidx)
    assert [(int(c["read_id"]), int(c["first"]), int(c["last"]), int(c["strand"]),
             int(c["valid"])) for c in got] == want
    w = cs.windows()
    jw = jr.join_cals(want, len(reads), len(ref), ext=30, max_gap=5000)
    assert [(int(x["read_id"]), int(x["ref_begin"]), int(x["len"]), int(x["strand"]))
            for x in w] == jw


def jr_dtype():
    return np.dtype([("read_id", "<u4"), ("first", "<u4"), ("last", "<u4"), ("strand", "u1"),
                     ("valid", "u1"), ("reserved", "<u2")])


def test_found_windows_hold_the_origins(ctx, seeded):
    """Score the windows the seeker found: every read copied from the reference
    (100 nt or longer) has a window on its own strand over at least half of its
    origin span, and its best window scores at least 2 per base."""
    ref, reads, origins, strands, db, cs, oidx = seeded
    hits = torch.empty((cs.n_cals, 3), dtype=torch.int32, device="cuda")
    bp = torch.empty(len(reads), dtype=torch.int32, device="cuda")
    bs = torch.empty(len(reads), dtype=torch.int32, device="cuda")
    sw.sw_batch_score(ctx, cs.view, SC, 0, hits)
    sw.sw_best_per_read(ctx, cs.view, hits, 0, bp, bs)
    torch.cuda.synchronize()
    w = cs.windows()
    bsn = bs.cpu().numpy()
    lens = np.array([len(q) for q in reads])
    by_read = {}
    for x in w:
        by_read.setdefault(int(x["read_id"]), []).append(x)
    covered = mapped = n = 0
    for r in range(len(reads)):
        if origins[r] < 0 or lens[r] < 100:
            continue
        n += 1
        o0, o1 = origins[r], origins[r] + lens[r]
        covered += any(int(x["strand"]) == strands[r] and
                       min(o1, int(x["ref_begin"]) + int(x["len"])) - max(o0, int(x["ref_begin"]))
                       >= 0.5 * lens[r] for x in by_read.get(r, []))
        mapped += bsn[r] >= 2 * lens[r]
    assert covered >= 0.995 * n and mapped >= 0.97 * n, (covered, mapped, n)


def test_stage_b_exact_and_skip(ctx):
    """Stage B on reads one edit or less from the reference (both strands, at
    the reference ends) and on mutated and random reads: every read's records
    equal the oracle's, and the CAL seeker then leaves the mapped reads out."""
    from oracle import stageb_ref as sb
    from seeker_inputs import one_edit_reads
    ref = reference_with_repeats(65, 800_000, families=10, copies=(2, 8))
    reads = one_edit_reads(66, ref, 3000) + reads_from(67, ref, 3000)[0]
    db = _db(ctx, ref, reads)
    idx = KmerIndex(ctx, db.ref2b, db.ref_len, k=15)
    cs = CandidateSeeker(ctx, db, idx, max_occ=40, stage_b=True)
    cs.run()
    torch.cuda.synchronize()
    recs, n_maps = cs.stage_b_maps()
    oidx = sr.build_index_fast(ref, 15)
    kinds = set()
    for r, q in enumerate(reads):
        want = sb.map_read(q, ref, oidx, 15, 12, 7, 40)
        n = int(n_maps[r])
        got = [(int(x["strand"]), int(x["first"]), int(x["last"]), int(x["edits"]), int(x["op"]),
                int(x["edit_pos"])) for x in recs[r, :n]]
        assert got == want, r
        assert (recs[r, n:]["first"] == 0).all() and (recs[r, n:]["edit_pos"] == 0).all()
        kinds |= {w[4] for w in want}
    assert kinds == {sb.EXACT, sb.SUBST, sb.DEL, sb.INS}
    assert (n_maps[:3000] > 0).mean() > 0.97
    got = cs.cals.cpu().numpy().view(jr_dtype())
    for r in range(len(reads)):
        row = got[r * sw.SW_SEEKER_MAX_CALS:(r + 1) * sw.SW_SEEKER_MAX_CALS]
        if n_maps[r]:
            assert not row["valid"].any()
        else:
            want = sr.cals(r, sr.regions(reads[r], oidx, 15, 12, 7, 40), 50, 20)
            assert [(int(c["read_id"]), int(c["first"]), int(c["last"]), int(c["strand"]), 1)
                    for c in row if c["valid"]] == want


def test_config2_reads_fifty_thousand(ctx):
    """50,000 reads of the benchmark workload (4 Mb GC-40 % reference, 1 %
    substitutions, 0.1 % indels, 5 % random reads) through the k = 15 index:
    every read's regions, CALs and stage B records equal the oracle's."""
    from oracle import stageb_ref as sb
    b = synth.config2(n_reads=50_000)
    db = sw.DeviceBatch(ctx, b.ref, b.reads, b.read_off, b.read_len, np.zeros(0, sw.WINDOW_DTYPE))
    idx = KmerIndex(ctx, db.ref2b, db.ref_len, k=15)
    cs = CandidateSeeker(ctx, db, idx, stage_b=True)
    cs.run()
    torch.cuda.synchronize()
    regs, end = cs.region_list()
    recs, n_maps = cs.stage_b_maps()
    cals = cs.cals.cpu().numpy().view(jr_dtype())
    ref = jr.codes_of(b.ref.tobytes())
    oidx = sr.build_index_fast(ref, 15)
    reads = [jr.codes_of(b.read(r)) for r in range(b.n_reads)]
    bgn = 0
    for r, q in enumerate(reads):
        want = sr.regions(q, oidx)
        e = int(end[r])
        got = [(int(x["strand"]), int(x["first"]), int(x["first"]) + 14, int(x["read_pos"]))
               for x in regs[bgn:e]]
        assert got == want, r
        bgn = e
        wb = sb.map_read(q, ref, oidx)
        n = int(n_maps[r])
        assert [(int(x["strand"]), int(x["first"]), int(x["last"]), int(x["edits"]),
                 int(x["op"]), int(x["edit_pos"])) for x in recs[r, :n]] == wb, r
        row = cals[r * sw.SW_SEEKER_MAX_CALS:(r + 1) * sw.SW_SEEKER_MAX_CALS]
        wc = [] if n else sr.cals(r, want, 50, 20)
        assert [(int(c["read_id"]), int(c["first"]), int(c["last"]), int(c["strand"]), 1)
                for c in row if c["valid"]] == wc, r
    assert 0.55 < (n_maps > 0).mean() < 0.75


def test_seed_regions_refuses_an_index_too_small_for_k(ctx):
    """An index built with k = 10 (or a size below what k = 15 needs) is refused
    for seeds of 15 bases before any kernel runs."""
    ref = reference_with_repeats(68, 200_000)
    db = _db(ctx, ref, [ref[1000:1100]])
    idx10 = KmerIndex(ctx, db.ref2b, db.ref_len, k=10)
    regions = torch.empty(64 * 8, dtype=torch.uint8, device="cuda")
    end = torch.empty(1, dtype=torch.int64, device="cuda")
    with pytest.raises(sw.SwError) as e:
        sw.sw_seed_regions(ctx, db, idx10.buf, (15, 12, 7, 64), regions, 64, end)
    assert e.value.status == sw.SW_E_RANGE
    idx15 = KmerIndex(ctx, db.ref2b, db.ref_len, k=15)
    with pytest.raises(sw.SwError) as e:
        sw.sw_seed_regions(ctx, db, idx15.buf, (15, 12, 7, 64), regions, 64, end,
                           index_bytes=idx15.nbytes - 4)
    assert e.value.status == sw.SW_E_RANGE
    sw.sw_seed_regions(ctx, db, idx15.buf, (15, 12, 7, 64), regions, 64, end)
    torch.cuda.synchronize()
    assert int(end[0].item()) > 0
