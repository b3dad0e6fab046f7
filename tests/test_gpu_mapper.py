"""Short-read mapping through stages B-E on the GPU (ShortReadMapper) against the
oracle's own chain: stage B records (oracle/stageb_ref.py) for the reads it
maps, and for the rest the oracle seeker's windows (oracle/seeker_ref.py,
oracle/junction_ref.py), their SW scores, the best window and its alignment
and CIGAR (oracle/gotoh.c)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1304_0681_amd as sw
import synth
from oracle import junction_ref as jr
from oracle import seeker_ref as sr
from oracle import stageb_ref as sb
from paper_1304_0681_amd.mapper import STAGE_B, STAGE_E, UNMAPPED, ShortReadMapper, cigar_string
from paper_1304_0681_amd.seeker import KmerIndex
from seeker_inputs import one_edit_reads, reads_from, reference_with_repeats

pytestmark = pytest.mark.gpu

SC = (5, -4, -10, -1)
T_MAP = 200


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = sw.sw_ctx_create(0)
    yield c
    sw.sw_ctx_destroy(c)


def _stage_b_cigar(m, op, pos):
    if op == sb.DEL:
        return f"{pos}M1D{m - pos}M"
    if op == sb.INS:
        return f"{pos}M1I{m - pos - 1}M"
    return f"{m}M"


def test_mapper_against_oracle_chain(ctx):
    ref = reference_with_repeats(70, 600_000, families=10, copies=(2, 8))
    reads = one_edit_reads(71, ref, 1500) + reads_from(72, ref, 2500, p_sub=0.03)[0]
    b = synth.custom(synth.ASCII[ref].tobytes(), [synth.ASCII[q].tobytes() for q in reads], [])
    db = sw.DeviceBatch(ctx, b.ref, b.reads, b.read_off, b.read_len, np.zeros(0, sw.WINDOW_DTYPE))
    idx = KmerIndex(ctx, db.ref2b, db.ref_len, k=15)
    mp = ShortReadMapper(ctx, db, idx, SC, t_map=T_MAP)
    mp.run()
    torch.cuda.synchronize()
    rec, ops, n_ops = mp.results()
    cig = [ops[r, :n_ops[r]] for r in range(len(rec))]

    oidx = sr.build_index_fast(ref, 15)
    n = len(reads)
    want_b = [sb.map_read(q, ref, oidx) for q in reads]
    # the oracle seeker's windows of the reads stage B leaves
    wins = []
    for r, q in enumerate(reads):
        if want_b[r]:
            continue
        c = sr.cals(0, sr.regions(q, oidx), 50, 20)
        wins += [(r, bb, nn, st, 0)
                 for _, bb, nn, st in jr.join_cals(c, 1, len(ref), ext=30, max_gap=5000)]
    win = np.array(wins, dtype=synth.WINDOW_DTYPE)
    ob = synth.Batch(ref=b.ref, reads=b.reads, read_off=b.read_off, read_len=b.read_len,
                     windows=win, truth={})
    res, _ = oracle.align_batch(ob, SC, mode=0)
    bp, bs = oracle.best_per_read(res["score"], win["read_id"].astype(np.int64), n)
    sel = np.nonzero((bp != 0xFFFFFFFF) & (bs >= T_MAP))[0]
    ra, rops = oracle.align_batch(ob, SC, mode=1, sel=bp[sel], ops_stride=64)
    ra_of = {int(r): k for k, r in enumerate(sel)}
    counts = {UNMAPPED: 0, STAGE_B: 0, STAGE_E: 0}
    for r in range(n):
        x = rec[r]
        counts[int(x["source"])] += 1
        if want_b[r]:
            s0, first, last, edits, op, pos = want_b[r][0]
            assert (int(x["source"]), int(x["strand"]), int(x["ref_begin"]), int(x["ref_end"]),
                    int(x["edits"]), int(x["n_records"])) == \
                (STAGE_B, s0, first, last, edits, len(want_b[r])), r
            assert cigar_string(cig[r]) == _stage_b_cigar(len(reads[r]), op, pos), r
        elif r in ra_of:
            a = ra[ra_of[r]]
            w = win[bp[r]]
            assert (int(x["source"]), int(x["strand"]), int(x["score"]), int(x["ref_begin"]),
                    int(x["ref_end"]), int(x["read_begin"]), int(x["read_end"])) == \
                (STAGE_E, int(w["strand"]), int(a["score"]),
                 int(w["ref_begin"]) + int(a["ref_begin"]), int(w["ref_begin"]) + int(a["ref_end"]),
                 int(a["read_begin"]), int(a["read_end"])), r
            k = int(a["n_ops"])
            assert list(cig[r]) == [int(o) for o in rops[ra_of[r], :k]], r
        else:
            assert int(x["source"]) == UNMAPPED, r
    # every source occurs, and stage B maps the one-edit reads
    assert min(counts.values()) > 50, counts
    assert sum(1 for r in range(1500) if rec[r]["source"] == STAGE_B) > 0.97 * 1500
