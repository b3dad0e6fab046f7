"""Streaming of paired-read chunks (double-buffered copies, filter, SW on the
kept pairs, best hit, traceback): every pass equals the eager filtered pass on
the same chunk, and the traced best hits equal the oracle's alignments."""
import numpy as np
import pytest
import torch

import oracle
import paper_1304_0681_amd as sw
import synth
from paper_1304_0681_amd import train as tr
from paper_1304_0681_amd.stream import HostChunk, StreamAligner

pytestmark = pytest.mark.gpu

SC = (5, -4, -10, -1)
T_MAP = 300          # 150-nt mates: 2 x read length
STRIDE = 64


def test_stream_matches_eager_and_oracle():
    torch.cuda.set_device(0)
    ctx = sw.sw_ctx_create(0)
    try:
        g = synth.rng(synth.BASE_SEED + 95)
        ref = synth.make_reference(g, 2_000_000)
        # filter trained and calibrated on chunks of their own
        b_tr = synth.paired_chunk(synth.BASE_SEED + 96, 4000, ref)
        db_tr = sw.DeviceBatch.from_synth(ctx, b_tr)
        p_tr = tr.plain_scores(ctx, db_tr)
        feat, y = tr.features_and_labels(ctx, db_tr, p_tr)
        mlp, _ = tr.train(ctx, feat, y, steps=300, batch=4096, seed=3)
        b_ca = synth.paired_chunk(synth.BASE_SEED + 97, 4000, ref)
        db_ca = sw.DeviceBatch.from_synth(ctx, b_ca)
        p_ca = tr.plain_scores(ctx, db_ca)
        f_ca, _ = tr.features_and_labels(ctx, db_ca, p_ca)
        z = tr.logits_of(ctx, mlp, f_ca).cpu().numpy()
        thr = tr.calibrate_output(z, p_ca.hits[:, 0].cpu().numpy(), p_ca.best_score.cpu().numpy(),
                                  b_ca.windows["read_id"].astype(np.int64), T_MAP, target=0.999)[:3]
        chunks = [synth.paired_chunk(synth.BASE_SEED + 98 + k, 1500, ref) for k in range(2)]
        # eager filtered pass per chunk (the expected results)
        exp = []
        for b in chunks:
            db = sw.DeviceBatch.from_synth(ctx, b)
            buf = tr.FilterBuffers(b.n_pairs, b.n_reads)
            tr.filtered_pass(ctx, mlp, db, thr[1], thr[2], buf, drop=thr[0])
            torch.cuda.synchronize()
            exp.append((buf.best_score.cpu().numpy(), int(buf.n_sel.item())))
        hcs = [HostChunk(b) for b in chunks]
        st = StreamAligner(ctx, chunks[0].ref, mlp, thr, T_MAP, reads_cap=3000,
                           bases_cap=3000 * 150, pairs_cap=3000 * 16, ops_stride=STRIDE)
        got = {}
        st.run([hcs[0], hcs[1], hcs[0], hcs[1]], lambda i, r: got.__setitem__(i, r))
        assert sorted(got) == [0, 1, 2, 3]
        for i, r in got.items():
            b = chunks[i % 2]
            best, kept = exp[i % 2]
            assert (r["best_score"] == best).all()
            assert r["kept"] == kept
            assert (r["mapped"] == (best >= T_MAP)).all()
            has = r["pair"] >= 0
            assert (has == (best >= 0)).all()
            # best window of a mapped mate: its traceback equals the oracle's
            sel = r["pair"][has].astype(np.uint32)
            ra, rops = oracle.align_batch(b, SC, mode=1, sel=sel, ops_stride=STRIDE)
            assert (ra["score"] == best[has]).all()
            a = r["aln"][has]
            for f in ("score", "read_begin", "read_end", "ref_begin", "ref_end", "n_ops", "status"):
                assert (a[f] == ra[f]).all(), f
            o = r["ops"][has]
            for k in range(len(sel)):
                n = int(ra[k]["n_ops"])
                assert (o[k, :n] == rops[k, :n]).all()
            assert (r["aln"]["status"][~has] == 2).all()     # no window kept: not aligned
        sw.sw_mlp_destroy(ctx, mlp)
    finally:
        sw.sw_ctx_destroy(ctx)


def test_stream_resumes_after_injected_failure(tmp_path):
    """A host hook fails the run before chunk 5 of 6; restarting with the same
    manifest processes only the chunks not yet handed out, and every chunk's
    results equal those of an uninterrupted run, each handed out once."""
    from paper_1304_0681_amd.stream import ChunkManifest
    torch.cuda.set_device(0)
    ctx = sw.sw_ctx_create(0)
    try:
        ref = synth.make_reference(synth.rng(synth.BASE_SEED + 105), 1_000_000)
        b_tr = synth.paired_chunk(synth.BASE_SEED + 106, 3000, ref)
        db_tr = sw.DeviceBatch.from_synth(ctx, b_tr)
        p_tr = tr.plain_scores(ctx, db_tr)
        feat, y = tr.features_and_labels(ctx, db_tr, p_tr)
        mlp, _ = tr.train(ctx, feat, y, steps=200, batch=4096, seed=4)
        thr = (-8.0, -4.0, -4.0)
        chunks = [synth.paired_chunk(synth.BASE_SEED + 107 + k, 1000, ref) for k in range(2)]
        hcs = [HostChunk(b) for b in chunks] * 3
        st = StreamAligner(ctx, chunks[0].ref, mlp, thr, T_MAP, reads_cap=2000,
                           bases_cap=2000 * 150, pairs_cap=2000 * 16, ops_stride=STRIDE)
        full = {}
        st.run(hcs, lambda i, r: full.__setitem__(i, r))
        assert sorted(full) == list(range(6))
        path = str(tmp_path / "stream.json")
        got, calls = {}, []

        def consume(i, r):
            calls.append(i)
            got[i] = r

        def fail_before_5(i):
            if i == 5:
                raise RuntimeError("injected chunk failure")

        with pytest.raises(RuntimeError, match="injected"):
            st.run(hcs, consume, manifest=ChunkManifest(path, 6, key="t"), hook=fail_before_5)
        first = sorted(calls)
        assert 0 < len(first) < 6 and first == list(range(len(first)))
        man = ChunkManifest(path, 6, key="t")
        assert man.pending() == list(range(len(first), 6))
        st.run(hcs, consume, manifest=man)
        assert sorted(calls) == list(range(6))           # each chunk handed out once
        assert man.complete
        for i in range(6):
            for f in ("best_score", "mapped", "pair", "kept"):
                assert np.array_equal(got[i][f], full[i][f]), (i, f)
            assert (got[i]["aln"] == full[i]["aln"]).all()
            assert (got[i]["ops"] == full[i]["ops"]).all()
        sw.sw_mlp_destroy(ctx, mlp)
    finally:
        sw.sw_ctx_destroy(ctx)
