"""Autotuning of the score kernels: the choice is a valid tile for every class,
results stay bit-exact, and the tuned context is used by later calls."""
import numpy as np
import pytest
import torch

import oracle
import paper_1304_0681_amd as sw
import synth

pytestmark = pytest.mark.gpu

SC = (5, -4, -10, -1)


def test_autotune_choice_and_parity():
    torch.cuda.set_device(0)
    ctx = sw.sw_ctx_create(0)
    try:
        b = synth.config2(n_reads=30_000, seed=synth.BASE_SEED + 81)
        sample = synth.config2(n_reads=30_000, seed=synth.BASE_SEED + 82)
        db_s = sw.DeviceBatch.from_synth(ctx, sample)
        for flags in (0, sw.SW_WANT_ENDS):
            tune = sw.sw_autotune(ctx, db_s, SC, flags=flags, repeats=2)
            assert len(tune) == sw.SW_NUM_CLASSES
            edges = [t["m_max"] for t in tune]
            assert edges == sorted(edges) and edges[-1] == 65535 and len(set(edges)) == len(edges)
            for c, t in enumerate(tune):
                assert t["blocks_per_cu"] in (1, 2, 4)
                if c < sw.SW_NUM_CLASSES - 1:
                    assert t["G"] * t["RPL"] >= t["m_max"]
                if t["path"]:
                    assert t["candidates"] >= 3
            # a choice is kept only when it measured faster than what it replaced
            # (each sum covers every pair of the sample)
            assert sum(t["ms"] for t in tune) <= 1.10 * sum(t["ms_default"] for t in tune)
            c100 = [c for c, t in enumerate(tune) if t["m_max"] >= 100][0]
            assert tune[c100]["path"] in ((1, 3) if flags == 0 else (2,))   # 100-nt reads ran
            db = sw.DeviceBatch.from_synth(ctx, b)
            hits = torch.empty((b.n_pairs, 3), dtype=torch.int32, device="cuda")
            sw.sw_batch_score(ctx, db, SC, flags, hits)
            torch.cuda.synchronize()
            ref, _ = oracle.align_batch(b, SC, mode=0)
            h = sw.hits_to_numpy(hits)
            assert (h["score"] == ref["score"]).all()
            if flags:
                assert (h["read_end"] == ref["read_end"]).all()
                assert (h["ref_end"] == ref["ref_end"]).all()
    finally:
        sw.sw_ctx_destroy(ctx)


def test_autotune_mixed_lengths_parity():
    """Reads of many lengths, so classes whose tuned tile and bounds differ
    from the default are exercised; scores stay bit-exact."""
    torch.cuda.set_device(0)
    ctx = sw.sw_ctx_create(0)
    try:
        g = np.random.default_rng(83)
        ref = g.integers(0, 4, 400_000).astype(np.uint8)
        reads, wins = [], []
        for i in range(3000):
            m = int(g.choice([20, 40, 70, 110, 140, 200, 300, 600]))
            b0 = int(g.integers(0, len(ref) - 2000))
            seg = ref[b0:b0 + m].copy()
            mut = g.random(m) < 0.03
            seg[mut] = (seg[mut] + 1) % 4
            reads.append(synth.ASCII[seg].tobytes())
            wins.append((i, max(b0 - int(g.integers(0, 200)), 0), int(g.integers(m, m + 400)), 0))
        b = synth.custom(synth.ASCII[ref].tobytes(), reads, wins)
        db = sw.DeviceBatch.from_synth(ctx, b)
        tune = sw.sw_autotune(ctx, db, SC, flags=0, repeats=1)
        # how many classes the tuned bounds keep is a timing decision (adjacent
        # classes may merge); they still hold every length of the sample
        used = [t for t in tune if t["path"]]
        assert len(used) >= 3 and max(t["m_max"] for t in used) >= 600
        hits = torch.empty((b.n_pairs, 3), dtype=torch.int32, device="cuda")
        sw.sw_batch_score(ctx, db, SC, 0, hits)
        torch.cuda.synchronize()
        r, _ = oracle.align_batch(b, SC, mode=0)
        assert (sw.hits_to_numpy(hits)["score"] == r["score"]).all()
    finally:
        sw.sw_ctx_destroy(ctx)


def _mixed(seed, n):
    g = np.random.default_rng(seed)
    ref = g.integers(0, 4, 400_000).astype(np.uint8)
    reads, wins = [], []
    for i in range(n):
        m = int(g.choice([20, 40, 50, 70, 90, 110, 140, 150, 200, 300, 600]))
        b0 = int(g.integers(0, len(ref) - 2000))
        seg = ref[b0:b0 + m].copy()
        mut = g.random(m) < 0.03
        seg[mut] = (seg[mut] + 1) % 4
        reads.append(synth.ASCII[seg].tobytes())
        for _ in range(int(g.integers(1, 5))):
            wins.append((i, max(b0 - int(g.integers(0, 200)), 0), int(g.integers(200, 800)),
                         int(g.integers(0, 2))))
    return synth.custom(synth.ASCII[ref].tobytes(), reads, wins)


def test_autotune_cache_round_trip(tmp_path):
    """The tuned choice goes to a JSON-lines cache; a fresh context with a sample
    of the same profile takes it from there without timing, and scores stay
    bit-exact under it; a damaged entry is ignored."""
    torch.cuda.set_device(0)
    path = str(tmp_path / "tune.jsonl")
    b = _mixed(91, 3000)
    ref, _ = oracle.align_batch(b, SC, mode=0)
    ctx = sw.sw_ctx_create(0)
    try:
        db = sw.DeviceBatch.from_synth(ctx, b)
        t1, hit = sw.sw_autotune_cached(ctx, db, SC, path, flags=0, repeats=1)
        assert not hit
        lines = open(path).read().splitlines()
        assert len(lines) == 1 and lines[0].startswith('{"key":"gfx950')
    finally:
        sw.sw_ctx_destroy(ctx)
    ctx = sw.sw_ctx_create(0)
    try:
        db = sw.DeviceBatch.from_synth(ctx, b)
        t2, hit = sw.sw_autotune_cached(ctx, db, SC, path, flags=0, repeats=1)
        assert hit
        for a, c in zip(t1, t2):
            assert (a["m_max"], a["G"], a["RPL"], a["blocks_per_cu"]) == \
                   (c["m_max"], c["G"], c["RPL"], c["blocks_per_cu"])
        hits = torch.empty((b.n_pairs, 3), dtype=torch.int32, device="cuda")
        sw.sw_batch_score(ctx, db, SC, 0, hits)
        torch.cuda.synchronize()
        assert (sw.hits_to_numpy(hits)["score"] == ref["score"]).all()
        # another scoring is another key; a damaged line with the key is skipped
        _, hit = sw.sw_autotune_cached(ctx, db, (2, -3, -4, -4), path, flags=0, repeats=1)
        assert not hit
        with open(path, "a") as f:
            f.write(lines[0].replace('"G":[', '"G":[99,'))
            f.write("\n")
        _, hit = sw.sw_autotune_cached(ctx, db, SC, path, flags=0, repeats=1)
        assert hit                     # the earlier valid entry still answers
    finally:
        sw.sw_ctx_destroy(ctx)
