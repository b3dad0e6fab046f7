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
            for c, t in enumerate(tune):
                assert t["blocks_per_cu"] in (1, 2, 4)
                if c < sw.SW_NUM_CLASSES - 1:
                    assert t["G"] * t["RPL"] >= t["m_max"]
                if t["path"]:
                    assert t["candidates"] >= 3 and t["ms"] <= t["ms_default"] + 1e-6
            assert tune[3]["path"] in ((1, 3) if flags == 0 else (2,))   # 100-nt reads ran
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
    """Reads of many lengths, so classes whose tuned tile differs from the
    default are exercised; scores stay bit-exact."""
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
        assert sum(1 for t in tune if t["path"]) >= 6
        hits = torch.empty((b.n_pairs, 3), dtype=torch.int32, device="cuda")
        sw.sw_batch_score(ctx, db, SC, 0, hits)
        torch.cuda.synchronize()
        r, _ = oracle.align_batch(b, SC, mode=0)
        assert (sw.hits_to_numpy(hits)["score"] == r["score"]).all()
    finally:
        sw.sw_ctx_destroy(ctx)
