"""Rules of graph capture on a context: while a captured graph is alive, no call
may move the scratch its kernels use, and the training calls (whose host-side
step count enters Adam's bias correction) cannot be captured."""
import numpy as np
import pytest
import torch

import oracle
import paper_1304_0681_amd as sw
import synth
from paper_1304_0681_amd import train as tr

pytestmark = pytest.mark.gpu

SC = (5, -4, -10, -1)


def test_live_graph_refuses_scratch_growth():
    print("graph rules: growth while a graph is alive", flush=True)
    torch.cuda.set_device(0)
    ctx = sw.sw_ctx_create(0)
    try:
        small = synth.config1(seed=synth.BASE_SEED + 81, n_reads=60)
        big = synth.config2(n_reads=20_000, seed=synth.BASE_SEED + 82)
        db, dbig = sw.DeviceBatch.from_synth(ctx, small), sw.DeviceBatch.from_synth(ctx, big)
        s = torch.cuda.Stream()
        hs = torch.empty((small.n_pairs, 3), dtype=torch.int32, device="cuda")
        hb = torch.empty((big.n_pairs, 3), dtype=torch.int32, device="cuda")
        with torch.cuda.stream(s):
            sw.sw_batch_score(ctx, db, SC, 0, hs, s)          # sizes the scratch for `small`
        s.synchronize()
        sw.sw_graph_begin(ctx, s)
        sw.sw_batch_score(ctx, db, SC, 0, hs, s)
        g = sw.sw_graph_end(ctx, s)
        try:
            with pytest.raises(sw.SwError, match="captured graph") as e:
                sw.sw_batch_score(ctx, dbig, SC, 0, hb)       # would grow the bucket scratch
            assert e.value.status == sw.SW_E_STATE
            # a larger traceback budget cannot be allocated either
            sw.sw_ctx_set_option(ctx, sw.SW_OPT_TB_SCRATCH_MB, 4096)
            ids = torch.arange(small.n_pairs, dtype=torch.int32, device="cuda")
            aln = torch.empty((small.n_pairs, 7), dtype=torch.int32, device="cuda")
            ops = torch.empty((small.n_pairs, 512), dtype=torch.int32, device="cuda")
            with pytest.raises(sw.SwError, match="captured graph"):
                sw.sw_batch_traceback(ctx, db, SC, ids, small.n_pairs, aln, ops, 512)
            sw.sw_ctx_set_option(ctx, sw.SW_OPT_TB_SCRATCH_MB, 64)
            # the graph still replays correctly on its own scratch
            hs.fill_(-5)
            sw.sw_graph_launch(ctx, g, s)
            s.synchronize()
            ref, _ = oracle.align_batch(small, SC, mode=0)
            assert (sw.hits_to_numpy(hs)["score"] == ref["score"]).all()
        finally:
            sw.sw_graph_destroy(ctx, g)
        # once the graph is gone the growing call runs
        sw.sw_batch_score(ctx, dbig, SC, 0, hb)
        torch.cuda.synchronize()
        sel = np.arange(0, big.n_pairs, 97, dtype=np.uint32)
        ref, _ = oracle.align_batch(big, SC, mode=0, sel=sel)
        assert (sw.hits_to_numpy(hb)["score"][sel] == ref["score"]).all()
    finally:
        sw.sw_ctx_destroy(ctx)


def test_training_calls_refuse_capture():
    print("graph rules: training calls under capture", flush=True)
    torch.cuda.set_device(0)
    ctx = sw.sw_ctx_create(0)
    mlp = sw.sw_mlp_create(ctx)
    try:
        sw.sw_mlp_set_params(ctx, mlp, tr.init_params(5))
        x = torch.zeros((64, 64), dtype=torch.int16, device="cuda")
        y = torch.zeros(64, dtype=torch.float32, device="cuda")
        grad = torch.empty(sw.SW_MLP_PARAMS, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        sw.sw_mlp_grad(ctx, mlp, x, y, 64, grad, loss)      # workspace sized eagerly
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        sw.sw_graph_begin(ctx, s)
        try:
            with pytest.raises(sw.SwError, match="cannot be captured"):
                sw.sw_mlp_train_step(ctx, mlp, x, y, 64, 1e-3, loss, s)
            with pytest.raises(sw.SwError, match="cannot be captured"):
                sw.sw_mlp_grad(ctx, mlp, x, y, 64, grad, loss, s)
        finally:
            try:
                sw.sw_graph_destroy(ctx, sw.sw_graph_end(ctx, s))
            except sw.SwError:
                pass
        torch.cuda.synchronize()
        # eagerly they still run
        sw.sw_mlp_train_step(ctx, mlp, x, y, 64, 1e-3, loss)
        torch.cuda.synchronize()
        assert np.isfinite(float(loss.item()))
    finally:
        sw.sw_mlp_destroy(ctx, mlp)
        sw.sw_ctx_destroy(ctx)
