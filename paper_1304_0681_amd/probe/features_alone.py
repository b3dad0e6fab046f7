"""The features kernel alone (sw_features) on the learned-filter workload: 1M
100-nt reads with exactly 16 windows of 200-600 nt each, three launches, each
timed with events.  A small program for counter runs of that one kernel:

    python3 paper_1304_0681_amd/probe/features_alone.py [n_reads]
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import torch  # noqa: E402

import paper_1304_0681_amd as sw  # noqa: E402
import synth  # noqa: E402


def main():
    n_reads = int(sys.argv[1]) if len(sys.argv) > 1 else 1_000_000
    torch.cuda.set_device(0)
    ctx = sw.sw_ctx_create(0)
    try:
        b = synth.config4(n_reads=n_reads)
        db = sw.DeviceBatch.from_synth(ctx, b)
        feat = torch.empty((b.n_pairs, 64), dtype=torch.int16, device="cuda")
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        for _ in range(3):
            ev[0].record()
            sw.sw_features(ctx, db, feat)
            ev[1].record()
            torch.cuda.synchronize()
            print("features ms", round(ev[0].elapsed_time(ev[1]), 3), flush=True)
    finally:
        sw.sw_ctx_destroy(ctx)


if __name__ == "__main__":
    main()
